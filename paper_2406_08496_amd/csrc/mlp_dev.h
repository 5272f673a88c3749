// mlp_dev.h -- shapes and kernel arguments of the surrogate perceptron.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lpsim_mlp {

constexpr int IN = 32;    // input features (padded)
constexpr int HID = 256;  // hidden width, three hidden layers
constexpr int OUT = 16;   // outputs (padded)
constexpr int TM = 64;    // rows per workgroup of the forward (2 waves per SIMD; 128 rows gave 1)
constexpr int LDX = IN + 8;    // LDS row pitch (bf16) of the input tile
constexpr int LDH = HID + 8;   // LDS row pitch of a hidden tile (bank spread)

struct MlpFwdArgs {
    const uint16_t *x;      // [n][IN] bf16
    const uint16_t *wt[4];  // layer l: [out_l][in_l] bf16
    const float *b[4];      // layer l: [out_l]
    float *y;               // [n][OUT]
    uint16_t *h[3];         // hidden activations [n][HID] bf16, or null
    int64_t n;
};

struct MlpBwdDataArgs {
    const uint16_t *dz;      // [n][N] bf16, gradient at this layer's output
    const uint16_t *w;       // [K][N] bf16 ("in x out")
    const uint16_t *h_prev;  // [n][K] bf16, this layer's input (ReLU output)
    uint16_t *dz_prev;       // [n][K] bf16
    int64_t n;
};

struct MlpBwdWeightArgs {
    const uint16_t *dz;  // [n][N] bf16
    const uint16_t *h;   // [n][K] bf16, layer input
    float *ws;           // [splits][N*K + N] partial sums
    int64_t n;
};

// Limits of the allocation-free backward (lpsim_mlp_backward_noalloc): its
// data-gradient buffers (2 x rows x HID bfloat16) and weight-gradient
// partials (slices x (HID x HID + HID) binary32) live in one static device
// array of NOALLOC_SCRATCH_BYTES (24.1 MiB) per GPU.
constexpr int64_t NOALLOC_MAX_ROWS = 8192;
constexpr int NOALLOC_MAX_SPLIT = 64;
constexpr size_t NOALLOC_DZ_BYTES = 2 * (size_t)NOALLOC_MAX_ROWS * HID * sizeof(uint16_t);
constexpr size_t NOALLOC_SCRATCH_BYTES =
    NOALLOC_DZ_BYTES + (size_t)NOALLOC_MAX_SPLIT * ((size_t)HID * HID + HID) * sizeof(float);

// device address of this GPU's static scratch array (looked up once per
// device, with that device current)
hipError_t noalloc_scratch(void **out);

hipError_t launch_fwd(const MlpFwdArgs &a, hipStream_t s);
hipError_t launch_bwd_data(int layer, const MlpBwdDataArgs &a, hipStream_t s);
hipError_t launch_bwd_weight(int layer, const MlpBwdWeightArgs &a, int n_split, hipStream_t s);
hipError_t launch_reduce(const float *ws, int n_split, int nn, int nk, float *dwt, float *db, hipStream_t s);
hipError_t launch_mse(const float *y, const float *t, const uint8_t *mask, int64_t n_elem, float inv_count,
                      uint16_t *dz, float *loss_sum, hipStream_t s);
hipError_t launch_adam(float *w, uint16_t *wt_bf, uint16_t *w_bf, const float *g, float *m, float *v, int rows,
                       int cols, float lr, float b1, float b2, float eps, float c1, float c2, hipStream_t s);

}  // namespace lpsim_mlp
