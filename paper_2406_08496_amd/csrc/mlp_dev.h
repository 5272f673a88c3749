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

// Fragment order.  The MFMA operand fragment of lane L (0..63) holds, for
// one 16-wide block of a matrix's non-contracted index ("feature" f) and one
// 32-long step of its contracted index ("row" r), feature f0 + L % 16 at rows
// 32 s + 8 (L / 16) .. +7.  Matrices that feed the matrix cores from memory
// are stored in that order, one 512-element (1 KiB) block per (step,
// feature block), blocks row-step-major:
//   (r, f) -> ((r / 32) * (C / 16) + f / 16) * 512 + (f % 16 + 16 ((r % 32) / 8)) * 8 + r % 8
// for C features.  A fragment is then one contiguous 1 KiB read, 16 bytes
// per lane in lane order, which the load path serves at full rate; in
// row-major order a fragment's lanes fall on 16 different lines and load
// several times slower.  Activations and gradients keep padded_rows(n)
// rows (a multiple of 64, the forward's tile); rows n .. padded_rows(n)-1
// hold finite values and meet zero gradients.
constexpr int PANEL = 64;
__host__ __device__ constexpr int64_t padded_rows(int64_t n) { return (n + PANEL - 1) / PANEL * PANEL; }
template <int C>
__device__ __forceinline__ size_t fo(int64_t r, int f) {
    return ((size_t)(r >> 5) * (C >> 4) + (size_t)(f >> 4)) * 512 + (size_t)(((f & 15) + 16 * ((int)(r & 31) >> 3)) * 8) +
           (size_t)(r & 7);
}
// first element of the block of features f0 .. f0+15 (f0 % 16 == 0), step s
template <int C>
__device__ __forceinline__ size_t fo_block(int64_t s, int f0) {
    return ((size_t)s * (C >> 4) + (size_t)(f0 >> 4)) * 512;
}

struct MlpFwdArgs {
    const uint16_t *x;      // [n][IN] bf16
    const uint16_t *wt[4];  // layer l: fragment order, rows in_l, features out_l, bf16
    const float *b[4];      // layer l: [out_l]
    float *y;               // [n][OUT]
    uint16_t *h[3];         // hidden activations, fragment order (HID features) bf16, or null
    int64_t n;
};

// Parameters in one flat binary32 vector, layer by layer: dwt_l ([out][in])
// then db_l.  The weight-gradient partials of one batch slice use this layout.
constexpr int PAR_W[4] = {0, IN * HID + HID, IN * HID + HID + HID * HID + HID,
                          IN * HID + HID + 2 * (HID * HID + HID)};
constexpr int PAR_COUNT = IN * HID + HID + 2 * (HID * HID + HID) + HID * OUT + OUT;  // 144,144

// The backward's workspace, carved from one caller (or static) buffer: the
// output gradients of the output layer (OUT features) and of the three hidden
// layers (HID features each) and the input x (IN features), all in fragment
// order, bf16, then n_split x PAR_COUNT binary32 partials.
struct MlpBwdArgs {
    const uint16_t *x;       // [n][IN] bf16
    const uint16_t *hT[3];   // forward's hidden activations, fragment order
    const uint16_t *dz_out;  // [n][OUT] bf16
    const uint16_t *w[4];    // layer l: fragment order, rows out_l (padded to 32), features in_l
    uint16_t *dzT[4];        // layer l's output gradient, fragment order
    uint16_t *xT;            // x, fragment order
    float *part;             // [n_split][PAR_COUNT]
    float *dwt[4];           // results, [out_l][in_l]
    float *db[4];
    int64_t n, rows;         // rows: padded_rows(n)
    int n_split;
};

inline size_t bwd_act_bytes(int64_t rows) { return (size_t)(OUT + 3 * HID + IN) * (size_t)rows * sizeof(uint16_t); }
inline size_t bwd_workspace_bytes(int64_t n, int n_split) {
    return bwd_act_bytes(padded_rows(n)) + (size_t)n_split * PAR_COUNT * sizeof(float);
}

// Limits of the allocation-free backward (lpsim_mlp_backward_noalloc): its
// workspace for NOALLOC_MAX_ROWS rows and NOALLOC_MAX_SPLIT slices lives in
// one static device array of NOALLOC_SCRATCH_BYTES (30.3 MiB) per GPU.
constexpr int64_t NOALLOC_MAX_ROWS = 8192;
constexpr int NOALLOC_MAX_SPLIT = 32;
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)(OUT + 3 * HID + IN) * NOALLOC_MAX_ROWS * sizeof(uint16_t) +
                                         (size_t)NOALLOC_MAX_SPLIT * PAR_COUNT * sizeof(float);

// device address of this GPU's static scratch array (looked up once per
// device, with that device current)
hipError_t noalloc_scratch(void **out);

hipError_t launch_fwd(const MlpFwdArgs &a, hipStream_t s);
hipError_t launch_bwd(const MlpBwdArgs &a, hipStream_t s);
hipError_t launch_mse(const float *y, const float *t, const uint8_t *mask, int64_t n_elem, float inv_count,
                      uint16_t *dz, float *loss_sum, hipStream_t s);
hipError_t launch_adam(float *w, uint16_t *wt_bf, uint16_t *w_bf, const float *g, float *m, float *v, int rows,
                       int cols, float lr, float b1, float b2, float eps, float c1, float c2, hipStream_t s);

}  // namespace lpsim_mlp
