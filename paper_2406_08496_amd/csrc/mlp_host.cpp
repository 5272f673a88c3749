// mlp_host.cpp -- C ABI of the surrogate perceptron kernels (include/lpsim.h).
#include <hip/hip_runtime.h>

#include <cmath>

#include "lpsim.h"
#include "mlp_dev.h"

using namespace lpsim_mlp;

static const int IN_OF[4] = {IN, HID, HID, HID};
static const int OUT_OF[4] = {HID, HID, HID, OUT};

static int32_t hip_status(hipError_t e) { return e == hipSuccess ? LPSIM_OK : LPSIM_EDEVICE; }

// the backward's launches, from the last layer to the first: weight-gradient
// partials per batch slice, their reduction in slice order, then the data
// gradient of the layer's input (ping-pong between the two halves of
// dz_scratch)
static int32_t run_backward(const uint16_t *x, const uint16_t *const *h, const uint16_t *dz_out,
                            const uint16_t *const *w, float *const *dwt, float *const *db, uint16_t *dz_scratch,
                            float *workspace, int32_t n_split, int64_t n, hipStream_t s) {
    const uint16_t *layer_in[4] = {x, h[0], h[1], h[2]};
    uint16_t *scratch[2] = {dz_scratch, dz_scratch + (size_t)n * HID};
    const uint16_t *dz = dz_out;
    int which = 0;
    for (int l = 3; l >= 0; --l) {
        MlpBwdWeightArgs wa{dz, layer_in[l], workspace, n};
        hipError_t e = launch_bwd_weight(l, wa, n_split, s);
        if (e != hipSuccess) return LPSIM_EDEVICE;
        e = launch_reduce(workspace, n_split, OUT_OF[l], IN_OF[l], dwt[l], db[l], s);
        if (e != hipSuccess) return LPSIM_EDEVICE;
        if (l == 0) break;
        MlpBwdDataArgs da{dz, w[l], layer_in[l], scratch[which], n};
        e = launch_bwd_data(l, da, s);
        if (e != hipSuccess) return LPSIM_EDEVICE;
        dz = scratch[which];
        which ^= 1;
    }
    return LPSIM_OK;
}

extern "C" {

int32_t lpsim_mlp_shape(int32_t *in_dim, int32_t *hidden, int32_t *out_dim) {
    if (in_dim) *in_dim = IN;
    if (hidden) *hidden = HID;
    if (out_dim) *out_dim = OUT;
    return LPSIM_OK;
}

int32_t lpsim_mlp_forward(const uint16_t *x, const uint16_t *const *wt, const float *const *bias, float *y,
                          uint16_t *const *h, int64_t n, void *stream) {
    if (n < 0 || !wt || !bias || (n > 0 && (!x || !y))) return LPSIM_EINVAL;
    MlpFwdArgs a{};
    a.x = x;
    for (int l = 0; l < 4; ++l) {
        if (!wt[l] || !bias[l]) return LPSIM_EINVAL;
        a.wt[l] = wt[l];
        a.b[l] = bias[l];
    }
    for (int l = 0; l < 3; ++l) a.h[l] = h ? h[l] : nullptr;
    a.y = y;
    a.n = n;
    return hip_status(launch_fwd(a, (hipStream_t)stream));
}

int32_t lpsim_mlp_loss_grad(const float *y, const float *target, const uint8_t *mask, int64_t n, float inv_count,
                            uint16_t *dz_out, float *loss_sum, void *stream) {
    if (n < 0 || (n > 0 && (!y || !target || !dz_out)) || !(inv_count >= 0.0f)) return LPSIM_EINVAL;
    if (n == 0) return LPSIM_OK;
    return hip_status(launch_mse(y, target, mask, n * OUT, inv_count, dz_out, loss_sum, (hipStream_t)stream));
}

size_t lpsim_mlp_workspace_bytes(int32_t n_split) {
    if (n_split < 1) return 0;
    return (size_t)n_split * ((size_t)HID * HID + HID) * sizeof(float);
}

int32_t lpsim_mlp_backward(const uint16_t *x, const uint16_t *const *h, const uint16_t *dz_out,
                           const uint16_t *const *w, float *const *dwt, float *const *db, uint16_t *dz_scratch,
                           float *workspace, int32_t n_split, int64_t n, void *stream) {
    if (n < 0 || n_split < 1 || n_split > 1024 || !h || !w || !dwt || !db) return LPSIM_EINVAL;
    for (int l = 0; l < 4; ++l)
        if (!w[l] || !dwt[l] || !db[l]) return LPSIM_EINVAL;
    if (n > 0 && (!x || !h[0] || !h[1] || !h[2] || !dz_out || !dz_scratch || !workspace)) return LPSIM_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    // with no rows every gradient is zero
    if (n == 0) {
        for (int l = 0; l < 4; ++l) {
            if (hipMemsetAsync(dwt[l], 0, (size_t)OUT_OF[l] * IN_OF[l] * 4, s) != hipSuccess) return LPSIM_EDEVICE;
            if (hipMemsetAsync(db[l], 0, (size_t)OUT_OF[l] * 4, s) != hipSuccess) return LPSIM_EDEVICE;
        }
        return LPSIM_OK;
    }
    return run_backward(x, h, dz_out, w, dwt, db, dz_scratch, workspace, n_split, n, s);
}

int32_t lpsim_mlp_backward_noalloc(const uint16_t *x, const uint16_t *const *h, const uint16_t *dz_out,
                                   const uint16_t *const *w, float *const *dwt, float *const *db, int32_t n_split,
                                   int64_t n, void *stream) {
    if (n < 0 || n_split < 1 || !h || !w || !dwt || !db) return LPSIM_EINVAL;
    if (n > NOALLOC_MAX_ROWS || n_split > NOALLOC_MAX_SPLIT) return LPSIM_ECAPACITY;
    for (int l = 0; l < 4; ++l)
        if (!w[l] || !dwt[l] || !db[l]) return LPSIM_EINVAL;
    if (n > 0 && (!x || !h[0] || !h[1] || !h[2] || !dz_out)) return LPSIM_EINVAL;
    void *base = nullptr;
    if (noalloc_scratch(&base) != hipSuccess) return LPSIM_EDEVICE;
    uint16_t *dz_scratch = static_cast<uint16_t *>(base);
    float *workspace = reinterpret_cast<float *>(static_cast<unsigned char *>(base) + NOALLOC_DZ_BYTES);
    // with no rows the kernels write zero partials and zero gradients (no
    // memset nodes, so the call can be captured in a graph)
    return run_backward(x, h, dz_out, w, dwt, db, dz_scratch, workspace, n_split, n, (hipStream_t)stream);
}

int32_t lpsim_mlp_adam(float *w, uint16_t *wt_bf16, uint16_t *w_bf16, const float *grad, float *m, float *v,
                       int32_t rows, int32_t cols, float lr, float beta1, float beta2, float eps, int32_t t,
                       void *stream) {
    if (!w || !grad || !m || !v || rows < 1 || cols < 1 || t < 1 || !(lr >= 0.0f) || !(beta1 >= 0.0f) ||
        !(beta1 < 1.0f) || !(beta2 >= 0.0f) || !(beta2 < 1.0f) || !(eps > 0.0f))
        return LPSIM_EINVAL;
    const float c1 = (float)(1.0 - std::pow((double)beta1, (double)t));
    const float c2 = (float)(1.0 - std::pow((double)beta2, (double)t));
    return hip_status(launch_adam(w, wt_bf16, w_bf16, grad, m, v, rows, cols, lr, beta1, beta2, eps, c1, c2,
                                  (hipStream_t)stream));
}

}  // extern "C"
