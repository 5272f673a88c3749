// mlp_host.cpp -- C ABI of the surrogate perceptron kernels (include/lpsim.h).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "lpsim.h"
#include "mlp_dev.h"

using namespace lpsim_mlp;

static int32_t hip_status(hipError_t e) { return e == hipSuccess ? LPSIM_OK : LPSIM_EDEVICE; }

static bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

// the backward's arguments, its workspace carved as mlp_dev.h lays it out
static MlpBwdArgs bwd_args(const uint16_t *x, const uint16_t *const *h, const uint16_t *dz_out,
                           const uint16_t *const *w, float *const *dwt, float *const *db, void *workspace,
                           int32_t n_split, int64_t n) {
    MlpBwdArgs a{};
    const int64_t rows = padded_rows(n);
    uint16_t *act = static_cast<uint16_t *>(workspace);
    a.x = x;
    for (int l = 0; l < 3; ++l) a.hT[l] = h[l];
    a.dz_out = dz_out;
    for (int l = 0; l < 4; ++l) {
        a.w[l] = w[l];
        a.dwt[l] = dwt[l];
        a.db[l] = db[l];
    }
    a.dzT[3] = act;
    a.dzT[2] = act + (size_t)OUT * rows;
    a.dzT[1] = act + (size_t)(OUT + HID) * rows;
    a.dzT[0] = act + (size_t)(OUT + 2 * HID) * rows;
    a.xT = act + (size_t)(OUT + 3 * HID) * rows;
    a.part = reinterpret_cast<float *>(static_cast<unsigned char *>(workspace) + bwd_act_bytes(rows));
    a.n = n;
    a.rows = rows;
    a.n_split = n_split;
    return a;
}

// arguments shared by both backward entry points
static int32_t check_bwd(const uint16_t *x, const uint16_t *const *h, const uint16_t *dz_out,
                         const uint16_t *const *w, float *const *dwt, float *const *db, int32_t n_split, int64_t n) {
    if (n < 0 || n_split < 1 || !h || !w || !dwt || !db) return LPSIM_EINVAL;
    for (int l = 0; l < 4; ++l)
        if (!w[l] || !dwt[l] || !db[l] || !aligned16(w[l])) return LPSIM_EINVAL;
    if (n > 0) {
        if (!x || !dz_out || !aligned16(x) || !aligned16(dz_out)) return LPSIM_EINVAL;
        for (int l = 0; l < 3; ++l)
            if (!h[l] || !aligned16(h[l])) return LPSIM_EINVAL;
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
    if (n < 0 || !wt || !bias || (n > 0 && (!x || !y || !aligned16(x)))) return LPSIM_EINVAL;
    MlpFwdArgs a{};
    a.x = x;
    for (int l = 0; l < 4; ++l) {
        if (!wt[l] || !bias[l]) return LPSIM_EINVAL;
        a.wt[l] = wt[l];
        a.b[l] = bias[l];
    }
    for (int l = 0; l < 3; ++l) {
        a.h[l] = h ? h[l] : nullptr;
        if (h && n > 0 && (!h[l] || !aligned16(h[l]))) return LPSIM_EINVAL;
    }
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

size_t lpsim_mlp_workspace_bytes(int64_t n, int32_t n_split) {
    if (n < 0 || n_split < 1 || n_split > 1024) return 0;
    return bwd_workspace_bytes(n, n_split);
}

int32_t lpsim_mlp_backward(const uint16_t *x, const uint16_t *const *h, const uint16_t *dz_out,
                           const uint16_t *const *w, float *const *dwt, float *const *db, void *workspace,
                           int32_t n_split, int64_t n, void *stream) {
    int32_t rc = check_bwd(x, h, dz_out, w, dwt, db, n_split, n);
    if (rc != LPSIM_OK) return rc;
    if (n_split > 1024 || !workspace || !aligned16(workspace)) return LPSIM_EINVAL;
    // with no rows the kernels write zero partials and zero gradients
    return hip_status(launch_bwd(bwd_args(x, h, dz_out, w, dwt, db, workspace, n_split, n), (hipStream_t)stream));
}

int32_t lpsim_mlp_backward_noalloc(const uint16_t *x, const uint16_t *const *h, const uint16_t *dz_out,
                                   const uint16_t *const *w, float *const *dwt, float *const *db, int32_t n_split,
                                   int64_t n, void *stream) {
    int32_t rc = check_bwd(x, h, dz_out, w, dwt, db, n_split, n);
    if (rc != LPSIM_OK) return rc;
    if (n > NOALLOC_MAX_ROWS || n_split > NOALLOC_MAX_SPLIT) return LPSIM_ECAPACITY;
    void *base = nullptr;
    if (noalloc_scratch(&base) != hipSuccess) return LPSIM_EDEVICE;
    return hip_status(launch_bwd(bwd_args(x, h, dz_out, w, dwt, db, base, n_split, n), (hipStream_t)stream));
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
