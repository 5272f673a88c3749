// mlp_kernels.hip -- the edge travel-time surrogate: a 4-layer perceptron
// (32 -> 256 -> 256 -> 256 -> 16, ReLU on the hidden layers) on gfx950 matrix
// cores.  Operands are bfloat16, accumulation is binary32
// (v_mfma_f32_16x16x32_bf16); hidden activations are rounded to bfloat16
// (round to nearest even) once, after bias and ReLU.
//
// Weight layouts: "wt" = [out][in] (rows contiguous along the input), used by
// the forward pass; "w" = [in][out], used by the backward data pass.  The
// optimizer keeps both bfloat16 copies in step with the binary32 master.
//
// MFMA 16x16x32 lane layout (64 lanes, l = lane): the A operand of lane l is
// row l%16, columns 8*(l/16) .. +7; the B operand is column l%16, rows
// 8*(l/16) .. +7; the result element i of lane l is row 4*(l/16)+i, column
// l%16.  Every fragment is therefore one contiguous 16-byte load when the
// contraction index is the fastest-varying one in memory.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "mlp_dev.h"

namespace lpsim_mlp {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f) {
    // round to nearest, ties to even (values here are finite)
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ bf16x8 frag(const uint16_t *p) {
    const uint4 u = *reinterpret_cast<const uint4 *>(p);
    return __builtin_bit_cast(bf16x8, u);
}

__device__ __forceinline__ bf16x8 zero_frag() { return __builtin_bit_cast(bf16x8, make_uint4(0, 0, 0, 0)); }

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// forward

// hidden layer on a tile of TM rows: out = bf16(relu(A Wt^T + bias)), N = HID.
// Wave w owns output column blocks 4w..4w+3 for all TM/16 row blocks.
template <int K>
__device__ __forceinline__ void hidden_layer(const uint16_t *A, int lda, const uint16_t *__restrict__ wt,
                                             const float *__restrict__ bias, uint16_t *out, int ldo,
                                             uint16_t *__restrict__ out_g, int64_t row0, int64_t n) {
    constexpr int RB = TM / 16, CB = HID / 16 / 4;
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int r16 = l & 15, kq = (l >> 4) * 8;
    f32x4 acc[RB][CB];
    for (int rb = 0; rb < RB; ++rb)
        for (int cb = 0; cb < CB; ++cb) acc[rb][cb] = f32x4{0.f, 0.f, 0.f, 0.f};
    // weight fragments come from L2; the next k-step's are loaded while the
    // current step's products run
    bf16x8 b[CB];
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) b[cb] = frag(wt + (size_t)((w * CB + cb) * 16 + r16) * K + kq);
#pragma unroll
    for (int k0 = 0; k0 < K; k0 += 32) {
        bf16x8 bn[CB];
        if (k0 + 32 < K) {
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) bn[cb] = frag(wt + (size_t)((w * CB + cb) * 16 + r16) * K + k0 + 32 + kq);
        }
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            const bf16x8 a = frag(A + (rb * 16 + r16) * lda + k0 + kq);
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) acc[rb][cb] = mfma(a, b[cb], acc[rb][cb]);
        }
        if (k0 + 32 < K) {
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) b[cb] = bn[cb];
        }
    }
    for (int cb = 0; cb < CB; ++cb) {
        const int col = (w * CB + cb) * 16 + r16;
        const float bc = bias[col];
        for (int rb = 0; rb < RB; ++rb) {
            for (int i = 0; i < 4; ++i) {
                const int row = rb * 16 + (l >> 4) * 4 + i;
                const float z = acc[rb][cb][i] + bc;
                const uint16_t h = f2bf(z > 0.0f ? z : 0.0f);
                out[row * ldo + col] = h;
                if (out_g && row0 + row < n) out_g[(size_t)(row0 + row) * HID + col] = h;
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_mlp_fwd(MlpFwdArgs a) {
    __shared__ __attribute__((aligned(16))) uint16_t xs[TM * LDX];
    __shared__ __attribute__((aligned(16))) uint16_t hs0[TM * LDH];
    __shared__ __attribute__((aligned(16))) uint16_t hs1[TM * LDH];
    const int64_t row0 = (int64_t)blockIdx.x * TM;
    // stage the input tile (rows past n are zero)
    for (int c = threadIdx.x; c < TM * IN / 8; c += blockDim.x) {
        const int r = c / (IN / 8), q = (c % (IN / 8)) * 8;
        uint4 v = make_uint4(0, 0, 0, 0);
        if (row0 + r < a.n) v = *reinterpret_cast<const uint4 *>(a.x + (size_t)(row0 + r) * IN + q);
        *reinterpret_cast<uint4 *>(xs + r * LDX + q) = v;
    }
    __syncthreads();
    hidden_layer<IN>(xs, LDX, a.wt[0], a.b[0], hs0, LDH, a.h[0], row0, a.n);
    __syncthreads();
    hidden_layer<HID>(hs0, LDH, a.wt[1], a.b[1], hs1, LDH, a.h[1], row0, a.n);
    __syncthreads();
    hidden_layer<HID>(hs1, LDH, a.wt[2], a.b[2], hs0, LDH, a.h[2], row0, a.n);
    __syncthreads();
    // output layer: N = OUT = 16, one column block; wave w owns row blocks 2w, 2w+1
    {
        const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
        const int r16 = l & 15, kq = (l >> 4) * 8;
        constexpr int RBW = TM / 16 / 4;
        f32x4 acc[RBW];
        for (int j = 0; j < RBW; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
        for (int k0 = 0; k0 < HID; k0 += 32) {
            const bf16x8 b = frag(a.wt[3] + (size_t)r16 * HID + k0 + kq);
            for (int j = 0; j < RBW; ++j) {
                const int rb = w * RBW + j;
                acc[j] = mfma(frag(hs0 + (rb * 16 + r16) * LDH + k0 + kq), b, acc[j]);
            }
        }
        const float bc = a.b[3][r16];
        for (int j = 0; j < RBW; ++j) {
            for (int i = 0; i < 4; ++i) {
                const int row = (w * RBW + j) * 16 + (l >> 4) * 4 + i;
                if (row0 + row < a.n) a.y[(size_t)(row0 + row) * OUT + r16] = acc[j][i] + bc;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// backward, data part: dz_prev = bf16(relu'(h_prev) * (dz @ W)), where W is
// [K][N] ("in x out") so that the contraction over N is contiguous.
// NC = contraction width padded to a multiple of 32.

// rows per tile of the data-gradient kernel: its accumulators take TMD / 4
// f32x4 per wave, which sets its occupancy (32 rows: 5 waves per SIMD,
// faster than 64 or 128 rows)
constexpr int TMD = 32;

template <int N, int K>
__global__ __launch_bounds__(256) void k_mlp_bwd_data(MlpBwdDataArgs a) {
    constexpr int NC = (N + 31) / 32 * 32;
    constexpr int LDZ = NC + 8;
    constexpr int RB = TMD / 16, CB = K / 16 / 4;
    __shared__ __attribute__((aligned(16))) uint16_t zs[TMD * LDZ];
    const int64_t row0 = (int64_t)blockIdx.x * TMD;
    for (int c = threadIdx.x; c < TMD * NC / 8; c += blockDim.x) {
        const int r = c / (NC / 8), q = (c % (NC / 8)) * 8;
        uint4 v = make_uint4(0, 0, 0, 0);
        if (row0 + r < a.n && q < N) v = *reinterpret_cast<const uint4 *>(a.dz + (size_t)(row0 + r) * N + q);
        *reinterpret_cast<uint4 *>(zs + r * LDZ + q) = v;
    }
    __syncthreads();
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int r16 = l & 15, kq = (l >> 4) * 8;
    // the loops over the accumulator tiles are unrolled so that acc stays in
    // registers (a rolled loop indexes it dynamically and puts it in scratch)
    f32x4 acc[RB][CB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) acc[rb][cb] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < NC; k0 += 32) {
        bf16x8 b[CB];
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
            const int col = (w * CB + cb) * 16 + r16;
            b[cb] = (k0 + kq < N) ? frag(a.w + (size_t)col * N + k0 + kq) : zero_frag();
        }
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            const bf16x8 av = frag(zs + (rb * 16 + r16) * LDZ + k0 + kq);
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) acc[rb][cb] = mfma(av, b[cb], acc[rb][cb]);
        }
    }
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
        const int col = (w * CB + cb) * 16 + r16;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int64_t row = row0 + rb * 16 + (l >> 4) * 4 + i;
                if (row >= a.n) continue;
                const uint16_t hp = a.h_prev[(size_t)row * K + col];
                const bool live = hp != 0 && !(hp & 0x8000u);  // relu output > 0
                a.dz_prev[(size_t)row * K + col] = f2bf(live ? acc[rb][cb][i] : 0.0f);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// rows per staging chunk of the weight-gradient kernel (a multiple of 32)
constexpr int WG_ROWS = 32;

// backward, weight part: partial dwt[n][k] = sum over a batch slice of
// dz[m][n] * h[m][k], and partial db[n] = sum dz[m][n].  Chunks of WG_ROWS
// rows are read with 16-byte loads and stored transposed in LDS, so both MFMA
// operands are contiguous along m; the next chunk is loaded into registers
// while the current one is multiplied.  Block tile: TN (n) x TK (k); its
// 16 x 16 output blocks are dealt evenly to the four waves, and each output
// element is summed by one MFMA chain in chunk order.

template <int N, int K>
__global__ __launch_bounds__(256) void k_mlp_bwd_weight(MlpBwdWeightArgs a) {
    constexpr int TN = N < 64 ? N : 64, TK = K < 64 ? K : 64;
    constexpr int MC = WG_ROWS, LT = MC + 8;
    static_assert(MC % 32 == 0, "chunks of whole MFMA steps");
    constexpr int NB = TN / 16, KB = TK / 16, PER_WAVE = NB * KB / 4;
    static_assert(NB * KB % 4 == 0 && PER_WAVE <= 4, "tile must split over four waves");
    constexpr int VP = MC * TN / 8, VQ = MC * TK / 8;  // 16-byte vectors per chunk
    constexpr int NVP = (VP + 255) / 256, NVQ = (VQ + 255) / 256;
    __shared__ __attribute__((aligned(16))) uint16_t pt[TN * LT];  // dz^T tile [n][m]
    __shared__ __attribute__((aligned(16))) uint16_t qt[TK * LT];  // h^T tile [k][m]
    constexpr int n_tiles_k = K / TK;
    const int tile = blockIdx.x;
    const int nt = tile / n_tiles_k, kt = tile % n_tiles_k;
    const int n0 = nt * TN, k0 = kt * TK;
    const int split = blockIdx.y, n_split = gridDim.y;
    const int64_t per = ((a.n + n_split - 1) / n_split + 31) / 32 * 32;
    const int64_t m_lo = per * split, m_hi = m_lo + per < a.n ? m_lo + per : a.n;
    const int t = threadIdx.x;
    const int l = t & 63, w = t >> 6;
    const int r16 = l & 15, mq = (l >> 4) * 8;
    uint4 vp[NVP], vq[NVQ];
    auto load = [&](int64_t m0) {
#pragma unroll
        for (int u = 0; u < NVP; ++u) {
            const int v = t + 256 * u, m = v / (TN / 8), c = (v % (TN / 8)) * 8;
            vp[u] = make_uint4(0, 0, 0, 0);
            if (v < VP && m0 + m < m_hi) vp[u] = *reinterpret_cast<const uint4 *>(a.dz + (size_t)(m0 + m) * N + n0 + c);
        }
#pragma unroll
        for (int u = 0; u < NVQ; ++u) {
            const int v = t + 256 * u, m = v / (TK / 8), c = (v % (TK / 8)) * 8;
            vq[u] = make_uint4(0, 0, 0, 0);
            if (v < VQ && m0 + m < m_hi) vq[u] = *reinterpret_cast<const uint4 *>(a.h + (size_t)(m0 + m) * K + k0 + c);
        }
    };
    f32x4 acc[PER_WAVE];
#pragma unroll
    for (int j = 0; j < PER_WAVE; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
    float dbias = 0.f;
    if (m_lo < m_hi) load(m_lo);
    for (int64_t m0 = m_lo; m0 < m_hi; m0 += MC) {
        __syncthreads();  // the previous chunk's fragments have been read
#pragma unroll
        for (int u = 0; u < NVP; ++u) {
            const int v = t + 256 * u, m = v / (TN / 8), c = (v % (TN / 8)) * 8;
            const uint32_t wv[4] = {vp[u].x, vp[u].y, vp[u].z, vp[u].w};
            if (v < VP)
                for (int j = 0; j < 8; ++j) pt[(c + j) * LT + m] = (uint16_t)(wv[j >> 1] >> (16 * (j & 1)));
        }
#pragma unroll
        for (int u = 0; u < NVQ; ++u) {
            const int v = t + 256 * u, m = v / (TK / 8), c = (v % (TK / 8)) * 8;
            const uint32_t wv[4] = {vq[u].x, vq[u].y, vq[u].z, vq[u].w};
            if (v < VQ)
                for (int j = 0; j < 8; ++j) qt[(c + j) * LT + m] = (uint16_t)(wv[j >> 1] >> (16 * (j & 1)));
        }
        __syncthreads();
        if (m0 + MC < m_hi) load(m0 + MC);
        // 32-row MFMA steps in increasing m: each element's sum keeps the row order
#pragma unroll
        for (int ms = 0; ms < MC; ms += 32)
#pragma unroll
            for (int j = 0; j < PER_WAVE; ++j) {
                const int b = w * PER_WAVE + j, nb = b / KB, kb = b % KB;
                acc[j] = mfma(frag(pt + (nb * 16 + r16) * LT + ms + mq), frag(qt + (kb * 16 + r16) * LT + ms + mq),
                              acc[j]);
            }
        if (kt == 0 && t < TN)
            for (int m = 0; m < MC; ++m) dbias += bf2f(pt[t * LT + m]);
    }
    float *part = a.ws + (size_t)split * (N * K + N);
#pragma unroll
    for (int j = 0; j < PER_WAVE; ++j) {
        const int b = w * PER_WAVE + j, nb = b / KB, kb = b % KB;
        for (int i = 0; i < 4; ++i) {
            const int nn = n0 + nb * 16 + (l >> 4) * 4 + i, kk = k0 + kb * 16 + r16;
            part[(size_t)nn * K + kk] = acc[j][i];
        }
    }
    if (kt == 0 && t < TN) part[N * K + n0 + t] = dbias;
}

// deterministic sum of the split partials
__global__ void k_mlp_reduce(const float *ws, int n_split, int n_elem, int stride, float *dwt, float *db, int nk) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_elem; i += gridDim.x * blockDim.x) {
        float s = 0.f;
        for (int p = 0; p < n_split; ++p) s += ws[(size_t)p * stride + i];
        if (i < nk) dwt[i] = s;
        else db[i - nk] = s;
    }
}

// ---------------------------------------------------------------------------
// loss: masked mean squared error; dy = 2 (y - t) mask / count, dz = bf16(dy)

__global__ void k_mlp_mse(const float *y, const float *t, const uint8_t *mask, int64_t n_elem, float inv_count,
                          uint16_t *dz, float *loss_sum) {
    float local = 0.f;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_elem; i += (int64_t)gridDim.x * blockDim.x) {
        float g = 0.f;
        if (!mask || mask[i]) {
            const float d = y[i] - t[i];
            g = (2.0f * d) * inv_count;
            local += (d * d) * inv_count;
        }
        dz[i] = f2bf(g);
    }
    if (loss_sum) {
        for (int off = 32; off > 0; off >>= 1) local += __shfl_down(local, off);
        if ((threadIdx.x & 63) == 0 && local != 0.f) atomicAdd(loss_sum, local);
    }
}

// ---------------------------------------------------------------------------
// Adam on one weight matrix of shape [rows][cols] ("wt" layout), bias vectors
// with rows = 1.  Updates the binary32 master and both bfloat16 copies.

__global__ void k_mlp_adam(float *w, uint16_t *wt_bf, uint16_t *w_bf, const float *g, float *m, float *v,
                           int rows, int cols, float lr, float b1, float b2, float eps, float c1, float c2) {
    const int n = rows * cols;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * (gi * gi);
        m[i] = mi;
        v[i] = vi;
        const float mh = mi / c1, vh = vi / c2;
        const float wi = w[i] - lr * (mh / (sqrtf(vh) + eps));
        w[i] = wi;
        const uint16_t hb = f2bf(wi);
        if (wt_bf) wt_bf[i] = hb;
        if (w_bf) {
            const int r = i / cols, c = i % cols;
            w_bf[(size_t)c * rows + r] = hb;
        }
    }
}

// ---------------------------------------------------------------------------

hipError_t launch_fwd(const MlpFwdArgs &a, hipStream_t s) {
    const unsigned g = (unsigned)((a.n + TM - 1) / TM);
    if (g) hipLaunchKernelGGL(k_mlp_fwd, dim3(g), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_bwd_data(int layer, const MlpBwdDataArgs &a, hipStream_t s) {
    const unsigned g = (unsigned)((a.n + TMD - 1) / TMD);
    if (!g) return hipSuccess;
    if (layer == 3) hipLaunchKernelGGL((k_mlp_bwd_data<OUT, HID>), dim3(g), dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_mlp_bwd_data<HID, HID>), dim3(g), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_bwd_weight(int layer, const MlpBwdWeightArgs &a, int n_split, hipStream_t s) {
    if (layer == 3) {
        hipLaunchKernelGGL((k_mlp_bwd_weight<OUT, HID>), dim3((OUT / 16) * (HID / 64), n_split), dim3(256), 0, s, a);
    } else if (layer == 0) {
        hipLaunchKernelGGL((k_mlp_bwd_weight<HID, IN>), dim3((HID / 64) * (IN / 32), n_split), dim3(256), 0, s, a);
    } else {
        hipLaunchKernelGGL((k_mlp_bwd_weight<HID, HID>), dim3((HID / 64) * (HID / 64), n_split), dim3(256), 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_reduce(const float *ws, int n_split, int nn, int nk, float *dwt, float *db, hipStream_t s) {
    const int n_elem = nn * nk + nn;
    hipLaunchKernelGGL(k_mlp_reduce, dim3((n_elem + 255) / 256), dim3(256), 0, s, ws, n_split, n_elem,
                       nn * nk + nn, dwt, db, nn * nk);
    return hipGetLastError();
}

hipError_t launch_mse(const float *y, const float *t, const uint8_t *mask, int64_t n_elem, float inv_count,
                      uint16_t *dz, float *loss_sum, hipStream_t s) {
    const int64_t blocks = (n_elem + 255) / 256;
    const unsigned g = (unsigned)(blocks < 4096 ? (blocks > 0 ? blocks : 1) : 4096);
    hipLaunchKernelGGL(k_mlp_mse, dim3(g), dim3(256), 0, s, y, t, mask, n_elem, inv_count, dz, loss_sum);
    return hipGetLastError();
}

hipError_t launch_adam(float *w, uint16_t *wt_bf, uint16_t *w_bf, const float *g, float *m, float *v, int rows,
                       int cols, float lr, float b1, float b2, float eps, float c1, float c2, hipStream_t s) {
    const int n = rows * cols;
    const unsigned grid = (unsigned)((n + 255) / 256 < 2048 ? (n + 255) / 256 : 2048);
    hipLaunchKernelGGL(k_mlp_adam, dim3(grid ? grid : 1), dim3(256), 0, s, w, wt_bf, w_bf, g, m, v, rows, cols, lr,
                       b1, b2, eps, c1, c2);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// static scratch of the allocation-free backward.  In host code the array's
// name stands for no device address: host code only ever uses the address
// that hipGetSymbolAddress returns for the current device.

static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
void *scratch_ptr[MAX_DEVICES] = {};
}  // namespace

hipError_t noalloc_scratch(void **out) {
    *out = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        scratch_ptr[dev] = p;
    }
    *out = scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace lpsim_mlp
