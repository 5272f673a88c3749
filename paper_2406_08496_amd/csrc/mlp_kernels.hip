// mlp_kernels.hip -- the edge travel-time surrogate: a 4-layer perceptron
// (32 -> 256 -> 256 -> 256 -> 16, ReLU on the hidden layers) on gfx950 matrix
// cores.  Operands are bfloat16, accumulation is binary32
// (v_mfma_f32_16x16x32_bf16); hidden activations are rounded to bfloat16
// (round to nearest even) once, after bias and ReLU.
//
// Weights: the binary32 master is [out][in].  The matrix cores read two
// bfloat16 copies in fragment order (mlp_dev.h): "wt" with rows = in
// (contracted by the forward) and features = out, "w" with rows = out
// (contracted by the backward data pass, padded to 32 with zeros) and
// features = in.  The optimizer keeps both copies in step with the master.
//
// MFMA 16x16x32 lane layout (64 lanes, l = lane): the A operand of lane l is
// row l%16, columns 8*(l/16) .. +7; the B operand is column l%16, rows
// 8*(l/16) .. +7; the result element i of lane l is row 4*(l/16)+i, column
// l%16.  An operand read from a row-major tile in LDS is one 16-byte read per
// lane; one read from global memory comes from a fragment-order array, 16
// bytes per lane in lane order.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "mlp_dev.h"

namespace lpsim_mlp {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int TMC_MAX = 64;  // largest row tile of the data-gradient chain

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

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// forward

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// two binary32 values rounded to bfloat16 (nearest even; one instruction on
// gfx950), packed low-first
__device__ __forceinline__ uint32_t pack_bf16(float lo, float hi) {
    const bf16x2 v = {(__bf16)lo, (__bf16)hi};
    return __builtin_bit_cast(uint32_t, v);
}

// hidden layer on a tile of TM rows: out = bf16(relu(A W^T + bias)), N = HID,
// computed transposed (out^T = W A^T: the weights are the MFMA's A operand,
// the activation tile its B operand) so that each lane's four results are
// four consecutive units of one row, written to LDS as one 8-byte store.
// Wave w owns units 64 w .. 64 w + 63 for all TM/16 row blocks.  With
// IN_PLACE the output overwrites the input tile once every wave has read it.
template <int K, bool IN_PLACE>
__device__ __forceinline__ void hidden_layer(const uint16_t *A, int lda, const uint16_t *__restrict__ wt,
                                             const float *__restrict__ bias, uint16_t *out, int ldo,
                                             uint16_t *__restrict__ out_g, int64_t row0) {
    constexpr int RB = TM / 16, FB = HID / 16 / 4;
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int r16 = l & 15, g = l >> 4, kq = g * 8;
    f32x4 acc[FB][RB];
#pragma unroll
    for (int fb = 0; fb < FB; ++fb)
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) acc[fb][rb] = f32x4{0.f, 0.f, 0.f, 0.f};
    // weight fragments come from L2; the next k-step's are loaded while the
    // current step's products run
    bf16x8 b[FB];
#pragma unroll
    for (int fb = 0; fb < FB; ++fb) b[fb] = frag(wt + fo_block<HID>(0, (w * FB + fb) * 16) + l * 8);
#pragma unroll
    for (int k0 = 0; k0 < K; k0 += 32) {
        bf16x8 bn[FB];
        if (k0 + 32 < K) {
#pragma unroll
            for (int fb = 0; fb < FB; ++fb) bn[fb] = frag(wt + fo_block<HID>(k0 / 32 + 1, (w * FB + fb) * 16) + l * 8);
        }
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            const bf16x8 a = frag(A + (rb * 16 + r16) * lda + k0 + kq);
#pragma unroll
            for (int fb = 0; fb < FB; ++fb) acc[fb][rb] = mfma(b[fb], a, acc[fb][rb]);
        }
        if (k0 + 32 < K) {
#pragma unroll
            for (int fb = 0; fb < FB; ++fb) b[fb] = bn[fb];
        }
    }
    if (IN_PLACE) __syncthreads();
#pragma unroll
    for (int fb = 0; fb < FB; ++fb) {
        const int f = (w * FB + fb) * 16 + g * 4;
        const float b0 = bias[f], b1 = bias[f + 1], b2 = bias[f + 2], b3 = bias[f + 3];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            const int row = rb * 16 + r16;
            const uint32_t p0 = pack_bf16(fmaxf(acc[fb][rb][0] + b0, 0.0f), fmaxf(acc[fb][rb][1] + b1, 0.0f));
            const uint32_t p1 = pack_bf16(fmaxf(acc[fb][rb][2] + b2, 0.0f), fmaxf(acc[fb][rb][3] + b3, 0.0f));
            *reinterpret_cast<uint2 *>(out + row * ldo + f) = make_uint2(p0, p1);
            // fragment-order copy for the backward; rows past n hold the
            // activations of a zero input and are never used with a nonzero
            // gradient
            if (out_g) {
                const int64_t r = row0 + row;
                out_g[fo<HID>(r, f)] = (uint16_t)p0;
                out_g[fo<HID>(r, f + 1)] = (uint16_t)(p0 >> 16);
                out_g[fo<HID>(r, f + 2)] = (uint16_t)p1;
                out_g[fo<HID>(r, f + 3)] = (uint16_t)(p1 >> 16);
            }
        }
    }
}

static_assert(TM == PANEL, "a forward tile is one panel of the kept activations");
static_assert(PANEL % TMC_MAX == 0, "a chain tile lies inside one panel");

__global__ __launch_bounds__(256) void k_mlp_fwd(MlpFwdArgs a) {
    // one hidden tile, overwritten layer by layer (39 KiB of LDS per block,
    // so that three blocks share a CU)
    __shared__ __attribute__((aligned(16))) uint16_t xs[TM * LDX];
    __shared__ __attribute__((aligned(16))) uint16_t hs0[TM * LDH];
    const int64_t row0 = (int64_t)blockIdx.x * TM;
    // stage the input tile (rows past n are zero)
    for (int c = threadIdx.x; c < TM * IN / 8; c += blockDim.x) {
        const int r = c / (IN / 8), q = (c % (IN / 8)) * 8;
        uint4 v = make_uint4(0, 0, 0, 0);
        if (row0 + r < a.n) v = *reinterpret_cast<const uint4 *>(a.x + (size_t)(row0 + r) * IN + q);
        *reinterpret_cast<uint4 *>(xs + r * LDX + q) = v;
    }
    __syncthreads();
    hidden_layer<IN, false>(xs, LDX, a.wt[0], a.b[0], hs0, LDH, a.h[0], row0);
    __syncthreads();
    hidden_layer<HID, true>(hs0, LDH, a.wt[1], a.b[1], hs0, LDH, a.h[1], row0);
    __syncthreads();
    hidden_layer<HID, true>(hs0, LDH, a.wt[2], a.b[2], hs0, LDH, a.h[2], row0);
    __syncthreads();
    // output layer: N = OUT = 16, one unit block, transposed like the hidden
    // layers; wave w owns the row blocks w RBW .. w RBW + RBW - 1
    {
        const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
        const int r16 = l & 15, g = l >> 4, kq = g * 8;
        constexpr int RBW = TM / 16 / 4;
        f32x4 acc[RBW];
#pragma unroll
        for (int j = 0; j < RBW; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int k0 = 0; k0 < HID; k0 += 32) {
            const bf16x8 b = frag(a.wt[3] + fo_block<OUT>(k0 / 32, 0) + l * 8);
#pragma unroll
            for (int j = 0; j < RBW; ++j) {
                const int rb = w * RBW + j;
                acc[j] = mfma(b, frag(hs0 + (rb * 16 + r16) * LDH + k0 + kq), acc[j]);
            }
        }
        const float *bo = a.b[3] + g * 4;
#pragma unroll
        for (int j = 0; j < RBW; ++j) {
            const int64_t row = row0 + (w * RBW + j) * 16 + r16;
            if (row < a.n) {
                float *yr = a.y + (size_t)row * OUT + g * 4;
#pragma unroll
                for (int i = 0; i < 4; ++i) yr[i] = acc[j][i] + bo[i];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// backward, in three launches:
//  1. k_mlp_bwd_chain: per tile of TMC rows, the data gradients of layers
//     3, 2 and 1 one after the other (a row's chain needs only its own row),
//     written feature-major; also x and dz_out feature-major.
//  2. k_mlp_bwd_wgrad: partial weight and bias gradients of all four layers,
//     one partial per batch slice.  With both operands feature-major the
//     contraction over rows is contiguous in memory, so every MFMA fragment
//     is one 16-byte load.
//  3. k_mlp_bwd_reduce: sum of the slice partials in slice order.

constexpr int TMC = 32;     // rows per block of the data-gradient chain (a multiple of 16)
static_assert(TMC % 16 == 0 && TMC <= TMC_MAX, "whole MFMA row blocks inside one panel");
constexpr int LDZ0 = 40;    // LDS pitch of the dz_out tile (16 columns padded to 32)

__device__ __forceinline__ bool relu_live(uint32_t h) { return h != 0 && !(h & 0x8000u); }

// data gradient of one layer on a TMC-row tile:
//   dz_prev[r][c] = bf16(relu'(h[r][c]) * sum_j dz[r][j] W[j][c])
// A (dz rows, contraction j contiguous) comes from LDS; W is the "w" copy
// (fragment order, rows j = the layer's N outputs padded to 32, features c).
// The result goes to LDS (next layer's A operand, if D) and to dz_prevT in
// fragment order.  Wave wv owns output columns 64 wv .. 64 wv + 63.
template <int N>
__device__ __forceinline__ void chain_layer(const uint16_t *A, int lda, const uint16_t *__restrict__ w,
                                            const uint16_t *__restrict__ hT, uint16_t *D,
                                            uint16_t *__restrict__ dzT, int64_t row0) {
    constexpr int NC = (N + 31) / 32 * 32, KS = NC / 32;
    constexpr int RB = TMC / 16, CB = HID / 16 / 4;
    const int l = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int r16 = l & 15, g = l >> 4, kq = g * 8;
    // the wave's weight fragments and ReLU masks, all issued before the products
    bf16x8 b[KS][CB];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
            b[ks][cb] = frag(w + fo_block<HID>(ks, (wv * CB + cb) * 16) + l * 8);
        }
    uint2 hm[RB][CB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
            const int col = (wv * CB + cb) * 16 + r16;
            hm[rb][cb] = *reinterpret_cast<const uint2 *>(hT + fo<HID>(row0 + rb * 16 + g * 4, col));
        }
    f32x4 acc[RB][CB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) acc[rb][cb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            const bf16x8 av = frag(A + (rb * 16 + r16) * lda + ks * 32 + kq);
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) acc[rb][cb] = mfma(av, b[ks][cb], acc[rb][cb]);
        }
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
        const int col = (wv * CB + cb) * 16 + r16;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            const uint32_t hw[4] = {hm[rb][cb].x & 0xffffu, hm[rb][cb].x >> 16, hm[rb][cb].y & 0xffffu,
                                    hm[rb][cb].y >> 16};
            uint32_t u[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                u[i] = f2bf(relu_live(hw[i]) ? acc[rb][cb][i] : 0.0f);
                if (D) D[(rb * 16 + g * 4 + i) * LDH + col] = (uint16_t)u[i];
            }
            *reinterpret_cast<uint2 *>(dzT + fo<HID>(row0 + rb * 16 + g * 4, col)) =
                make_uint2(u[0] | u[1] << 16, u[2] | u[3] << 16);
        }
    }
}

// gather 8 consecutive rows of column c of an LDS tile into one vector
__device__ __forceinline__ uint4 lds_column8(const uint16_t *t, int pitch, int r, int c) {
    uint32_t v[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) v[j] = (uint32_t)t[(r + 2 * j) * pitch + c] | (uint32_t)t[(r + 2 * j + 1) * pitch + c] << 16;
    return make_uint4(v[0], v[1], v[2], v[3]);
}

__global__ __launch_bounds__(256) void k_mlp_bwd_chain(MlpBwdArgs a) {
    __shared__ __attribute__((aligned(16))) uint16_t zs[TMC * LDZ0];
    __shared__ __attribute__((aligned(16))) uint16_t xs[TMC * LDX];
    __shared__ __attribute__((aligned(16))) uint16_t d0[TMC * LDH];
    __shared__ __attribute__((aligned(16))) uint16_t d1[TMC * LDH];
    const int64_t row0 = (int64_t)blockIdx.x * TMC;
    const int t = threadIdx.x;
    // stage dz_out (columns 16..31 zero) and x; rows past n are zero
    for (int u = t; u < 2 * TMC * 4; u += 256) {
        const int v = u % (TMC * 4), r = v >> 2, q = (v & 3) * 8;
        uint4 val = make_uint4(0, 0, 0, 0);
        if (u < TMC * 4) {
            if (q < OUT && row0 + r < a.n) val = *reinterpret_cast<const uint4 *>(a.dz_out + (size_t)(row0 + r) * OUT + q);
            *reinterpret_cast<uint4 *>(zs + r * LDZ0 + q) = val;
        } else {
            if (row0 + r < a.n) val = *reinterpret_cast<const uint4 *>(a.x + (size_t)(row0 + r) * IN + q);
            *reinterpret_cast<uint4 *>(xs + r * LDX + q) = val;
        }
    }
    __syncthreads();
    // fragment-order copies of dz_out and x for the weight gradients
    constexpr int RG = TMC / 8;
    for (int u = t; u < (OUT + IN) * RG; u += 256) {
        if (u < OUT * RG) {
            const int c = u / RG, r = (u % RG) * 8;
            *reinterpret_cast<uint4 *>(a.dzT[3] + fo<OUT>(row0 + r, c)) = lds_column8(zs, LDZ0, r, c);
        } else {
            const int w = u - OUT * RG, c = w / RG, r = (w % RG) * 8;
            *reinterpret_cast<uint4 *>(a.xT + fo<IN>(row0 + r, c)) = lds_column8(xs, LDX, r, c);
        }
    }
    chain_layer<OUT>(zs, LDZ0, a.w[3], a.hT[2], d0, a.dzT[2], row0);
    __syncthreads();
    chain_layer<HID>(d0, LDH, a.w[2], a.hT[1], d1, a.dzT[1], row0);
    __syncthreads();
    chain_layer<HID>(d1, LDH, a.w[1], a.hT[0], nullptr, a.dzT[0], row0);
}

// partial gradient of layer L over one batch slice, output tile
// [o0, o0 + TO) x [i0, i0 + TI) of dwt_L (and db_L when i0 = 0):
//   dwt[o][i] = sum_r dz[r][o] in[r][i],  db[o] = sum_r dz[r][o]
// dz and in are in fragment order, whose rows are the contracted index here.
// Each of the block's four waves takes a quarter of the slice's rows and sums
// them in one MFMA chain, the next 32-row step's fragments loading while the
// current one multiplies; the bias sums are the same products with an operand
// of ones.  The four wave sums are added in wave order through LDS.
constexpr int WG_TILES = 4 + 16 + 16 + 4;  // output tiles per slice (layers 0..3)
constexpr int WG_RED = 64 * 64;            // largest tile

template <int L>
__device__ __forceinline__ void wgrad_tile(const MlpBwdArgs &a, int o0, int i0, int s, float *red) {
    constexpr int NI = L == 0 ? IN : HID, NO = L == 3 ? OUT : HID;
    constexpr int TO = NO < 64 ? NO : 64, TI = NI < 64 ? NI : 64;
    constexpr int OB = TO / 16, IB = TI / 16;
    const uint16_t *__restrict__ A = a.dzT[L];
    const uint16_t *__restrict__ B = L == 0 ? a.xT : a.hT[L - 1];
    const int t = threadIdx.x, l = t & 63, wv = t >> 6;
    const int r16 = l & 15, g = l >> 4;
    // the wave's rows: [lo, hi), whole 32-row steps (rows is a multiple of 64)
    const int64_t rows = a.rows, quarters = 4 * (int64_t)a.n_split;
    const int64_t per = ((rows + quarters - 1) / quarters + 31) / 32 * 32;
    const int64_t lo = ((int64_t)s * 4 + wv) * per;
    const int64_t hi = lo + per < rows ? lo + per : rows;
    const bool bias = i0 == 0;
    const bf16x8 ones = __builtin_bit_cast(bf16x8, make_uint4(0x3f803f80u, 0x3f803f80u, 0x3f803f80u, 0x3f803f80u));
    f32x4 acc[OB][IB], accb[OB];
#pragma unroll
    for (int ob = 0; ob < OB; ++ob) {
        accb[ob] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ib = 0; ib < IB; ++ib) acc[ob][ib] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
    // fragments of features f .. f+15 over one 32-row step, one contiguous
    // 1 KiB read each; two steps stay in flight while the products run.  Steps past hi
    // (a prefetch at the end) reread step lo and are not multiplied.
    auto load = [&](int64_t r0, uint4 *va, uint4 *vb) {
        const int64_t st = (r0 < hi ? r0 : lo) / 32;
#pragma unroll
        for (int ob = 0; ob < OB; ++ob) va[ob] = *reinterpret_cast<const uint4 *>(A + fo_block<NO>(st, o0 + ob * 16) + l * 8);
#pragma unroll
        for (int ib = 0; ib < IB; ++ib) vb[ib] = *reinterpret_cast<const uint4 *>(B + fo_block<NI>(st, i0 + ib * 16) + l * 8);
    };
    auto step = [&](const uint4 *va, const uint4 *vb) {
#pragma unroll
        for (int ob = 0; ob < OB; ++ob) {
            const bf16x8 fa = __builtin_bit_cast(bf16x8, va[ob]);
#pragma unroll
            for (int ib = 0; ib < IB; ++ib) acc[ob][ib] = mfma(fa, __builtin_bit_cast(bf16x8, vb[ib]), acc[ob][ib]);
            if (bias) accb[ob] = mfma(fa, ones, accb[ob]);
        }
    };
    if (lo < hi) {
        uint4 a0[OB], b0[IB], a1[OB], b1[IB];
        load(lo, a0, b0);
        load(lo + 32, a1, b1);
        for (int64_t r0 = lo; r0 < hi; r0 += 64) {
            step(a0, b0);
            load(r0 + 64, a0, b0);
            if (r0 + 32 < hi) step(a1, b1);
            load(r0 + 96, a1, b1);
        }
    }
    // wave sums to LDS, then their sum in wave order into the slice's partial
    float *mine = red + wv * (WG_RED + 64);
#pragma unroll
    for (int ob = 0; ob < OB; ++ob) {
#pragma unroll
        for (int ib = 0; ib < IB; ++ib)
#pragma unroll
            for (int i = 0; i < 4; ++i) mine[(ob * 16 + g * 4 + i) * TI + ib * 16 + r16] = acc[ob][ib][i];
        if (bias && r16 == 0)
#pragma unroll
            for (int i = 0; i < 4; ++i) mine[WG_RED + ob * 16 + g * 4 + i] = accb[ob][i];
    }
    __syncthreads();
    float *part = a.part + (size_t)s * PAR_COUNT + PAR_W[L];
    for (int e = t; e < TO * TI; e += 256) {
        const float v = ((red[e] + red[(WG_RED + 64) + e]) + red[2 * (WG_RED + 64) + e]) + red[3 * (WG_RED + 64) + e];
        part[(size_t)(o0 + e / TI) * NI + i0 + e % TI] = v;
    }
    if (bias && t < TO) {
        const int e = WG_RED + t;
        const float v = ((red[e] + red[(WG_RED + 64) + e]) + red[2 * (WG_RED + 64) + e]) + red[3 * (WG_RED + 64) + e];
        part[NO * NI + o0 + t] = v;
    }
}

// block b: slice b mod n_split (so that, with a multiple of 8 slices, a
// slice's blocks share one XCD and its L2), tile b / n_split
__global__ __launch_bounds__(256) void k_mlp_bwd_wgrad(MlpBwdArgs a) {
    __shared__ float red[4 * (WG_RED + 64)];
    const int s = blockIdx.x % a.n_split, tile = blockIdx.x / a.n_split;
    if (tile < 4) {
        wgrad_tile<0>(a, tile * 64, 0, s, red);
    } else if (tile < 20) {
        const int u = tile - 4;
        wgrad_tile<1>(a, (u / 4) * 64, (u % 4) * 64, s, red);
    } else if (tile < 36) {
        const int u = tile - 20;
        wgrad_tile<2>(a, (u / 4) * 64, (u % 4) * 64, s, red);
    } else {
        wgrad_tile<3>(a, 0, (tile - 36) * 64, s, red);
    }
}

// gradients = sum of the slice partials, in slice order; four consecutive
// parameters per thread (layer segments are multiples of four long)
__global__ __launch_bounds__(256) void k_mlp_bwd_reduce(MlpBwdArgs a) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= PAR_COUNT / 4) return;
    const float4 *p = reinterpret_cast<const float4 *>(a.part) + q;
    // eight slices' loads in flight at a time, added in slice order
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int k0 = 0; k0 < a.n_split; k0 += 8) {
        float4 u[8];
#pragma unroll
        for (int j = 0; j < 8; ++j)
            if (k0 + j < a.n_split) u[j] = p[(size_t)(k0 + j) * (PAR_COUNT / 4)];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            if (k0 + j >= a.n_split) break;
            if (k0 + j == 0) {
                v = u[0];
                continue;
            }
            v.x += u[j].x;
            v.y += u[j].y;
            v.z += u[j].z;
            v.w += u[j].w;
        }
    }
    const int e = 4 * q;
    const int L = e >= PAR_W[3] ? 3 : e >= PAR_W[2] ? 2 : e >= PAR_W[1] ? 1 : 0;
    const int nw = (L == 3 ? OUT : HID) * (L == 0 ? IN : HID);
    const int off = e - (L == 3 ? PAR_W[3] : L == 2 ? PAR_W[2] : L == 1 ? PAR_W[1] : 0);
    float *dst;
    switch (L) {
        case 0: dst = off < nw ? a.dwt[0] + off : a.db[0] + (off - nw); break;
        case 1: dst = off < nw ? a.dwt[1] + off : a.db[1] + (off - nw); break;
        case 2: dst = off < nw ? a.dwt[2] + off : a.db[2] + (off - nw); break;
        default: dst = off < nw ? a.dwt[3] + off : a.db[3] + (off - nw); break;
    }
    dst[0] = v.x;
    dst[1] = v.y;
    dst[2] = v.z;
    dst[3] = v.w;
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
// Adam on one weight matrix of shape [rows][cols] = [out][in] (a bias:
// rows = 1).  Updates the binary32 master and both bfloat16 copies in
// fragment order: wt (rows in, features out) and w (rows out, features in).

__device__ __forceinline__ size_t fo_rt(int r, int f, int c) {
    return ((size_t)(r >> 5) * (c >> 4) + (size_t)(f >> 4)) * 512 + (size_t)(((f & 15) + 16 * ((r & 31) >> 3)) * 8) +
           (size_t)(r & 7);
}

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
        const int o = i / cols, k = i % cols;
        if (wt_bf) wt_bf[fo_rt(k, o, rows)] = hb;
        if (w_bf) w_bf[fo_rt(o, k, cols)] = hb;
    }
}

// ---------------------------------------------------------------------------

hipError_t launch_fwd(const MlpFwdArgs &a, hipStream_t s) {
    const unsigned g = (unsigned)((a.n + TM - 1) / TM);
    if (g) hipLaunchKernelGGL(k_mlp_fwd, dim3(g), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_bwd(const MlpBwdArgs &a, hipStream_t s) {
    const unsigned g1 = (unsigned)(a.rows / TMC);
    if (g1) hipLaunchKernelGGL(k_mlp_bwd_chain, dim3(g1), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_mlp_bwd_wgrad, dim3(WG_TILES * a.n_split), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_mlp_bwd_reduce, dim3((PAR_COUNT / 4 + 255) / 256), dim3(256), 0, s, a);
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
