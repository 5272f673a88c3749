// stats_kernels.hip -- the binned per-edge statistics handed over on the
// device, in input edge order: inflow, exits and travel-time sums per
// (edge, bin) as the step kept them, and the occupancy completed with the
// steps that the vehicles still on an edge have spent there so far (the
// same figures lpsim_edge_stats copies to the host).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lpsim_dev.h"

namespace lpsim {

// row i of each internal-order [E][B] array goes to row ext[i]
__global__ __launch_bounds__(256) void k_stats_rows(const int32_t *ext, int32_t E, int32_t B, const int32_t *in_i,
                                                    const int32_t *ex_i, const unsigned long long *tt_i,
                                                    const unsigned long long *occ_i, int32_t *in_o, int32_t *ex_o,
                                                    unsigned long long *tt_o, unsigned long long *occ_o) {
    const size_t total = (size_t)E * (size_t)B;
    for (size_t j = (size_t)blockIdx.x * blockDim.x + threadIdx.x; j < total; j += (size_t)gridDim.x * blockDim.x) {
        const size_t i = j / (size_t)B, b = j - i * (size_t)B;
        const size_t o = (size_t)ext[i] * (size_t)B + b;
        if (in_o) in_o[o] = in_i[j];
        if (ex_o) ex_o[o] = ex_i[j];
        if (tt_o) tt_o[o] = tt_i[j];
        if (occ_o) occ_o[o] = occ_i[j];
    }
}

// every live vehicle adds the steps from its entry to the current step, split
// over the bins they fall in (the last bin takes everything after it); the
// slot count and the step come from the control block `ct` on the device
__global__ __launch_bounds__(256) void k_stats_live(const Ctrl *ct, Slots S0, Slots S1, const int32_t *ext,
                                                    int32_t B, int32_t bin_steps, unsigned long long *occ_o) {
    const uint32_t n = ct->n_slots + ct->n_new;
    const int32_t k = ct->k;
    const Slots &S = ct->cur ? S1 : S0;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        if (S.m[i] & M_DEAD) continue;
        const int32_t en = S.ent[i], ex = k;
        if (ex <= en) continue;
        const int32_t b0 = min(en / bin_steps, B - 1), b1 = min((ex - 1) / bin_steps, B - 1);
        unsigned long long *row = occ_o + (size_t)ext[S.e[i]] * (size_t)B;
        for (int32_t b = b0; b <= b1; ++b) {
            const int32_t lo = b * bin_steps, hi = b == B - 1 ? 0x7fffffff : lo + bin_steps;
            atomicAdd(&row[b], (unsigned long long)(min(ex, hi) - max(en, lo)));
        }
    }
}

hipError_t launch_stats_device(const Dev &d, const Ctrl *ct, const int32_t *ext, int32_t E, int32_t B,
                               int32_t bin_steps, uint32_t slot_cap, int32_t *inflow, int32_t *exits,
                               unsigned long long *tt, unsigned long long *occ, hipStream_t s) {
    const size_t total = (size_t)E * (size_t)B;
    if (total && (inflow || exits || tt || occ)) {
        const size_t g = (total + 255) / 256 < 8192 ? (total + 255) / 256 : 8192;
        hipLaunchKernelGGL(k_stats_rows, dim3((unsigned)g), dim3(256), 0, s, ext, E, B, d.inflow_bin, d.exits_bin,
                           d.tt_bin, d.occ_bin, inflow, exits, tt, occ);
    }
    if (occ && slot_cap) {
        const uint32_t g = (slot_cap + 255) / 256 < 2048 ? (slot_cap + 255) / 256 : 2048;
        hipLaunchKernelGGL(k_stats_live, dim3(g), dim3(256), 0, s, ct, d.buf[0], d.buf[1], ext, B, bin_steps, occ);
    }
    return hipGetLastError();
}

}  // namespace lpsim
