// surrogate_kernels.hip -- the data path around the travel-time perceptron in
// the traffic-assignment loop: network loading under estimated travel times,
// perceptron features, training targets from simulator statistics, and the
// damped travel-time update.  Bins are the simulator's statistics bins; a
// sample is one (edge, window of 12 bins).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lpsim.h"

namespace lpsim_sur {

constexpr int WIN = 12;   // bins per perceptron sample
constexpr int NX = 32;    // features per sample (27 used)
constexpr int NY = 16;    // outputs per sample (12 used)

__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// Each trip walks its route from its departure: it enters the first edge at
// depart + 1, spends round(tt) >= 1 steps on an edge entered in bin b
// (tt of that edge and bin), and stops at the horizon.  Entries count in the
// entry bin; the steps spent on an edge count in the bins they fall in.
__global__ void k_load(const int64_t *route_off, const int32_t *route, const int32_t *depart, int64_t n_trips,
                       const float *tt, int32_t n_bins, int32_t bin_steps, int32_t horizon, int32_t *inflow,
                       unsigned long long *occ) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_trips;
         i += (int64_t)gridDim.x * blockDim.x) {
        int64_t t = (int64_t)depart[i] + 1;
        for (int64_t j = route_off[i]; j < route_off[i + 1] && t < horizon; ++j) {
            const int32_t e = route[j];
            const int64_t row = (int64_t)e * n_bins;
            const int32_t b0 = (int32_t)min<int64_t>(t / bin_steps, n_bins - 1);
            atomicAdd(&inflow[row + b0], 1);
            const float est = tt[row + b0];
            const int32_t tau = est >= 1.0f ? (int32_t)rintf(est) : 1;
            const int64_t t_out = min<int64_t>(t + tau, horizon);
            const int32_t b1 = (int32_t)min<int64_t>((t_out - 1) / bin_steps, n_bins - 1);
            for (int32_t b = b0; b <= b1; ++b) {
                const int64_t lo = (int64_t)b * bin_steps;
                const int64_t hi = (b == n_bins - 1) ? INT64_MAX : lo + bin_steps;
                const int64_t s = t > lo ? t : lo, u = t_out < hi ? t_out : hi;
                atomicAdd(&occ[row + b], (unsigned long long)(u - s));
            }
            t += tau;
        }
    }
}

// features of sample (e, w): log1p(inflow) x12, density x12 (mean vehicles per
// metre of lane during the bin, times the jam spacing), log(length),
// lanes / 4, speed limit / 22.4
__global__ void k_features(int32_t n_edges, int32_t n_bins, int32_t bin_steps, float jam, const int32_t *inflow,
                           const int64_t *occ, const float *length, const uint8_t *lanes, const float *speed,
                           uint16_t *x) {
    const int32_t nw = n_bins / WIN;
    const int64_t n = (int64_t)n_edges * nw;
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n; s += (int64_t)gridDim.x * blockDim.x) {
        const int32_t e = (int32_t)(s / nw), w = (int32_t)(s % nw);
        const int64_t row = (int64_t)e * n_bins + (int64_t)w * WIN;
        const float cap = (float)bin_steps * ceilf(length[e]) * (float)lanes[e];
        uint16_t *o = x + s * NX;
        for (int j = 0; j < WIN; ++j) o[j] = f2bf(log1pf((float)inflow[row + j]));
        for (int j = 0; j < WIN; ++j) o[WIN + j] = f2bf(((float)occ[row + j] / cap) * jam);
        o[24] = f2bf(logf(length[e]));
        o[25] = f2bf((float)lanes[e] * 0.25f);
        o[26] = f2bf(speed[e] / 22.4f);
        for (int j = 27; j < NX; ++j) o[j] = 0;
    }
}

// targets of sample (e, w): log(mean travel time / free-flow time) per bin,
// masked where no traversal entered in that bin
__global__ void k_targets(int32_t n_edges, int32_t n_bins, const int32_t *exits, const int64_t *tt_sum,
                          const float *tt_free, float *y, uint8_t *mask) {
    const int32_t nw = n_bins / WIN;
    const int64_t n = (int64_t)n_edges * nw;
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n; s += (int64_t)gridDim.x * blockDim.x) {
        const int32_t e = (int32_t)(s / nw), w = (int32_t)(s % nw);
        const int64_t row = (int64_t)e * n_bins + (int64_t)w * WIN;
        for (int j = 0; j < NY; ++j) {
            float v = 0.0f;
            uint8_t m = 0;
            if (j < WIN && exits[row + j] > 0) {
                const float mean = (float)tt_sum[row + j] / (float)exits[row + j];
                v = logf(mean / tt_free[e]);
                m = 1;
            }
            y[s * NY + j] = v;
            mask[s * NY + j] = m;
        }
    }
}

// damped update of the travel-time estimate from predictions:
// tt <- (1 - damping) tt + damping * clamp(tt_free * exp(y), 1, tt_max)
__global__ void k_tt(int32_t n_edges, int32_t n_bins, const float *y, const float *tt_free, float damping,
                     float tt_max, float *tt) {
    const int32_t nw = n_bins / WIN;
    const int64_t n = (int64_t)n_edges * nw;
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n; s += (int64_t)gridDim.x * blockDim.x) {
        const int32_t e = (int32_t)(s / nw), w = (int32_t)(s % nw);
        const int64_t row = (int64_t)e * n_bins + (int64_t)w * WIN;
        for (int j = 0; j < WIN; ++j) {
            float p = tt_free[e] * expf(y[s * NY + j]);
            p = p < 1.0f ? 1.0f : (p > tt_max ? tt_max : p);
            tt[row + j] = (1.0f - damping) * tt[row + j] + damping * p;
        }
    }
}

// anchored estimate: the last simulated travel time of each (edge, bin),
// moved by the perceptron's predicted change of log travel time between the
// anchor loading and the new one (the change clamped to +-max_shift), then
// clamped to [1, tt_max]
__global__ void k_shift(int32_t n_edges, int32_t n_bins, const float *y_new, const float *y_anchor,
                        const float *anchor_tt, float max_shift, float tt_max, float *tt_out) {
    const int64_t n = (int64_t)n_edges * n_bins;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
        const int32_t b = (int32_t)(q % n_bins);
        const int64_t s = (q / n_bins) * (n_bins / WIN) + b / WIN;
        const int32_t j = b % WIN;
        float dlt = y_new[s * NY + j] - y_anchor[s * NY + j];
        dlt = dlt < -max_shift ? -max_shift : (dlt > max_shift ? max_shift : dlt);
        float t = anchor_tt[q] * expf(dlt);
        tt_out[q] = t < 1.0f ? 1.0f : (t > tt_max ? tt_max : t);
    }
}

// routing cost of an edge in seconds: the entry-weighted mean over bins of
// the travel time in steps, free flow where nobody entered, at least one step
__global__ void k_edge_tt(int32_t n_edges, int32_t n_bins, const int32_t *inflow, const float *tt,
                          const float *tt_free, float dt, double *out) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n_edges;
         e += (int64_t)gridDim.x * blockDim.x) {
        double num = 0.0, den = 0.0;
        for (int32_t b = 0; b < n_bins; ++b) {
            const double f = (double)inflow[e * n_bins + b];
            num += f * (double)tt[e * n_bins + b];
            den += f;
        }
        double t = den > 0.0 ? num / den : (double)tt_free[e];
        out[e] = (t > 1.0 ? t : 1.0) * (double)dt;
    }
}

static unsigned grid_for(int64_t n) {
    const int64_t b = (n + 255) / 256;
    return (unsigned)(b < 1 ? 1 : (b > 8192 ? 8192 : b));
}

// mean travel time per (edge, bin) in steps: the float64 quotient rounded
// once to float32, or the edge's free-flow time where nothing entered
__global__ void k_tt_bins(int32_t n_edges, int32_t n_bins, const int64_t *tt_sum, const int32_t *exits,
                          const double *tt_free, float *out) {
    const int64_t n = (int64_t)n_edges * n_bins;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = exits[i] > 0 ? (float)((double)tt_sum[i] / (double)exits[i]) : (float)tt_free[i / n_bins];
}

}  // namespace lpsim_sur

using namespace lpsim_sur;

extern "C" {

int32_t lpsim_surrogate_load(const int64_t *route_off, const int32_t *route_edges, const int32_t *depart_step,
                             int64_t n_trips, const float *tt_steps, int32_t n_edges, int32_t n_bins,
                             int32_t bin_steps, int32_t horizon, int32_t *inflow_bin, int64_t *occ_steps_bin,
                             void *stream) {
    if (n_trips < 0 || n_edges < 1 || n_bins < 1 || bin_steps < 1 || horizon < 0 || !tt_steps || !inflow_bin ||
        !occ_steps_bin || (n_trips > 0 && (!route_off || !route_edges || !depart_step)))
        return LPSIM_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const size_t nb = (size_t)n_edges * n_bins;
    if (hipMemsetAsync(inflow_bin, 0, nb * 4, s) != hipSuccess) return LPSIM_EDEVICE;
    if (hipMemsetAsync(occ_steps_bin, 0, nb * 8, s) != hipSuccess) return LPSIM_EDEVICE;
    if (n_trips == 0) return LPSIM_OK;
    hipLaunchKernelGGL(k_load, dim3(grid_for(n_trips)), dim3(256), 0, s, route_off, route_edges, depart_step, n_trips,
                       tt_steps, n_bins, bin_steps, horizon, inflow_bin, (unsigned long long *)occ_steps_bin);
    return hipGetLastError() == hipSuccess ? LPSIM_OK : LPSIM_EDEVICE;
}

int32_t lpsim_edge_tt_bins_device(int32_t n_edges, int32_t n_bins, const int64_t *tt_sum_bin, const int32_t *exits_bin,
                                  const double *tt_free_steps, float *out_steps, void *stream) {
    if (n_edges < 0 || n_bins < 1 || (n_edges > 0 && (!tt_sum_bin || !exits_bin || !tt_free_steps || !out_steps)))
        return LPSIM_EINVAL;
    if (n_edges == 0) return LPSIM_OK;
    const int64_t n = (int64_t)n_edges * n_bins;
    hipLaunchKernelGGL(k_tt_bins, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, n_edges, n_bins, tt_sum_bin,
                       exits_bin, tt_free_steps, out_steps);
    return hipGetLastError() == hipSuccess ? LPSIM_OK : LPSIM_EDEVICE;
}

int32_t lpsim_surrogate_features(int32_t n_edges, int32_t n_bins, int32_t bin_steps, float jam_spacing,
                                 const int32_t *inflow_bin, const int64_t *occ_steps_bin, const float *length_m,
                                 const uint8_t *lanes, const float *speed_mps, uint16_t *x_out, void *stream) {
    if (n_edges < 1 || n_bins < WIN || n_bins % WIN || bin_steps < 1 || !inflow_bin || !occ_steps_bin ||
        !length_m || !lanes || !speed_mps || !x_out)
        return LPSIM_EINVAL;
    const int64_t n = (int64_t)n_edges * (n_bins / WIN);
    hipLaunchKernelGGL(k_features, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, n_edges, n_bins, bin_steps,
                       jam_spacing, inflow_bin, occ_steps_bin, length_m, lanes, speed_mps, x_out);
    return hipGetLastError() == hipSuccess ? LPSIM_OK : LPSIM_EDEVICE;
}

int32_t lpsim_surrogate_targets(int32_t n_edges, int32_t n_bins, const int32_t *exits_bin, const int64_t *tt_sum_bin,
                                const float *tt_free_steps, float *y_out, uint8_t *mask_out, void *stream) {
    if (n_edges < 1 || n_bins < WIN || n_bins % WIN || !exits_bin || !tt_sum_bin || !tt_free_steps || !y_out ||
        !mask_out)
        return LPSIM_EINVAL;
    const int64_t n = (int64_t)n_edges * (n_bins / WIN);
    hipLaunchKernelGGL(k_targets, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, n_edges, n_bins, exits_bin,
                       tt_sum_bin, tt_free_steps, y_out, mask_out);
    return hipGetLastError() == hipSuccess ? LPSIM_OK : LPSIM_EDEVICE;
}

int32_t lpsim_surrogate_tt(int32_t n_edges, int32_t n_bins, const float *y_pred, const float *tt_free_steps,
                           float damping, float tt_max, float *tt_steps, void *stream) {
    if (n_edges < 1 || n_bins < WIN || n_bins % WIN || !y_pred || !tt_free_steps || !tt_steps ||
        !(damping >= 0.0f && damping <= 1.0f) || !(tt_max >= 1.0f))
        return LPSIM_EINVAL;
    const int64_t n = (int64_t)n_edges * (n_bins / WIN);
    hipLaunchKernelGGL(k_tt, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, n_edges, n_bins, y_pred,
                       tt_free_steps, damping, tt_max, tt_steps);
    return hipGetLastError() == hipSuccess ? LPSIM_OK : LPSIM_EDEVICE;
}

int32_t lpsim_surrogate_shift(int32_t n_edges, int32_t n_bins, const float *y_new, const float *y_anchor,
                              const float *anchor_tt_steps, float max_shift, float tt_max, float *tt_steps_out,
                              void *stream) {
    if (n_edges < 1 || n_bins < WIN || n_bins % WIN || !y_new || !y_anchor || !anchor_tt_steps || !tt_steps_out ||
        !(max_shift >= 0.0f) || !(tt_max >= 1.0f))
        return LPSIM_EINVAL;
    const int64_t n = (int64_t)n_edges * n_bins;
    hipLaunchKernelGGL(k_shift, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, n_edges, n_bins, y_new,
                       y_anchor, anchor_tt_steps, max_shift, tt_max, tt_steps_out);
    return hipGetLastError() == hipSuccess ? LPSIM_OK : LPSIM_EDEVICE;
}

int32_t lpsim_surrogate_edge_tt(int32_t n_edges, int32_t n_bins, const int32_t *inflow_bin, const float *tt_steps,
                                const float *tt_free_steps, float dt, double *edge_tt_s, void *stream) {
    if (n_edges < 1 || n_bins < 1 || !inflow_bin || !tt_steps || !tt_free_steps || !edge_tt_s || !(dt > 0.0f))
        return LPSIM_EINVAL;
    hipLaunchKernelGGL(k_edge_tt, dim3(grid_for(n_edges)), dim3(256), 0, (hipStream_t)stream, n_edges, n_bins,
                       inflow_bin, tt_steps, tt_free_steps, dt, edge_tt_s);
    return hipGetLastError() == hipSuccess ? LPSIM_OK : LPSIM_EDEVICE;
}

}  // extern "C"
