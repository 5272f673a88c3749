// lpsim_kernels.hip -- gfx950 kernels of one simulation step.
//
// One step k -> k+1 (paper Section 3.1, vehicle-dynamics equation: every new
// state depends on step-k state only; Algorithm 1 per vehicle) runs as four
// kernels, each a grid of fixed shape that walks the current work list:
//
//   move     reads the lane map of step k: leader scan, IDM / free move,
//            stop line, crossing; entry requests of crossing vehicles and of
//            departing trips go into one 32-bit word per target lane by
//            atomicMin of the trip id (exclusive entry, lowest id wins);
//   resolve  winners enter, losers wait at the last cell, arrivals leave;
//            each vehicle clears its old cell byte and writes its new one --
//            no two vehicles touch the same byte in this kernel (a mover never
//            lands on a cell another vehicle occupied at step k, entries need
//            the first W cells free); per-edge statistics by atomics;
//   lanechg  mandatory lane change decided on the post-move map;
//   commit   writes the accepted lane changes into the map, then the last
//            block to finish does the step's bookkeeping (clock, counts).
//   compact  (every few steps) moves live vehicle slots together.
//
// Vehicle state lives in slots (structure of arrays) that only hold vehicles
// on the road; the per-step control words live in device memory so that a
// captured HIP graph of many steps replays without host involvement.
//
// All floating point is binary32 with no contraction (-ffp-contract=off) and
// IEEE division, in exactly the order of the method's definition, so results
// are identical to the CPU oracle bit for bit.

#include "lpsim_dev.h"

namespace lpsim {

__device__ __forceinline__ uint32_t logical_block() {
    const uint32_t G = gridDim.x, b = blockIdx.x;
    // Blocks are dispatched round-robin over the 8 XCDs; give each XCD one
    // contiguous eighth of the work list so neighbouring vehicles (which read
    // neighbouring lane-map bytes) share that XCD's L2.
    if ((G & 7u) == 0u) return (b & 7u) * (G >> 3) + (b >> 3);
    return b;
}

__device__ __forceinline__ void block_range(uint64_t total, uint64_t &lo, uint64_t &hi) {
    const uint64_t G = gridDim.x;
    uint64_t chunk = (total + G - 1) / G;
    chunk = (chunk + 63) & ~uint64_t(63);
    lo = (uint64_t)logical_block() * chunk;
    hi = lo + chunk;
    if (hi > total) hi = total;
    if (lo > total) lo = total;
}

__device__ __forceinline__ uint8_t speed_byte(float v) {
    float c = v < 254.0f ? v : 254.0f;
    return (uint8_t)(int32_t)c;
}

__device__ __forceinline__ int32_t bin_of(const Params &p, int32_t step) {
    int32_t b = step / p.bin_steps;
    return b < p.n_bins - 1 ? b : p.n_bins - 1;
}

// first occupied cell in [lo, hi] of one lane, or -1
__device__ __forceinline__ int32_t first_occ(const uint8_t *lane, int32_t lo, int32_t hi) {
    for (int32_t c = lo; c <= hi; ++c)
        if (lane[c] != FREE_BYTE) return c;
    return -1;
}

// first occupied cell going down from hi to lo, or -1
__device__ __forceinline__ int32_t last_occ(const uint8_t *lane, int32_t hi, int32_t lo) {
    for (int32_t c = hi; c >= lo; --c)
        if (lane[c] != FREE_BYTE) return c;
    return -1;
}

__device__ __forceinline__ bool entry_free(const Dev &d, const uint4 &E, int32_t e, int32_t l) {
    if (d.aux[e] & AUX_BLOCKED) return false;
    const int32_t C = E_CELLS(E);
    const uint8_t *lp = d.map + E.x + (uint32_t)l * (uint32_t)C;
    for (int32_t c = 0; c < d.p.W; ++c)
        if (lp[c] != FREE_BYTE) return false;
    return true;
}

__device__ __forceinline__ void idm_follow(const Params &p, float x, float v, float v0, float gap,
                                           float vl, float &xn, float &vn) {
    if (gap <= 0.0f) {
        vn = 0.0f;
        xn = x;
        return;
    }
    const float dv = v - vl;
    const float t = (v * p.T) + ((v * dv) / p.tsab);
    const float ss = p.s0 + (t > 0.0f ? t : 0.0f);
    const float r = v / v0;
    const float r2 = r * r;
    const float r4 = r2 * r2;
    const float q = ss / gap;
    const float q2 = q * q;
    const float acc = p.a * ((1.0f - r4) - q2);
    const float nv = v + acc * p.dt;
    vn = nv > 0.0f ? nv : 0.0f;
    xn = x + (v + vn) * p.half_dt;
}

__device__ __forceinline__ void free_move(const Params &p, float x, float v, float v0, float &xn,
                                          float &vn) {
    if (p.free_mode == 0) {
        vn = v0;
        xn = x + vn * p.dt;
    } else {
        const float r = v / v0;
        const float r2 = r * r;
        const float r4 = r2 * r2;
        const float acc = p.a * (1.0f - r4);
        const float nv = v + acc * p.dt;
        vn = nv > 0.0f ? nv : 0.0f;
        xn = x + (v + vn) * p.half_dt;
    }
}

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    // SplitMix64 output function (Steele, Lea & Flood 2014)
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

__device__ __forceinline__ void add_exit(const Dev &d, int32_t e, int32_t enter, int32_t ex) {
    const int32_t tt = ex - enter;
    const Params &p = d.p;
    atomicAdd(&d.n_exits[e], 1);
    atomicAdd(&d.tt_sum[e], (unsigned long long)tt);
    const int64_t row = (int64_t)e * p.n_bins;
    const int32_t b0 = bin_of(p, enter);
    atomicAdd(&d.exits_bin[row + b0], 1);
    atomicAdd(&d.tt_bin[row + b0], (unsigned long long)tt);
    const int32_t b1 = bin_of(p, ex - 1);
    for (int32_t b = b0; b <= b1; ++b) {
        const int32_t lo = b * p.bin_steps;
        const int32_t hi = (b == p.n_bins - 1) ? 0x7fffffff : lo + p.bin_steps;
        const int32_t s = enter > lo ? enter : lo;
        const int32_t t = ex < hi ? ex : hi;
        atomicAdd(&d.occ_bin[row + b], (unsigned long long)(t - s));
    }
}

__device__ __forceinline__ void add_entry(const Dev &d, int32_t e, int32_t step) {
    atomicAdd(&d.inflow_bin[(int64_t)e * d.p.n_bins + bin_of(d.p, step)], 1);
}

__device__ __forceinline__ uint32_t dep_hi_of(const Dev &d, int32_t k) {
    return k < d.n_dep_hi ? d.dep_hi[k] : d.n_trips;
}

// per-block event counters, flushed without atomics into this block's row
struct BlockCounts {
    unsigned int c[NPART];
};

__device__ __forceinline__ void counts_init(BlockCounts *s) {
    if (threadIdx.x < NPART) s->c[threadIdx.x] = 0;
    __syncthreads();
}

__device__ __forceinline__ void counts_flush(const Dev &d, BlockCounts *s) {
    __syncthreads();
    if (threadIdx.x < NPART) {
        const unsigned int v = s->c[threadIdx.x];
        if (v) d.partial[(uint64_t)logical_block() * NPART + threadIdx.x] += v;
    }
}

// ---------------------------------------------------------------------------
// move: longitudinal intent from step-k state

__global__ __launch_bounds__(1024) void k_move(Dev d) {
    __shared__ BlockCounts cnt;
    counts_init(&cnt);
    const Ctrl *ctl = d.ctrl;
    const int32_t k = ctl->k;
    const uint32_t n = ctl->n_slots;
    const uint32_t wlo = ctl->wait_lo;
    const uint32_t dhi = dep_hi_of(d, k);
    const uint32_t ncand = dhi > wlo ? dhi - wlo : 0;
    const Slots S = d.buf[ctl->cur];
    const Params &p = d.p;
    uint64_t lo, hi;
    block_range((uint64_t)n + ncand, lo, hi);
    unsigned int alive = 0, scanned = 0;
    for (uint64_t it = lo + threadIdx.x; it < hi; it += blockDim.x) {
        if (it < n) {
            const uint32_t i = (uint32_t)it;
            const uint32_t m = S.m[i];
            if (m & M_DEAD) continue;
            ++alive;
            const float x = S.x[i], v = S.v[i];
            const int32_t e = S.e[i];
            const uint32_t lane = m & M_LANE;
            const uint4 E = d.edge[e];
            const int32_t C = E_CELLS(E), D = E_LOOK(E);
            const float v0 = __uint_as_float(E.z);
            const uint8_t *lp = d.map + E.x + lane * (uint32_t)C;
            const int32_t c = (int32_t)x;
            const int32_t top = c + D < C - 1 ? c + D : C - 1;
            const int32_t cl = first_occ(lp, c + 1, top);
            float x2, v2;
            uint32_t rp = 0, re = 0;
            bool have_route = false;
            scanned += (uint32_t)((cl >= 0 ? cl : top) - c);
            if (cl >= 0) {
                const float vl = (float)lp[cl];
                const float gap = ((float)cl - x) - p.L;
                idm_follow(p, x, v, v0, gap, vl, x2, v2);
                const float lim = (float)cl - p.L;
                if (x2 > lim) {
                    x2 = x > lim ? x : lim;
                    v2 = v2 < vl ? v2 : vl;
                }
            } else {
                bool stop = false;
                if (c + D >= C) {
                    rp = S.rp[i];
                    re = S.rend[i];
                    have_route = true;
                    if (rp + 1 < re) {
                        const int32_t en = (int32_t)d.route[rp + 1];
                        const uint4 En = d.edge[en];
                        const int32_t nle = E_LANES(En);
                        const int32_t ln = (int32_t)lane < nle - 1 ? (int32_t)lane : nle - 1;
                        stop = !entry_free(d, En, en, ln);
                        // route position (8), next edge record (16) and flags (4), entry window
                        scanned += 28u + (uint32_t)p.W;
                    }
                }
                if (stop) {
                    const float gap = (float)C - x;
                    idm_follow(p, x, v, v0, gap, 0.0f, x2, v2);
                    const float lim = (float)(C - 1);
                    if (x2 > lim) {
                        x2 = x > lim ? x : lim;
                        v2 = 0.0f;
                    }
                } else {
                    free_move(p, x, v, v0, x2, v2);
                }
            }
            uint32_t kind = K_MOVE;
            if (x2 >= (float)C) {
                if (!have_route) {
                    rp = S.rp[i];
                    re = S.rend[i];
                }
                if (rp + 1 >= re) {
                    kind = K_ARRIVE;
                } else {
                    const int32_t en = (int32_t)d.route[rp + 1];
                    const uint4 En = d.edge[en];
                    const int32_t nle = E_LANES(En);
                    const int32_t ln = (int32_t)lane < nle - 1 ? (int32_t)lane : nle - 1;
                    const uint32_t tgt = En.w + (uint32_t)ln;
                    kind = K_CLAIM;
                    d.scl[i] = tgt;
                    d.sxo[i] = x;
                    atomicMin(&d.claims[tgt], S.id[i]);
                }
            }
            S.x[i] = x2;
            S.v[i] = v2;
            S.m[i] = lane | (kind << M_KIND_SHIFT) | ((uint32_t)c << M_CELL_SHIFT);
        } else {
            const uint32_t pos = wlo + (uint32_t)(it - n);
            const uint32_t j = d.dep_order[pos];
            if (d.status[j] != ST_WAIT) continue;
            const uint32_t r0 = d.route_off[j];
            const int32_t e0 = (int32_t)d.route[r0];
            const uint4 E0 = d.edge[e0];
            const uint32_t loc = j - d.scen_tbase[d.escen[e0]];
            const int32_t l0 = (int32_t)(loc % (uint32_t)E_LANES(E0));
            const bool ok = entry_free(d, E0, e0, l0);
            d.dclaim[j] = ok ? 1 : 0;
            if (ok) atomicMin(&d.claims[E0.w + (uint32_t)l0], j);
        }
    }
    if (alive) atomicAdd(&cnt.c[P_VSTEPS], alive);
    if (scanned) atomicAdd(&cnt.c[P_SCAN], scanned);
    counts_flush(d, &cnt);
}

// ---------------------------------------------------------------------------
// resolve: apply entries, losses, arrivals; commit occupancy; statistics

__global__ __launch_bounds__(1024) void k_resolve(Dev d) {
    __shared__ BlockCounts cnt;
    __shared__ unsigned int s_wmin, s_arr, s_ev;
    if (threadIdx.x == 0) {
        s_wmin = 0xffffffffu;
        s_arr = 0;
        s_ev = 0;
    }
    counts_init(&cnt);
    Ctrl *ctl = d.ctrl;
    const int32_t k = ctl->k;
    const uint32_t n = ctl->n_slots;
    const uint32_t wlo = ctl->wait_lo;
    const uint32_t dhi = dep_hi_of(d, k);
    const uint32_t ncand = dhi > wlo ? dhi - wlo : 0;
    const Slots S = d.buf[ctl->cur];
    uint64_t lo, hi;
    block_range((uint64_t)n + ncand, lo, hi);
    for (uint64_t it = lo + threadIdx.x; it < hi; it += blockDim.x) {
        if (it < n) {
            const uint32_t i = (uint32_t)it;
            const uint32_t m = S.m[i];
            if (m & M_DEAD) continue;
            const uint32_t kind = (m >> M_KIND_SHIFT) & 3u;
            const uint32_t lane = m & M_LANE;
            const int32_t oc = (int32_t)(m >> M_CELL_SHIFT);
            const int32_t e = S.e[i];
            const uint4 E = d.edge[e];
            const int32_t C = E_CELLS(E);
            uint8_t *lp = d.map + E.x + lane * (uint32_t)C;
            if (kind == K_ARRIVE) {
                lp[oc] = FREE_BYTE;
                const uint32_t id = S.id[i];
                d.status[id] = ST_DONE;
                d.arrival[id] = k + 1;
                add_exit(d, e, S.ent[i], k + 1);
                S.m[i] = M_DEAD;
                atomicAdd(&cnt.c[P_ARRIVED], 1u);
                atomicAdd(&s_arr, 1u);
                s_ev = 1;
            } else if (kind == K_CLAIM) {
                const uint32_t tgt = d.scl[i];
                const uint32_t id = S.id[i];
                if (d.claims[tgt] == id) {
                    d.claims[tgt] = 0xffffffffu;
                    lp[oc] = FREE_BYTE;
                    const uint32_t rp = S.rp[i] + 1;
                    const int32_t en = (int32_t)d.route[rp];
                    const uint4 En = d.edge[en];
                    const uint32_t ln = tgt - En.w;
                    const float v2 = S.v[i];
                    d.map[En.x + ln * (uint32_t)E_CELLS(En)] = speed_byte(v2);
                    add_exit(d, e, S.ent[i], k + 1);
                    add_entry(d, en, k + 1);
                    S.e[i] = en;
                    S.x[i] = 0.0f;
                    S.rp[i] = rp;
                    S.ent[i] = k + 1;
                    S.m[i] = ln | M_ENTERED;
                    atomicAdd(&cnt.c[P_TRANSFERS], 1u);
                    s_ev = 1;
                } else {
                    const float xo = d.sxo[i];
                    const float lim = (float)(C - 1);
                    const float xn = xo > lim ? xo : lim;
                    S.x[i] = xn;
                    S.v[i] = 0.0f;
                    const int32_t nc = (int32_t)xn;
                    if (nc != oc) lp[oc] = FREE_BYTE;
                    lp[nc] = speed_byte(0.0f);
                    atomicAdd(&cnt.c[P_LOST], 1u);
                }
            } else {
                const int32_t nc = (int32_t)S.x[i];
                if (nc != oc) lp[oc] = FREE_BYTE;
                lp[nc] = speed_byte(S.v[i]);
            }
        } else {
            const uint32_t pos = wlo + (uint32_t)(it - n);
            const uint32_t j = d.dep_order[pos];
            if (d.status[j] != ST_WAIT) continue;
            const uint32_t r0 = d.route_off[j];
            const int32_t e0 = (int32_t)d.route[r0];
            const uint4 E0 = d.edge[e0];
            const uint32_t loc = j - d.scen_tbase[d.escen[e0]];
            const uint32_t l0 = loc % (uint32_t)E_LANES(E0);
            const uint32_t tgt = E0.w + l0;
            if (d.claims[tgt] == j) {
                d.claims[tgt] = 0xffffffffu;
                d.status[j] = ST_ACTIVE;
                const uint32_t ns = n + atomicAdd(&ctl->n_new, 1u);
                S.x[ns] = 0.0f;
                S.v[ns] = 0.0f;
                S.e[ns] = e0;
                S.m[ns] = l0 | M_ENTERED;
                S.id[ns] = j;
                S.rp[ns] = r0;
                S.rend[ns] = d.route_off[j + 1];
                S.ent[ns] = k + 1;
                d.map[E0.x + l0 * (uint32_t)E_CELLS(E0)] = speed_byte(0.0f);
                add_entry(d, e0, k + 1);
                atomicAdd(&cnt.c[P_DEPARTS], 1u);
                s_ev = 1;
            } else {
                if (d.dclaim[j]) atomicAdd(&cnt.c[P_LOST], 1u);
                atomicMin(&s_wmin, pos);
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (s_wmin != 0xffffffffu) atomicMin(&ctl->wait_lo_next, s_wmin);
        if (s_arr) atomicAdd(&ctl->arr_step, s_arr);
        if (s_ev) ctl->events = 1;
    }
    counts_flush(d, &cnt);
}

// ---------------------------------------------------------------------------
// lane change: decided on the map after the longitudinal move

__global__ __launch_bounds__(1024) void k_lanechg(Dev d) {
    __shared__ BlockCounts cnt;
    counts_init(&cnt);
    Ctrl *ctl = d.ctrl;
    const int32_t k = ctl->k;
    const uint32_t n = ctl->n_slots;  // vehicles that departed this step sit above n
    const Slots S = d.buf[ctl->cur];
    const Params &p = d.p;
    uint64_t lo, hi;
    block_range(n, lo, hi);
    for (uint64_t it = lo + threadIdx.x; it < hi; it += blockDim.x) {
        const uint32_t i = (uint32_t)it;
        const uint32_t m = S.m[i];
        if (m & (M_DEAD | M_ENTERED)) continue;
        const float x = S.x[i];
        const int32_t e = S.e[i];
        const uint4 E = d.edge[e];
        const int32_t C = E_CELLS(E);
        const float dist = (float)C - x;
        if (!(dist < p.x0)) continue;  // probability 0: no draw can succeed
        const uint32_t rp = S.rp[i];
        if (rp + 1 >= S.rend[i]) continue;  // last edge
        const int32_t en = (int32_t)d.route[rp + 1];
        const uint32_t ax = d.aux[en];
        const int32_t rank = (int32_t)(ax & 0xffu), deg = (int32_t)((ax >> 8) & 0xffu);
        const int32_t lane = (int32_t)(m & M_LANE);
        const int32_t req = (rank * E_LANES(E)) / deg;
        if (req == lane) continue;
        const int32_t dir = req > lane ? 1 : -1;
        if (((k & 1) == 0 && dir > 0) || ((k & 1) == 1 && dir < 0)) continue;
        const float prob = 1.0f - dist / p.x0;
        const int32_t sc = d.escen[e];
        const uint32_t loc = S.id[i] - d.scen_tbase[sc];
        const uint64_t h = mix64(d.scen_seed[sc] ^ (((uint64_t)loc << 32) | (uint64_t)(uint32_t)k));
        if (!((float)(h >> 40) < prob * 16777216.0f)) continue;
        atomicAdd(&cnt.c[P_LC_TRY], 1u);
        const int32_t lt = lane + dir;
        const int32_t c = (int32_t)x;
        const uint8_t *lp = d.map + E.x + (uint32_t)lt * (uint32_t)C;
        if (lp[c] != FREE_BYTE) continue;
        const float v = S.v[i];
        const int32_t D = E_LOOK(E);
        bool ok = true;
        const int32_t top = c + D < C - 1 ? c + D : C - 1;
        const int32_t ca = first_occ(lp, c + 1, top);
        if (ca >= 0) {
            const float va = (float)lp[ca];
            const float g_lead = ((float)ca - x) - p.L;
            const float t = (p.al_i * v) - (p.al_a * va);
            const float crit = p.g_a + (t > 0.0f ? t : 0.0f);
            if (!(g_lead >= crit)) ok = false;
        }
        const int32_t bot = c - D > 0 ? c - D : 0;
        const int32_t cb = last_occ(lp, c - 1, bot);
        if (ok && cb >= 0) {
            const float vb = (float)lp[cb];
            const float g_lag = (x - p.L) - (float)(cb + 1);
            const float t = (p.al_b * vb) - (p.al_i * v);
            const float crit = p.g_b + (t > 0.0f ? t : 0.0f);
            if (!(g_lag >= crit)) ok = false;
        }
        if (ok) {
            S.m[i] = (uint32_t)lt | ((uint32_t)lane << M_OLDLANE_SHIFT);
            d.lc_list[atomicAdd(&ctl->n_lc, 1u)] = i;
            atomicAdd(&cnt.c[P_LC_OK], 1u);
        }
    }
    counts_flush(d, &cnt);
}

// ---------------------------------------------------------------------------
// commit: lane changes into the map; the last block closes the step

__device__ void end_of_step(const Dev &d) {
    Ctrl *c = d.ctrl;
    const int32_t k = c->k;
    const uint32_t dhi = dep_hi_of(d, k);
    const int64_t alive0 = c->n_alive;
    c->watchdog = (alive0 > 0 && c->events == 0) ? c->watchdog + 1 : 0;
    c->n_alive = alive0 + (int64_t)c->n_new - (int64_t)c->arr_step;
    c->n_slots += c->n_new;
    c->n_new = 0;
    c->arr_step = 0;
    c->n_lc = 0;
    c->events = 0;
    const uint32_t wn = c->wait_lo_next;
    c->wait_lo = wn < dhi ? wn : dhi;
    c->wait_lo_next = 0xffffffffu;
    c->k = k + 1;
}

__global__ __launch_bounds__(1024) void k_commit(Dev d) {
    Ctrl *ctl = d.ctrl;
    const uint32_t nlc = ctl->n_lc;
    const Slots S = d.buf[ctl->cur];
    for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < nlc; q += gridDim.x * blockDim.x) {
        const uint32_t i = d.lc_list[q];
        const uint32_t m = S.m[i];
        const uint32_t lt = m & M_LANE, lo = (m >> M_OLDLANE_SHIFT) & M_LANE;
        const uint4 E = d.edge[S.e[i]];
        const uint32_t C = (uint32_t)E_CELLS(E);
        const uint32_t c = (uint32_t)(int32_t)S.x[i];
        d.map[E.x + lo * C + c] = FREE_BYTE;
        d.map[E.x + lt * C + c] = speed_byte(S.v[i]);
        S.m[i] = lt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned int t = atomicAdd(&ctl->done_commit, 1u);
        if (t == gridDim.x - 1) {
            __threadfence();
            end_of_step(d);
            ctl->done_commit = 0;
        }
    }
}

// ---------------------------------------------------------------------------
// compact: live slots of the current buffer -> the other buffer

__global__ __launch_bounds__(1024) void k_compact(Dev d) {
    Ctrl *ctl = d.ctrl;
    const uint32_t n = ctl->n_slots;
    const uint32_t cur = ctl->cur;
    const Slots A = d.buf[cur], B = d.buf[cur ^ 1u];
    uint64_t lo, hi;
    block_range(n, lo, hi);
    const uint32_t lane = threadIdx.x & 63u;
    for (uint64_t base = lo; base < hi; base += blockDim.x) {
        const uint64_t it = base + threadIdx.x;
        const bool live = it < hi && !(A.m[(uint32_t)it] & M_DEAD);
        const uint64_t mask = __ballot(live);
        uint32_t dst = 0;
        if (lane == 0 && mask) dst = atomicAdd(&ctl->n_comp, (uint32_t)__popcll(mask));
        dst = __shfl(dst, 0);
        if (live) {
            const uint32_t i = (uint32_t)it;
            const uint32_t o = dst + (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
            B.x[o] = A.x[i];
            B.v[o] = A.v[i];
            B.e[o] = A.e[i];
            B.m[o] = A.m[i];
            B.id[o] = A.id[i];
            B.rp[o] = A.rp[i];
            B.rend[o] = A.rend[i];
            B.ent[o] = A.ent[i];
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned int t = atomicAdd(&ctl->done_compact, 1u);
        if (t == gridDim.x - 1) {
            __threadfence();
            ctl->n_slots = ctl->n_comp;
            ctl->n_comp = 0;
            ctl->cur = cur ^ 1u;
            ctl->done_compact = 0;
        }
    }
}

// ---------------------------------------------------------------------------

void launch_move(const Dev &d, int blocks, int threads, hipStream_t s) {
    hipLaunchKernelGGL(k_move, dim3(blocks), dim3(threads), 0, s, d);
}
void launch_resolve(const Dev &d, int blocks, int threads, hipStream_t s) {
    hipLaunchKernelGGL(k_resolve, dim3(blocks), dim3(threads), 0, s, d);
}
void launch_lanechg(const Dev &d, int blocks, int threads, hipStream_t s) {
    hipLaunchKernelGGL(k_lanechg, dim3(blocks), dim3(threads), 0, s, d);
}
void launch_commit(const Dev &d, int blocks, int threads, hipStream_t s) {
    hipLaunchKernelGGL(k_commit, dim3(blocks), dim3(threads), 0, s, d);
}
void launch_compact(const Dev &d, int blocks, int threads, hipStream_t s) {
    hipLaunchKernelGGL(k_compact, dim3(blocks), dim3(threads), 0, s, d);
}

}  // namespace lpsim
