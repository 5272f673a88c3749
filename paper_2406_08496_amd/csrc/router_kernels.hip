// router_kernels.hip -- shortest-time trees toward many destinations at once
// on the GPU, for the traffic-assignment loop's routing step.
//
// For every destination t the trees solve, in float64,
//     dist[t] = 0,   dist[x] = min over out-edges e = (x -> y) of dist[y] + cost[e],
// the fixed point that a backward Dijkstra settles, and give each node the
// lowest-numbered out-edge that attains the minimum (so the tree does not
// depend on any processing order).  The distances come from label-correcting
// relaxation over a frontier of (destination, node) pairs: a pair whose
// distance dropped relaxes the in-edges of its node with a 64-bit atomic
// minimum on the distance bits (non-negative doubles order like their bit
// patterns), and every drop queues the upstream pair once.  The fixed point
// is unique, so the order of relaxations does not change it.
//
// Relaxing in hop order alone settles a pair many times over (about 23
// times on the regional network with congested costs), so the frontier is
// split by distance (near-far, Davidson et al. 2014): a round relaxes only
// pairs at most a threshold tau from their destination; drops above tau wait
// in a far pile, and when the near frontier runs dry tau moves up by delta
// (or to the nearest waiting pair) and the far pile is split again.
//
// The tree edges are then picked in a separate pass that compares each
// out-edge's candidate with the final distance, exactly as the Dijkstra's
// tie rule does.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "lpsim.h"

namespace lpsim_route {

constexpr unsigned long long INF_BITS = 0x7ff0000000000000ull;  // +infinity
constexpr int THREADS = 256;
constexpr int GRID = 2048;         // blocks of the grid-stride kernels
constexpr int PUSH_BUF = 4 * THREADS;  // per-block staging of queued pairs
constexpr double DELTA_COSTS = 16.0;    // near-far threshold step, in mean edge costs
constexpr int32_t ROUNDS_AHEAD = 16;    // first group of rounds launched between reads of the state

// Round state of one destination batch's relaxation, on the device: a
// one-thread kernel after each round takes the step between rounds, so the
// host launches rounds ahead and only reads `done` every few rounds.
struct RoundCtl {
    uint32_t count[3];             // near frontier sizes, by round mod 3
    uint32_t far_count[2];         // the two far piles
    uint32_t done;                 // both frontiers empty
    uint32_t split;                // the pile was split after round `round`: the
                                   // next round is round + 1 with the piles switched
    int32_t round, fc;             // round number, far pile being filled
    unsigned long long far_min;    // least distance bits entering the pile
    double tau, delta;             // threshold and its step
};

struct GpuRouter {
    int32_t n = 0, m = 0;
    // incoming edges per node (CSR) with their upstream node; outgoing
    // edges per node in increasing edge id with their downstream node
    int32_t *in_off = nullptr, *in_src = nullptr, *in_edge = nullptr;
    int32_t *out_off = nullptr, *out_dst = nullptr, *out_edge = nullptr;
    double *in_cost = nullptr, *out_cost = nullptr, *cost = nullptr;
    // per destination batch
    size_t cap_pairs = 0;        // destinations x nodes the buffers hold
    unsigned long long *dist = nullptr;
    uint2 *front[2] = {nullptr, nullptr};
    uint32_t *flags[2] = {nullptr, nullptr};  // one bit per pair
    RoundCtl *ctl = nullptr;
    uint32_t *count = nullptr;                // ctl->count
    int32_t *targets = nullptr;
    // tree edge of every (destination, node) of the last solve
    int32_t *nx = nullptr;
    size_t nx_cap = 0;
    // trips of the last solve: origin node, destination index; destination
    // nodes; downstream node of each edge (for walking the trees)
    int32_t *trip_origin = nullptr, *trip_dest = nullptr, *dest_node = nullptr, *edge_dst = nullptr;
    size_t trip_cap = 0, dest_cap = 0;
    int64_t n_trips = 0;
    uint8_t *take = nullptr;       // [n_trips] trips that take their new route
    int32_t *len = nullptr;        // [n_trips] new route lengths
    int64_t *poff = nullptr;       // [n_trips + 1] offsets of the packed new routes
    int32_t *packed = nullptr;     // the new routes, packed
    size_t packed_cap = 0;
    bool take_all = true;          // the last length walk took every trip
    // page-locked host copies of the offsets and of the packed routes, kept
    // across calls (fast transfers, no fresh pages per call)
    int64_t *poff_h = nullptr;
    size_t poff_h_cap = 0;
    RoundCtl *ctl_h = nullptr;     // page-locked copy of ctl read between groups of rounds
    int32_t *packed_h = nullptr;
    size_t packed_h_cap = 0;
    uint32_t *bad = nullptr;       // a trip whose destination cannot be reached
    // far pile: pairs whose distance dropped above the threshold
    uint2 *far[2] = {nullptr, nullptr};
    uint32_t *far_flags = nullptr;             // one bit per pair in the pile
    uint32_t *far_count = nullptr;             // ctl->far_count
    unsigned long long *far_min = nullptr;     // &ctl->far_min
    std::vector<void *> allocs;
};

__global__ void k_costs(GpuRouter g) {
    for (int32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < g.m; j += gridDim.x * blockDim.x) {
        g.in_cost[j] = g.cost[g.in_edge[j]];
        g.out_cost[j] = g.cost[g.out_edge[j]];
    }
}

// all distances infinite but each destination's own, which starts the frontier
__global__ void k_init(GpuRouter g, int32_t nd) {
    const size_t total = (size_t)nd * g.n;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x)
        g.dist[i] = INF_BITS;
    const size_t words = (total + 31) / 32;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += (size_t)gridDim.x * blockDim.x) {
        g.flags[0][i] = 0;
        g.flags[1][i] = 0;
        g.far_flags[i] = 0;
    }
}

__global__ void k_seed(GpuRouter g, int32_t nd, double delta) {
    for (int32_t d = blockIdx.x * blockDim.x + threadIdx.x; d < nd; d += gridDim.x * blockDim.x) {
        const size_t pair = (size_t)d * g.n + (size_t)g.targets[d];
        g.dist[pair] = 0ull;
        g.front[0][d] = make_uint2((uint32_t)d, (uint32_t)g.targets[d]);
        atomicOr(&g.flags[0][pair >> 5], 1u << (pair & 31));
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        g.count[0] = (uint32_t)nd;
        g.count[1] = 0;
        g.count[2] = 0;
        g.far_count[0] = 0;
        g.far_count[1] = 0;
        *g.far_min = ~0ull;
        g.ctl->done = 0;
        g.ctl->split = 0;
        g.ctl->round = 0;
        g.ctl->fc = 0;
        g.ctl->tau = delta;
        g.ctl->delta = delta;
    }
}

// queue of one block's pushes, flushed into a list with one atomic
struct PushBuf {
    uint2 item[PUSH_BUF / 2];
    uint32_t n, base;
};

__device__ __forceinline__ void push(PushBuf &b, uint2 *list, uint32_t *count, uint2 it) {
    const uint32_t k = atomicAdd(&b.n, 1u);
    if (k < PUSH_BUF / 2) b.item[k] = it;
    else list[atomicAdd(count, 1u)] = it;
}

__device__ __forceinline__ void flush(PushBuf &b, uint2 *list, uint32_t *count) {
    const uint32_t nb = b.n < PUSH_BUF / 2 ? b.n : PUSH_BUF / 2;
    if (threadIdx.x == 0 && nb) b.base = atomicAdd(count, nb);
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < nb; k += blockDim.x) list[b.base + k] = b.item[k];
}

// least of the block's values, then one atomic for the block
__device__ __forceinline__ void block_min(unsigned long long v, unsigned long long *dst, unsigned long long *s_min) {
    if (v != ~0ull) atomicMin(s_min, v);
    __syncthreads();
    if (threadIdx.x == 0 && *s_min != ~0ull) atomicMin(dst, *s_min);
}

// round r: every queued pair of near frontier r % 2 relaxes the in-edges of
// its node; a drop to at most tau queues the upstream pair (once) in the
// other near frontier, a drop above tau puts it (once) in the far pile.  A
// processed pair's queue flag is cleared here (nothing queues into this
// round's frontier during the round), and the size counter of round r + 2 is
// reset (round r - 1, its last reader, has finished).  Nothing runs once the
// batch is done (the host launches rounds ahead).
__global__ __launch_bounds__(THREADS) void k_relax(GpuRouter g) {
    __shared__ PushBuf bn, bf;
    __shared__ unsigned long long s_min;
    const RoundCtl *const c = g.ctl;
    const uint32_t done = c->done, split = c->split;
    const int32_t round = c->round + (int32_t)split, fc = c->fc ^ (int32_t)split;
    const double tau = c->tau;
    if (done) return;
    const int32_t cur = round & 1;
    const uint32_t nf = g.count[round % 3];
    const uint2 *front = g.front[cur];
    uint32_t *flags = g.flags[cur];
    uint2 *next = g.front[cur ^ 1];
    uint32_t *nflags = g.flags[cur ^ 1];
    uint32_t *ncount = &g.count[(round + 1) % 3];
    const unsigned long long tau_b = (unsigned long long)__double_as_longlong(tau);
    if (blockIdx.x == 0 && threadIdx.x == 0) g.count[(round + 2) % 3] = 0;
    for (uint32_t t0 = blockIdx.x * blockDim.x; t0 < nf; t0 += gridDim.x * blockDim.x) {
        if (threadIdx.x == 0) {
            bn.n = 0;
            bf.n = 0;
            s_min = ~0ull;
        }
        __syncthreads();
        unsigned long long fmin = ~0ull;
        const uint32_t t = t0 + threadIdx.x;
        if (t < nf) {
            const uint2 it = front[t];
            const size_t row = (size_t)it.x * g.n;
            {
                // leaves the queue; other pairs of the same flag word are in
                // this frontier too, so the word can simply be cleared
                const size_t pair = row + it.y;
                flags[pair >> 5] = 0u;
            }
            unsigned long long *dd = g.dist + row;
            const double dy = __longlong_as_double((long long)dd[it.y]);
            for (int32_t j = g.in_off[it.y]; j < g.in_off[it.y + 1]; ++j) {
                const int32_t x = g.in_src[j];
                const unsigned long long cb = (unsigned long long)__double_as_longlong(dy + g.in_cost[j]);
                if (cb >= dd[x]) continue;
                const unsigned long long old = atomicMin(&dd[x], cb);
                if (cb >= old) continue;
                const size_t pair = row + (size_t)x;
                const uint32_t bit = 1u << (pair & 31);
                if (cb <= tau_b) {
                    if (atomicOr(&nflags[pair >> 5], bit) & bit) continue;  // already queued
                    push(bn, next, ncount, make_uint2(it.x, (uint32_t)x));
                } else {
                    fmin = cb < fmin ? cb : fmin;
                    if (atomicOr(&g.far_flags[pair >> 5], bit) & bit) continue;  // already in the pile
                    push(bf, g.far[fc], &g.far_count[fc], make_uint2(it.x, (uint32_t)x));
                }
            }
        }
        __syncthreads();
        flush(bn, next, ncount);
        flush(bf, g.far[fc], &g.far_count[fc]);
        block_min(fmin, g.far_min, &s_min);
        __syncthreads();
    }
}

// the step between rounds, after round r: with the next near frontier empty
// the batch is done if the pile is empty too; else tau moves up by delta, or
// at once to the nearest waiting pair, and the pile is split (k_split) before
// round r + 1
__global__ void k_round_ctl(GpuRouter g) {
    RoundCtl *const c = g.ctl;
    const RoundCtl v = *c;  // the whole block in one round trip
    if (v.done) return;
    // the round that just ran followed a split if one is pending
    const int32_t round = v.round + (int32_t)v.split, fc = v.fc ^ (int32_t)v.split;
    c->fc = fc;
    c->split = 0;
    if (v.count[(round + 1) % 3] != 0) {
        c->round = round + 1;
    } else if (v.far_count[fc] == 0) {
        c->round = round;
        c->done = 1;
    } else {
        const double fmin = __longlong_as_double((long long)v.far_min);
        const double up = v.tau + v.delta;
        c->round = round;
        c->tau = up < fmin ? fmin : up;
        c->far_count[fc ^ 1] = 0;
        c->far_min = ~0ull;
        c->split = 1;
    }
}

// the near frontier ran dry: the far pile (buffer fc) is split by the new
// threshold tau; pairs now within it join the next near frontier (round r +
// 1), the others move to pile fc ^ 1, whose least distance is recorded.
// Launched after every round, it does nothing unless k_round_ctl asked for it.
__global__ __launch_bounds__(THREADS) void k_split(GpuRouter g) {
    __shared__ PushBuf bn, bf;
    __shared__ unsigned long long s_min;
    const RoundCtl *const c = g.ctl;
    const uint32_t done = c->done, split = c->split;
    const int32_t round = c->round, fc = c->fc;
    const double tau = c->tau;
    if (done || !split) return;
    const int32_t nxt = (round + 1) & 1;
    uint2 *next = g.front[nxt];
    uint32_t *nflags = g.flags[nxt];
    uint32_t *ncount = &g.count[(round + 1) % 3];
    const uint32_t nfar = g.far_count[fc];
    const unsigned long long tau_b = (unsigned long long)__double_as_longlong(tau);
    for (uint32_t t0 = blockIdx.x * blockDim.x; t0 < nfar; t0 += gridDim.x * blockDim.x) {
        if (threadIdx.x == 0) {
            bn.n = 0;
            bf.n = 0;
            s_min = ~0ull;
        }
        __syncthreads();
        unsigned long long fmin = ~0ull;
        const uint32_t t = t0 + threadIdx.x;
        if (t < nfar) {
            const uint2 it = g.far[fc][t];
            const size_t pair = (size_t)it.x * g.n + it.y;
            const uint32_t bit = 1u << (pair & 31);
            const unsigned long long db = g.dist[pair];
            if (db <= tau_b) {
                atomicAnd(&g.far_flags[pair >> 5], ~bit);
                if (!(atomicOr(&nflags[pair >> 5], bit) & bit)) push(bn, next, ncount, it);
            } else {
                fmin = db;
                push(bf, g.far[fc ^ 1], &g.far_count[fc ^ 1], it);
            }
        }
        __syncthreads();
        flush(bn, next, ncount);
        flush(bf, g.far[fc ^ 1], &g.far_count[fc ^ 1]);
        block_min(fmin, g.far_min, &s_min);
        __syncthreads();
    }
}

// tree edge of every (destination, node): the lowest out-edge whose
// candidate equals the node's distance (-1 at the destination or if the
// destination cannot be reached)
__global__ void k_ties(GpuRouter g, int32_t nd, int32_t d0) {
    const size_t total = (size_t)nd * g.n;
    int32_t *nx = g.nx + (size_t)d0 * g.n;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
        const int32_t d = (int32_t)(i / g.n), x = (int32_t)(i - (size_t)d * g.n);
        int32_t best = -1;
        const unsigned long long dx = g.dist[i];
        if (x != g.targets[d] && dx != INF_BITS) {
            const unsigned long long *dd = g.dist + (size_t)d * g.n;
            for (int32_t j = g.out_off[x]; j < g.out_off[x + 1]; ++j) {
                const double cand = __longlong_as_double((long long)dd[g.out_dst[j]]) + g.out_cost[j];
                if ((unsigned long long)__double_as_longlong(cand) == dx) {
                    best = g.out_edge[j];
                    break;
                }
            }
        }
        nx[i] = best;
    }
}

// every trip's origin has a tree edge toward its destination
__global__ void k_reachable(GpuRouter g) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < g.n_trips;
         i += (int64_t)gridDim.x * blockDim.x)
        if (g.nx[(size_t)g.trip_dest[i] * g.n + g.trip_origin[i]] < 0) atomicOr(g.bad, 1u);
}

// length of each new route: the walk down the destination's tree
__global__ void k_walk_len(GpuRouter g) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < g.n_trips;
         i += (int64_t)gridDim.x * blockDim.x) {
        int32_t l = 0;
        if (g.take == nullptr || g.take[i]) {
            const int32_t d = g.trip_dest[i], t = g.dest_node[d];
            const int32_t *nx = g.nx + (size_t)d * g.n;
            int32_t u = g.trip_origin[i];
            while (u != t && l <= g.n) {
                u = g.edge_dst[nx[u]];
                ++l;
            }
        }
        g.len[i] = l;
    }
}

// the new routes, packed at offsets poff
__global__ void k_walk_write(GpuRouter g) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < g.n_trips;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (g.take != nullptr && !g.take[i]) continue;
        const int32_t d = g.trip_dest[i], t = g.dest_node[d];
        const int32_t *nx = g.nx + (size_t)d * g.n;
        int32_t *o = g.packed + g.poff[i];
        int32_t *const end = g.packed + g.poff[i + 1];
        int32_t u = g.trip_origin[i];
        while (u != t && o < end) {
            const int32_t e = nx[u];
            *o++ = e;
            u = g.edge_dst[e];
        }
    }
}

static int32_t status(hipError_t e) { return e == hipSuccess ? LPSIM_OK : LPSIM_EDEVICE; }

template <class T>
static hipError_t alloc(GpuRouter *g, T *&p, size_t n) {
    void *q = nullptr;
    const hipError_t e = hipMalloc(&q, std::max<size_t>(n, 1) * sizeof(T));
    if (e != hipSuccess) return e;
    g->allocs.push_back(q);
    p = static_cast<T *>(q);
    return hipSuccess;
}

void gpu_router_free(GpuRouter *g) {
    if (!g) return;
    for (void *p : g->allocs) (void)hipFree(p);
    if (g->poff_h) (void)hipHostFree(g->poff_h);
    if (g->ctl_h) (void)hipHostFree(g->ctl_h);
    if (g->packed_h) (void)hipHostFree(g->packed_h);
    delete g;
}

#define RCHK(call)                                   \
    do {                                             \
        const hipError_t e_ = (call);                \
        if (e_ != hipSuccess) return status(e_);     \
    } while (0)

// Trees toward `nd` destinations (host ids) for edge costs `cost` (host,
// n_edges): next_edge (host, nd x n_nodes) receives each node's tree edge.
// The graph (host CSR arrays) is uploaded on the first call.
int32_t gpu_router_solve(GpuRouter **gp, int32_t n_nodes, int32_t n_edges, const int64_t *in_off_h,
                         const int32_t *in_edges_h, const int32_t *in_src_h, const int32_t *src_h,
                         const int32_t *dst_h, const double *cost_h, const int32_t *dests, int32_t nd,
                         int64_t n_trips, const int32_t *origin_h, const int32_t *dest_idx_h, hipStream_t s) {
    if (!*gp) {
        GpuRouter *g = new (std::nothrow) GpuRouter();
        if (!g) return LPSIM_ENOMEM;
        *gp = g;
        g->n = n_nodes;
        g->m = n_edges;
        std::vector<int32_t> io((size_t)n_nodes + 1), oo((size_t)n_nodes + 1, 0), od((size_t)n_edges),
            oe((size_t)n_edges);
        for (size_t u = 0; u <= (size_t)n_nodes; ++u) io[u] = (int32_t)in_off_h[u];
        for (int32_t e = 0; e < n_edges; ++e) oo[(size_t)src_h[e] + 1]++;
        for (int32_t u = 0; u < n_nodes; ++u) oo[(size_t)u + 1] += oo[(size_t)u];
        {
            std::vector<int32_t> pos(oo.begin(), oo.end() - 1);
            for (int32_t e = 0; e < n_edges; ++e) {  // increasing edge id within each node
                const int32_t k = pos[(size_t)src_h[e]]++;
                oe[(size_t)k] = e;
                od[(size_t)k] = dst_h[e];
            }
        }
        RCHK(alloc(g, g->in_off, (size_t)n_nodes + 1));
        RCHK(alloc(g, g->in_src, (size_t)n_edges));
        RCHK(alloc(g, g->in_edge, (size_t)n_edges));
        RCHK(alloc(g, g->out_off, (size_t)n_nodes + 1));
        RCHK(alloc(g, g->out_dst, (size_t)n_edges));
        RCHK(alloc(g, g->out_edge, (size_t)n_edges));
        RCHK(alloc(g, g->in_cost, (size_t)n_edges));
        RCHK(alloc(g, g->out_cost, (size_t)n_edges));
        RCHK(alloc(g, g->cost, (size_t)n_edges));
        RCHK(alloc(g, g->ctl, 1));
        g->count = g->ctl->count;
        g->far_count = g->ctl->far_count;
        g->far_min = &g->ctl->far_min;
        RCHK(hipHostMalloc((void **)&g->ctl_h, sizeof(RoundCtl), hipHostMallocDefault));
        RCHK(alloc(g, g->bad, 1));
        RCHK(alloc(g, g->edge_dst, (size_t)n_edges));
        RCHK(hipMemcpy(g->edge_dst, dst_h, (size_t)n_edges * 4, hipMemcpyHostToDevice));
        RCHK(hipMemcpy(g->in_off, io.data(), io.size() * 4, hipMemcpyHostToDevice));
        RCHK(hipMemcpy(g->in_src, in_src_h, (size_t)n_edges * 4, hipMemcpyHostToDevice));
        RCHK(hipMemcpy(g->in_edge, in_edges_h, (size_t)n_edges * 4, hipMemcpyHostToDevice));
        RCHK(hipMemcpy(g->out_off, oo.data(), oo.size() * 4, hipMemcpyHostToDevice));
        RCHK(hipMemcpy(g->out_dst, od.data(), od.size() * 4, hipMemcpyHostToDevice));
        RCHK(hipMemcpy(g->out_edge, oe.data(), oe.size() * 4, hipMemcpyHostToDevice));
    }
    GpuRouter *g = *gp;
    if (g->n != n_nodes || g->m != n_edges) return LPSIM_EINVAL;
    // destinations per batch: distances, frontiers and flags of at most 256M pairs (about 7 GB)
    const int32_t per = std::max<int32_t>(1, std::min<int32_t>(nd, (int32_t)((256ll << 20) / n_nodes)));
    const size_t pairs = (size_t)per * (size_t)n_nodes;
    if (g->cap_pairs < pairs) {
        // grow the batch buffers (freed with the router)
        RCHK(alloc(g, g->dist, pairs));
        RCHK(alloc(g, g->front[0], pairs));
        RCHK(alloc(g, g->front[1], pairs));
        RCHK(alloc(g, g->flags[0], (pairs + 31) / 32));
        RCHK(alloc(g, g->flags[1], (pairs + 31) / 32));
        RCHK(alloc(g, g->targets, (size_t)per));
        RCHK(alloc(g, g->far[0], pairs));
        RCHK(alloc(g, g->far[1], pairs));
        RCHK(alloc(g, g->far_flags, (pairs + 31) / 32));
        g->cap_pairs = pairs;
    }
    // trees of all destinations, the trips and their destinations
    if (g->nx_cap < (size_t)nd * n_nodes) {
        RCHK(alloc(g, g->nx, (size_t)nd * n_nodes));
        g->nx_cap = (size_t)nd * n_nodes;
    }
    if (g->trip_cap < (size_t)n_trips) {
        RCHK(alloc(g, g->trip_origin, (size_t)n_trips));
        RCHK(alloc(g, g->trip_dest, (size_t)n_trips));
        RCHK(alloc(g, g->take, (size_t)n_trips));
        RCHK(alloc(g, g->len, (size_t)n_trips));
        RCHK(alloc(g, g->poff, (size_t)n_trips + 1));
        g->trip_cap = (size_t)n_trips;
    }
    if (g->dest_cap < (size_t)nd) {
        RCHK(alloc(g, g->dest_node, (size_t)nd));
        g->dest_cap = (size_t)nd;
    }
    g->n_trips = n_trips;
    RCHK(hipMemcpyAsync(g->trip_origin, origin_h, (size_t)n_trips * 4, hipMemcpyHostToDevice, s));
    RCHK(hipMemcpyAsync(g->trip_dest, dest_idx_h, (size_t)n_trips * 4, hipMemcpyHostToDevice, s));
    RCHK(hipMemcpyAsync(g->dest_node, dests, (size_t)nd * 4, hipMemcpyHostToDevice, s));
    // threshold step of the near-far split: a few mean edge costs
    double mean_cost = 0.0;
    for (int32_t e = 0; e < n_edges; ++e) mean_cost += cost_h[e];
    mean_cost /= std::max(1, n_edges);
    const double delta = DELTA_COSTS * mean_cost;
    RCHK(hipMemcpyAsync(g->cost, cost_h, (size_t)n_edges * 8, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_costs, dim3(GRID), dim3(THREADS), 0, s, *g);
    RCHK(hipGetLastError());
    for (int32_t d0 = 0; d0 < nd; d0 += per) {
        const int32_t nb = std::min(per, nd - d0);
        RCHK(hipMemcpyAsync(g->targets, dests + d0, (size_t)nb * 4, hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_init, dim3(GRID), dim3(THREADS), 0, s, *g, nb);
        hipLaunchKernelGGL(k_seed, dim3((nb + THREADS - 1) / THREADS), dim3(THREADS), 0, s, *g, nb, delta);
        RCHK(hipGetLastError());
        // rounds until the near frontier and the far pile are both empty,
        // launched ahead in groups; the host reads the state between groups
        // (rounds after the last one return at once).  Each round settles at
        // least one more hop of every shortest path within the threshold,
        // and the threshold only rises; past this bound something is wrong
        // (it cannot happen with finite positive costs)
        const int64_t max_rounds = 4ll * n_nodes + 1024;
        for (int32_t group = ROUNDS_AHEAD;; group = std::min(2 * group, 4 * ROUNDS_AHEAD)) {
            for (int32_t k = 0; k < group; ++k) {
                hipLaunchKernelGGL(k_relax, dim3(GRID), dim3(THREADS), 0, s, *g);
                hipLaunchKernelGGL(k_round_ctl, dim3(1), dim3(1), 0, s, *g);
                hipLaunchKernelGGL(k_split, dim3(GRID), dim3(THREADS), 0, s, *g);
            }
            RCHK(hipGetLastError());
            RCHK(hipMemcpyAsync(g->ctl_h, g->ctl, sizeof(RoundCtl), hipMemcpyDeviceToHost, s));
            RCHK(hipStreamSynchronize(s));
            if (g->ctl_h->done) break;
            if (g->ctl_h->round > max_rounds) return LPSIM_EDEVICE;
        }
        hipLaunchKernelGGL(k_ties, dim3(GRID), dim3(THREADS), 0, s, *g, nb, d0);
        RCHK(hipGetLastError());
    }
    const uint32_t zero = 0;
    uint32_t bad = 0;
    RCHK(hipMemcpyAsync(g->bad, &zero, 4, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_reachable, dim3(GRID), dim3(THREADS), 0, s, *g);
    RCHK(hipGetLastError());
    RCHK(hipMemcpyAsync(&bad, g->bad, 4, hipMemcpyDeviceToHost, s));
    RCHK(hipStreamSynchronize(s));
    return bad ? LPSIM_EINVAL : LPSIM_OK;
}

// Lengths of the new routes of the last GPU solve: new_len (host, n_trips)
// receives the length of each new route (0 where take[i] == 0; take NULL
// takes all).  The choice stays on the device for gpu_router_write.
int32_t gpu_router_lengths(GpuRouter *g, const uint8_t *take_h, int32_t *new_len, hipStream_t s) {
    if (!g) return LPSIM_ESTATE;
    const int64_t n = g->n_trips;
    if (take_h) RCHK(hipMemcpyAsync(g->take, take_h, (size_t)n, hipMemcpyHostToDevice, s));
    g->take_all = take_h == nullptr;
    GpuRouter gv = *g;
    if (g->take_all) gv.take = nullptr;
    hipLaunchKernelGGL(k_walk_len, dim3(GRID), dim3(THREADS), 0, s, gv);
    RCHK(hipGetLastError());
    RCHK(hipMemcpyAsync(new_len, g->len, (size_t)n * 4, hipMemcpyDeviceToHost, s));
    return status(hipStreamSynchronize(s));
}

// Page-locked host buffer of n_trips + 1 offsets for gpu_router_write (NULL
// if it cannot be allocated); the caller fills it with the exclusive prefix
// of the lengths from gpu_router_lengths.
int64_t *gpu_router_offsets(GpuRouter *g) {
    if (!g) return nullptr;
    const size_t need = (size_t)g->n_trips + 1;
    if (g->poff_h_cap < need) {
        if (g->poff_h) (void)hipHostFree(g->poff_h);
        g->poff_h = nullptr;
        g->poff_h_cap = 0;
        if (hipHostMalloc((void **)&g->poff_h, need * 8, hipHostMallocDefault) != hipSuccess) {
            g->poff_h = nullptr;
            return nullptr;
        }
        g->poff_h_cap = need;
    }
    return g->poff_h;
}

// The new routes of the trips chosen by the last gpu_router_lengths, walked
// on the device and copied back packed at the offsets in gpu_router_offsets'
// buffer; *packed points at them (page-locked, valid until the next call).
int32_t gpu_router_write(GpuRouter *g, const int32_t **packed, hipStream_t s) {
    if (!g || !g->poff_h) return LPSIM_ESTATE;
    const int64_t n = g->n_trips;
    const size_t total = (size_t)g->poff_h[n];
    if (g->packed_cap < total) {
        RCHK(alloc(g, g->packed, total));
        g->packed_cap = total;
    }
    if (g->packed_h_cap < std::max<size_t>(total, 1)) {
        if (g->packed_h) (void)hipHostFree(g->packed_h);
        g->packed_h = nullptr;
        g->packed_h_cap = 0;
        const size_t cap = std::max<size_t>(total, 1);
        if (hipHostMalloc((void **)&g->packed_h, cap * 4, hipHostMallocDefault) != hipSuccess) {
            g->packed_h = nullptr;
            return LPSIM_ENOMEM;
        }
        g->packed_h_cap = cap;
    }
    GpuRouter gv = *g;
    if (g->take_all) gv.take = nullptr;
    RCHK(hipMemcpyAsync(g->poff, g->poff_h, (size_t)(n + 1) * 8, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_walk_write, dim3(GRID), dim3(THREADS), 0, s, gv);
    RCHK(hipGetLastError());
    if (total) RCHK(hipMemcpyAsync(g->packed_h, g->packed, total * 4, hipMemcpyDeviceToHost, s));
    *packed = g->packed_h;
    return status(hipStreamSynchronize(s));
}

}  // namespace lpsim_route
