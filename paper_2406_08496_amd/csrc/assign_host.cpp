// assign_host.cpp -- static shortest-time routing for the traffic-assignment
// loop (the paper's title: accelerated traffic assignment; routes are the
// simulator's input, Section 3.1 vehicle data).
//
// For every distinct destination a backward Dijkstra (binary heap, float64
// costs) gives, for every node, the edge to take toward that destination.
// Among equally short choices the lower edge id wins, which makes the result
// independent of heap order and of the number of threads.  Destinations are
// spread over std::thread workers.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include <hip/hip_runtime.h>

#include "lpsim.h"

namespace lpsim_route {
struct GpuRouter;
void gpu_router_free(GpuRouter *g);
int32_t gpu_router_solve(GpuRouter **gp, int32_t n_nodes, int32_t n_edges, const int64_t *in_off_h,
                         const int32_t *in_edges_h, const int32_t *in_src_h, const int32_t *src_h,
                         const int32_t *dst_h, const double *cost_h, const int32_t *dests, int32_t nd,
                         int64_t n_trips, const int32_t *origin_h, const int32_t *dest_idx_h, hipStream_t s);
int32_t gpu_router_lengths(GpuRouter *g, const uint8_t *take_h, int32_t *new_len, hipStream_t s);
int64_t *gpu_router_offsets(GpuRouter *g);
int32_t gpu_router_write(GpuRouter *g, const int32_t **packed, hipStream_t s);
}  // namespace lpsim_route

struct lpsim_router {
    int32_t n_nodes = 0, n_edges = 0, n_threads = 1;
    std::vector<int32_t> src, dst;
    std::vector<int64_t> in_off;   // incoming edges per node (CSR)
    std::vector<int32_t> in_edges;
    std::vector<int32_t> in_src;   // upstream node of each in_edges entry
    std::vector<double> in_cost;   // cost of each in_edges entry (this solve)
    // last solve
    std::vector<int32_t> dests;      // distinct destination nodes
    std::vector<int32_t> dest_idx;   // per trip
    std::vector<int32_t> origin;     // per trip
    // tree edge per [dest][node] of the last host solve (a GPU solve keeps
    // its trees on the device and walks them there)
    std::vector<int32_t> next_edge;
    bool on_gpu = false;         // the last solve ran on the GPU
    void *gpu_stream = nullptr;  // and on this stream
    std::vector<int32_t> len;        // per trip, new route length (trips taking one)
    // lengths in len are those of the trips chosen by len_take (all trips if
    // len_all) for the last solve
    bool len_ok = false, len_all = false;
    std::vector<uint8_t> len_take;
    bool solved = false;
    lpsim_route::GpuRouter *gpu = nullptr;  // device copy of the graph (GPU solves)
};

namespace {

struct HeapItem {
    double key;
    int32_t node;
};

void tree_to(const lpsim_router &r, const double *cost, int32_t target, int32_t *nx, std::vector<double> &dist,
             std::vector<uint8_t> &done, std::vector<HeapItem> &heap) {
    const int32_t n = r.n_nodes;
    std::fill(dist.begin(), dist.end(), std::numeric_limits<double>::infinity());
    std::fill(done.begin(), done.end(), 0);
    for (int32_t u = 0; u < n; ++u) nx[u] = -1;
    auto cmp = [](const HeapItem &a, const HeapItem &b) { return a.key > b.key; };
    heap.clear();
    dist[target] = 0.0;
    heap.push_back({0.0, target});
    while (!heap.empty()) {
        std::pop_heap(heap.begin(), heap.end(), cmp);
        const HeapItem it = heap.back();
        heap.pop_back();
        const int32_t y = it.node;
        if (done[y]) continue;
        done[y] = 1;
        // incoming edges with their upstream node and cost stored side by
        // side: sequential reads instead of two gathers per edge
        for (int64_t j = r.in_off[y]; j < r.in_off[y + 1]; ++j) {
            const int32_t e = r.in_edges[j];
            const int32_t x = r.in_src[j];
            if (done[x]) continue;
            const double cand = dist[y] + r.in_cost[j];
            if (cand < dist[x] || (cand == dist[x] && e < nx[x])) {
                dist[x] = cand;
                nx[x] = e;
                heap.push_back({cand, x});
                std::push_heap(heap.begin(), heap.end(), cmp);
            }
        }
    }
}

template <class F>
void parallel_for(int32_t n_items, int32_t n_threads, F &&f) {
    std::atomic<int32_t> next{0};
    auto worker = [&]() {
        for (;;) {
            const int32_t i = next.fetch_add(1);
            if (i >= n_items) break;
            f(i);
        }
    };
    const int32_t nt = std::max(1, std::min(n_threads, n_items));
    std::vector<std::thread> pool;
    for (int32_t t = 1; t < nt; ++t) pool.emplace_back(worker);
    worker();
    for (auto &t : pool) t.join();
}

// out[0] = 0, out[i + 1] = out[i] + len_of(i) for i < n: chunk sums on the
// router's threads, their running total, then every chunk from its start
template <class F>
void prefix_sum(int64_t n, int32_t n_threads, int64_t *out, F &&len_of) {
    const int64_t chunk = 65536;
    const int32_t n_chunks = (int32_t)((n + chunk - 1) / chunk);
    std::vector<int64_t> start((size_t)n_chunks + 1, 0);
    parallel_for(n_chunks, n_threads, [&](int32_t ci) {
        int64_t s = 0;
        for (int64_t i = ci * chunk; i < std::min<int64_t>(n, (ci + 1) * chunk); ++i) s += len_of(i);
        start[(size_t)ci + 1] = s;
    });
    for (int32_t ci = 0; ci < n_chunks; ++ci) start[(size_t)ci + 1] += start[(size_t)ci];
    out[0] = 0;
    parallel_for(n_chunks, n_threads, [&](int32_t ci) {
        int64_t s = start[(size_t)ci];
        for (int64_t i = ci * chunk; i < std::min<int64_t>(n, (ci + 1) * chunk); ++i) {
            s += len_of(i);
            out[i + 1] = s;
        }
    });
}

// the new routes' buffer shares memory with the old routes' (which the
// fill still reads)
bool routes_overlap(const int64_t *old_off, const int32_t *old_edges, const int64_t *out_off,
                    const int32_t *out_edges, int64_t n) {
    if (!old_edges || !out_edges) return false;
    const uintptr_t ob = (uintptr_t)old_edges, oe = ob + (uintptr_t)old_off[n] * 4;
    const uintptr_t nb = (uintptr_t)out_edges, ne = nb + (uintptr_t)out_off[n] * 4;
    return nb < oe && ob < ne;
}

}  // namespace

extern "C" {

int32_t lpsim_router_create(int32_t n_nodes, int32_t n_edges, const int32_t *src, const int32_t *dst,
                            int32_t n_threads, lpsim_router **out) {
    if (!out || n_nodes <= 0 || n_edges <= 0 || !src || !dst) return LPSIM_EINVAL;
    *out = nullptr;
    for (int32_t e = 0; e < n_edges; ++e)
        if (src[e] < 0 || src[e] >= n_nodes || dst[e] < 0 || dst[e] >= n_nodes) return LPSIM_EINVAL;
    lpsim_router *r = new (std::nothrow) lpsim_router();
    if (!r) return LPSIM_ENOMEM;
    try {
        r->n_nodes = n_nodes;
        r->n_edges = n_edges;
        r->n_threads = n_threads > 0 ? n_threads : (int32_t)std::max(1u, std::thread::hardware_concurrency());
        r->src.assign(src, src + n_edges);
        r->dst.assign(dst, dst + n_edges);
        r->in_off.assign((size_t)n_nodes + 1, 0);
        for (int32_t e = 0; e < n_edges; ++e) r->in_off[(size_t)dst[e] + 1]++;
        for (int32_t u = 0; u < n_nodes; ++u) r->in_off[(size_t)u + 1] += r->in_off[(size_t)u];
        r->in_edges.resize((size_t)n_edges);
        std::vector<int64_t> pos(r->in_off.begin(), r->in_off.end() - 1);
        for (int32_t e = 0; e < n_edges; ++e) r->in_edges[(size_t)pos[(size_t)dst[e]]++] = e;
        r->in_src.resize((size_t)n_edges);
        for (size_t j = 0; j < r->in_edges.size(); ++j) r->in_src[j] = src[r->in_edges[j]];
    } catch (...) {
        delete r;
        return LPSIM_ENOMEM;
    }
    *out = r;
    return LPSIM_OK;
}

void lpsim_router_destroy(lpsim_router *r) {
    if (!r) return;
    lpsim_route::gpu_router_free(r->gpu);
    delete r;
}

// both solves: the trees toward every distinct destination, on the host
// (std::thread workers) or on the GPU on `stream`
static int32_t router_solve(lpsim_router *r, const double *cost, int64_t n_trips, const int32_t *origin,
                            const int32_t *dest, bool on_gpu, void *stream) {
    if (!r || !cost || n_trips < 0 || (n_trips > 0 && (!origin || !dest))) return LPSIM_EINVAL;
    for (int32_t e = 0; e < r->n_edges; ++e)
        if (!(cost[e] > 0.0) || !std::isfinite(cost[e])) return LPSIM_EINVAL;
    r->solved = false;
    r->len_ok = false;
    try {
        // distinct destinations in order of first appearance
        std::vector<int32_t> idx((size_t)r->n_nodes, -1);
        r->dests.clear();
        r->dest_idx.resize((size_t)n_trips);
        r->origin.assign(origin, origin + n_trips);
        for (int64_t i = 0; i < n_trips; ++i) {
            const int32_t t = dest[i];
            if (t < 0 || t >= r->n_nodes || origin[i] < 0 || origin[i] >= r->n_nodes || origin[i] == t)
                return LPSIM_EINVAL;
            if (idx[(size_t)t] < 0) {
                idx[(size_t)t] = (int32_t)r->dests.size();
                r->dests.push_back(t);
            }
            r->dest_idx[(size_t)i] = idx[(size_t)t];
        }
        const int32_t nd = (int32_t)r->dests.size();
        r->on_gpu = on_gpu;
        r->gpu_stream = stream;
        if (on_gpu) {
            // the trees stay on the device, which also checks that every
            // trip's destination can be reached
            const int32_t rc = lpsim_route::gpu_router_solve(
                &r->gpu, r->n_nodes, r->n_edges, r->in_off.data(), r->in_edges.data(), r->in_src.data(),
                r->src.data(), r->dst.data(), cost, r->dests.data(), nd, n_trips, r->origin.data(),
                r->dest_idx.data(), (hipStream_t)stream);
            if (rc) return rc;
            r->len.assign((size_t)n_trips, 0);
            r->solved = true;
            return LPSIM_OK;
        }
        // every entry is written by the solve (-1 where there is no tree edge)
        r->next_edge.resize((size_t)nd * r->n_nodes);
        r->in_cost.resize(r->in_edges.size());
        for (size_t j = 0; j < r->in_edges.size(); ++j) r->in_cost[j] = cost[r->in_edges[j]];
        const int32_t nw = std::max(1, std::min(r->n_threads, nd));
        std::vector<std::vector<double>> dist(nw, std::vector<double>((size_t)r->n_nodes));
        std::vector<std::vector<uint8_t>> done(nw, std::vector<uint8_t>((size_t)r->n_nodes));
        std::vector<std::vector<HeapItem>> heap(nw);
        std::atomic<int32_t> next{0};
        auto worker = [&](int32_t w) {
            for (;;) {
                const int32_t d = next.fetch_add(1);
                if (d >= nd) break;
                tree_to(*r, cost, r->dests[(size_t)d], r->next_edge.data() + (size_t)d * r->n_nodes, dist[w],
                        done[w], heap[w]);
            }
        };
        {
            std::vector<std::thread> pool;
            for (int32_t w = 1; w < nw; ++w) pool.emplace_back(worker, w);
            worker(0);
            for (auto &t : pool) t.join();
        }
        // every destination reachable: the origin has an edge toward it (a
        // shortest-path tree then leads there); route lengths are measured
        // by lpsim_router_fill for the trips that take a new route
        for (int64_t i = 0; i < n_trips; ++i)
            if (r->next_edge[(size_t)r->dest_idx[(size_t)i] * r->n_nodes + (size_t)r->origin[(size_t)i]] < 0)
                return LPSIM_EINVAL;
        r->len.assign((size_t)n_trips, 0);
    } catch (...) {
        return LPSIM_ENOMEM;
    }
    r->solved = true;
    return LPSIM_OK;
}

int32_t lpsim_router_solve(lpsim_router *r, const double *cost, int64_t n_trips, const int32_t *origin,
                           const int32_t *dest) {
    return router_solve(r, cost, n_trips, origin, dest, false, nullptr);
}

int32_t lpsim_msa_switch(int64_t n_trips, int32_t n, uint64_t seed, uint8_t *take) {
    if (n_trips < 0 || n < 1 || (n_trips > 0 && !take)) return LPSIM_EINVAL;
    auto mix = [](uint64_t z) {  // SplitMix64 output function
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
        z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
        return z ^ (z >> 31);
    };
    for (int64_t i = 0; i < n_trips; ++i)
        take[i] = mix(seed ^ ((uint64_t)i << 8) ^ (uint64_t)n) % (uint64_t)(n + 1) == 0 ? 1 : 0;
    return LPSIM_OK;
}

int32_t lpsim_edge_tt(int32_t n_edges, const int64_t *tt_sum_steps, const int32_t *n_exits,
                      const double *tt_free_steps, double dt, double *out_s) {
    if (n_edges < 0 || !(dt > 0) || (n_edges > 0 && (!tt_sum_steps || !n_exits || !tt_free_steps || !out_s)))
        return LPSIM_EINVAL;
    for (int32_t e = 0; e < n_edges; ++e) {
        const double mean = n_exits[e] > 0 ? (double)tt_sum_steps[e] / (double)n_exits[e] : tt_free_steps[e];
        out_s[e] = (mean > 1.0 ? mean : 1.0) * dt;
    }
    return LPSIM_OK;
}

int32_t lpsim_edge_tt_bins(int32_t n_edges, int32_t n_bins, const int64_t *tt_sum_bin, const int32_t *exits_bin,
                           const double *tt_free_steps, float *out_steps) {
    if (n_edges < 0 || n_bins < 1 ||
        (n_edges > 0 && (!tt_sum_bin || !exits_bin || !tt_free_steps || !out_steps)))
        return LPSIM_EINVAL;
    for (int64_t e = 0; e < n_edges; ++e)
        for (int64_t b = 0; b < n_bins; ++b) {
            const int64_t i = e * n_bins + b;
            out_steps[i] = exits_bin[i] > 0 ? (float)((double)tt_sum_bin[i] / (double)exits_bin[i])
                                            : (float)tt_free_steps[e];
        }
    return LPSIM_OK;
}

int32_t lpsim_router_solve_gpu(lpsim_router *r, const double *cost, int64_t n_trips, const int32_t *origin,
                               const int32_t *dest, void *stream) {
    return router_solve(r, cost, n_trips, origin, dest, true, stream);
}

int32_t lpsim_router_fill(lpsim_router *r, const int64_t *old_off, const int32_t *old_edges, const uint8_t *take_new,
                          int64_t *out_off, int32_t *out_edges) {
    if (!r || !r->solved || !out_off) return LPSIM_ESTATE;
    const int64_t n = (int64_t)r->len.size();
    if (take_new && (!old_off || !old_edges)) return LPSIM_EINVAL;
    const int64_t chunk = 65536;
    const int32_t n_chunks = (int32_t)((n + chunk - 1) / chunk);
    if (take_new) {
        // the old routes that are kept must have non-negative lengths
        std::atomic<bool> bad{false};
        parallel_for(n_chunks, r->n_threads, [&](int32_t ci) {
            for (int64_t i = ci * chunk; i < std::min<int64_t>(n, (ci + 1) * chunk); ++i)
                if (!take_new[i] && old_off[i + 1] < old_off[i]) bad.store(true, std::memory_order_relaxed);
        });
        if (bad.load()) return LPSIM_EINVAL;
    }
    if (r->on_gpu) {
        // lengths of the new routes from walks on the device; a call that
        // follows a sizing call for the same choice of trips reuses them
        const bool same = r->len_ok && (take_new ? !r->len_all && r->len_take.size() == (size_t)n &&
                                                       std::memcmp(r->len_take.data(), take_new, (size_t)n) == 0
                                                 : r->len_all);
        if (!same) {
            r->len_ok = false;
            const int32_t rc = lpsim_route::gpu_router_lengths(r->gpu, take_new, r->len.data(),
                                                               (hipStream_t)r->gpu_stream);
            if (rc) return rc;
            try {
                if (take_new) r->len_take.assign(take_new, take_new + n);
            } catch (...) {
                return LPSIM_ENOMEM;
            }
            r->len_all = !take_new;
            r->len_ok = true;
        }
        const int32_t *len = r->len.data();
        prefix_sum(n, r->n_threads, out_off, [&](int64_t i) -> int64_t {
            return !take_new || take_new[i] ? len[i] : old_off[i + 1] - old_off[i];
        });
        if (!out_edges) return LPSIM_OK;
        if (take_new && routes_overlap(old_off, old_edges, out_off, out_edges, n)) return LPSIM_EINVAL;
        // the new routes come back packed (page-locked), the old ones are
        // copied on the host
        int64_t *poff = lpsim_route::gpu_router_offsets(r->gpu);
        if (!poff) return LPSIM_ENOMEM;
        prefix_sum(n, r->n_threads, poff, [&](int64_t i) -> int64_t { return len[i]; });
        const int32_t *packed = nullptr;
        const int32_t rc2 = lpsim_route::gpu_router_write(r->gpu, &packed, (hipStream_t)r->gpu_stream);
        if (rc2) return rc2;
        parallel_for(n_chunks, r->n_threads, [&](int32_t ci) {
            for (int64_t i = ci * chunk; i < std::min<int64_t>(n, (ci + 1) * chunk); ++i) {
                int32_t *o = out_edges + out_off[i];
                if (take_new && !take_new[i])
                    std::memcpy(o, old_edges + old_off[i], (size_t)(old_off[i + 1] - old_off[i]) * 4);
                else
                    std::memcpy(o, packed + poff[i], (size_t)len[i] * 4);
            }
        });
        return LPSIM_OK;
    }
    {
        // lengths of the new routes (walks down the destination's tree);
        // measured on every call, so a call that writes the edges without a
        // sizing call first still gets its offsets right
        parallel_for(n_chunks, r->n_threads, [&](int32_t ci) {
            for (int64_t i = ci * chunk; i < std::min<int64_t>(n, (ci + 1) * chunk); ++i) {
                if (take_new && !take_new[i]) continue;
                const int32_t *nx = r->next_edge.data() + (size_t)r->dest_idx[(size_t)i] * r->n_nodes;
                const int32_t t = r->dests[(size_t)r->dest_idx[(size_t)i]];
                int32_t u = r->origin[(size_t)i], l = 0;
                while (u != t && l <= r->n_nodes) {
                    u = r->dst[(size_t)nx[u]];
                    ++l;
                }
                r->len[(size_t)i] = l;
            }
        });
    }
    {
        const int32_t *len = r->len.data();
        prefix_sum(n, r->n_threads, out_off, [&](int64_t i) -> int64_t {
            return !take_new || take_new[i] ? len[i] : old_off[i + 1] - old_off[i];
        });
    }
    if (!out_edges) return LPSIM_OK;
    if (take_new && routes_overlap(old_off, old_edges, out_off, out_edges, n)) return LPSIM_EINVAL;
    parallel_for(n_chunks, r->n_threads, [&](int32_t ci) {
        for (int64_t i = ci * chunk; i < std::min<int64_t>(n, (ci + 1) * chunk); ++i) {
            int32_t *o = out_edges + out_off[i];
            if (take_new && !take_new[i]) {
                std::memcpy(o, old_edges + old_off[i], (size_t)(old_off[i + 1] - old_off[i]) * 4);
                continue;
            }
            const int32_t *nx = r->next_edge.data() + (size_t)r->dest_idx[(size_t)i] * r->n_nodes;
            const int32_t t = r->dests[(size_t)r->dest_idx[(size_t)i]];
            int32_t u = r->origin[(size_t)i];
            while (u != t) {
                const int32_t e = nx[u];
                *o++ = e;
                u = r->dst[(size_t)e];
            }
        }
    });
    return LPSIM_OK;
}

}  // extern "C"
