// lpsim_host.cpp -- host side of the C ABI declared in include/lpsim.h:
// validation, device layout, HIP graph capture of the step kernels, read-back.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "lpsim.h"
#include "lpsim_dev.h"

using namespace lpsim;

namespace {

constexpr int N_PHASES = 5;
constexpr uint64_t SNAP_MAGIC = 0x4c5053494d534e32ull;  // "LPSIMSN2"

}  // namespace

struct lpsim_ctx {
    lpsim_params P{};
    Params dp{};
    int device = 0;
    hipStream_t own = nullptr;
    hipStream_t last = nullptr;   // stream of the last enqueued step work
    hipEvent_t order_ev = nullptr;  // orders a call on a new stream after the last one
    std::string err;
    bool poisoned = false;
    void *(*ualloc)(size_t, void *) = nullptr;
    void (*ufree)(void *, void *) = nullptr;
    void *uuser = nullptr;
    std::vector<void *> net_allocs, trip_allocs;

    // network (all scenarios)
    int32_t n_scen = 0;
    std::vector<int32_t> edge_off, node_off;   // per scenario, global ranges
    std::vector<int32_t> look;                 // per scenario lookahead D
    std::vector<int32_t> ext_of_int;           // internal edge -> global input edge id
    std::vector<int32_t> int_of_ext;           // global input edge id -> internal
    int32_t *ext_d = nullptr;                  // ext_of_int on the device
    std::vector<int32_t> src_g, dst_g;         // global input edge order, local node ids
    std::vector<uint32_t> aux_h;               // internal order
    uint2 *sig_d = nullptr;                    // signal words (allocated on first use)
    int32_t n_edges = 0;
    uint64_t map_bytes = 0;
    uint32_t n_lane_slots = 0;
    uint32_t due0 = 0;  // trips due at step 0 (departure-order positions)
    bool have_net = false;

    // trips
    int64_t n_trips = 0;
    // page-locked staging of the translated routes, kept across loads (an
    // assignment loop reloads every iteration)
    uint32_t *route_pin = nullptr;
    size_t route_pin_cap = 0;
    std::vector<int64_t> trip_off;
    bool have_trips = false;
    uint32_t slot_cap = 0;

    Dev d{};      // device view with the control pair of parity 0
    int32_t k = 0;  // current step (its parity picks the control buffer)

    // launch shape: 640 work blocks of 512 threads (plus the helper blocks)
    // stay resident in one round on 256 CUs at the move kernel's occupancy
    int threads = 512;
    int blocks = 640;
    // steps per graph, which is also the interval of the slot reorder (64 is
    // within 0.5% of the best of 16..128 on the benchmark workloads)
    int graph_steps = 64;
    // graphs of graph_steps steps (+ reorder) and of one step, by the parity
    // of the step they start at
    hipGraphExec_t g_full[2] = {nullptr, nullptr}, g_one[2] = {nullptr, nullptr};
    // graphs of fewer than graph_steps steps, for calls (or the ends of
    // calls) shorter than a full graph: keyed by length, starting parity and
    // the step after which the slot reorder falls (0: none); a few are kept,
    // the oldest replaced first
    struct PartGraph {
        int n, par, reorder_after;
        hipGraphExec_t ex;
    };
    std::vector<PartGraph> parts;
    // steps since the last slot reorder, whichever way they were launched
    int since_reorder = 0;

    // timing
    bool timing = false;
    double ms[N_PHASES] = {0};
    int64_t launches[N_PHASES] = {0};
    std::vector<hipEvent_t> ev;   // begin/end pairs
    std::vector<int> ev_phase;    // phase of each recorded pair
    int ev_used = 0;              // pairs recorded and not yet harvested
};

// ---------------------------------------------------------------------------
// errors

static int32_t fail(lpsim_ctx *c, int32_t code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) {
        c->err = buf;
        if (code == LPSIM_EDEVICE) c->poisoned = true;
    }
    return code;
}

#define HIPCHK(c, call)                                                                     \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail((c), LPSIM_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

// ---------------------------------------------------------------------------
// memory

static void *dev_alloc(lpsim_ctx *c, size_t bytes, std::vector<void *> &owner) {
    if (bytes == 0) bytes = 16;
    bytes = (bytes + 255) & ~size_t(255);
    void *p = nullptr;
    if (c->ualloc) {
        p = c->ualloc(bytes, c->uuser);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        p = nullptr;
    }
    if (p) owner.push_back(p);
    return p;
}

static void dev_free_all(lpsim_ctx *c, std::vector<void *> &owner) {
    for (void *p : owner) {
        if (c->ufree) c->ufree(p, c->uuser);
        else (void)hipFree(p);
    }
    owner.clear();
}

static void drop_graphs(lpsim_ctx *c) {
    for (int p = 0; p < 2; ++p) {
        if (c->g_full[p]) (void)hipGraphExecDestroy(c->g_full[p]);
        if (c->g_one[p]) (void)hipGraphExecDestroy(c->g_one[p]);
        c->g_full[p] = c->g_one[p] = nullptr;
    }
    for (auto &g : c->parts) (void)hipGraphExecDestroy(g.ex);
    c->parts.clear();
}

// the device view for a step of parity `par`: its control block is buffer
// par, the next step's is the other one
static Dev dev_at(const lpsim_ctx *c, int par) {
    Dev d = c->d;
    d.ctrl = c->d.ctrl + par;
    d.ctrl_next = c->d.ctrl + (par ^ 1);
    return d;
}

static int32_t sync_all(lpsim_ctx *c) {
    if (c->last) HIPCHK(c, hipStreamSynchronize(c->last));
    HIPCHK(c, hipStreamSynchronize(c->own));
    return LPSIM_OK;
}

template <class T>
static int32_t upload(lpsim_ctx *c, T *&dst, const T *src, size_t n, std::vector<void *> &owner) {
    dst = (T *)dev_alloc(c, n * sizeof(T), owner);
    if (!dst) return fail(c, LPSIM_ENOMEM, "device allocation of %zu bytes failed", n * sizeof(T));
    if (n) HIPCHK(c, hipMemcpy(dst, src, n * sizeof(T), hipMemcpyHostToDevice));
    return LPSIM_OK;
}

template <class T>
static int32_t alloc_n(lpsim_ctx *c, T *&dst, size_t n, std::vector<void *> &owner) {
    dst = (T *)dev_alloc(c, n * sizeof(T), owner);
    if (!dst) return fail(c, LPSIM_ENOMEM, "device allocation of %zu bytes failed", n * sizeof(T));
    return LPSIM_OK;
}

// ---------------------------------------------------------------------------
// recursive coordinate bisection of nodes: a locality order

static void rcb(std::vector<int32_t> &idx, size_t lo, size_t hi, const float *xy, size_t leaf) {
    if (hi - lo <= leaf) return;
    float xmin = INFINITY, xmax = -INFINITY, ymin = INFINITY, ymax = -INFINITY;
    for (size_t i = lo; i < hi; ++i) {
        const float x = xy[2 * (size_t)idx[i]], y = xy[2 * (size_t)idx[i] + 1];
        xmin = std::min(xmin, x); xmax = std::max(xmax, x);
        ymin = std::min(ymin, y); ymax = std::max(ymax, y);
    }
    const int axis = (xmax - xmin) >= (ymax - ymin) ? 0 : 1;
    const size_t mid = lo + (hi - lo) / 2;
    std::nth_element(idx.begin() + lo, idx.begin() + mid, idx.begin() + hi,
                     [&](int32_t a, int32_t b) {
                         const float pa = xy[2 * (size_t)a + axis], pb = xy[2 * (size_t)b + axis];
                         return pa < pb || (pa == pb && a < b);
                     });
    rcb(idx, lo, mid, xy, leaf);
    rcb(idx, mid, hi, xy, leaf);
}

// ---------------------------------------------------------------------------
// network

static void release_trips(lpsim_ctx *c) {
    // work still queued on the context's streams may read what is freed
    // here (steps, or statistics handed over on the device)
    if (c->last) (void)hipStreamSynchronize(c->last);
    if (c->own) (void)hipStreamSynchronize(c->own);
    drop_graphs(c);
    dev_free_all(c, c->trip_allocs);
    c->have_trips = false;
    c->n_trips = 0;
}

static void release_net(lpsim_ctx *c) {
    release_trips(c);
    dev_free_all(c, c->net_allocs);
    c->ext_d = nullptr;
    c->sig_d = nullptr;
    c->d.sig = nullptr;
    c->have_net = false;
}

struct NetIn {
    int32_t n_scen;
    const int32_t *node_off, *edge_off;
    const float *node_xy;
    const int32_t *src, *dst;
    const float *length;
    const uint8_t *lanes;
    const float *speed;
};

static int32_t build_network(lpsim_ctx *c, const NetIn &in) {
    const lpsim_params &P = c->P;
    const int32_t S = in.n_scen;
    if (S < 1) return fail(c, LPSIM_EINVAL, "need at least one scenario");
    if (in.node_off[0] != 0 || in.edge_off[0] != 0) return fail(c, LPSIM_EINVAL, "offsets must start at 0");
    for (int32_t s = 0; s < S; ++s) {
        if (in.node_off[s + 1] <= in.node_off[s] || in.edge_off[s + 1] <= in.edge_off[s])
            return fail(c, LPSIM_EINVAL, "scenario %d has no nodes or no edges", s);
    }
    const int32_t E = in.edge_off[S];
    const int32_t W = c->dp.W;
    std::vector<int32_t> look(S);
    std::vector<int32_t> cells(E);
    for (int32_t s = 0; s < S; ++s) {
        const int32_t nn = in.node_off[s + 1] - in.node_off[s];
        double vmax = 0.0;
        for (int32_t e = in.edge_off[s]; e < in.edge_off[s + 1]; ++e) {
            if (in.src[e] < 0 || in.src[e] >= nn || in.dst[e] < 0 || in.dst[e] >= nn)
                return fail(c, LPSIM_EINVAL, "edge %d: node id out of range", e);
            if (in.lanes[e] < 1 || in.lanes[e] > 8)
                return fail(c, LPSIM_EINVAL, "edge %d: lanes must be 1..8", e);
            if (!(in.speed[e] > 0.0f && in.speed[e] <= 254.0f))
                return fail(c, LPSIM_EINVAL, "edge %d: speed limit must be in (0, 254]", e);
            if (!(in.length[e] > 0.0f)) return fail(c, LPSIM_EINVAL, "edge %d: length must be > 0", e);
            const double cl = std::ceil((double)in.length[e]);
            if (cl < (double)(W + 1) || cl > 65535.0)
                return fail(c, LPSIM_EINVAL, "edge %d: %g cells, need %d..65535", e, cl, W + 1);
            cells[e] = (int32_t)cl;
            vmax = std::max(vmax, (double)in.speed[e]);
        }
        // leader look-ahead: at least 2*dt*v (the paper's bound), extended to
        // the IDM desired gap s0 + T*v at the scenario's top speed
        const double reach = 2.0 * (double)P.dt * vmax;
        const double desired = (double)P.s0 + (double)P.T * vmax;
        const double Dd = std::ceil((double)P.veh_len + std::max(reach, desired));
        if (Dd > 255.0) return fail(c, LPSIM_ECAPACITY, "look-ahead of %g cells exceeds 255", Dd);
        look[s] = (int32_t)Dd;
    }

    // internal order: per scenario, RCB order of the upstream node, then id
    std::vector<int32_t> ext_of_int(E), int_of_ext(E);
    for (int32_t s = 0; s < S; ++s) {
        const int32_t e0 = in.edge_off[s], e1 = in.edge_off[s + 1];
        const int32_t nn = in.node_off[s + 1] - in.node_off[s];
        std::vector<int32_t> order(e1 - e0);
        std::iota(order.begin(), order.end(), e0);
        if (in.node_xy) {
            std::vector<int32_t> nodes(nn);
            std::iota(nodes.begin(), nodes.end(), 0);
            rcb(nodes, 0, nodes.size(), in.node_xy + 2 * (size_t)in.node_off[s], 1024);
            std::vector<int32_t> rank(nn);
            for (int32_t i = 0; i < nn; ++i) rank[nodes[i]] = i;
            std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
                return rank[in.src[a]] < rank[in.src[b]];
            });
        }
        for (int32_t i = 0; i < e1 - e0; ++i) {
            ext_of_int[e0 + i] = order[i];
            int_of_ext[order[i]] = e0 + i;
        }
    }

    // out-edge rank (by input id) and out-degree per edge, per scenario
    std::vector<uint32_t> rank_e(E), deg_e(E);
    for (int32_t s = 0; s < S; ++s) {
        const int32_t nn = in.node_off[s + 1] - in.node_off[s];
        std::vector<int32_t> deg(nn, 0);
        for (int32_t e = in.edge_off[s]; e < in.edge_off[s + 1]; ++e) rank_e[e] = deg[in.src[e]]++;
        for (int32_t e = in.edge_off[s]; e < in.edge_off[s + 1]; ++e) {
            deg_e[e] = deg[in.src[e]];
            if (deg_e[e] > 255) return fail(c, LPSIM_ECAPACITY, "node with more than 255 out-edges");
        }
    }

    std::vector<uint4> rec(E);
    std::vector<uint32_t> aux(E);
    std::vector<int32_t> escen(E);
    uint64_t off = 0;
    uint64_t slot = 0;
    for (int32_t s = 0; s < S; ++s) {
        for (int32_t i = in.edge_off[s]; i < in.edge_off[s + 1]; ++i) {
            const int32_t e = ext_of_int[i];
            const uint32_t C = (uint32_t)cells[e], nl = in.lanes[e];
            float v0 = in.speed[e];
            uint32_t v0b;
            std::memcpy(&v0b, &v0, 4);
            rec[i] = make_uint4((uint32_t)off, C | (nl << 16) | ((uint32_t)look[s] << 24), v0b, (uint32_t)slot);
            aux[i] = rank_e[e] | (deg_e[e] << 8);
            escen[i] = s;
            off += (uint64_t)C * nl;
            slot += nl;
            if (off > 0xffffff00ull) return fail(c, LPSIM_ECAPACITY, "lane map exceeds 4 GiB");
        }
    }

    release_net(c);
    c->n_scen = S;
    c->edge_off.assign(in.edge_off, in.edge_off + S + 1);
    c->node_off.assign(in.node_off, in.node_off + S + 1);
    c->look = look;
    c->ext_of_int = ext_of_int;
    c->int_of_ext = int_of_ext;
    c->src_g.assign(in.src, in.src + E);
    c->dst_g.assign(in.dst, in.dst + E);
    c->aux_h = aux;
    c->n_edges = E;
    c->map_bytes = off;
    c->n_lane_slots = (uint32_t)slot;

    Dev &d = c->d;
    int32_t rc;
    const uint4 *edge_d;
    if ((rc = upload(c, *(uint4 **)&edge_d, rec.data(), rec.size(), c->net_allocs))) return rc;
    d.edge = edge_d;
    if ((rc = upload(c, d.aux, aux.data(), aux.size(), c->net_allocs))) return rc;
    const int32_t *escen_d;
    if ((rc = upload(c, *(int32_t **)&escen_d, escen.data(), escen.size(), c->net_allocs))) return rc;
    d.escen = escen_d;
    d.n_scen = S;
    if ((rc = upload(c, c->ext_d, ext_of_int.data(), ext_of_int.size(), c->net_allocs))) return rc;
    if ((rc = alloc_n(c, d.map, off + 256, c->net_allocs))) return rc;
    if ((rc = alloc_n(c, d.claims, (size_t)slot, c->net_allocs))) return rc;
    const size_t nb = (size_t)E * (size_t)c->dp.n_bins;
    if ((rc = alloc_n(c, d.n_exits, (size_t)E, c->net_allocs))) return rc;
    if ((rc = alloc_n(c, d.tt_sum, (size_t)E, c->net_allocs))) return rc;
    if ((rc = alloc_n(c, d.inflow_bin, nb, c->net_allocs))) return rc;
    if ((rc = alloc_n(c, d.exits_bin, nb, c->net_allocs))) return rc;
    if ((rc = alloc_n(c, d.tt_bin, nb, c->net_allocs))) return rc;
    if ((rc = alloc_n(c, d.occ_bin, nb, c->net_allocs))) return rc;
    if ((rc = alloc_n(c, d.partial, (size_t)PART_ROWS * NPART, c->net_allocs))) return rc;
    const size_t n_chunks = ((size_t)E + SORT_CHUNK - 1) / SORT_CHUNK;
    if ((rc = alloc_n(c, d.ecnt, (size_t)E, c->net_allocs))) return rc;
    if ((rc = alloc_n(c, d.eoff, (size_t)E, c->net_allocs))) return rc;
    if ((rc = alloc_n(c, d.csum, n_chunks + 1, c->net_allocs))) return rc;
    HIPCHK(c, hipMemset(d.ecnt, 0, (size_t)E * 4));
    d.n_edges = E;
    if ((rc = alloc_n(c, d.ctrl, 2, c->net_allocs))) return rc;
    d.ctrl_next = d.ctrl + 1;
    HIPCHK(c, hipMemset(d.map, 0xff, off + 256));
    HIPCHK(c, hipMemset(d.claims, 0xff, (size_t)slot * 4));
    c->have_net = true;
    return LPSIM_OK;
}

struct TripIn {
    const int64_t *trip_off;       // per scenario, n_scen+1
    const int32_t *depart;         // global
    const int64_t *route_offsets;  // per scenario (count+1 each), concatenated
    const int32_t *route_edges;    // concatenated, local edge ids
    const uint64_t *seeds;
};

static int32_t reset_run_state(lpsim_ctx *c) {
    Dev &d = c->d;
    const size_t E = (size_t)c->n_edges, nb = E * (size_t)c->dp.n_bins;
    const size_t N = (size_t)c->n_trips;
    HIPCHK(c, hipMemset(d.map, 0xff, c->map_bytes + 256));
    HIPCHK(c, hipMemset(d.claims, 0xff, (size_t)c->n_lane_slots * 4));
    HIPCHK(c, hipMemset(d.n_exits, 0, E * 4));
    HIPCHK(c, hipMemset(d.tt_sum, 0, E * 8));
    HIPCHK(c, hipMemset(d.inflow_bin, 0, nb * 4));
    HIPCHK(c, hipMemset(d.exits_bin, 0, nb * 4));
    HIPCHK(c, hipMemset(d.tt_bin, 0, nb * 8));
    HIPCHK(c, hipMemset(d.occ_bin, 0, nb * 8));
    HIPCHK(c, hipMemset(d.partial, 0, (size_t)PART_ROWS * NPART * 8));
    HIPCHK(c, hipMemset(d.status, 0, N + 1));
    HIPCHK(c, hipMemset(d.arrival, 0xff, (N + 1) * 4));
    HIPCHK(c, hipMemset(d.dclaim, 0, (size_t)d.n_ol + 1));
    HIPCHK(c, hipMemset(d.ol_bits, 0, (N / 32 + 1) * 4));
    HIPCHK(c, hipMemset(d.ol_head, 0xff, ((size_t)d.n_ol + 1) * 8));
    HIPCHK(c, hipMemset(d.ol_cnt, 0, ((size_t)d.n_ol + 1) * 4));
    HIPCHK(c, hipMemset(d.aq_n, 0, 2 * 4));
    HIPCHK(c, hipMemset(d.ecnt, 0, E * 4));
    for (uint32_t *a : {d.rl_cnt, d.lcc_cnt, d.lc_cnt, d.blk_arr, d.blk_ev})
        HIPCHK(c, hipMemset(a, 0, (size_t)MAX_BLOCKS * 4));
    // the trips due at step 0 wait in their origin lanes' sets
    Ctrl ct{};
    ct.dep_done = c->due0;
    ct.n_wq = c->due0;
    HIPCHK(c, hipMemcpy(d.ctrl, &ct, sizeof ct, hipMemcpyHostToDevice));
    launch_enqueue(d, 0, c->due0, 0, nullptr);
    HIPCHK(c, hipGetLastError());
    c->k = 0;
    // the blocked flags survive a reload of trips
    HIPCHK(c, hipMemcpy(d.aux, c->aux_h.data(), c->aux_h.size() * 4, hipMemcpyHostToDevice));
    HIPCHK(c, hipDeviceSynchronize());
    return LPSIM_OK;
}

// f(begin, end) over [0, n) in chunks on the host's hardware threads
template <class F>
static void host_parallel(int64_t n, F &&f) {
    const int64_t chunk = 1 << 16;
    const int64_t n_chunks = (n + chunk - 1) / chunk;
    const int32_t nt = (int32_t)std::max<int64_t>(
        1, std::min<int64_t>(n_chunks, std::min<unsigned>(32u, std::max(1u, std::thread::hardware_concurrency()))));
    std::atomic<int64_t> next{0};
    auto worker = [&]() {
        for (;;) {
            const int64_t ci = next.fetch_add(1);
            if (ci >= n_chunks) break;
            f(ci * chunk, std::min(n, (ci + 1) * chunk));
        }
    };
    std::vector<std::thread> pool;
    for (int32_t t = 1; t < nt; ++t) pool.emplace_back(worker);
    worker();
    for (auto &t : pool) t.join();
}

static int32_t build_trips(lpsim_ctx *c, const TripIn &in) {
    if (!c->have_net) return fail(c, LPSIM_ESTATE, "load a network first");
    const int32_t S = c->n_scen;
    if (in.trip_off[0] != 0) return fail(c, LPSIM_EINVAL, "trip offsets must start at 0");
    for (int32_t s = 0; s < S; ++s)
        if (in.trip_off[s + 1] < in.trip_off[s]) return fail(c, LPSIM_EINVAL, "trip offsets decrease");
    const int64_t N = in.trip_off[S];
    if (N > 0x7ffffffeLL) return fail(c, LPSIM_ECAPACITY, "more than 2^31-2 trips");
    // absolute offsets, then the routes checked (edge ids in range,
    // contiguous) and translated to internal ids in one pass on all host
    // threads, straight into the page-locked staging buffer
    std::vector<uint32_t> roff((size_t)N + 1);
    uint64_t total = 0;
    {
        const int64_t *ro = in.route_offsets;
        for (int32_t s = 0; s < S; ++s) {
            const int64_t t0 = in.trip_off[s], nt = in.trip_off[s + 1] - t0;
            if (ro[0] != 0) return fail(c, LPSIM_EINVAL, "scenario %d: route offsets must start at 0", s);
            for (int64_t t = 0; t < nt; ++t) {
                const int64_t a0 = ro[t], b0 = ro[t + 1];
                if (b0 <= a0) return fail(c, LPSIM_EINVAL, "trip %lld has an empty route", (long long)(t0 + t));
                if (in.depart[t0 + t] < 0)
                    return fail(c, LPSIM_EINVAL, "trip %lld departs before 0", (long long)(t0 + t));
                roff[(size_t)(t0 + t)] = (uint32_t)(total + (uint64_t)a0);
            }
            total += (uint64_t)ro[nt];
            if (total > 0xfffffff0ull) return fail(c, LPSIM_ECAPACITY, "more than 2^32-16 route entries");
            ro += nt + 1;
        }
        roff[(size_t)N] = (uint32_t)total;
    }
    if (c->route_pin_cap < total + 1) {
        if (c->route_pin) HIPCHK(c, hipHostFree(c->route_pin));
        c->route_pin = nullptr;
        c->route_pin_cap = 0;
        void *p = nullptr;
        const size_t cap = (size_t)(total + 1) + (size_t)(total + 1) / 8;  // room for longer routes later
        if (hipHostMalloc(&p, cap * sizeof(uint32_t), hipHostMallocDefault) != hipSuccess || !p)
            return fail(c, LPSIM_ENOMEM, "page-locked staging of %zu route entries failed", cap);
        c->route_pin = static_cast<uint32_t *>(p);
        c->route_pin_cap = cap;
    }
    uint32_t *route = c->route_pin;
    {
        const int64_t *ro = in.route_offsets;
        const int32_t *re = in.route_edges;
        uint32_t *out = route;
        for (int32_t s = 0; s < S; ++s) {
            const int64_t t0 = in.trip_off[s], nt = in.trip_off[s + 1] - t0;
            const int32_t eb = c->edge_off[s], ne = c->edge_off[s + 1] - eb;
            // the lowest failing trip is reported
            std::atomic<int64_t> bad_range{INT64_MAX}, bad_gap{INT64_MAX};
            host_parallel(nt, [&](int64_t t_lo, int64_t t_hi) {
                for (int64_t t = t_lo; t < t_hi; ++t) {
                    for (int64_t j = ro[t]; j < ro[t + 1]; ++j) {
                        const int32_t e = re[j];
                        if (e < 0 || e >= ne) {
                            int64_t cur = bad_range.load();
                            while (t < cur && !bad_range.compare_exchange_weak(cur, t)) {
                            }
                            break;
                        }
                        if (j > ro[t] && c->dst_g[eb + re[j - 1]] != c->src_g[eb + e]) {
                            int64_t cur = bad_gap.load();
                            while (t < cur && !bad_gap.compare_exchange_weak(cur, t)) {
                            }
                            break;
                        }
                        out[j] = (uint32_t)c->int_of_ext[eb + e];
                    }
                }
            });
            if (bad_range.load() != INT64_MAX || bad_gap.load() != INT64_MAX) {
                if (bad_range.load() <= bad_gap.load())
                    return fail(c, LPSIM_EINVAL, "trip %lld: edge id out of range",
                                (long long)(t0 + bad_range.load()));
                return fail(c, LPSIM_EINVAL, "trip %lld: route is not contiguous", (long long)(t0 + bad_gap.load()));
            }
            const int64_t len = ro[nt];
            re += len;
            out += len;
            ro += nt + 1;
        }
        route[total] = 0;
    }
    // departure order and the count of trips due by each step
    int32_t maxdep = -1;
    for (int64_t t = 0; t < N; ++t) maxdep = std::max(maxdep, in.depart[t]);
    if (maxdep >= (1 << 26)) return fail(c, LPSIM_ECAPACITY, "departure step beyond 2^26");
    std::vector<uint32_t> cnt((size_t)maxdep + 2, 0);
    for (int64_t t = 0; t < N; ++t) cnt[(size_t)in.depart[t] + 1]++;
    for (size_t k = 1; k < cnt.size(); ++k) cnt[k] += cnt[k - 1];
    std::vector<uint32_t> order((size_t)std::max<int64_t>(N, 1));
    {
        std::vector<uint32_t> pos(cnt.begin(), cnt.end() - 1);
        for (int64_t t = 0; t < N; ++t) order[pos[(size_t)in.depart[t]]++] = (uint32_t)t;
    }
    std::vector<uint32_t> dep_hi((size_t)maxdep + 2, (uint32_t)N);  // one spare entry
    for (int32_t k = 0; k <= maxdep; ++k) dep_hi[(size_t)k] = cnt[(size_t)k + 1];
    // per-trip origin: claim word, lane-map offset of the start lane, first
    // edge (start lane = scenario-local id mod lanes)
    std::vector<uint4> orig((size_t)std::max<int64_t>(N, 1));
    // and what a departing trip's slot needs from its route: route index of
    // the first edge, route end, second edge (NO_NEXT if none)
    std::vector<uint4> dep_rec((size_t)std::max<int64_t>(N, 1));
    {
        std::vector<uint4> rec_h(c->n_edges);
        HIPCHK(c, hipMemcpy(rec_h.data(), c->d.edge, (size_t)c->n_edges * 16, hipMemcpyDeviceToHost));
        for (int32_t s = 0; s < S; ++s) {
            const int64_t t0 = in.trip_off[s];
            host_parallel(in.trip_off[s + 1] - t0, [&](int64_t lo, int64_t hi) {
                for (int64_t t = t0 + lo; t < t0 + hi; ++t) {
                    const uint32_t r0 = roff[(size_t)t];
                    const uint32_t e0 = route[r0];
                    const uint4 R = rec_h[e0];
                    const uint32_t C = R.y & 0xffffu, nl = (R.y >> 16) & 0xffu;
                    const uint32_t l0 = (uint32_t)(t - t0) % nl;
                    orig[(size_t)t] = make_uint4(R.w + l0, R.x + l0 * C, e0, 0u);
                    const uint32_t rend = roff[(size_t)t + 1];
                    dep_rec[(size_t)t] = make_uint4(r0, rend, r0 + 1 < rend ? route[r0 + 1] : NO_NEXT, 0u);
                }
            });
        }
    }
    // origin lanes (the lanes trips start on), numbered in claim-word order,
    // each with its trips in increasing id: counted and filled on all host
    // threads (relaxed atomic counters), then each lane's few trips sorted
    std::vector<uint32_t> ol_of((size_t)c->n_lane_slots + 1, 0);  // trips per claim word, then lane number
    host_parallel(N, [&](int64_t lo, int64_t hi) {
        for (int64_t t = lo; t < hi; ++t) __atomic_fetch_add(&ol_of[orig[(size_t)t].x], 1u, __ATOMIC_RELAXED);
    });
    std::vector<uint4> ol_rec;
    uint32_t n_ol = 0;
    {
        uint32_t off = 0;
        for (uint32_t w = 0; w < c->n_lane_slots; ++w) {
            const uint32_t m = ol_of[w];
            if (!m) {
                ol_of[w] = NO_NEXT;
                continue;
            }
            ol_of[w] = n_ol++;
            ol_rec.push_back(make_uint4(w, 0u, 0u, off));
            off += m;
        }
        ol_rec.push_back(make_uint4(0u, 0u, 0u, off));
    }
    std::vector<uint32_t> ol_trips((size_t)std::max<int64_t>(N, 1));
    std::vector<uint2> trip_ol((size_t)std::max<int64_t>(N, 1));
    {
        std::vector<uint32_t> fill(n_ol, 0);
        host_parallel(N, [&](int64_t lo, int64_t hi) {
            for (int64_t t = lo; t < hi; ++t) {
                const uint32_t l = ol_of[orig[(size_t)t].x];
                ol_trips[ol_rec[l].w + __atomic_fetch_add(&fill[l], 1u, __ATOMIC_RELAXED)] = (uint32_t)t;
            }
        });
        host_parallel(n_ol, [&](int64_t lo, int64_t hi) {
            for (int64_t l = lo; l < hi; ++l) {
                const uint32_t beg = ol_rec[(size_t)l].w, end = ol_rec[(size_t)l + 1].w;
                std::sort(ol_trips.begin() + beg, ol_trips.begin() + end);
                const uint4 o = orig[ol_trips[beg]];
                ol_rec[(size_t)l].y = o.y;
                ol_rec[(size_t)l].z = o.z;
                for (uint32_t p = beg; p < end; ++p) trip_ol[ol_trips[p]] = make_uint2((uint32_t)l, p);
            }
        });
    }
    std::vector<uint64_t> seeds(S);
    std::vector<uint32_t> tbase(S);
    for (int32_t s = 0; s < S; ++s) {
        seeds[s] = in.seeds ? in.seeds[s] : c->P.seed;
        tbase[s] = (uint32_t)in.trip_off[s];
    }

    release_trips(c);
    Dev &d = c->d;
    int32_t rc;
    c->n_trips = N;
    c->trip_off.assign(in.trip_off, in.trip_off + S + 1);
    const size_t cap = (size_t)std::max<int64_t>(N, 1);
    c->slot_cap = (uint32_t)cap;
    const uint32_t *route_d, *roff_d, *order_d, *dephi_d, *tbase_d;
    const uint64_t *seeds_d;
    if ((rc = upload(c, *(uint32_t **)&route_d, route, (size_t)total + 1, c->trip_allocs))) return rc;
    if ((rc = upload(c, *(uint32_t **)&roff_d, roff.data(), roff.size(), c->trip_allocs))) return rc;
    if ((rc = upload(c, *(uint32_t **)&order_d, order.data(), order.size(), c->trip_allocs))) return rc;
    if ((rc = upload(c, *(uint32_t **)&dephi_d, dep_hi.data(), dep_hi.size(), c->trip_allocs))) return rc;
    if ((rc = upload(c, *(uint64_t **)&seeds_d, seeds.data(), seeds.size(), c->trip_allocs))) return rc;
    const uint4 *olrec_d;
    if ((rc = upload(c, *(uint4 **)&olrec_d, ol_rec.data(), ol_rec.size(), c->trip_allocs))) return rc;
    d.ol_rec = olrec_d;
    const uint32_t *oltrips_d;
    if ((rc = upload(c, *(uint32_t **)&oltrips_d, ol_trips.data(), ol_trips.size(), c->trip_allocs))) return rc;
    d.ol_trips = oltrips_d;
    const uint2 *tripol_d;
    if ((rc = upload(c, *(uint2 **)&tripol_d, trip_ol.data(), trip_ol.size(), c->trip_allocs))) return rc;
    d.trip_ol = tripol_d;
    d.n_ol = n_ol;
    if ((rc = alloc_n(c, d.ol_bits, (size_t)N / 32 + 1, c->trip_allocs))) return rc;
    if ((rc = alloc_n(c, d.ol_head, (size_t)n_ol + 1, c->trip_allocs))) return rc;
    if ((rc = alloc_n(c, d.ol_cnt, (size_t)n_ol + 1, c->trip_allocs))) return rc;
    if ((rc = alloc_n(c, d.aq[0], (size_t)n_ol + 1, c->trip_allocs))) return rc;
    if ((rc = alloc_n(c, d.aq[1], (size_t)n_ol + 1, c->trip_allocs))) return rc;
    if ((rc = alloc_n(c, d.aq_n, (size_t)2, c->trip_allocs))) return rc;
    c->due0 = N > 0 ? dep_hi[0] : 0u;
    const uint4 *deprec_d;
    if ((rc = upload(c, *(uint4 **)&deprec_d, dep_rec.data(), dep_rec.size(), c->trip_allocs))) return rc;
    d.dep_rec = deprec_d;
    if ((rc = upload(c, *(uint32_t **)&tbase_d, tbase.data(), tbase.size(), c->trip_allocs))) return rc;
    d.route = route_d;
    d.route_off = roff_d;
    d.dep_order = order_d;
    d.dep_hi = dephi_d;
    d.n_dep_hi = maxdep + 1;
    d.n_trips = (uint32_t)N;
    d.scen_seed = seeds_d;
    d.scen_tbase = tbase_d;
    if ((rc = alloc_n(c, d.status, cap + 1, c->trip_allocs))) return rc;
    if ((rc = alloc_n(c, d.arrival, cap + 1, c->trip_allocs))) return rc;
    if ((rc = alloc_n(c, d.dclaim, (size_t)n_ol + 1, c->trip_allocs))) return rc;
    for (int b = 0; b < 2; ++b) {
        Slots &s = d.buf[b];
        if ((rc = alloc_n(c, s.x, cap, c->trip_allocs))) return rc;
        if ((rc = alloc_n(c, s.v, cap, c->trip_allocs))) return rc;
        if ((rc = alloc_n(c, s.e, cap, c->trip_allocs))) return rc;
        if ((rc = alloc_n(c, s.en, cap, c->trip_allocs))) return rc;
        if ((rc = alloc_n(c, s.m, cap, c->trip_allocs))) return rc;
        if ((rc = alloc_n(c, s.id, cap, c->trip_allocs))) return rc;
        if ((rc = alloc_n(c, s.rp, cap, c->trip_allocs))) return rc;
        if ((rc = alloc_n(c, s.rend, cap, c->trip_allocs))) return rc;
        if ((rc = alloc_n(c, s.ent, cap, c->trip_allocs))) return rc;
        if ((rc = alloc_n(c, s.lb, cap, c->trip_allocs))) return rc;
        if ((rc = alloc_n(c, s.cd, cap, c->trip_allocs))) return rc;
        if ((rc = alloc_n(c, s.v0, cap, c->trip_allocs))) return rc;
        if ((rc = alloc_n(c, s.tlb, cap, c->trip_allocs))) return rc;
        if ((rc = alloc_n(c, s.tgt, cap, c->trip_allocs))) return rc;
    }
    if ((rc = alloc_n(c, d.scl, cap, c->trip_allocs))) return rc;
    if ((rc = alloc_n(c, d.sxo, cap, c->trip_allocs))) return rc;
    if ((rc = alloc_n(c, d.lc_list, cap + LIST_SPARE, c->trip_allocs))) return rc;
    if ((rc = alloc_n(c, d.rl_list, cap + LIST_SPARE, c->trip_allocs))) return rc;
    if ((rc = alloc_n(c, d.lcc_list, cap + LIST_SPARE, c->trip_allocs))) return rc;
    d.slot_cap = (uint32_t)cap;
    if ((rc = alloc_n(c, d.rl_cnt, (size_t)MAX_BLOCKS, c->trip_allocs))) return rc;
    if ((rc = alloc_n(c, d.lcc_cnt, (size_t)MAX_BLOCKS, c->trip_allocs))) return rc;
    if ((rc = alloc_n(c, d.lc_cnt, (size_t)MAX_BLOCKS, c->trip_allocs))) return rc;
    if ((rc = alloc_n(c, d.blk_arr, (size_t)MAX_BLOCKS, c->trip_allocs))) return rc;
    if ((rc = alloc_n(c, d.blk_ev, (size_t)MAX_BLOCKS, c->trip_allocs))) return rc;
    if ((rc = alloc_n(c, d.srank, cap, c->trip_allocs))) return rc;
    if ((rc = reset_run_state(c))) return rc;
    c->have_trips = true;
    c->since_reorder = 0;
    return LPSIM_OK;
}

// ---------------------------------------------------------------------------
// stepping

// one step whose control block has parity `par`
static void enqueue_step(lpsim_ctx *c, hipStream_t s, int par) {
    const Dev d = dev_at(c, par);
    launch_move(d, c->blocks, c->threads, s);
    launch_resolve(d, c->blocks, c->threads, s);
    if (c->dp.lane_change) launch_lanechg(d, c->blocks, c->threads, s);
    launch_commit(d, c->blocks, c->threads, s);
}

static int32_t build_graphs(lpsim_ctx *c) {
    drop_graphs(c);
    for (int which = 0; which < 4; ++which) {
        const int p0 = which & 1;
        const bool full = which < 2;
        hipGraph_t g = nullptr;
        HIPCHK(c, hipStreamBeginCapture(c->own, hipStreamCaptureModeThreadLocal));
        const int n = full ? c->graph_steps : 1;
        for (int t = 0; t < n; ++t) enqueue_step(c, c->own, (p0 + t) & 1);
        if (full) launch_reorder(dev_at(c, (p0 + n) & 1), c->blocks, c->threads, c->own);
        HIPCHK(c, hipStreamEndCapture(c->own, &g));
        hipGraphExec_t ex = nullptr;
        HIPCHK(c, hipGraphInstantiate(&ex, g, nullptr, nullptr, 0));
        (void)hipGraphDestroy(g);
        (full ? c->g_full : c->g_one)[p0] = ex;
    }
    return LPSIM_OK;
}

static constexpr size_t MAX_PART_GRAPHS = 8;

// the graph of `n` (< graph_steps) steps from the current step, with the
// slot reorder after step `reorder_after` of them (0: none); captured on
// first use
static int32_t part_graph(lpsim_ctx *c, int n, int reorder_after, hipGraphExec_t *out) {
    const int par = c->k & 1;
    for (auto &g : c->parts)
        if (g.n == n && g.par == par && g.reorder_after == reorder_after) {
            *out = g.ex;
            return LPSIM_OK;
        }
    if (c->parts.size() >= MAX_PART_GRAPHS) {
        (void)hipGraphExecDestroy(c->parts.front().ex);
        c->parts.erase(c->parts.begin());
    }
    hipGraph_t g = nullptr;
    HIPCHK(c, hipStreamBeginCapture(c->own, hipStreamCaptureModeThreadLocal));
    for (int t = 0; t < n; ++t) {
        enqueue_step(c, c->own, (par + t) & 1);
        if (t + 1 == reorder_after) launch_reorder(dev_at(c, (par + t + 1) & 1), c->blocks, c->threads, c->own);
    }
    HIPCHK(c, hipStreamEndCapture(c->own, &g));
    hipGraphExec_t ex = nullptr;
    const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HIPCHK(c, e);
    c->parts.push_back({n, par, reorder_after, ex});
    *out = ex;
    return LPSIM_OK;
}

static int32_t harvest_events(lpsim_ctx *c) {
    for (int i = 0; i < c->ev_used; ++i) {
        HIPCHK(c, hipEventSynchronize(c->ev[2 * i + 1]));
        float ms = 0.f;
        HIPCHK(c, hipEventElapsedTime(&ms, c->ev[2 * i], c->ev[2 * i + 1]));
        c->ms[c->ev_phase[i]] += ms;
        c->launches[c->ev_phase[i]] += 1;
    }
    c->ev_used = 0;
    return LPSIM_OK;
}

// the next free event pair, for phase `phase`
static int32_t next_events(lpsim_ctx *c, int phase, KernelEvents &ev) {
    if ((size_t)(c->ev_used + 1) * 2 > c->ev.size()) {
        int32_t rc = harvest_events(c);
        if (rc) return rc;
    }
    const int i = c->ev_used++;
    c->ev_phase[i] = phase;
    ev.start = c->ev[2 * i];
    ev.stop = c->ev[2 * i + 1];
    return LPSIM_OK;
}

// one kernel launch whose events take the dispatch's own start and end
// timestamps (hipExtLaunchKernel): the kernel's execution time
static int32_t timed(lpsim_ctx *c, const Dev &d, int phase, hipStream_t s,
                     void (*fn)(const Dev &, int, int, hipStream_t, KernelEvents)) {
    KernelEvents ev;
    int32_t rc = next_events(c, phase, ev);
    if (rc) return rc;
    fn(d, c->blocks, c->threads, s, ev);
    return LPSIM_OK;
}

static int reorder_interval(const lpsim_ctx *c) { return c->graph_steps > 0 ? c->graph_steps : 64; }

// the step (1-based) of a run of n steps after which the slot reorder falls,
// or 0 if the reorder interval does not end within them
static int reorder_point(const lpsim_ctx *c, int n) {
    const int r = reorder_interval(c) - c->since_reorder;
    return (r >= 1 && r <= n) ? r : 0;
}

static int32_t step_direct(lpsim_ctx *c, hipStream_t s) {
    int32_t rc;
    const Dev d = dev_at(c, c->k & 1);
    if (c->timing) {
        if ((rc = timed(c, d, 0, s, launch_move))) return rc;
        if ((rc = timed(c, d, 1, s, launch_resolve))) return rc;
        if (c->dp.lane_change && (rc = timed(c, d, 2, s, launch_lanechg))) return rc;
        if ((rc = timed(c, d, 3, s, launch_commit))) return rc;
    } else {
        enqueue_step(c, s, c->k & 1);
    }
    ++c->k;
    // the same reorder interval as the graphs (64 when kernels are launched singly)
    if (++c->since_reorder >= reorder_interval(c)) {
        const Dev dn = dev_at(c, c->k & 1);
        if (c->timing) {
            // several kernels: an event pair recorded around them
            KernelEvents ev;
            if ((rc = next_events(c, 4, ev))) return rc;
            HIPCHK(c, hipEventRecord(ev.start, s));
            launch_reorder(dn, c->blocks, c->threads, s);
            HIPCHK(c, hipEventRecord(ev.stop, s));
        } else {
            launch_reorder(dn, c->blocks, c->threads, s);
        }
        c->since_reorder = 0;
    }
    HIPCHK(c, hipGetLastError());
    return LPSIM_OK;
}

// ---------------------------------------------------------------------------
// read-back helpers

struct HostSlots {
    std::vector<float> x, v;
    std::vector<int32_t> e, ent;
    std::vector<uint32_t> m, id;
};

static int32_t read_ctrl(lpsim_ctx *c, Ctrl &ct) {
    HIPCHK(c, hipMemcpy(&ct, c->d.ctrl + (c->k & 1), sizeof ct, hipMemcpyDeviceToHost));
    return LPSIM_OK;
}

static int32_t read_slots(lpsim_ctx *c, const Ctrl &ct, HostSlots &h) {
    const uint32_t n = ct.n_slots + ct.n_new;
    const Slots &S = c->d.buf[ct.cur];
    h.x.resize(n); h.v.resize(n); h.e.resize(n); h.ent.resize(n); h.m.resize(n); h.id.resize(n);
    if (!n) return LPSIM_OK;
    HIPCHK(c, hipMemcpy(h.x.data(), S.x, n * 4, hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(h.v.data(), S.v, n * 4, hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(h.e.data(), S.e, n * 4, hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(h.ent.data(), S.ent, n * 4, hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(h.m.data(), S.m, n * 4, hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(h.id.data(), S.id, n * 4, hipMemcpyDeviceToHost));
    return LPSIM_OK;
}

static int32_t check_ready(lpsim_ctx *c, bool need_trips) {
    if (!c) return LPSIM_EINVAL;
    if (c->poisoned) return fail(c, LPSIM_EDEVICE, "context poisoned by an earlier device error: %s", c->err.c_str());
    if (!c->have_net) return fail(c, LPSIM_ESTATE, "no network loaded");
    if (need_trips && !c->have_trips) return fail(c, LPSIM_ESTATE, "no trips loaded");
    HIPCHK(c, hipSetDevice(c->device));
    return LPSIM_OK;
}

// ---------------------------------------------------------------------------
// ABI

extern "C" {

int32_t lpsim_create(const lpsim_params *p, lpsim_ctx **out) {
    if (!p || !out) return LPSIM_EINVAL;
    *out = nullptr;
    if (!(p->dt > 0 && p->a > 0 && p->b > 0 && p->s0 > 0 && p->T > 0 && p->veh_len > 0 && p->x0 > 0 &&
          p->g_a >= 0 && p->g_b >= 0 && p->alpha_i >= 0 && p->alpha_a >= 0 && p->alpha_b >= 0 &&
          p->eps_a >= 0 && p->eps_a <= 100 && p->eps_b >= 0 && p->eps_b <= 100 &&
          p->bin_seconds > 0 && p->delta == 4 && p->n_bins >= 1 &&
          (p->free_mode == LPSIM_FREE_JUMP || p->free_mode == LPSIM_FREE_IDM) &&
          (p->lane_change == 0 || p->lane_change == 1)))
        return LPSIM_EINVAL;
    const double bs = p->bin_seconds / (double)p->dt;
    const double bsr = std::nearbyint(bs);
    if (bsr < 1.0 || std::fabs(bs - bsr) > 1e-9 || bsr > 1e9) return LPSIM_EINVAL;
    lpsim_ctx *c = new (std::nothrow) lpsim_ctx();
    if (!c) return LPSIM_ENOMEM;
    c->P = *p;
    Params &dp = c->dp;
    dp.dt = p->dt; dp.a = p->a; dp.b = p->b; dp.s0 = p->s0; dp.T = p->T; dp.L = p->veh_len;
    dp.x0 = p->x0; dp.g_a = p->g_a; dp.g_b = p->g_b;
    dp.al_i = p->alpha_i; dp.al_a = p->alpha_a; dp.al_b = p->alpha_b;
    dp.eps_a = p->eps_a; dp.eps_b = p->eps_b;
    dp.tsab = (float)(2.0 * std::sqrt((double)p->a * (double)p->b));
    dp.half_dt = 0.5f * p->dt;
    dp.W = (int32_t)std::ceil((double)p->veh_len + (double)p->s0);
    dp.bin_steps = (int32_t)bsr;
    dp.n_bins = p->n_bins;
    dp.free_mode = p->free_mode;
    dp.lane_change = p->lane_change;
    c->d.p = dp;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        (void)hipGetLastError();
        delete c;
        return LPSIM_EDEVICE;
    }
    if (hipGetDevice(&c->device) != hipSuccess ||
        hipStreamCreateWithFlags(&c->own, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        delete c;
        return LPSIM_EDEVICE;
    }
    if (hipEventCreateWithFlags(&c->order_ev, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipStreamDestroy(c->own);
        delete c;
        return LPSIM_EDEVICE;
    }
    c->ev.resize(2 * 512);
    c->ev_phase.resize(512);
    // timing events without the system-scope fence: they order work on the
    // device only, so recording them adds as little as possible to a launch
    for (auto &e : c->ev) {
        if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) {
            (void)hipGetLastError();
            e = nullptr;
        }
    }
    *out = c;
    return LPSIM_OK;
}

void lpsim_destroy(lpsim_ctx *c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    if (c->last) (void)hipStreamSynchronize(c->last);
    if (c->own) (void)hipStreamSynchronize(c->own);
    release_net(c);
    if (c->route_pin) (void)hipHostFree(c->route_pin);
    for (auto &e : c->ev)
        if (e) (void)hipEventDestroy(e);
    if (c->order_ev) (void)hipEventDestroy(c->order_ev);
    if (c->own) (void)hipStreamDestroy(c->own);
    delete c;
}

int32_t lpsim_set_allocator(lpsim_ctx *c, void *(*alloc)(size_t, void *), void (*release)(void *, void *),
                            void *user) {
    if (!c || (alloc == nullptr) != (release == nullptr)) return LPSIM_EINVAL;
    if (c->have_net) return fail(c, LPSIM_ESTATE, "set the allocator before loading");
    c->ualloc = alloc;
    c->ufree = release;
    c->uuser = user;
    return LPSIM_OK;
}

int32_t lpsim_load_network(lpsim_ctx *c, int32_t n_nodes, const float *node_xy, int32_t n_edges,
                           const int32_t *src, const int32_t *dst, const float *length_m,
                           const uint8_t *lanes, const float *speed_limit_mps) {
    if (!c) return LPSIM_EINVAL;
    if (c->poisoned) return fail(c, LPSIM_EDEVICE, "context poisoned");
    if (n_nodes <= 0 || n_edges <= 0 || !src || !dst || !length_m || !lanes || !speed_limit_mps)
        return fail(c, LPSIM_EINVAL, "bad network arguments");
    HIPCHK(c, hipSetDevice(c->device));
    const int32_t noff[2] = {0, n_nodes}, eoff[2] = {0, n_edges};
    NetIn in{1, noff, eoff, node_xy, src, dst, length_m, lanes, speed_limit_mps};
    return build_network(c, in);
}

int32_t lpsim_load_trips(lpsim_ctx *c, int64_t n_trips, const int32_t *depart_step,
                         const int64_t *route_offsets, const int32_t *route_edges) {
    if (!c) return LPSIM_EINVAL;
    if (c->poisoned) return fail(c, LPSIM_EDEVICE, "context poisoned");
    if (!c->have_net) return fail(c, LPSIM_ESTATE, "load a network first");
    if (c->n_scen != 1) return fail(c, LPSIM_ESTATE, "context holds a batch; use lpsim_batch_load");
    if (n_trips < 0 || (n_trips > 0 && (!depart_step || !route_offsets || !route_edges)))
        return fail(c, LPSIM_EINVAL, "bad trip arguments");
    HIPCHK(c, hipSetDevice(c->device));
    const int64_t toff[2] = {0, n_trips};
    const int64_t zero = 0;
    TripIn in{toff, depart_step, n_trips ? route_offsets : &zero, route_edges, nullptr};
    return build_trips(c, in);
}

int32_t lpsim_batch_load(lpsim_ctx *c, int32_t n_scen, const int32_t *node_off, const int32_t *edge_off,
                         const int64_t *trip_off, const float *node_xy, const int32_t *src,
                         const int32_t *dst, const float *length_m, const uint8_t *lanes,
                         const float *speed_limit_mps, const int32_t *depart_step,
                         const int64_t *route_offsets, const int32_t *route_edges, const uint64_t *seeds) {
    if (!c) return LPSIM_EINVAL;
    if (c->poisoned) return fail(c, LPSIM_EDEVICE, "context poisoned");
    if (n_scen < 1 || !node_off || !edge_off || !trip_off || !src || !dst || !length_m || !lanes ||
        !speed_limit_mps || !route_offsets)
        return fail(c, LPSIM_EINVAL, "bad batch arguments");
    HIPCHK(c, hipSetDevice(c->device));
    NetIn in{n_scen, node_off, edge_off, node_xy, src, dst, length_m, lanes, speed_limit_mps};
    int32_t rc = build_network(c, in);
    if (rc) return rc;
    TripIn tin{trip_off, depart_step, route_offsets, route_edges, seeds};
    return build_trips(c, tin);
}

int32_t lpsim_step(lpsim_ctx *c, int32_t n_steps, void *hip_stream) {
    int32_t rc = check_ready(c, true);
    if (rc) return rc;
    if (n_steps < 0) return fail(c, LPSIM_EINVAL, "n_steps < 0");
    hipStream_t s = hip_stream ? (hipStream_t)hip_stream : c->own;
    if (c->last && c->last != s) {
        // work the previous call queued on another stream comes first
        HIPCHK(c, hipEventRecord(c->order_ev, c->last));
        HIPCHK(c, hipStreamWaitEvent(s, c->order_ev, 0));
    }
    c->last = s;
    if (c->timing || c->graph_steps == 0) {
        for (int32_t t = 0; t < n_steps; ++t)
            if ((rc = step_direct(c, s))) return rc;
    } else {
        if (!c->g_full[0] && (rc = build_graphs(c))) return rc;
        int32_t left = n_steps;
        while (left >= c->graph_steps) {
            HIPCHK(c, hipGraphLaunch(c->g_full[c->k & 1], s));
            c->k += c->graph_steps;
            left -= c->graph_steps;
            c->since_reorder = 0;  // the graph ends with a reorder
        }
        if (left > 1) {
            // the rest in one shorter graph; its steps count toward the same
            // reorder interval, so calls shorter than a graph still compact
            // the slots
            const int r = reorder_point(c, left);
            hipGraphExec_t ex = nullptr;
            if ((rc = part_graph(c, left, r, &ex))) return rc;
            HIPCHK(c, hipGraphLaunch(ex, s));
            c->k += left;
            c->since_reorder = r ? left - r : c->since_reorder + left;
        } else if (left == 1) {
            HIPCHK(c, hipGraphLaunch(c->g_one[c->k & 1], s));
            ++c->k;
            if (++c->since_reorder >= reorder_interval(c)) {
                launch_reorder(dev_at(c, c->k & 1), c->blocks, c->threads, s);
                HIPCHK(c, hipGetLastError());
                c->since_reorder = 0;
            }
        }
    }
    if (!hip_stream) HIPCHK(c, hipStreamSynchronize(s));
    return LPSIM_OK;
}

int32_t lpsim_prepare_steps(lpsim_ctx *c, int32_t n_steps) {
    int32_t rc = check_ready(c, true);
    if (rc) return rc;
    if (n_steps < 0) return fail(c, LPSIM_EINVAL, "n_steps < 0");
    if (c->timing || c->graph_steps == 0) return LPSIM_OK;
    if (!c->g_full[0] && (rc = build_graphs(c))) return rc;
    // the same walk as lpsim_step, without launching
    const int left = n_steps % c->graph_steps;
    if (left > 1) {
        const int k0 = c->k, s0 = c->since_reorder;
        const int full = n_steps / c->graph_steps;
        c->k += full * c->graph_steps;
        if (full) c->since_reorder = 0;
        hipGraphExec_t ex = nullptr;
        rc = part_graph(c, left, reorder_point(c, left), &ex);
        c->k = k0;
        c->since_reorder = s0;
        if (rc) return rc;
    }
    return LPSIM_OK;
}

int32_t lpsim_edge_stats(lpsim_ctx *c, int64_t *tt_sum_steps, int32_t *n_exits, int32_t *inflow_bin,
                         int32_t *exits_bin, int64_t *tt_sum_bin, int64_t *occ_steps_bin) {
    int32_t rc = check_ready(c, true);
    if (rc) return rc;
    if ((rc = sync_all(c))) return rc;
    const size_t E = (size_t)c->n_edges, B = (size_t)c->dp.n_bins;
    const Dev &d = c->d;
    auto perm_rows = [&](auto *dst_ext, const auto &src_int, size_t width) {
        for (size_t i = 0; i < E; ++i) {
            const size_t e = (size_t)c->ext_of_int[i];
            std::memcpy(dst_ext + e * width, src_int.data() + i * width, width * sizeof(src_int[0]));
        }
    };
    if (tt_sum_steps) {
        std::vector<int64_t> t(E);
        HIPCHK(c, hipMemcpy(t.data(), d.tt_sum, E * 8, hipMemcpyDeviceToHost));
        perm_rows(tt_sum_steps, t, 1);
    }
    if (n_exits) {
        std::vector<int32_t> t(E);
        HIPCHK(c, hipMemcpy(t.data(), d.n_exits, E * 4, hipMemcpyDeviceToHost));
        perm_rows(n_exits, t, 1);
    }
    if (inflow_bin) {
        std::vector<int32_t> t(E * B);
        HIPCHK(c, hipMemcpy(t.data(), d.inflow_bin, E * B * 4, hipMemcpyDeviceToHost));
        perm_rows(inflow_bin, t, B);
    }
    if (exits_bin) {
        std::vector<int32_t> t(E * B);
        HIPCHK(c, hipMemcpy(t.data(), d.exits_bin, E * B * 4, hipMemcpyDeviceToHost));
        perm_rows(exits_bin, t, B);
    }
    if (tt_sum_bin) {
        std::vector<int64_t> t(E * B);
        HIPCHK(c, hipMemcpy(t.data(), d.tt_bin, E * B * 8, hipMemcpyDeviceToHost));
        perm_rows(tt_sum_bin, t, B);
    }
    if (occ_steps_bin) {
        std::vector<int64_t> t(E * B);
        HIPCHK(c, hipMemcpy(t.data(), d.occ_bin, E * B * 8, hipMemcpyDeviceToHost));
        // vehicles still on an edge: the steps they have spent there so far
        Ctrl ct;
        if ((rc = read_ctrl(c, ct))) return rc;
        HostSlots h;
        if ((rc = read_slots(c, ct, h))) return rc;
        const int32_t bs = c->dp.bin_steps, nb = c->dp.n_bins;
        for (size_t i = 0; i < h.m.size(); ++i) {
            if (h.m[i] & M_DEAD) continue;
            const int32_t en = h.ent[i], ex = ct.k;
            if (ex <= en) continue;
            const int32_t b0 = std::min(en / bs, nb - 1), b1 = std::min((ex - 1) / bs, nb - 1);
            for (int32_t b = b0; b <= b1; ++b) {
                const int32_t lo = b * bs, hi = (b == nb - 1) ? 0x7fffffff : lo + bs;
                t[(size_t)h.e[i] * B + (size_t)b] += std::min(ex, hi) - std::max(en, lo);
            }
        }
        perm_rows(occ_steps_bin, t, B);
    }
    return LPSIM_OK;
}

int32_t lpsim_edge_stats_device(lpsim_ctx *c, int32_t *inflow_bin, int32_t *exits_bin, int64_t *tt_sum_bin,
                                int64_t *occ_steps_bin, void *hip_stream) {
    int32_t rc = check_ready(c, true);
    if (rc) return rc;
    hipStream_t s = hip_stream ? (hipStream_t)hip_stream : c->own;
    if (c->last && c->last != s) {
        // the steps queued on another stream come first
        HIPCHK(c, hipEventRecord(c->order_ev, c->last));
        HIPCHK(c, hipStreamWaitEvent(s, c->order_ev, 0));
    }
    c->last = s;
    HIPCHK(c, launch_stats_device(c->d, c->d.ctrl + (c->k & 1), c->ext_d, c->n_edges, c->dp.n_bins,
                                  c->dp.bin_steps, c->slot_cap, inflow_bin, exits_bin,
                                  (unsigned long long *)tt_sum_bin, (unsigned long long *)occ_steps_bin, s));
    return LPSIM_OK;
}

int32_t lpsim_get_vehicles(lpsim_ctx *c, int32_t *edge, uint8_t *lane, int32_t *cell, float *x, float *v,
                           int32_t *arrival_step, uint8_t *status) {
    int32_t rc = check_ready(c, true);
    if (rc) return rc;
    if ((rc = sync_all(c))) return rc;
    const size_t N = (size_t)c->n_trips;
    std::vector<uint8_t> st(N + 1);
    std::vector<int32_t> arr(N + 1);
    HIPCHK(c, hipMemcpy(st.data(), c->d.status, N + 1, hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(arr.data(), c->d.arrival, (N + 1) * 4, hipMemcpyDeviceToHost));
    for (size_t i = 0; i < N; ++i) {
        if (edge) edge[i] = -1;
        if (lane) lane[i] = 0;
        if (cell) cell[i] = -1;
        if (x) x[i] = 0.0f;
        if (v) v[i] = 0.0f;
        if (arrival_step) arrival_step[i] = arr[i];
        if (status) status[i] = st[i];
    }
    Ctrl ct;
    if ((rc = read_ctrl(c, ct))) return rc;
    HostSlots h;
    if ((rc = read_slots(c, ct, h))) return rc;
    for (size_t i = 0; i < h.m.size(); ++i) {
        if (h.m[i] & M_DEAD) continue;
        const size_t id = h.id[i];
        if (id >= N) return fail(c, LPSIM_EINVAL, "corrupt slot %zu", i);
        if (edge) {
            // global input edge id -> scenario-local id
            const int32_t g = c->ext_of_int[h.e[i]];
            const int32_t s = (int32_t)(std::upper_bound(c->edge_off.begin(), c->edge_off.end(), g) -
                                        c->edge_off.begin()) - 1;
            edge[id] = g - c->edge_off[s];
        }
        if (lane) lane[id] = (uint8_t)(h.m[i] & M_LANE);
        if (cell) cell[id] = (int32_t)h.x[i];
        if (x) x[id] = h.x[i];
        if (v) v[id] = h.v[i];
    }
    return LPSIM_OK;
}

int32_t lpsim_get_counters(lpsim_ctx *c, lpsim_counters *out) {
    if (!out) return LPSIM_EINVAL;
    int32_t rc = check_ready(c, true);
    if (rc) return rc;
    if ((rc = sync_all(c))) return rc;
    std::vector<unsigned long long> part((size_t)PART_ROWS * NPART);
    HIPCHK(c, hipMemcpy(part.data(), c->d.partial, part.size() * 8, hipMemcpyDeviceToHost));
    unsigned long long tot[NPART] = {0};
    for (size_t b = 0; b < (size_t)PART_ROWS; ++b)
        for (int j = 0; j < NPART; ++j) tot[j] += part[b * NPART + j];
    Ctrl ct;
    if ((rc = read_ctrl(c, ct))) return rc;
    out->step = ct.k;
    out->active = ct.n_alive;
    out->departures = (int64_t)tot[P_DEPARTS];
    out->waiting = c->n_trips - out->departures;
    out->arrived = (int64_t)tot[P_ARRIVED];
    out->vehicle_steps = (int64_t)tot[P_VSTEPS];
    out->transfers = (int64_t)tot[P_TRANSFERS];
    out->claims_lost = (int64_t)tot[P_LOST];
    out->lc_attempts = (int64_t)tot[P_LC_TRY];
    out->lc_accepts = (int64_t)tot[P_LC_OK];
    out->watchdog = ct.watchdog;
    out->scan_bytes = (int64_t)tot[P_SCAN];
    return LPSIM_OK;
}

int32_t lpsim_block_edge(lpsim_ctx *c, int32_t edge, int32_t on) {
    int32_t rc = check_ready(c, false);
    if (rc) return rc;
    if (c->n_scen != 1) return fail(c, LPSIM_EINVAL, "block_edge takes a single-scenario context");
    if (edge < 0 || edge >= c->n_edges) return fail(c, LPSIM_EINVAL, "edge out of range");
    if ((rc = sync_all(c))) return rc;
    const int32_t i = c->int_of_ext[edge];
    if (on) c->aux_h[i] |= AUX_BLOCKED;
    else c->aux_h[i] &= ~AUX_BLOCKED;
    HIPCHK(c, hipMemcpy(c->d.aux + i, &c->aux_h[i], 4, hipMemcpyHostToDevice));
    if (c->have_trips) {
        // vehicles already heading for this edge carry its flag in their cache
        launch_set_next_blocked(dev_at(c, c->k & 1), i, on != 0, c->own);
        HIPCHK(c, hipGetLastError());
        HIPCHK(c, hipStreamSynchronize(c->own));
    }
    return LPSIM_OK;
}

int32_t lpsim_set_signals(lpsim_ctx *c, const int32_t *n_phases, const int32_t *green, const int32_t *allred,
                          const int32_t *offset, const int32_t *edge_phase) {
    int32_t rc = check_ready(c, false);
    if (rc) return rc;
    const int32_t E = c->n_edges;
    std::vector<uint2> w((size_t)E, make_uint2(0u, 0u));
    if (n_phases) {
        if (!green || !allred || !offset || !edge_phase) return fail(c, LPSIM_EINVAL, "null signal array");
        const int32_t n_nodes = c->node_off[c->n_scen];
        for (int32_t n = 0; n < n_nodes; ++n) {
            if (n_phases[n] < 0 || n_phases[n] > 15) return fail(c, LPSIM_EINVAL, "node %d: phases not in 0..15", n);
            if (n_phases[n] == 0) continue;
            if (green[n] < 1 || allred[n] < 0) return fail(c, LPSIM_EINVAL, "node %d: bad green or all-red", n);
            const int64_t cyc = (int64_t)n_phases[n] * ((int64_t)green[n] + allred[n]);
            if (cyc > 65535) return fail(c, LPSIM_EINVAL, "node %d: cycle above 65535 steps", n);
            if (offset[n] < 0 || offset[n] >= cyc) return fail(c, LPSIM_EINVAL, "node %d: offset outside the cycle", n);
        }
        for (int32_t s = 0; s < c->n_scen; ++s) {
            for (int32_t e = c->edge_off[s]; e < c->edge_off[s + 1]; ++e) {
                const int32_t n = c->node_off[s] + c->dst_g[e];
                const int32_t ph = edge_phase[e];
                if (ph < -1 || ph >= n_phases[n]) return fail(c, LPSIM_EINVAL, "edge %d: phase not served by its node", e);
                if (ph < 0) continue;
                const uint32_t per = (uint32_t)(green[n] + allred[n]);
                const uint32_t cyc = per * (uint32_t)n_phases[n];
                const uint32_t g0 = (uint32_t)ph * per;
                w[(size_t)c->int_of_ext[e]] = make_uint2(cyc | ((uint32_t)offset[n] << 16),
                                                         g0 | ((g0 + (uint32_t)green[n]) << 16));
            }
        }
    }
    if ((rc = sync_all(c))) return rc;
    if (n_phases) {
        if (!c->sig_d && (rc = alloc_n(c, c->sig_d, (size_t)E, c->net_allocs))) return rc;
        HIPCHK(c, hipMemcpy(c->sig_d, w.data(), (size_t)E * sizeof(uint2), hipMemcpyHostToDevice));
    }
    c->d.sig = n_phases ? c->sig_d : nullptr;
    // captured graphs hold the old device view
    drop_graphs(c);
    if (c->have_trips) {
        // vehicles already on the road carry the flag of their edge
        launch_refresh_flags(dev_at(c, c->k & 1), c->own);
        HIPCHK(c, hipGetLastError());
        HIPCHK(c, hipStreamSynchronize(c->own));
    }
    return LPSIM_OK;
}

int32_t lpsim_set_launch(lpsim_ctx *c, int32_t block_size, int32_t n_blocks, int32_t graph_steps) {
    if (!c) return LPSIM_EINVAL;
    if (block_size < 64 || block_size > 1024 || block_size % 64 || n_blocks < 8 || n_blocks > MAX_BLOCKS ||
        n_blocks % 8 || graph_steps < 0 || graph_steps > 4096)
        return fail(c, LPSIM_EINVAL, "bad launch shape");
    if (c->have_trips) {
        int32_t rc = sync_all(c);
        if (rc) return rc;
    }
    c->threads = block_size;
    c->blocks = n_blocks;
    c->graph_steps = graph_steps;
    drop_graphs(c);
    return LPSIM_OK;
}

int32_t lpsim_set_timing(lpsim_ctx *c, int32_t on) {
    if (!c) return LPSIM_EINVAL;
    for (const auto &e : c->ev)
        if (!e) return fail(c, LPSIM_EDEVICE, "timing events unavailable");
    if (c->have_trips) {
        int32_t rc = sync_all(c);
        if (rc) return rc;
    }
    c->timing = on != 0;
    c->ev_used = 0;
    for (int i = 0; i < N_PHASES; ++i) {
        c->ms[i] = 0.0;
        c->launches[i] = 0;
    }
    return LPSIM_OK;
}

int32_t lpsim_kernel_times(lpsim_ctx *c, double *ms_out, int64_t *launches_out, int32_t n_phases) {
    if (!c || n_phases < 0) return LPSIM_EINVAL;
    int32_t rc = harvest_events(c);
    if (rc) return rc;
    for (int i = 0; i < n_phases && i < N_PHASES; ++i) {
        if (ms_out) ms_out[i] = c->ms[i];
        if (launches_out) launches_out[i] = c->launches[i];
    }
    return LPSIM_OK;
}

// snapshot layout: header, ctrl, partial counters, lane map, trip status and
// arrival, statistics, live slots, the waiting sets (bits, heads, counts)
// and the live list of origin lanes with waiting trips
struct SnapHeader {
    uint64_t magic;
    uint64_t n_trips, n_edges, map_bytes, n_bins, n_slots, n_aq;
};

static size_t snap_size(const lpsim_ctx *c, uint64_t n_slots, uint64_t n_aq) {
    const size_t N = (size_t)c->n_trips, E = (size_t)c->n_edges, B = (size_t)c->dp.n_bins;
    return sizeof(SnapHeader) + sizeof(Ctrl) + (size_t)PART_ROWS * NPART * 8 + c->map_bytes + (N + 1) * 5 +
           E * 12 + E * B * 24 + (size_t)n_slots * 56 + (N / 32 + 1) * 4 + ((size_t)c->d.n_ol + 1) * 12 +
           (size_t)n_aq * 16;
}

// origin lanes in the live waiting list
static int32_t read_n_aq(lpsim_ctx *c, const Ctrl &ct, uint32_t &n_aq) {
    HIPCHK(c, hipMemcpy(&n_aq, c->d.aq_n + (ct.aq_cur & 1u), 4, hipMemcpyDeviceToHost));
    return LPSIM_OK;
}

int32_t lpsim_state_size(lpsim_ctx *c, size_t *bytes) {
    if (!bytes) return LPSIM_EINVAL;
    int32_t rc = check_ready(c, true);
    if (rc) return rc;
    if ((rc = sync_all(c))) return rc;
    Ctrl ct;
    if ((rc = read_ctrl(c, ct))) return rc;
    uint32_t n_aq;
    if ((rc = read_n_aq(c, ct, n_aq))) return rc;
    *bytes = snap_size(c, ct.n_slots, n_aq);
    return LPSIM_OK;
}

int32_t lpsim_save_state(lpsim_ctx *c, void *buf, size_t bytes) {
    int32_t rc = check_ready(c, true);
    if (rc) return rc;
    if (!buf) return LPSIM_EINVAL;
    if ((rc = sync_all(c))) return rc;
    Ctrl ct;
    if ((rc = read_ctrl(c, ct))) return rc;
    uint32_t n_aq;
    if ((rc = read_n_aq(c, ct, n_aq))) return rc;
    if (bytes < snap_size(c, ct.n_slots, n_aq)) return fail(c, LPSIM_EINVAL, "snapshot buffer too small");
    const Dev &d = c->d;
    const size_t N = (size_t)c->n_trips, E = (size_t)c->n_edges, B = (size_t)c->dp.n_bins;
    char *p = (char *)buf;
    SnapHeader h{SNAP_MAGIC, N, E, c->map_bytes, B, ct.n_slots, n_aq};
    std::memcpy(p, &h, sizeof h); p += sizeof h;
    std::memcpy(p, &ct, sizeof ct); p += sizeof ct;
    auto get = [&](const void *src, size_t n) -> int32_t {
        HIPCHK(c, hipMemcpy(p, src, n, hipMemcpyDeviceToHost));
        p += n;
        return LPSIM_OK;
    };
    if ((rc = get(d.partial, (size_t)PART_ROWS * NPART * 8))) return rc;
    if ((rc = get(d.map, c->map_bytes))) return rc;
    if ((rc = get(d.status, N + 1))) return rc;
    if ((rc = get(d.arrival, (N + 1) * 4))) return rc;
    if ((rc = get(d.n_exits, E * 4))) return rc;
    if ((rc = get(d.tt_sum, E * 8))) return rc;
    if ((rc = get(d.inflow_bin, E * B * 4))) return rc;
    if ((rc = get(d.exits_bin, E * B * 4))) return rc;
    if ((rc = get(d.tt_bin, E * B * 8))) return rc;
    if ((rc = get(d.occ_bin, E * B * 8))) return rc;
    const Slots &S = d.buf[ct.cur];
    const size_t n = ct.n_slots;
    if ((rc = get(S.x, n * 4))) return rc;
    if ((rc = get(S.v, n * 4))) return rc;
    if ((rc = get(S.e, n * 4))) return rc;
    if ((rc = get(S.en, n * 4))) return rc;
    if ((rc = get(S.m, n * 4))) return rc;
    if ((rc = get(S.id, n * 4))) return rc;
    if ((rc = get(S.rp, n * 4))) return rc;
    if ((rc = get(S.rend, n * 4))) return rc;
    if ((rc = get(S.ent, n * 4))) return rc;
    if ((rc = get(S.lb, n * 4))) return rc;
    if ((rc = get(S.cd, n * 4))) return rc;
    if ((rc = get(S.v0, n * 4))) return rc;
    if ((rc = get(S.tlb, n * 4))) return rc;
    if ((rc = get(S.tgt, n * 4))) return rc;
    if ((rc = get(d.ol_bits, (N / 32 + 1) * 4))) return rc;
    if ((rc = get(d.ol_head, ((size_t)d.n_ol + 1) * 8))) return rc;
    if ((rc = get(d.ol_cnt, ((size_t)d.n_ol + 1) * 4))) return rc;
    if ((rc = get(d.aq[ct.aq_cur & 1u], (size_t)n_aq * 16))) return rc;
    return LPSIM_OK;
}

int32_t lpsim_restore_state(lpsim_ctx *c, const void *buf, size_t bytes) {
    int32_t rc = check_ready(c, true);
    if (rc) return rc;
    if (!buf || bytes < sizeof(SnapHeader) + sizeof(Ctrl)) return fail(c, LPSIM_EINVAL, "snapshot too small");
    if ((rc = sync_all(c))) return rc;
    const char *p = (const char *)buf;
    SnapHeader h;
    std::memcpy(&h, p, sizeof h); p += sizeof h;
    const Dev &d = c->d;
    const size_t N = (size_t)c->n_trips, E = (size_t)c->n_edges, B = (size_t)c->dp.n_bins;
    if (h.magic != SNAP_MAGIC || h.n_trips != N || h.n_edges != E || h.map_bytes != c->map_bytes || h.n_bins != B ||
        h.n_slots > c->slot_cap || h.n_aq > c->d.n_ol || bytes < snap_size(c, h.n_slots, h.n_aq))
        return fail(c, LPSIM_EINVAL, "snapshot does not match this instance");
    Ctrl ct;
    std::memcpy(&ct, p, sizeof ct); p += sizeof ct;
    ct.cur = 0;
    ct.aq_cur = 0;
    auto put = [&](void *dst, size_t n) -> int32_t {
        HIPCHK(c, hipMemcpy(dst, p, n, hipMemcpyHostToDevice));
        p += n;
        return LPSIM_OK;
    };
    if ((rc = put(d.partial, (size_t)PART_ROWS * NPART * 8))) return rc;
    if ((rc = put(d.map, c->map_bytes))) return rc;
    if ((rc = put(d.status, N + 1))) return rc;
    if ((rc = put(d.arrival, (N + 1) * 4))) return rc;
    if ((rc = put(d.n_exits, E * 4))) return rc;
    if ((rc = put(d.tt_sum, E * 8))) return rc;
    if ((rc = put(d.inflow_bin, E * B * 4))) return rc;
    if ((rc = put(d.exits_bin, E * B * 4))) return rc;
    if ((rc = put(d.tt_bin, E * B * 8))) return rc;
    if ((rc = put(d.occ_bin, E * B * 8))) return rc;
    const Slots &S = d.buf[0];
    const size_t n = h.n_slots;
    if ((rc = put(S.x, n * 4))) return rc;
    if ((rc = put(S.v, n * 4))) return rc;
    if ((rc = put(S.e, n * 4))) return rc;
    if ((rc = put(S.en, n * 4))) return rc;
    if ((rc = put(S.m, n * 4))) return rc;
    if ((rc = put(S.id, n * 4))) return rc;
    if ((rc = put(S.rp, n * 4))) return rc;
    if ((rc = put(S.rend, n * 4))) return rc;
    if ((rc = put(S.ent, n * 4))) return rc;
    if ((rc = put(S.lb, n * 4))) return rc;
    if ((rc = put(S.cd, n * 4))) return rc;
    if ((rc = put(S.v0, n * 4))) return rc;
    if ((rc = put(S.tlb, n * 4))) return rc;
    if ((rc = put(S.tgt, n * 4))) return rc;
    if ((rc = put(d.ol_bits, (N / 32 + 1) * 4))) return rc;
    if ((rc = put(d.ol_head, ((size_t)d.n_ol + 1) * 8))) return rc;
    if ((rc = put(d.ol_cnt, ((size_t)d.n_ol + 1) * 4))) return rc;
    if ((rc = put(d.aq[0], (size_t)h.n_aq * 16))) return rc;
    const uint32_t aq_n[2] = {(uint32_t)h.n_aq, 0u};
    HIPCHK(c, hipMemcpy(d.aq_n, aq_n, sizeof aq_n, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemset(d.claims, 0xff, (size_t)c->n_lane_slots * 4));
    HIPCHK(c, hipMemset(d.ecnt, 0, (size_t)c->n_edges * 4));
    HIPCHK(c, hipMemcpy(d.ctrl + (ct.k & 1), &ct, sizeof ct, hipMemcpyHostToDevice));
    c->k = ct.k;
    c->since_reorder = 0;
    // the snapshot's cached edge flags follow the signal plan and blocked
    // edges of now, not of when it was taken
    launch_refresh_flags(dev_at(c, c->k & 1), c->own);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipDeviceSynchronize());
    return LPSIM_OK;
}

int32_t lpsim_autotune(lpsim_ctx *c, int32_t n_steps, const int32_t *block_sizes, int32_t n_bs,
                       const int32_t *block_counts, int32_t n_bc, int32_t *best_out, double *trial_us) {
    int32_t rc = check_ready(c, true);
    if (rc) return rc;
    if (n_steps < 1 || n_bs < 1 || n_bc < 1 || !block_sizes || !block_counts || !best_out)
        return fail(c, LPSIM_EINVAL, "bad autotune arguments");
    for (int32_t i = 0; i < n_bs; ++i)
        if (block_sizes[i] < 64 || block_sizes[i] > 1024 || block_sizes[i] % 64)
            return fail(c, LPSIM_EINVAL, "bad block size %d", block_sizes[i]);
    for (int32_t j = 0; j < n_bc; ++j)
        if (block_counts[j] < 8 || block_counts[j] > MAX_BLOCKS || block_counts[j] % 8)
            return fail(c, LPSIM_EINVAL, "bad block count %d", block_counts[j]);
    if (c->timing) return fail(c, LPSIM_ESTATE, "turn kernel timing off before autotuning");
    size_t bytes = 0;
    if ((rc = lpsim_state_size(c, &bytes))) return rc;
    std::vector<uint8_t> snap;
    try {
        snap.resize(bytes);
    } catch (...) {
        return fail(c, LPSIM_ENOMEM, "no host memory for the autotune snapshot");
    }
    if ((rc = lpsim_save_state(c, snap.data(), bytes))) return rc;
    const int keep_threads = c->threads, keep_blocks = c->blocks;
    hipEvent_t t0 = nullptr, t1 = nullptr;
    HIPCHK(c, hipEventCreate(&t0));
    HIPCHK(c, hipEventCreate(&t1));
    double best = 1e300;
    int best_t = keep_threads, best_b = keep_blocks;
    for (int32_t i = 0; i < n_bs; ++i) {
        for (int32_t j = 0; j < n_bc; ++j) {
            c->threads = block_sizes[i];
            c->blocks = block_counts[j];
            drop_graphs(c);
            if ((rc = lpsim_restore_state(c, snap.data(), bytes))) break;
            // one untimed graph replay to build and warm the graphs, then rewind
            if ((rc = lpsim_step(c, std::min(n_steps, std::max(c->graph_steps, 1)), c->own))) break;
            if ((rc = lpsim_restore_state(c, snap.data(), bytes))) break;
            HIPCHK(c, hipEventRecord(t0, c->own));
            if ((rc = lpsim_step(c, n_steps, c->own))) break;
            HIPCHK(c, hipEventRecord(t1, c->own));
            HIPCHK(c, hipEventSynchronize(t1));
            float ms = 0.f;
            HIPCHK(c, hipEventElapsedTime(&ms, t0, t1));
            const double us = 1000.0 * (double)ms / n_steps;
            if (trial_us) trial_us[i * n_bc + j] = us;
            if (us < best) {
                best = us;
                best_t = c->threads;
                best_b = c->blocks;
            }
        }
        if (rc) break;
    }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    c->threads = rc ? keep_threads : best_t;
    c->blocks = rc ? keep_blocks : best_b;
    drop_graphs(c);
    int32_t rc2 = lpsim_restore_state(c, snap.data(), bytes);
    if (rc) return rc;
    if (rc2) return rc2;
    best_out[0] = best_t;
    best_out[1] = best_b;
    best_out[2] = (int32_t)std::lround(best);
    return LPSIM_OK;
}

int32_t lpsim_query(const lpsim_ctx *c, int32_t which) {
    if (!c) return LPSIM_EINVAL;
    if (which == 0) return c->dp.W;
    if (which == 1) return c->look.empty() ? LPSIM_ESTATE : c->look[0];
    if (which == 2) return c->dp.bin_steps;
    return LPSIM_EINVAL;
}

const char *lpsim_last_error(const lpsim_ctx *c) { return c ? c->err.c_str() : ""; }

}  // extern "C"
