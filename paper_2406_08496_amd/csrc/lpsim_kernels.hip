// lpsim_kernels.hip -- gfx950 kernels of one simulation step.
//
// One step k -> k+1 (paper Section 3.1, vehicle-dynamics equation: every new
// state depends on step-k state only; Algorithm 1 per vehicle) runs as four
// kernels, each a grid of fixed shape that walks the current work list:
//
//   move     reads the lane map of step k: leader scan, IDM / free move,
//            stop line, crossing; entry requests of crossing vehicles and of
//            due trips go into one 32-bit word per target lane by atomicMin
//            of the trip id (exclusive entry, lowest id wins); due trips wait
//            in per-origin-lane sets, and only each set's lowest id asks;
//   resolve  winners enter, losers wait at the last cell, arrivals leave;
//            each vehicle clears its old cell byte and writes its new one --
//            no two vehicles touch the same byte in this kernel (a mover never
//            lands on a cell another vehicle occupied at step k, entries need
//            the first W cells free); per-edge statistics by atomics; trips
//            that could not enter keep waiting in their lane's set;
//   lanechg  mandatory lane change decided on the post-move map;
//   commit   writes the accepted lane changes into the map; its helper
//            blocks end the step (clock, counts) and queue the trips that
//            fall due at the next step.
//   reorder  (every few steps) a counting sort of the live vehicle slots by
//            edge: drops finished vehicles and puts vehicles of one edge next
//            to each other, so neighbouring lanes share cache lines.
//
// Vehicle state lives in slots (structure of arrays) that only hold vehicles
// on the road; the per-step control words live in device memory so that a
// captured HIP graph of many steps replays without host involvement.  Every
// loop walks whole wavefronts (64 lanes) together so that list appends can be
// aggregated per wavefront with a ballot.
//
// All floating point is binary32 with no contraction (-ffp-contract=off) and
// IEEE division, in exactly the order of the method's definition, so results
// are identical to the CPU oracle bit for bit.

#include <hip/hip_ext.h>

#include "lpsim_dev.h"

namespace lpsim {

// Work block b of G (b counted after any leading helper blocks, whose number
// is a multiple of 8) -> its share of the work list.  Blocks are dispatched
// round-robin over the 8 XCDs; give each XCD one contiguous eighth of the
// list so neighbouring vehicles (which read neighbouring lane-map bytes)
// share that XCD's L2.
__device__ __forceinline__ uint32_t logical_block(uint32_t b, uint32_t G) {
    if ((G & 7u) == 0u) return (b & 7u) * (G >> 3) + (b >> 3);
    return b;
}

// [lo, hi) of a list of `total` items for logical block lb of G
__device__ __forceinline__ void block_range(uint64_t total, uint32_t lb, uint32_t G, uint64_t &lo, uint64_t &hi) {
    uint64_t chunk = (total + G - 1) / G;
    chunk = (chunk + 63) & ~uint64_t(63);
    lo = (uint64_t)lb * chunk;
    hi = lo + chunk;
    if (hi > total) hi = total;
    if (lo > total) lo = total;
}

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & 63u; }

// An empty statement that takes loaded values: the loads before it are all
// issued before the code after it runs, so a test of one loaded value cannot
// make the compiler sink the other loads below that test (one memory round
// trip for all of them instead of two or more in a row).
#define ISSUED_TOGETHER6(a, b, c, d, e, f) \
    __asm__ volatile("" : "+v"(a), "+v"(b), "+v"(c), "+v"(d), "+v"(e), "+v"(f))
#define ISSUED_TOGETHER7(a, b, c, d, e, f, g) \
    __asm__ volatile("" : "+v"(a), "+v"(b), "+v"(c), "+v"(d), "+v"(e), "+v"(f), "+v"(g))
#define ISSUED_TOGETHER4(a, b, c, d) __asm__ volatile("" : "+v"(a), "+v"(b), "+v"(c), "+v"(d))
#define ISSUED_TOGETHER9(a, b, c, d, e, f, g, h, i)                                                     \
    __asm__ volatile("" : "+v"(a), "+v"(b), "+v"(c), "+v"(d), "+v"(e), "+v"(f), "+v"(g), "+v"(h), \
                     "+v"(i))

// wavefront-aggregated append: returns this lane's index in `list` (valid if pred)
__device__ __forceinline__ uint32_t wave_append(uint32_t *counter, bool pred) {
    const uint64_t mask = __ballot(pred);
    uint32_t base = 0;
    if (mask) {
        const uint32_t leader = (uint32_t)__ffsll((long long)mask) - 1u;
        if (lane_id() == leader) base = atomicAdd(counter, (uint32_t)__popcll(mask));
        base = __shfl(base, (int)leader);
    }
    return base + (uint32_t)__popcll(mask & ((1ull << lane_id()) - 1ull));
}

__device__ __forceinline__ uint8_t speed_byte(float v) {
    float c = v < 254.0f ? v : 254.0f;
    return (uint8_t)(int32_t)c;
}

__device__ __forceinline__ int32_t bin_of(const Params &p, int32_t step) {
    int32_t b = step / p.bin_steps;
    return b < p.n_bins - 1 ? b : p.n_bins - 1;
}

// ---------------------------------------------------------------------------
// lane-map scans.  A window of cells is read as 16-byte chunks from the
// dword boundary at or below its first byte (the memory system takes 16-byte
// loads at any dword boundary; the map starts 256-aligned and has 256 spare
// bytes at its end, so every chunk is readable), three chunks per group: one
// group covers any window of up to 45 cells, so the default look-ahead of 41
// cells is one round trip.  Inside a group the chunk holding the wanted byte
// is picked first, then the dword inside it, with selects and no branches.

constexpr uint32_t FREE_WORD = 0xffffffffu;

__device__ __forceinline__ uint4 ld16(const uint8_t *map, uint32_t a) {
    typedef uint32_t u32x4_a4 __attribute__((ext_vector_type(4), aligned(4)));
    const u32x4_a4 r = *reinterpret_cast<const u32x4_a4 *>(map + a);
    return make_uint4(r.x, r.y, r.z, r.w);
}

// occupied bits of a dword: a byte is occupied unless it is 0xFF, so any set
// bit of ~w marks an occupied byte; the lowest set bit lies in the first one
__device__ __forceinline__ uint32_t first_byte(uint32_t t) {
    return (uint32_t)__builtin_ctz(t | 0x80000000u) >> 3;  // t != 0
}
__device__ __forceinline__ uint32_t last_byte(uint32_t t) {
    return (31u - (uint32_t)__builtin_clz(t | 1u)) >> 3;  // t != 0
}

// one group: three chunks from map offset a (dword-aligned); chunks that
// start after the window's last byte e are not read and stand as free
struct Group3 {
    uint4 c0, c1, c2;
};

__device__ __forceinline__ Group3 load_group(const uint8_t *map, uint32_t a, uint32_t e) {
    const uint4 f = make_uint4(FREE_WORD, FREE_WORD, FREE_WORD, FREE_WORD);
    const uint32_t span = e - a;
    Group3 g;
    g.c0 = ld16(map, a);
    g.c1 = span >= 16u ? ld16(map, a + 16) : f;
    g.c2 = span >= 32u ? ld16(map, a + 32) : f;
    return g;
}

// first occupied byte at or after s (a <= s <= a + 3) inside a group loaded
// from a: its offset from a, or 48 if none; *w receives its dword
__device__ __forceinline__ uint32_t group_first(Group3 g, uint32_t a, uint32_t s, uint32_t *w) {
    g.c0.x |= ~(FREE_WORD << (8u * (s - a)));  // bytes before s read as free
    const bool h0 = (g.c0.x & g.c0.y & g.c0.z & g.c0.w) != FREE_WORD;
    const bool h1 = (g.c1.x & g.c1.y & g.c1.z & g.c1.w) != FREE_WORD;
    const bool h2 = (g.c2.x & g.c2.y & g.c2.z & g.c2.w) != FREE_WORD;
    // the first chunk with an occupied byte, then its first such dword
    const uint4 c = h0 ? g.c0 : (h1 ? g.c1 : g.c2);
    const uint32_t cb = h0 ? 0u : (h1 ? 16u : 32u);
    const uint32_t tx = ~c.x, ty = ~c.y, tz = ~c.z, tw = ~c.w;
    *w = tx ? c.x : (ty ? c.y : (tz ? c.z : c.w));
    const uint32_t t = tx ? tx : (ty ? ty : (tz ? tz : tw));
    const uint32_t wb = tx ? 0u : (ty ? 4u : (tz ? 8u : 12u));
    return (h0 || h1 || h2) ? cb + wb + first_byte(t) : 48u;
}

// first occupied cell in [lo, hi] of the lane starting at map offset `lane`,
// or -1; *val receives its byte (the occupant's shown speed).  Finds the
// first occupied byte at or after the window's start and compares it with
// the window's end, which gives the same answer.  `g`, when given, is the
// first group, already loaded from (lane + lo) & ~3.
__device__ __forceinline__ int32_t first_occ_in(const uint8_t *map, uint32_t lane, int32_t lo, int32_t hi,
                                                uint32_t *val, const Group3 *g0) {
    if (lo > hi) return -1;
    const uint32_t s = lane + (uint32_t)lo, e = lane + (uint32_t)hi;
    uint32_t a = s & ~3u, from = s;
    for (bool first = true;; first = false) {
        const Group3 g = (first && g0) ? *g0 : load_group(map, a, e);
        uint32_t w;
        const uint32_t off = group_first(g, a, from, &w);
        if (off < 48u) {
            const uint32_t pos = a + off;
            if (pos > e) return -1;
            if (val) *val = (w >> (8u * (pos & 3u))) & 0xffu;
            return (int32_t)(pos - lane);
        }
        if (e - a < 48u) return -1;
        a += 48u;
        from = a;
    }
}

__device__ __forceinline__ int32_t first_occ(const uint8_t *map, uint32_t lane, int32_t lo, int32_t hi,
                                             uint32_t *val = nullptr) {
    return first_occ_in(map, lane, lo, hi, val, nullptr);
}

// highest occupied cell in [lo, hi], or -1; *val receives its byte.  Groups
// are laid out from the window's first dword as in first_occ and taken from
// the last one down; bytes after the window's end are read as free.
// `g0`, when given, is the group at (lane + lo) & ~3, already loaded.
__device__ __forceinline__ int32_t last_occ_in(const uint8_t *map, uint32_t lane, int32_t lo, int32_t hi,
                                               uint32_t *val, const Group3 *g0) {
    if (lo > hi) return -1;
    const uint32_t s = lane + (uint32_t)lo, e = lane + (uint32_t)hi;
    const uint32_t a0 = s & ~3u;
    for (uint32_t a = a0 + (e - a0) / 48u * 48u;; a -= 48u) {
        const uint32_t span = e - a;  // 0..47 for the last group, more below it
        const Group3 g = (g0 && a == a0) ? *g0 : load_group(map, a, e);
        uint4 c0m = g.c0, c1 = g.c1, c2 = g.c2;
        // bytes after e read as free: e lies in chunk span / 16, dword (span / 4) % 4
        if (span < 48u) {
            const uint32_t je = span >> 2;  // dword of e, 0..11
            const uint32_t keep = FREE_WORD >> (8u * (3u - (span & 3u)));  // bytes up to e
            auto cut = [je, keep](uint32_t w, uint32_t j) {
                return j < je ? w : (j == je ? (w | ~keep) : FREE_WORD);
            };
            c0m = make_uint4(cut(c0m.x, 0), cut(c0m.y, 1), cut(c0m.z, 2), cut(c0m.w, 3));
            c1 = make_uint4(cut(c1.x, 4), cut(c1.y, 5), cut(c1.z, 6), cut(c1.w, 7));
            c2 = make_uint4(cut(c2.x, 8), cut(c2.y, 9), cut(c2.z, 10), cut(c2.w, 11));
        }
        const bool h0 = (c0m.x & c0m.y & c0m.z & c0m.w) != FREE_WORD;
        const bool h1 = (c1.x & c1.y & c1.z & c1.w) != FREE_WORD;
        const bool h2 = (c2.x & c2.y & c2.z & c2.w) != FREE_WORD;
        if (h0 || h1 || h2) {
            const uint4 c = h2 ? c2 : (h1 ? c1 : c0m);
            const uint32_t cb = h2 ? 32u : (h1 ? 16u : 0u);
            const uint32_t tx = ~c.x, ty = ~c.y, tz = ~c.z, tw = ~c.w;
            const uint32_t w = tw ? c.w : (tz ? c.z : (ty ? c.y : c.x));
            const uint32_t t = tw ? tw : (tz ? tz : (ty ? ty : tx));
            const uint32_t wb = tw ? 12u : (tz ? 8u : (ty ? 4u : 0u));
            const uint32_t k = last_byte(t);
            const uint32_t pos = a + cb + wb + k;
            if (pos < s) return -1;
            if (val) *val = (w >> (8u * k)) & 0xffu;
            return (int32_t)(pos - lane);
        }
        if (a == a0) return -1;
    }
}

__device__ __forceinline__ int32_t last_occ(const uint8_t *map, uint32_t lane, int32_t lo, int32_t hi,
                                            uint32_t *val = nullptr) {
    return last_occ_in(map, lane, lo, hi, val, nullptr);
}

__device__ __forceinline__ uint32_t lane_base(const uint4 &E, uint32_t l) {
    return E.x + l * (uint32_t)E_CELLS(E);
}

__device__ __forceinline__ bool entry_free(const Dev &d, const uint4 &E, int32_t e, uint32_t l) {
    if (d.aux[e] & AUX_BLOCKED) return false;
    return first_occ(d.map, lane_base(E, l), 0, d.p.W - 1) < 0;
}

// ---------------------------------------------------------------------------
// car following

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

// key of the random gap terms' hash stream (an arbitrary odd constant)
constexpr uint64_t GAP_TERM_KEY = 0xD6E8FEB86659FD93ull;

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    // SplitMix64 output function (Steele, Lea & Flood 2014)
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

// ---------------------------------------------------------------------------
// statistics

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

__device__ __forceinline__ void counts_flush(const Dev &d, BlockCounts *s, uint32_t row) {
    __syncthreads();
    if (threadIdx.x < NPART) {
        const unsigned int v = s->c[threadIdx.x];
        if (v) d.partial[(uint64_t)row * NPART + threadIdx.x] += v;
    }
}

// an origin lane's waiting set: the bits of ol_bits over its ol_trips
// segment [beg, end) (neighbouring lanes may share a word).  First waiting
// position after position p of the segment, or NO_NEXT.
__device__ __forceinline__ uint32_t next_waiting(const Dev &d, uint32_t p, uint32_t end) {
    const uint32_t q = p + 1;
    if (q >= end) return NO_NEXT;
    const uint32_t w_end = (end + 31) >> 5;
    uint32_t w = q >> 5;
    uint32_t bits = d.ol_bits[w] & (0xffffffffu << (q & 31));
    while (bits == 0u) {
        if (++w >= w_end) return NO_NEXT;
        bits = d.ol_bits[w];
    }
    const uint32_t r = (w << 5) + (uint32_t)__builtin_ctz(bits);
    return r < end ? r : NO_NEXT;
}

// exclusive scan of one value per thread over the block (blockDim.x a
// multiple of 64, at most 1024); wsum: 32 words of LDS
__device__ __forceinline__ uint32_t block_scan(uint32_t v, uint32_t *wsum, uint32_t &total) {
    const uint32_t lane = lane_id(), w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    uint32_t x = v;
    for (int dlt = 1; dlt < 64; dlt <<= 1) {
        const uint32_t t = __shfl_up(x, dlt);
        if (lane >= (uint32_t)dlt) x += t;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    if (threadIdx.x < 16) {
        uint32_t y = threadIdx.x < nw ? wsum[threadIdx.x] : 0u;
        for (int dlt = 1; dlt < 16; dlt <<= 1) {
            const uint32_t t = __shfl_up(y, dlt);
            if (threadIdx.x >= (uint32_t)dlt) y += t;
        }
        wsum[16 + threadIdx.x] = y;
    }
    __syncthreads();
    total = wsum[16 + nw - 1];
    const uint32_t before = w ? wsum[16 + w - 1] : 0u;
    return before + x - v;
}

// Even shares of the move blocks' work lists.  cnt[0..G) are the lengths of
// the G list segments (segment s starts at slot s * chunk, where chunk is the
// move blocks' share); s_pre (LDS, G + 1 words) receives their exclusive
// prefix, and this logical block lb takes the entries [q0, q1) of the
// concatenation.  Balances blocks whose lists are long (intersections)
// against blocks whose lists are empty.
__device__ __forceinline__ void share_lists(const uint32_t *cnt, uint32_t G, uint32_t lb, uint32_t *s_pre,
                                            uint32_t *wsum, uint32_t &q0, uint32_t &q1) {
    const uint32_t per = (G + blockDim.x - 1) / blockDim.x;
    const uint32_t b0 = threadIdx.x * per;
    uint32_t mine = 0;
    if (per <= 4) {
        // up to four counts per thread, loaded in one round trip
        uint32_t c0 = 0, c1 = 0, c2 = 0, c3 = 0;
        if (b0 < G) c0 = cnt[b0];
        if (per > 1 && b0 + 1 < G) c1 = cnt[b0 + 1];
        if (per > 2 && b0 + 2 < G) c2 = cnt[b0 + 2];
        if (per > 3 && b0 + 3 < G) c3 = cnt[b0 + 3];
        ISSUED_TOGETHER4(c0, c1, c2, c3);
        const uint32_t cs[4] = {c0, c1, c2, c3};
#pragma unroll
        for (uint32_t j = 0; j < 4; ++j)
            if (j < per && b0 + j < G) {
                s_pre[b0 + j] = cs[j];
                mine += cs[j];
            }
    } else {
        for (uint32_t j = 0; j < per; ++j)
            if (b0 + j < G) {
                const uint32_t c = cnt[b0 + j];
                s_pre[b0 + j] = c;
                mine += c;
            }
    }
    uint32_t total;
    uint32_t run = block_scan(mine, wsum, total);
    for (uint32_t j = 0; j < per; ++j)
        if (b0 + j < G) {
            const uint32_t c = s_pre[b0 + j];
            s_pre[b0 + j] = run;
            run += c;
        }
    if (threadIdx.x == 0) s_pre[G] = total;
    __syncthreads();
    q0 = (uint32_t)((uint64_t)total * lb / G);
    q1 = (uint32_t)((uint64_t)total * (lb + 1) / G);
}

// segment of entry q (s_pre[0] <= q < s_pre[G]): the largest s with s_pre[s] <= q
__device__ __forceinline__ uint32_t seg_of(const uint32_t *s_pre, uint32_t G, uint32_t q) {
    uint32_t lo = 0, hi = G;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (s_pre[mid] <= q) lo = mid;
        else hi = mid;
    }
    return lo;
}

// share of the slot list per move block (as block_range)
__device__ __forceinline__ uint64_t share_chunk(uint64_t total, uint32_t G) {
    uint64_t chunk = (total + G - 1) / G;
    return (chunk + 63) & ~uint64_t(63);
}

// work-list segment per move block: a block's share of the slots at any
// slot count (at most slot_cap) fits in it
__device__ __forceinline__ uint64_t list_seg(const Dev &d, uint32_t G) { return share_chunk(d.slot_cap, G); }

// lane required to leave toward edge `en`: the node's out-edges split the
// lanes of the incoming edge in proportion to their rank
__device__ __forceinline__ uint32_t required_lane(const Dev &d, int32_t en, int32_t lanes_e) {
    const uint32_t ax = d.aux[en];
    return (uint32_t)(((int32_t)(ax & 0xffu) * lanes_e) / (int32_t)((ax >> 8) & 0xffu));
}

// ---------------------------------------------------------------------------
// move: longitudinal intent from step-k state

// may vehicles pass the signal at the end of their edge at step k?  w is the
// edge's signal word: the cycle position of step k must lie in the green
// part of the phase that serves the edge
__device__ __forceinline__ bool signal_green(uint2 w, int32_t k) {
    const uint32_t cyc = w.x & 0xffffu, off = w.x >> 16;
    const uint32_t t = ((uint32_t)k % cyc + off) % cyc;
    return t >= (w.y & 0xffffu) && t < (w.y >> 16);
}

__device__ __forceinline__ bool has_signal(const Dev &d, int32_t e) {
    return d.sig != nullptr && d.sig[e].x != 0u;
}

// refresh a vehicle's cached edge data from records already loaded: it is on
// an edge with record E in `lane` (`sig`: a signal ends that edge), next edge
// en (-1 on the last edge) with record En and aux word ax_n
__device__ __forceinline__ void set_cache_from(const Slots &S, uint32_t i, const uint4 &E, uint32_t lane, bool sig,
                                               int32_t en, const uint4 &En, uint32_t ax_n) {
    S.lb[i] = lane_base(E, lane);
    S.v0[i] = __uint_as_float(E.z);
    uint32_t cd = (uint32_t)E_CELLS(E) | ((uint32_t)E_LOOK(E) << 16);
    if (sig) cd |= CD_SIGNAL;
    if (en >= 0) {
        if (ax_n & AUX_BLOCKED) cd |= CD_NEXT_BLOCKED;
        const uint32_t nle = (uint32_t)E_LANES(En);
        const uint32_t ln = lane < nle - 1 ? lane : nle - 1;
        S.tlb[i] = lane_base(En, ln);
        S.tgt[i] = En.w + ln;
    } else {
        S.tlb[i] = NO_NEXT;
        S.tgt[i] = 0;
    }
    S.cd[i] = cd;
}

// the lane required to leave toward an edge with aux word ax
__device__ __forceinline__ uint32_t required_lane_of(uint32_t ax, int32_t lanes_e) {
    return (uint32_t)(((int32_t)(ax & 0xffu) * lanes_e) / (int32_t)((ax >> 8) & 0xffu));
}

// refresh a vehicle's cached edge data: it is on edge `e` (record E) in
// `lane`, next edge `en` (-1 on the last edge)
__device__ __forceinline__ void set_cache(const Dev &d, const Slots &S, uint32_t i, int32_t e, const uint4 &E,
                                          uint32_t lane, int32_t en) {
    S.lb[i] = lane_base(E, lane);
    S.v0[i] = __uint_as_float(E.z);
    uint32_t cd = (uint32_t)E_CELLS(E) | ((uint32_t)E_LOOK(E) << 16);
    if (has_signal(d, e)) cd |= CD_SIGNAL;
    if (en >= 0) {
        const uint4 En = d.edge[en];
        if (d.aux[en] & AUX_BLOCKED) cd |= CD_NEXT_BLOCKED;
        const uint32_t nle = (uint32_t)E_LANES(En);
        const uint32_t ln = lane < nle - 1 ? lane : nle - 1;
        S.tlb[i] = lane_base(En, ln);
        S.tgt[i] = En.w + ln;
    } else {
        S.tlb[i] = NO_NEXT;
        S.tgt[i] = 0;
    }
    S.cd[i] = cd;
}

// ---------------------------------------------------------------------------
// departure candidates: due trips request their start lane (reads step k)

// runs in the X leading blocks of the move launch (hb = 0..X-1), beside the
// move: it reads the same step-k map and only adds claims.  One request per
// origin lane with waiting trips, for its lowest trip id: the lane's trips
// share the entry window and the first edge, so no other of them can win.
// Its bytes (list entry 16, head 8, the first edge's flags 4, the entry
// window W, the request flag 1) count into row MAX_BLOCKS + hb.
__device__ __forceinline__ void cand_part(const Dev &d, uint32_t hb, uint32_t X) {
    __shared__ BlockCounts cnt;
    counts_init(&cnt);
    const Ctrl *ctl = d.ctrl;
    const uint32_t cur = ctl->aq_cur;
    // the next step's lane list starts empty (last read by the previous step)
    if (hb == 0 && threadIdx.x == 0) d.aq_n[cur ^ 1u] = 0u;
    const uint32_t nc = d.aq_n[cur];
    const uint4 *aq = d.aq[cur];
    const uint32_t W = (uint32_t)d.p.W;
    uint32_t bytes = 0;
    for (uint32_t q = hb * blockDim.x + threadIdx.x; q < nc; q += X * blockDim.x) {
        const uint4 A = aq[q];
        const unsigned long long head = d.ol_head[A.w];  // a listed lane has a waiting trip
        const uint32_t j = (uint32_t)head;
        const bool ok = head != NO_HEAD && !(d.aux[A.z] & AUX_BLOCKED) && first_occ(d.map, A.y, 0, (int32_t)W - 1) < 0;
        d.dclaim[q] = ok ? 1 : 0;
        if (ok) atomicMin(&d.claims[A.x], j);
        bytes += 16u + 8u + 4u + W + 1u;
    }
    if (bytes) atomicAdd(&cnt.c[P_SCAN], bytes);
    counts_flush(d, &cnt, MAX_BLOCKS + hb);
}

// launch: X leading helper blocks (departure requests), then G work blocks.
// At most 72 VGPRs (7 wavefronts per SIMD, no spills): this kernel is bound
// by memory latency, so resident wavefronts matter more than registers.
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(7, 8))) void k_move(Dev d, uint32_t X) {
    if (blockIdx.x < X) {
        cand_part(d, blockIdx.x, X);
        return;
    }
    const uint32_t G = gridDim.x - X;
    const uint32_t lb = logical_block(blockIdx.x - X, G);
    __shared__ BlockCounts cnt;
    __shared__ uint32_t s_rl, s_lcc;
    if (threadIdx.x == 0) {
        s_rl = 0;
        s_lcc = 0;
    }
    counts_init(&cnt);
    const Ctrl *ctl = d.ctrl;
    const int32_t k = ctl->k;
    const uint32_t n = ctl->n_slots;
    const Slots S = ctl->cur ? d.buf[1] : d.buf[0];
    const Params &p = d.p;
    uint64_t lo64, hi64;
    block_range(n, lb, G, lo64, hi64);
    const uint32_t vlo = (uint32_t)lo64, nv = (uint32_t)(hi64 - lo64);
    const uint64_t lbase = (uint64_t)lb * list_seg(d, G);
    unsigned int alive = 0, scanned = 0;
    for (uint32_t base = 0; base < nv; base += blockDim.x) {
        const uint32_t it = base + threadIdx.x;
        const uint32_t i = vlo + it;
        bool need_resolve = false, lc_cand = false;
        uint4 rl = make_uint4(0, 0, 0, 0);
        if (it < nv) {
            uint32_t m = S.m[i];
            float x = S.x[i], v = S.v[i];
            uint32_t lb = S.lb[i], cd = S.cd[i], tlb = S.tlb[i];
            float v0 = S.v0[i];
            ISSUED_TOGETHER7(m, x, v, lb, cd, tlb, v0);
            if (!(m & M_DEAD)) {
                ++alive;
                const uint32_t lane = m & M_LANE;
                const int32_t C = (int32_t)(cd & 0xffffu), D = (int32_t)((cd >> 16) & 0xffu);
                const int32_t c = (int32_t)x;
                // stop line inside the look-ahead: the next edge's entry matters
                const bool near = tlb != NO_NEXT && c + D >= C;
                const int32_t top = c + D < C - 1 ? c + D : C - 1;
                const bool scan_own = c + 1 <= top;
                Group3 g = {};
                if (scan_own) g = load_group(d.map, (lb + (uint32_t)(c + 1)) & ~3u, lb + (uint32_t)top);
                uint32_t vlb = 0;
                const int32_t cl = first_occ_in(d.map, lb, c + 1, top, &vlb, &g);
                scanned += (uint32_t)((cl >= 0 ? cl : top) - c);
                // the obstacle ahead: the leader (at its cell, with its
                // byte's speed), or a closed stop line (at C, speed 0); the
                // no-overlap clamp caps the position at lim and the speed at
                // vcap.  One car-following evaluation serves both.
                bool follow = cl >= 0;
                float gap = 0.0f, vl = 0.0f, lim = 0.0f, vcap = 0.0f;
                if (follow) {
                    vl = (float)vlb;
                    gap = ((float)cl - x) - p.L;
                    lim = (float)cl - p.L;
                    vcap = vl;
                } else if (near) {
                    // a red signal at the stop line (edge id and signal word
                    // read only here), or the next edge's entry window taken
                    // (its blocked flag is cached)
                    bool stop = false;
                    if (cd & CD_SIGNAL) {
                        stop = !signal_green(d.sig[S.e[i]], k);
                        scanned += 12u;
                    }
                    stop = stop || (cd & CD_NEXT_BLOCKED) || first_occ(d.map, tlb, 0, p.W - 1) >= 0;
                    scanned += (uint32_t)p.W;
                    if (stop) {
                        follow = true;
                        gap = (float)C - x;
                        lim = (float)(C - 1);
                    }
                }
                float x2, v2;
                if (follow) {
                    idm_follow(p, x, v, v0, gap, vl, x2, v2);
                    if (x2 > lim) {
                        x2 = x > lim ? x : lim;
                        v2 = v2 < vcap ? v2 : vcap;
                    }
                } else {
                    free_move(p, x, v, v0, x2, v2);
                }
                uint32_t kind = K_MOVE;
                if (x2 >= (float)C) {
                    if (tlb == NO_NEXT) {
                        kind = K_ARRIVE;
                    } else {
                        // entry request: trip id and claim word are read
                        // only here (8 bytes), request written (8) and the
                        // claim word updated (4)
                        const uint32_t tgt = S.tgt[i], id = S.id[i];
                        kind = K_CLAIM;
                        d.scl[i] = tgt;
                        d.sxo[i] = x;
                        atomicMin(&d.claims[tgt], id);
                        scanned += 20u;
                    }
                }
                const int32_t c2 = kind == K_MOVE ? (int32_t)x2 : c;
                const uint32_t b2 = speed_byte(v2);
                need_resolve = kind != K_MOVE || c2 != c || b2 != speed_byte(v);
                rl = make_uint4(i, lb, (uint32_t)c | ((uint32_t)c2 << 16), b2 | (kind << 8));
                S.x[i] = x2;
                S.v[i] = v2;
                S.m[i] = (m & M_REQ) | lane | (kind << M_KIND_SHIFT) | ((uint32_t)c << M_CELL_SHIFT);
                // may want a lane change: wrong lane for the next edge, the
                // direction allowed at this step, and within x0 of the end
                if (p.lane_change && tlb != NO_NEXT) {
                    const uint32_t req = (m & M_REQ) >> M_REQ_SHIFT;
                    const bool dir_ok = (k & 1) == 0 ? req < lane : req > lane;
                    lc_cand = dir_ok && ((float)C - x2 < p.x0);
                }
            }
        }
        const uint32_t r = wave_append(&s_rl, need_resolve);
        if (need_resolve) d.rl_list[lbase + r] = rl;
        const uint32_t q = wave_append(&s_lcc, lc_cand);
        if (lc_cand) d.lcc_list[lbase + q] = i;
    }
    if (alive) atomicAdd(&cnt.c[P_VSTEPS], alive);
    if (scanned) atomicAdd(&cnt.c[P_SCAN], scanned);
    counts_flush(d, &cnt, lb);
    if (threadIdx.x == 0) {
        d.rl_cnt[lb] = s_rl;
        d.lcc_cnt[lb] = s_lcc;
    }
}

// ---------------------------------------------------------------------------
// depart: the lowest waiting trip of an origin lane that won its claim
// becomes a vehicle and leaves the lane's set; lanes that still hold waiting
// trips go to the next step's list.  Both lists are built with block-wide
// scans, so a block makes one atomic per list per pass.

// runs in the X leading blocks of the resolve launch (hb = 0..X-1); its
// counters go to row MAX_BLOCKS + hb
__device__ __forceinline__ void depart_part(const Dev &d, uint32_t hb, uint32_t X) {
    __shared__ BlockCounts cnt;
    __shared__ uint32_t wsum[32];
    __shared__ uint32_t s_base[2];
    counts_init(&cnt);
    Ctrl *ctl = d.ctrl;
    const int32_t k = ctl->k;
    const uint32_t cur = ctl->aq_cur;
    const uint32_t nc = d.aq_n[cur];
    const uint4 *aq = d.aq[cur];
    uint4 *aq_next = d.aq[cur ^ 1u];
    const uint32_t n = ctl->n_slots;
    const Slots S = ctl->cur ? d.buf[1] : d.buf[0];
    bool any_dep = false;
    for (uint32_t pass0 = hb * blockDim.x; pass0 < nc; pass0 += X * blockDim.x) {
        const uint32_t q = pass0 + threadIdx.x;
        bool dep = false, rq = false;
        uint32_t j = 0;
        uint4 A = make_uint4(0, 0, 0, 0);
        // a winner's edge records and route data, read before the block
        // scans: with the claim word for lanes that made a request, then the
        // second edge's record and aux word for winners
        uint4 E0 = make_uint4(0, 0, 0, 0), dr = make_uint4(0, 0, NO_NEXT, 0), En0 = make_uint4(0, 0, 0, 0);
        uint32_t ax0 = 0, sg0 = 0;
        if (q < nc) {
            A = aq[q];
            const uint32_t o = A.w;
            const unsigned long long head = d.ol_head[o];
            uint32_t wc = d.ol_cnt[o];
            uint32_t claimed = d.dclaim[q];
            uint32_t cw = d.claims[A.x];
            j = (uint32_t)head;
            if (claimed) {
                E0 = d.edge[A.z];
                dr = d.dep_rec[j];
                if (d.sig != nullptr) sg0 = d.sig[A.z].x;
            }
            ISSUED_TOGETHER4(claimed, cw, E0.x, dr.x);
            if (claimed && cw == j) {
                d.claims[A.x] = 0xffffffffu;
                dep = true;
                if (dr.z != NO_NEXT) {
                    En0 = d.edge[dr.z];
                    ax0 = d.aux[dr.z];
                }
                // leave the set: clear the bit (a word may hold bits of a
                // neighbouring lane), find the next waiting trip
                const uint32_t h = (uint32_t)(head >> 32);
                atomicAnd(&d.ol_bits[h >> 5], ~(1u << (h & 31)));
                wc -= 1u;
                d.ol_cnt[o] = wc;
                const uint32_t nh = wc ? next_waiting(d, h, d.ol_rec[o + 1].w) : NO_NEXT;
                d.ol_head[o] = nh != NO_NEXT ? ((unsigned long long)nh << 32) | d.ol_trips[nh] : NO_HEAD;
                rq = nh != NO_NEXT;
            } else {
                rq = head != NO_HEAD;
            }
            // every other trip of a lane that asked lost its request
            if (claimed && wc) atomicAdd(&cnt.c[P_LOST], wc);
        }
        uint32_t tot_dep, tot_rq;
        const uint32_t my_dep = block_scan(dep ? 1u : 0u, wsum, tot_dep);
        __syncthreads();
        const uint32_t my_rq = block_scan(rq ? 1u : 0u, wsum, tot_rq);
        if (threadIdx.x == 0) {
            s_base[0] = tot_dep ? atomicAdd(&ctl->n_new, tot_dep) : 0u;
            s_base[1] = tot_rq ? atomicAdd(&d.aq_n[cur ^ 1u], tot_rq) : 0u;
        }
        __syncthreads();
        if (rq) aq_next[s_base[1] + my_rq] = A;
        if (dep) {
            any_dep = true;
            const uint32_t ns = n + s_base[0] + my_dep;
            const int32_t e0 = (int32_t)A.z;
            const uint32_t l0 = A.x - E0.w;
            const int32_t en0 = dr.z != NO_NEXT ? (int32_t)dr.z : -1;
            const uint32_t req0 = en0 >= 0 ? required_lane_of(ax0, E_LANES(E0)) : 0u;
            d.status[j] = ST_ACTIVE;
            S.x[ns] = 0.0f;
            S.v[ns] = 0.0f;
            S.e[ns] = e0;
            S.en[ns] = en0;
            S.m[ns] = l0 | M_ENTERED | (req0 << M_REQ_SHIFT);
            S.id[ns] = j;
            S.rp[ns] = dr.x;
            S.rend[ns] = dr.y;
            S.ent[ns] = k + 1;
            set_cache_from(S, ns, E0, l0, sg0 != 0u, en0, En0, ax0);
            d.map[A.y] = speed_byte(0.0f);
            add_entry(d, e0, k + 1);
            atomicAdd(&cnt.c[P_DEPARTS], 1u);
        }
        __syncthreads();
    }
    if (any_dep) ctl->dep_ev = 1;
    counts_flush(d, &cnt, MAX_BLOCKS + hb);
}

// ---------------------------------------------------------------------------
// resolve: apply entries, losses, arrivals; commit occupancy; statistics

// launch: X leading helper blocks (departures), then G work blocks
__global__ __launch_bounds__(1024) void k_resolve(Dev d, uint32_t X) {
    if (blockIdx.x < X) {
        depart_part(d, blockIdx.x, X);
        return;
    }
    const uint32_t G = gridDim.x - X;
    const uint32_t lb = logical_block(blockIdx.x - X, G);
    __shared__ BlockCounts cnt;
    __shared__ unsigned int s_arr, s_ev;
    if (threadIdx.x == 0) {
        s_arr = 0;
        s_ev = 0;
    }
    counts_init(&cnt);
    const Ctrl *ctl = d.ctrl;
    const int32_t k = ctl->k;
    const uint32_t n = ctl->n_slots;
    const Slots S = ctl->cur ? d.buf[1] : d.buf[0];
    // an even share of all move blocks' resolve lists
    extern __shared__ uint32_t s_pre[];
    __shared__ uint32_t wsum[32];
    uint32_t q0, q1;
    share_lists(d.rl_cnt, G, lb, s_pre, wsum, q0, q1);
    const uint64_t seg = list_seg(d, G);
    for (uint32_t q = q0 + threadIdx.x; q < q1; q += blockDim.x) {
        const uint32_t sg = seg_of(s_pre, G, q);
        uint4 r = d.rl_list[(uint64_t)sg * seg + (q - s_pre[sg])];
        ISSUED_TOGETHER4(r.x, r.y, r.z, r.w);
        const uint32_t kind = r.w >> 8;
        const int32_t oc = (int32_t)(r.z & 0xffffu), nc = (int32_t)(r.z >> 16);
        uint8_t *lp = d.map + r.y;
        if (kind == K_MOVE) {
            if (nc != oc) lp[oc] = FREE_BYTE;
            lp[nc] = (uint8_t)(r.w & 0xffu);
            continue;
        }
        const uint32_t i = r.x;
        if (kind == K_ARRIVE) {
            const int32_t e = S.e[i], ent = S.ent[i];
            const uint32_t id = S.id[i];
            lp[oc] = FREE_BYTE;
            d.status[id] = ST_DONE;
            d.arrival[id] = k + 1;
            add_exit(d, e, ent, k + 1);
            S.m[i] = M_DEAD;
            atomicAdd(&cnt.c[P_ARRIVED], 1u);
            atomicAdd(&s_arr, 1u);
            s_ev = 1;
            continue;
        }
        // entry request.  Round trip 1: what the slot holds for a winner or
        // a loser; 2: the claim word, the next edge's record and the route's
        // edge after it; 3 (winners): that edge's record and aux word
        uint32_t tgt = d.scl[i], id = S.id[i], rp = S.rp[i], rend = S.rend[i], cdw = S.cd[i];
        int32_t e = S.e[i], en = S.en[i], ent = S.ent[i];
        float xo = d.sxo[i];
        ISSUED_TOGETHER9(tgt, id, rp, rend, cdw, e, en, ent, xo);
        uint32_t cw = d.claims[tgt];
        uint4 En = d.edge[en];
        int32_t en2 = rp + 2 < rend ? (int32_t)d.route[rp + 2] : -1;
        uint32_t sig_n = d.sig != nullptr ? d.sig[en].x : 0u;
        ISSUED_TOGETHER4(cw, En.x, en2, sig_n);
        if (cw == id) {
            uint4 En2 = make_uint4(0, 0, 0, 0);
            uint32_t ax2 = 0;
            if (en2 >= 0) {
                En2 = d.edge[en2];
                ax2 = d.aux[en2];
            }
            d.claims[tgt] = 0xffffffffu;
            lp[oc] = FREE_BYTE;
            const uint32_t ln = tgt - En.w;
            d.map[lane_base(En, ln)] = (uint8_t)(r.w & 0xffu);
            add_exit(d, e, ent, k + 1);
            add_entry(d, en, k + 1);
            const uint32_t req2 = en2 >= 0 ? required_lane_of(ax2, E_LANES(En)) : 0u;
            S.e[i] = en;
            S.en[i] = en2;
            S.x[i] = 0.0f;
            S.rp[i] = rp + 1;
            S.ent[i] = k + 1;
            S.m[i] = ln | M_ENTERED | (req2 << M_REQ_SHIFT);
            set_cache_from(S, i, En, ln, sig_n != 0u, en2, En2, ax2);
            atomicAdd(&cnt.c[P_TRANSFERS], 1u);
            s_ev = 1;
        } else {
            const float lim = (float)((int32_t)(cdw & 0xffffu) - 1);
            const float xn = xo > lim ? xo : lim;
            S.x[i] = xn;
            S.v[i] = 0.0f;
            const int32_t c2 = (int32_t)xn;
            if (c2 != oc) lp[oc] = FREE_BYTE;
            lp[c2] = speed_byte(0.0f);
            atomicAdd(&cnt.c[P_LOST], 1u);
        }
    }
    counts_flush(d, &cnt, lb);
    if (threadIdx.x == 0) {
        d.blk_arr[lb] = s_arr;
        d.blk_ev[lb] = s_ev;
    }
}

// ---------------------------------------------------------------------------
// lane change: decided on the map after the longitudinal move

__global__ __launch_bounds__(1024) void k_lanechg(Dev d) {
    __shared__ BlockCounts cnt;
    __shared__ uint32_t s_lc;
    // one round trip for the control block, this block's candidate count
    // and each thread's first candidate (read ahead of the count; the list
    // has spare entries for it)
    const uint32_t lb = logical_block(blockIdx.x, gridDim.x);
    const uint64_t lo = (uint64_t)lb * list_seg(d, gridDim.x);
    Ctrl *ctl = d.ctrl;
    const uint32_t ncand = d.lcc_cnt[lb];
    const uint32_t i_first = d.lcc_list[lo + threadIdx.x];
    const int32_t k = ctl->k;
    const Slots S = ctl->cur ? d.buf[1] : d.buf[0];
    const Params &p = d.p;
    // a single scenario's draw seed and trip base, read once beside the control block
    const bool one_scen = d.n_scen == 1;
    uint64_t seed0 = 0;
    uint32_t tbase0 = 0;
    if (one_scen) {
        seed0 = d.scen_seed[0];
        tbase0 = d.scen_tbase[0];
    }
    if (threadIdx.x == 0) s_lc = 0;
    counts_init(&cnt);
    for (uint32_t base = 0; base < ncand; base += blockDim.x) {
        const uint32_t it = base + threadIdx.x;
        bool accept = false;
        uint32_t i = 0;
        do {
            if (it >= ncand) break;
            i = base == 0 ? i_first : d.lcc_list[lo + it];
            uint32_t m = S.m[i];
            float x = S.x[i], v = S.v[i];
            uint32_t cd = S.cd[i], lb0 = S.lb[i], id = S.id[i];
            int32_t e = S.e[i];
            ISSUED_TOGETHER7(m, x, v, cd, lb0, id, e);
            if (m & (M_DEAD | M_ENTERED)) break;  // entered its edge this step
            const int32_t C = (int32_t)(cd & 0xffffu);
            const float dist = (float)C - x;
            if (!(dist < p.x0)) break;  // probability 0: no draw can succeed
            const int32_t lane = (int32_t)(m & M_LANE);
            const int32_t req = (int32_t)((m & M_REQ) >> M_REQ_SHIFT);
            if (req == lane) break;
            const int32_t dir = req > lane ? 1 : -1;
            if (((k & 1) == 0 && dir > 0) || ((k & 1) == 1 && dir < 0)) break;
            const float prob = 1.0f - dist / p.x0;
            uint64_t seed = seed0;
            uint32_t tbase = tbase0;
            if (!one_scen) {
                const int32_t sc = d.escen[e];
                seed = d.scen_seed[sc];
                tbase = d.scen_tbase[sc];
            }
            const uint32_t loc = id - tbase;
            const uint64_t h = mix64(seed ^ (((uint64_t)loc << 32) | (uint64_t)(uint32_t)k));
            if (!((float)(h >> 40) < prob * 16777216.0f)) break;
            atomicAdd(&cnt.c[P_LC_TRY], 1u);
            // random gap terms from a second stream of the same key: 24 bits
            // each, uniform on [-eps, eps) in steps of eps * 2^-23
            float ea = 0.0f, eb = 0.0f;
            if (p.eps_a > 0.0f || p.eps_b > 0.0f) {
                const uint64_t h2 = mix64(seed ^ GAP_TERM_KEY ^ (((uint64_t)loc << 32) | (uint64_t)(uint32_t)k));
                ea = p.eps_a * ((float)(uint32_t)(h2 >> 40) * 0x1p-23f - 1.0f);
                eb = p.eps_b * ((float)(uint32_t)((h2 >> 16) & 0xffffffu) * 0x1p-23f - 1.0f);
            }
            const int32_t lt = lane + dir;
            const int32_t c = (int32_t)x;
            const uint32_t lb = lb0 + (uint32_t)(dir * C);  // lane lt of the same edge
            const int32_t D = (int32_t)((cd >> 16) & 0xffu);
            uint32_t vtmp = 0;
            const int32_t top = c + D < C - 1 ? c + D : C - 1;
            const int32_t bot = c - D > 0 ? c - D : 0;
            // the lead window's and the lag window's first groups, read
            // together (one round trip for both scans)
            Group3 g_lead = load_group(d.map, (lb + (uint32_t)c) & ~3u, lb + (uint32_t)top);
            Group3 g_lag = {};
            const bool lag_win = bot <= c - 1;
            if (lag_win) g_lag = load_group(d.map, (lb + (uint32_t)bot) & ~3u, lb + (uint32_t)(c - 1));
            ISSUED_TOGETHER6(g_lead.c0.x, g_lead.c1.x, g_lead.c2.x, g_lag.c0.x, g_lag.c1.x, g_lag.c2.x);
            // one scan from the target cell: occupied target cell -> no
            // change; else the first occupied cell is the lead; then the lag
            const int32_t ca = first_occ_in(d.map, lb, c, top, &vtmp, &g_lead);
            if (ca == c) break;
            if (ca >= 0) {
                const float va = (float)vtmp;
                const float g_lead = ((float)ca - x) - p.L;
                const float t = ((p.al_i * v) - (p.al_a * va)) + ea;
                const float crit = p.g_a + (t > 0.0f ? t : 0.0f);
                if (!(g_lead >= crit)) break;
            }
            const int32_t cb = last_occ_in(d.map, lb, bot, c - 1, &vtmp, &g_lag);  // -1 if bot > c - 1
            if (cb >= 0) {
                const float vb = (float)vtmp;
                const float g_lag = (x - p.L) - (float)(cb + 1);
                const float t = ((p.al_b * vb) - (p.al_i * v)) + eb;
                const float crit = p.g_b + (t > 0.0f ? t : 0.0f);
                if (!(g_lag >= crit)) break;
            }
            S.m[i] = (uint32_t)lt | ((uint32_t)lane << M_OLDLANE_SHIFT) | (m & M_REQ);
            accept = true;
        } while (false);
        const uint32_t q = wave_append(&s_lc, accept);
        if (accept) {
            d.lc_list[lo + q] = i;
            atomicAdd(&cnt.c[P_LC_OK], 1u);
        }
    }
    counts_flush(d, &cnt, lb);
    if (threadIdx.x == 0) d.lc_cnt[lb] = s_lc;
}

// ---------------------------------------------------------------------------
// commit: lane changes into the map

// the trips at departure-order positions [lo, hi) join their origin lanes'
// waiting sets; a lane whose set was empty joins list aq[which] (exactly one
// of the trips joining an empty set sees the empty head).  Runs after the
// step's departures (the lane's bits, count and head are not touched
// concurrently by anything else).  Helper block hb of nb.
__device__ __forceinline__ void enqueue_part(const Dev &d, uint32_t lo, uint32_t hi, uint32_t which, uint32_t hb,
                                             uint32_t nb) {
    for (uint32_t q = lo + hb * blockDim.x + threadIdx.x; q < hi; q += nb * blockDim.x) {
        const uint32_t j = d.dep_order[q];
        const uint2 t = d.trip_ol[j];
        const uint4 R = d.ol_rec[t.x];  // issued beside the head's minimum, used by one trip per lane
        atomicOr(&d.ol_bits[t.y >> 5], 1u << (t.y & 31));
        atomicAdd(&d.ol_cnt[t.x], 1u);
        if (atomicMin(&d.ol_head[t.x], ((unsigned long long)t.y << 32) | j) == NO_HEAD)
            d.aq[which][atomicAdd(&d.aq_n[which], 1u)] = make_uint4(R.x, R.y, R.z, t.x);
    }
}

__global__ __launch_bounds__(1024) void k_enqueue(Dev d, uint32_t lo, uint32_t hi, uint32_t which) {
    enqueue_part(d, lo, hi, which, blockIdx.x, gridDim.x);
}

void launch_enqueue(const Dev &d, uint32_t lo, uint32_t hi, uint32_t which, hipStream_t s) {
    if (hi <= lo) return;
    const uint32_t n = hi - lo, g = (n + 255) / 256 < 1024 ? (n + 255) / 256 : 1024;
    hipLaunchKernelGGL(k_enqueue, dim3(g), dim3(256), 0, s, d, lo, hi, which);
}

// end of step (first helper block of the commit launch): sums the per-block
// arrival and event flags of the resolve phase over the G work blocks and
// writes the next step's control block
__device__ __forceinline__ void end_part(const Dev &d, uint32_t G) {
    __shared__ uint32_t s_arr, s_ev;
    // the control block and the per-block flags in one round trip
    Ctrl c{};
    if (threadIdx.x == 0) c = *d.ctrl;
    uint32_t arr = 0, ev = 0;
    for (uint32_t b = threadIdx.x; b < G; b += blockDim.x) {
        arr += d.blk_arr[b];
        ev |= d.blk_ev[b];
    }
    if (threadIdx.x == 0) {
        s_arr = 0;
        s_ev = 0;
    }
    __syncthreads();
    if (arr) atomicAdd(&s_arr, arr);
    if (ev) s_ev = 1;
    __syncthreads();
    if (threadIdx.x == 0) {
        Ctrl nx = c;
        const bool any = s_ev != 0 || c.dep_ev != 0;
        nx.watchdog = (c.n_alive > 0 && !any) ? c.watchdog + 1 : 0;
        nx.dep_ev = 0;
        nx.n_alive = c.n_alive + (int64_t)c.n_new - (int64_t)s_arr;
        nx.n_slots = c.n_slots + c.n_new;
        nx.n_new = 0;
        // the trips due at the next step join the waiting sets in this launch
        const uint32_t due_next = dep_hi_of(d, c.k + 1);
        nx.dep_done = due_next;
        nx.aq_cur = c.aq_cur ^ 1u;
        nx.n_wq = c.n_wq - c.n_new + (due_next - c.dep_done);
        nx.k = c.k + 1;
        *d.ctrl_next = nx;
    }
}

// launch: X leading helper blocks (the first ends the step), then G_lc work
// blocks that write the accepted lane changes into the map (G_lc = 0 when
// lane changes are off); G = work blocks of the step's other kernels
__global__ __launch_bounds__(1024) void k_commit(Dev d, uint32_t X, uint32_t G) {
    if (blockIdx.x < X) {
        if (blockIdx.x == 0) {
            end_part(d, G);
        } else {
            const Ctrl *ctl = d.ctrl;
            enqueue_part(d, ctl->dep_done, dep_hi_of(d, ctl->k + 1), ctl->aq_cur ^ 1u, blockIdx.x - 1, X - 1);
        }
        return;
    }
    const Ctrl *ctl = d.ctrl;
    const uint32_t lb = logical_block(blockIdx.x - X, G);
    const uint64_t lo = (uint64_t)lb * list_seg(d, G);
    // the count and each thread's first entry in one round trip with the
    // control block (the list has spare entries for the read ahead)
    const uint32_t nlc = d.lc_cnt[lb];
    const uint32_t i_first = d.lc_list[lo + threadIdx.x];
    const Slots S = ctl->cur ? d.buf[1] : d.buf[0];
    for (uint32_t q = threadIdx.x; q < nlc; q += blockDim.x) {
        const uint32_t i = q == threadIdx.x ? i_first : d.lc_list[lo + q];
        uint32_t m = S.m[i], cd = S.cd[i], lb_old = S.lb[i];
        float x = S.x[i], v = S.v[i];
        int32_t en = S.en[i];
        ISSUED_TOGETHER6(m, cd, lb_old, x, v, en);
        const uint32_t lt = m & M_LANE, lold = (m >> M_OLDLANE_SHIFT) & M_LANE;
        const uint32_t C = cd & 0xffffu;
        const uint32_t lb_new = lb_old + (lt - lold) * C;  // unsigned wrap handles lt < lold
        const uint32_t c = (uint32_t)(int32_t)x;
        d.map[lb_old + c] = FREE_BYTE;
        d.map[lb_new + c] = speed_byte(v);
        S.m[i] = lt | (m & M_REQ);
        S.lb[i] = lb_new;
        if (en >= 0) {  // entry lane on the next edge follows the lane index
            const uint4 En = d.edge[en];
            const uint32_t nle = (uint32_t)E_LANES(En);
            const uint32_t ln = lt < nle - 1 ? lt : nle - 1;
            S.tlb[i] = lane_base(En, ln);
            S.tgt[i] = En.w + ln;
        }
    }
}

// ---------------------------------------------------------------------------
// reorder: counting sort of the live slots by edge into the other buffer

__global__ __launch_bounds__(1024) void k_sort_count(Dev d) {
    const Ctrl *ctl = d.ctrl;
    const uint32_t n = ctl->n_slots;
    const Slots S = ctl->cur ? d.buf[1] : d.buf[0];
    uint64_t lo, hi;
    block_range(n, logical_block(blockIdx.x, gridDim.x), gridDim.x, lo, hi);
    const uint32_t lane = lane_id();
    for (uint64_t base = lo; base < hi; base += blockDim.x) {
        const uint64_t it = base + threadIdx.x;
        const uint32_t i = (uint32_t)it;
        int32_t e = -1;
        if (it < hi && !(S.m[i] & M_DEAD)) e = S.e[i];
        // slots are mostly sorted by edge already: one atomic per run of
        // equal edges inside the wavefront, not one per vehicle
        const int32_t prev = __shfl_up(e, 1);
        const bool head = lane == 0 || prev != e;
        const uint64_t heads = __ballot(head);
        const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
        const uint32_t hl = 63u - (uint32_t)__builtin_clzll(heads & upto);
        const uint64_t after = heads & ~upto;
        const uint32_t end = after ? (uint32_t)__builtin_ctzll(after) : 64u;
        uint32_t b0 = 0;
        if (lane == hl && e >= 0) b0 = atomicAdd(&d.ecnt[e], end - hl);
        b0 = __shfl(b0, (int)hl);
        if (e >= 0) d.srank[i] = b0 + (lane - hl);
    }
}

// per 4096-edge chunk: exclusive offsets inside the chunk, chunk total; clears counts
__global__ __launch_bounds__(1024) void k_sort_scan1(Dev d) {
    __shared__ uint32_t wsum[32];
    const uint32_t e0 = blockIdx.x * SORT_CHUNK + threadIdx.x * 4;
    uint32_t c[4];
    for (int j = 0; j < 4; ++j) c[j] = (e0 + j < (uint32_t)d.n_edges) ? d.ecnt[e0 + j] : 0u;
    const uint32_t mine = c[0] + c[1] + c[2] + c[3];
    uint32_t total;
    uint32_t run = block_scan(mine, wsum, total);
    for (int j = 0; j < 4; ++j) {
        if (e0 + j < (uint32_t)d.n_edges) {
            d.eoff[e0 + j] = run;
            d.ecnt[e0 + j] = 0;
        }
        run += c[j];
    }
    if (threadIdx.x == 0) d.csum[blockIdx.x] = total;
}

// exclusive scan of the chunk totals (one block); total live count -> ctrl
__global__ __launch_bounds__(1024) void k_sort_scan2(Dev d, uint32_t n_chunks) {
    __shared__ uint32_t wsum[32];
    const uint32_t per = (n_chunks + 1023) / 1024;
    const uint32_t b0 = threadIdx.x * per;
    uint32_t mine = 0;
    for (uint32_t j = 0; j < per; ++j)
        if (b0 + j < n_chunks) mine += d.csum[b0 + j];
    uint32_t total;
    uint32_t run = block_scan(mine, wsum, total);
    for (uint32_t j = 0; j < per; ++j) {
        if (b0 + j < n_chunks) {
            const uint32_t cj = d.csum[b0 + j];
            d.csum[b0 + j] = run;
            run += cj;
        }
    }
    if (threadIdx.x == 0) d.ctrl->n_comp = total;
}

__global__ __launch_bounds__(1024) void k_sort_scatter(Dev d) {
    Ctrl *ctl = d.ctrl;
    const uint32_t n = ctl->n_slots;
    const uint32_t cur = ctl->cur;
    const Slots A = cur ? d.buf[1] : d.buf[0];
    const Slots B = cur ? d.buf[0] : d.buf[1];
    uint64_t lo, hi;
    block_range(n, logical_block(blockIdx.x, gridDim.x), gridDim.x, lo, hi);
    for (uint64_t it = lo + threadIdx.x; it < hi; it += blockDim.x) {
        const uint32_t i = (uint32_t)it;
        const uint32_t m = A.m[i];
        if (m & M_DEAD) continue;
        const int32_t e = A.e[i];
        const uint32_t o = d.csum[(uint32_t)e / SORT_CHUNK] + d.eoff[e] + d.srank[i];
        B.x[o] = A.x[i];
        B.v[o] = A.v[i];
        B.e[o] = e;
        B.en[o] = A.en[i];
        B.m[o] = m;
        B.id[o] = A.id[i];
        B.rp[o] = A.rp[i];
        B.rend[o] = A.rend[i];
        B.ent[o] = A.ent[i];
        B.lb[o] = A.lb[i];
        B.cd[o] = A.cd[i];
        B.v0[o] = A.v0[i];
        B.tlb[o] = A.tlb[i];
        B.tgt[o] = A.tgt[i];
    }
}

__global__ void k_sort_finish(Dev d) {
    if (threadIdx.x == 0) {
        Ctrl *c = d.ctrl;
        c->n_slots = c->n_comp;
        c->n_comp = 0;
        c->cur ^= 1u;
    }
}

// the cached blocked flag of every live vehicle whose next edge is `edge`
__global__ __launch_bounds__(1024) void k_set_next_blocked(Dev d, int32_t edge, uint32_t on) {
    const Ctrl *ctl = d.ctrl;
    const uint32_t n = ctl->n_slots;
    const Slots S = ctl->cur ? d.buf[1] : d.buf[0];
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        if ((S.m[i] & M_DEAD) || S.en[i] != edge) continue;
        const uint32_t cd = S.cd[i];
        S.cd[i] = on ? (cd | CD_NEXT_BLOCKED) : (cd & ~CD_NEXT_BLOCKED);
    }
}

void launch_set_next_blocked(const Dev &d, int32_t edge, bool on, hipStream_t s) {
    hipLaunchKernelGGL(k_set_next_blocked, dim3(1024), dim3(256), 0, s, d, edge, on ? 1u : 0u);
}

// both cached edge flags of every live vehicle, recomputed from the edge
// state (after a signal plan change or a restored snapshot)
__global__ __launch_bounds__(1024) void k_refresh_flags(Dev d) {
    const Ctrl *ctl = d.ctrl;
    const uint32_t n = ctl->n_slots;
    const Slots S = ctl->cur ? d.buf[1] : d.buf[0];
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        if (S.m[i] & M_DEAD) continue;
        const int32_t en = S.en[i];
        uint32_t cd = S.cd[i] & ~(CD_SIGNAL | CD_NEXT_BLOCKED);
        if (has_signal(d, S.e[i])) cd |= CD_SIGNAL;
        if (en >= 0 && (d.aux[en] & AUX_BLOCKED)) cd |= CD_NEXT_BLOCKED;
        S.cd[i] = cd;
    }
}

void launch_refresh_flags(const Dev &d, hipStream_t s) {
    hipLaunchKernelGGL(k_refresh_flags, dim3(1024), dim3(256), 0, s, d);
}

// ---------------------------------------------------------------------------

// launch on stream s; with timing events given, they take the dispatch's own
// start and end timestamps (the kernel's execution interval)
#define LPSIM_LAUNCH_SHM(kern, grid, block, shm, s, ev, ...)                                          \
    do {                                                                                              \
        if ((ev).start)                                                                               \
            hipExtLaunchKernelGGL(kern, grid, block, shm, s, (ev).start, (ev).stop, 0, __VA_ARGS__); \
        else                                                                                          \
            hipLaunchKernelGGL(kern, grid, block, shm, s, __VA_ARGS__);                               \
    } while (0)
#define LPSIM_LAUNCH(kern, grid, block, s, ev, ...) LPSIM_LAUNCH_SHM(kern, grid, block, 0, s, ev, __VA_ARGS__)

void launch_move(const Dev &d, int blocks, int threads, hipStream_t s, KernelEvents ev) {
    const uint32_t X = helper_blocks(threads);
    LPSIM_LAUNCH(k_move, dim3(X + (uint32_t)blocks), dim3(threads), s, ev, d, X);
}
void launch_resolve(const Dev &d, int blocks, int threads, hipStream_t s, KernelEvents ev) {
    const uint32_t X = helper_blocks(threads);
    // dynamic LDS: prefix of the G list lengths
    LPSIM_LAUNCH_SHM(k_resolve, dim3(X + (uint32_t)blocks), dim3(threads), ((size_t)blocks + 1) * 4, s, ev, d, X);
}
void launch_lanechg(const Dev &d, int blocks, int threads, hipStream_t s, KernelEvents ev) {
    LPSIM_LAUNCH(k_lanechg, dim3(blocks), dim3(threads), s, ev, d);
}
void launch_commit(const Dev &d, int blocks, int threads, hipStream_t s, KernelEvents ev) {
    const uint32_t g_lc = d.p.lane_change ? (uint32_t)blocks : 0u;
    LPSIM_LAUNCH(k_commit, dim3(END_HELPERS + g_lc), dim3(threads), s, ev, d, END_HELPERS, (uint32_t)blocks);
}
void launch_reorder(const Dev &d, int blocks, int threads, hipStream_t s) {
    const uint32_t n_chunks = ((uint32_t)d.n_edges + SORT_CHUNK - 1) / SORT_CHUNK;
    hipLaunchKernelGGL(k_sort_count, dim3(blocks), dim3(threads), 0, s, d);
    hipLaunchKernelGGL(k_sort_scan1, dim3(n_chunks), dim3(1024), 0, s, d);
    hipLaunchKernelGGL(k_sort_scan2, dim3(1), dim3(1024), 0, s, d, n_chunks);
    hipLaunchKernelGGL(k_sort_scatter, dim3(blocks), dim3(threads), 0, s, d);
    hipLaunchKernelGGL(k_sort_finish, dim3(1), dim3(64), 0, s, d);
}

}  // namespace lpsim
