// lpsim_dev.h -- device data layout shared by the kernels and the host side
// of the GPU library (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lpsim {

constexpr uint8_t FREE_BYTE = 255;  // lane-map byte of an empty cell

// trip status
constexpr uint8_t ST_WAIT = 0, ST_ACTIVE = 1, ST_DONE = 2;

// slot meta word: lane | flags | step kind | old lane | required lane | old cell
constexpr uint32_t M_LANE = 7u;             // bits 0-2
constexpr uint32_t M_DEAD = 1u << 3;        // slot no longer holds a vehicle
constexpr uint32_t M_ENTERED = 1u << 4;     // entered its edge in this step
constexpr uint32_t M_KIND_SHIFT = 6;        // bits 6-7: K_MOVE / K_ARRIVE / K_CLAIM
constexpr uint32_t M_OLDLANE_SHIFT = 8;     // bits 8-10 (accepted lane change)
constexpr uint32_t M_REQ_SHIFT = 11;        // bits 11-13: lane required for the next edge
constexpr uint32_t M_REQ = 7u << M_REQ_SHIFT;
constexpr uint32_t M_CELL_SHIFT = 16;       // bits 16-31: cell at step start
constexpr uint32_t K_MOVE = 0, K_ARRIVE = 1, K_CLAIM = 2;

// edge record: x = lane-map byte offset, y = cells | lanes<<16 | lookahead<<24,
// z = speed limit (float bits), w = first entry-claim word of the edge
#define E_CELLS(E) ((int32_t)((E).y & 0xffffu))
#define E_LANES(E) ((int32_t)(((E).y >> 16) & 0xffu))
#define E_LOOK(E) ((int32_t)((E).y >> 24))

// aux word: rank among the source node's out-edges | out-degree<<8 | blocked
constexpr uint32_t AUX_BLOCKED = 1u << 16;

// per-block counter rows
constexpr int P_VSTEPS = 0, P_TRANSFERS = 1, P_DEPARTS = 2, P_LOST = 3, P_LC_TRY = 4,
              P_LC_OK = 5, P_ARRIVED = 6, P_SCAN = 7, NPART = 8;
constexpr int MAX_BLOCKS = 8192;
// work-list entries beyond slot_cap: segments are rounded up to 64 entries per
// block, and a block may read one entry per thread of its segment ahead of
// knowing its count
constexpr uint32_t LIST_SPARE = 64u * MAX_BLOCKS + 1024u;

struct Params {
    float dt, a, b, s0, T, L, x0, g_a, g_b, al_i, al_a, al_b;
    float eps_a, eps_b;  // half-widths of the random gap terms (0: none)
    float tsab;     // 2 sqrt(a b), rounded once from fp64
    float half_dt;  // 0.5 dt
    int32_t W;      // entry window in cells
    int32_t bin_steps, n_bins, free_mode, lane_change;
};

// step control block, device resident so captured graphs replay on their own
struct Ctrl {
    int64_t n_alive;       // vehicles on the road
    int64_t watchdog;      // steps in a row with vehicles but no entry/exit
    int32_t k;             // current step
    uint32_t cur;          // which slot buffer is live
    uint32_t n_slots;      // slots in use in the live buffer (some may be dead)
    uint32_t n_new;        // departures appended this step (above n_slots)
    uint32_t n_comp;       // live slots counted by the reorder
    uint32_t aq_cur;       // which list of origin lanes with waiting trips is live
    uint32_t n_wq;         // due trips still waiting
    uint32_t dep_ev;       // a trip departed this step
    uint32_t dep_done;     // departure-order positions already queued (due by now)
};

struct Slots {
    float *x, *v;
    int32_t *e;     // internal edge id
    int32_t *en;    // next edge on the route (internal id), -1 on the last edge
    uint32_t *m;    // meta word
    uint32_t *id;   // trip id (global)
    uint32_t *rp;   // absolute route index of the current edge
    uint32_t *rend; // absolute route end (exclusive)
    int32_t *ent;   // step the current edge was entered
    // per-vehicle copies of what the move phase needs, refreshed when the
    // vehicle enters an edge or changes lane (saves dependent loads)
    uint32_t *lb;   // lane-map offset of the vehicle's lane
    uint32_t *cd;   // cells | look-ahead << 16 of the current edge | CD_NEXT_BLOCKED
    float *v0;      // speed limit of the current edge
    uint32_t *tlb;  // lane-map offset of the entry lane on the next edge (NO_NEXT on the last edge)
    uint32_t *tgt;  // claim word of that entry lane
};

constexpr uint32_t NO_NEXT = 0xffffffffu;
constexpr unsigned long long NO_HEAD = ~0ull;
constexpr uint32_t CD_NEXT_BLOCKED = 1u << 31;  // the next edge accepts no entries
constexpr uint32_t CD_SIGNAL = 1u << 30;        // the current edge ends at a signal serving it

struct Dev {
    Params p;
    // Control of step k lives in buffer k & 1: the kernels of the step read
    // `ctrl`, and the end of the step (in the commit launch) writes the next
    // step's control into `ctrl_next`, so no kernel reads a control block
    // while it is being rewritten.  The host launches each step with the
    // pair for its parity.
    Ctrl *ctrl;
    Ctrl *ctrl_next;
    Slots buf[2];
    uint32_t *scl;  // claim word of a crossing vehicle (this step)
    float *sxo;     // its position before the move
    // per-step work lists, one segment per move block: move block b owns
    // entries [b * seg, b * seg + count[b]), where seg = list_seg(slot_cap,
    // G) covers any block's share of the slots (so no global counter is
    // contended, and a list's position does not depend on the step's slot
    // count).  Lists hold slot_cap + LIST_SPARE entries.  The resolve kernel deals
    // the concatenated resolve entries out evenly (share_lists); the lane
    // change and its commit keep the move block's segment.
    uint4 *rl_list;     // vehicles with an entry request, an arrival or a changed map
                        // byte: {slot, lane-map offset of its lane, old | new cell << 16,
                        // new speed byte | step kind << 8}
    uint32_t *lcc_list; // slots that may change lane
    uint32_t *lc_list;  // accepted lane changes
    uint32_t *rl_cnt, *lcc_cnt, *lc_cnt;  // [MAX_BLOCKS]
    uint32_t slot_cap;    // slots per buffer (vehicles that can be on the road)
    uint32_t *blk_arr;  // [MAX_BLOCKS] arrivals of the block this step
    uint32_t *blk_ev;   // [MAX_BLOCKS] any entry or exit in the block this step
    const uint4 *edge;
    uint32_t *aux;
    // fixed-time signal of each approach edge (null: no signals):
    // x = cycle | offset << 16, y = green start | green end << 16, in steps of
    // the cycle; x = 0 for an edge no signal stops
    const uint2 *sig;
    int32_t n_scen;       // scenarios in this context (1 unless batched)
    const int32_t *escen;
    const uint64_t *scen_seed;
    const uint32_t *scen_tbase;
    uint8_t *map;
    uint32_t *claims;
    const uint32_t *route;
    const uint32_t *route_off;  // per trip, absolute (n_trips + 1)
    const uint32_t *dep_order;  // trips by (departure, id)
    const uint32_t *dep_hi;     // trips with departure <= k, for k < n_dep_hi
    int32_t n_dep_hi;
    uint32_t n_trips;
    uint8_t *status;
    int32_t *arrival;
    // Due trips that have not entered yet, one set per origin lane (a lane
    // some trip starts on).  Only the lowest trip id of a lane can win its
    // entry (all of the lane's trips see the same entry window), so each
    // step makes one request per origin lane with waiting trips.
    //   ol_rec[o]   {claim word, lane-map offset, first edge, start of the
    //               lane's segment in ol_trips} (n_ol + 1 records; the last
    //               holds only the end of the final segment)
    //   ol_trips    each lane's trips in increasing id, lane after lane
    //   ol_bits     one bit per ol_trips entry: due and not yet entered
    //   ol_head[o]  the lane's lowest waiting trip: its position in ol_trips
    //               << 32 | its trip id (NO_HEAD when none waits; the two
    //               orders agree within a lane, so one 64-bit minimum
    //               keeps both)
    //   ol_cnt[o]   waiting trips of the lane
    //   trip_ol[j]  {origin lane, position in ol_trips}
    //   aq[2]       origin lanes with waiting trips, as {claim word, lane-map
    //               offset, first edge, origin lane}: this step's list and
    //               the next step's, counts in aq_n[2] (the move launch
    //               clears the next one's count)
    const uint4 *ol_rec;
    const uint32_t *ol_trips;
    uint32_t *ol_bits;
    unsigned long long *ol_head;
    uint32_t *ol_cnt;
    const uint2 *trip_ol;
    uint4 *aq[2];
    uint32_t *aq_n;
    uint32_t n_ol;
    uint8_t *dclaim;      // [position in this step's lane list] the lane's request was made
    const uint4 *dep_rec; // per trip: route index of the first edge, route end,
                          // second edge (NO_NEXT if none), 0
    // per-edge counting sort of the slots (locality), every few steps
    int32_t n_edges;
    uint32_t *ecnt;       // [n_edges] vehicles per edge, zero between sorts
    uint32_t *eoff;       // [n_edges] offset inside the edge's 4096-edge chunk
    uint32_t *csum;       // [chunks] chunk offsets
    uint32_t *srank;      // [slot] rank inside its edge
    int32_t *n_exits;
    unsigned long long *tt_sum;
    int32_t *inflow_bin, *exits_bin;
    unsigned long long *tt_bin, *occ_bin;
    unsigned long long *partial;  // [PART_ROWS][NPART]
};

// optional timing events of one kernel launch (both null: untimed)
struct KernelEvents {
    hipEvent_t start = nullptr, stop = nullptr;
};

// The move and resolve launches carry the departure work in helper blocks
// placed before their `blocks` work blocks: enough threads for one pass over
// DEP_THREADS candidates, a multiple of 8 blocks (so the work blocks keep
// their XCD placement), at most MAX_HELPERS.
constexpr uint32_t DEP_THREADS = 65536;
constexpr uint32_t MAX_HELPERS = 2048;
inline uint32_t helper_blocks(int threads) {
    uint32_t x = (DEP_THREADS + (uint32_t)threads - 1) / (uint32_t)threads;
    x = (x + 7u) & ~7u;
    return x < MAX_HELPERS ? x : MAX_HELPERS;
}
// rows of per-block counters: work blocks, then helper blocks
constexpr int PART_ROWS = MAX_BLOCKS + (int)MAX_HELPERS;

// refresh the cached blocked flag of vehicles heading for (internal) `edge`
void launch_set_next_blocked(const Dev &d, int32_t edge, bool on, hipStream_t s);
// recompute the cached signal and blocked flags of every live vehicle
void launch_refresh_flags(const Dev &d, hipStream_t s);
// queue the trips at departure-order positions [lo, hi) into their origin
// lanes; lanes that had no waiting trip join list aq[which]
void launch_enqueue(const Dev &d, uint32_t lo, uint32_t hi, uint32_t which, hipStream_t s);
// move (with departure requests in helper blocks)
void launch_move(const Dev &d, int blocks, int threads, hipStream_t s, KernelEvents ev = {});
// resolve (with departures in helper blocks)
void launch_resolve(const Dev &d, int blocks, int threads, hipStream_t s, KernelEvents ev = {});
void launch_lanechg(const Dev &d, int blocks, int threads, hipStream_t s, KernelEvents ev = {});
// lane-change commit (if lane changes are on) and the end of the step, in
// END_HELPERS leading blocks (the first ends the step, the others queue the
// trips that fall due at the next step; 8 keeps the work blocks' XCD
// placement)
constexpr uint32_t END_HELPERS = 8;
void launch_commit(const Dev &d, int blocks, int threads, hipStream_t s, KernelEvents ev = {});
void launch_reorder(const Dev &d, int blocks, int threads, hipStream_t s);
// binned statistics in input edge order into device arrays (any may be
// NULL), the occupancy completed for the vehicles still on an edge; `ct` is
// the current control block, `ext` maps internal to input edge ids
hipError_t launch_stats_device(const Dev &d, const Ctrl *ct, const int32_t *ext, int32_t E, int32_t B,
                               int32_t bin_steps, uint32_t slot_cap, int32_t *inflow, int32_t *exits,
                               unsigned long long *tt, unsigned long long *occ, hipStream_t s);
constexpr int SORT_CHUNK = 4096;  // edges per scan block

}  // namespace lpsim
