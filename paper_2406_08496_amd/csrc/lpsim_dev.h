// lpsim_dev.h -- device data layout shared by the kernels and the host side
// of the GPU library (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lpsim {

constexpr uint8_t FREE_BYTE = 255;  // lane-map byte of an empty cell

// trip status
constexpr uint8_t ST_WAIT = 0, ST_ACTIVE = 1, ST_DONE = 2;

// slot meta word: lane | flags | step kind | old lane | old cell
constexpr uint32_t M_LANE = 7u;             // bits 0-2
constexpr uint32_t M_DEAD = 1u << 3;        // slot no longer holds a vehicle
constexpr uint32_t M_ENTERED = 1u << 4;     // entered its edge in this step
constexpr uint32_t M_KIND_SHIFT = 6;        // bits 6-7: K_MOVE / K_ARRIVE / K_CLAIM
constexpr uint32_t M_OLDLANE_SHIFT = 8;     // bits 8-10 (accepted lane change)
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

struct Params {
    float dt, a, b, s0, T, L, x0, g_a, g_b, al_i, al_a, al_b;
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
    uint32_t n_lc;         // accepted lane changes this step
    uint32_t n_comp;       // compaction output count
    uint32_t wait_lo;      // first departure-order position that may still wait
    uint32_t wait_lo_next;
    uint32_t arr_step;     // arrivals this step
    uint32_t events;       // any entry or exit this step
    uint32_t done_commit;  // last-block counters
    uint32_t done_compact;
};

struct Slots {
    float *x, *v;
    int32_t *e;     // internal edge id
    uint32_t *m;    // meta word
    uint32_t *id;   // trip id (global)
    uint32_t *rp;   // absolute route index of the current edge
    uint32_t *rend; // absolute route end (exclusive)
    int32_t *ent;   // step the current edge was entered
};

struct Dev {
    Params p;
    Ctrl *ctrl;
    Slots buf[2];
    uint32_t *scl;  // claim word of a crossing vehicle (this step)
    float *sxo;     // its position before the move
    uint32_t *lc_list;
    const uint4 *edge;
    uint32_t *aux;
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
    uint8_t *dclaim;
    int32_t *n_exits;
    unsigned long long *tt_sum;
    int32_t *inflow_bin, *exits_bin;
    unsigned long long *tt_bin, *occ_bin;
    unsigned long long *partial;  // [MAX_BLOCKS][NPART]
};

void launch_move(const Dev &d, int blocks, int threads, hipStream_t s);
void launch_resolve(const Dev &d, int blocks, int threads, hipStream_t s);
void launch_lanechg(const Dev &d, int blocks, int threads, hipStream_t s);
void launch_commit(const Dev &d, int blocks, int threads, hipStream_t s);
void launch_compact(const Dev &d, int blocks, int threads, hipStream_t s);

}  // namespace lpsim
