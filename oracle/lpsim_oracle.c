/*
 * lpsim_oracle.c -- plain, slow, deliberately obvious CPU reference of the
 * LPSim per-timestep vehicle update (Jiang, Sengupta, Demmel, Williams,
 * "Large Scale Multi-GPU Based Parallel Traffic Simulation for Accelerated
 * Traffic Assignment and Propagation").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker that the GPU library is
 * compared against.  It shares no code, header, table or constant generator
 * with the GPU path, and only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load it.
 *
 * What it computes, and where each piece comes from:
 *   - Lane map (Section 3.1, "Lane Map"): one byte per metre of lane, lanes of
 *     an edge stored one after another; 255 = free, 0..254 = occupied, value =
 *     the occupant's speed in m/s (truncated toward zero).
 *   - Synchronous update (Section 3.1, the vehicle-dynamics equation): the new
 *     state of every vehicle is a function of step-k state only.  Here that
 *     is taken literally: every longitudinal decision reads the map of step k;
 *     the one documented exception is the lane change, which reads the map
 *     after the longitudinal move (the paper leaves the order inside a step
 *     open; Algorithm 1 evaluates lane change after car following).
 *   - Car following (Section 3.1, Car Following equation; IDM with the
 *     notation-table parameters a, v0, delta=4, s0, T, b).  Leader found by a
 *     forward scan of the lane map (Algorithm 1, front-car check); without a
 *     leader the speed jumps to the edge's free speed (Algorithm 1, else
 *     branch), or, as a variant, follows IDM free-road acceleration.
 *   - Intersections (Section 3.1 Remarks; Algorithm 1 intersection branch;
 *     Section 3.3 first-byte rule): a vehicle may move onto its next edge only
 *     if the entry cells of the target lane are free; otherwise it waits
 *     behind the stop line.  Exclusive entry (Remarks, atomic switch) is
 *     resolved deterministically: the lowest trip id among all claimants of a
 *     target lane wins, departures and transfers pooled.
 *   - Signal control (Algorithm 1 intersection branch; Section 3.3 keeps
 *     signal states with the rest of a partition's local data).  The paper
 *     gives no signal model, so this reading is a fixed-time plan per node:
 *     n_phases phases, each `green` steps followed by `allred` steps, the
 *     cycle shifted by `offset` steps; every approach edge of the node serves
 *     in one phase (or in none: never stopped).  At step k the approach may
 *     hand vehicles to the next edge only inside the green part of its phase;
 *     otherwise the stop line is a standing obstacle, as for a full entry
 *     window.  Departures (which enter at the upstream end of their first
 *     edge) and arrivals (which leave at the end of the last edge) do not
 *     pass a signal.
 *   - Departure (Algorithm 1, first test): a trip whose departure time has
 *     come enters its first edge when that edge's entry cells are free.
 *   - Mandatory lane change and gap acceptance (Section 3.1, Lane Change and
 *     Gap Acceptance equations): the probability ramps up linearly inside x0
 *     of the edge end; critical lead/lag gaps are linear in the anticipation
 *     times alpha.  The equations' random components eps_a, eps_b (notation
 *     table) have no stated distribution; here each is uniform on
 *     [-eps, eps), drawn per attempt from a second counter-based stream, and
 *     enters the speed term of the critical gap before its clamp at zero, so
 *     a critical gap never falls below g_a (g_b).  eps = 0 (the default)
 *     leaves the terms out.
 *   - Edge entry time t_start (Algorithm 1, new-edge bookkeeping) gives the
 *     per-edge travel times; travel-time estimation is the simulator's stated
 *     purpose (abstract).
 *
 * All floating point is binary32, one rounding per operation, no contraction
 * (compile with -ffp-contract=off), evaluated in the written order.  Integer
 * and byte results are exact.
 *
 * Built twice from this one file: single-threaded (the parity reference), and
 * with OpenMP over all host cores.  Only per-vehicle loops run in parallel:
 * the longitudinal intent, the departure candidates' entry checks and the
 * lane change each write nothing but the vehicle's own result slots; a
 * vehicle that stays on its edge writes only its own new position and lane;
 * painting or erasing the map writes only the vehicle's own cell.  Claims and
 * statistics, which several vehicles touch, stay in serial loops in vehicle
 * order, so both builds give identical results.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ENOMEM (-2)
#define OR_ESTATE (-4)

#define ST_WAIT 0
#define ST_ACTIVE 1
#define ST_DONE 2

#define FREE_BYTE 255

typedef struct {
    float dt, a, b, s0, T, veh_len, x0, g_a, g_b, alpha_i, alpha_a, alpha_b;
    double bin_seconds;
    int32_t delta;
    int32_t n_bins;
    uint64_t seed;
    int32_t free_mode;   /* 0: speed jumps to v0 without a leader; 1: IDM free road */
    int32_t lane_change; /* 0 off, 1 on */
    float eps_a, eps_b;  /* half-widths of the random lead / lag gap terms (0: none) */
} or_params;

typedef struct {
    int64_t step, active, waiting, arrived, vehicle_steps, transfers, departures,
        claims_lost, lc_attempts, lc_accepts, watchdog;
} or_counters;

typedef struct {
    or_params p;
    /* derived constants */
    int32_t W, D, bin_steps;
    float two_sqrt_ab, half_dt;
    /* network */
    int32_t n_nodes, n_edges;
    int32_t *src, *dst, *cells, *lanes, *rank, *outdeg;
    float *v0;
    int64_t *lane_off, *slot_off;
    uint8_t *blocked;
    /* fixed-time signals (NULL: none): per node phases, green, all-red and
       offset in steps; per edge the phase it is served in (-1 none) */
    int32_t *sig_nph, *sig_green, *sig_allred, *sig_off, *sig_phase;
    int64_t map_bytes, n_slots;
    uint8_t *map;
    /* trips */
    int64_t n_trips;
    int32_t *depart;
    int64_t *route_off;
    int32_t *route;
    uint8_t *status;
    int32_t *edge, *lane, *rp, *enter_step, *arrival_step;
    float *x, *v;
    /* departure bookkeeping: trips sorted by (depart, id), next unstarted, stuck list */
    int64_t *dep_order;
    int64_t dep_next;
    int64_t *stuck;
    int64_t n_stuck;
    /* active list */
    int64_t *act;
    int64_t n_act;
    /* per-step scratch, sized once per trip set */
    int32_t *kind, *tlane, *new_lane;
    float *xn, *vn;
    int64_t *target, *cand, *cand_slot, *next_act, *claim_min, *touched;
    uint8_t *cand_claims, *moved_edge;
    int64_t n_touched;
    /* stats */
    int32_t *n_exits;
    int64_t *tt_sum;
    int32_t *inflow_bin, *exits_bin;
    int64_t *tt_bin, *occ_bin;
    or_counters c;
    int32_t k;
    int32_t loaded_net, loaded_trips;
    int32_t invariant_broken;
} or_sim;

/* ------------------------------------------------------------------------ */

static void *xcalloc(size_t n, size_t s) { return calloc(n ? n : 1, s ? s : 1); }

void or_destroy(or_sim *s) {
    if (!s) return;
    free(s->src); free(s->dst); free(s->cells); free(s->lanes); free(s->rank);
    free(s->outdeg); free(s->v0); free(s->lane_off); free(s->slot_off);
    free(s->blocked); free(s->map);
    free(s->sig_nph); free(s->sig_green); free(s->sig_allred); free(s->sig_off); free(s->sig_phase);
    free(s->depart); free(s->route_off); free(s->route); free(s->status);
    free(s->edge); free(s->lane); free(s->rp); free(s->enter_step);
    free(s->arrival_step); free(s->x); free(s->v); free(s->dep_order);
    free(s->stuck); free(s->act);
    free(s->kind); free(s->tlane); free(s->new_lane); free(s->xn); free(s->vn);
    free(s->target); free(s->cand); free(s->cand_slot); free(s->next_act);
    free(s->claim_min); free(s->touched); free(s->cand_claims); free(s->moved_edge);
    free(s->n_exits); free(s->tt_sum); free(s->inflow_bin); free(s->exits_bin);
    free(s->tt_bin); free(s->occ_bin);
    free(s);
}

int or_create(const or_params *p, or_sim **out) {
    if (!p || !out) return OR_EINVAL;
    if (!(p->dt > 0 && p->a > 0 && p->b > 0 && p->s0 > 0 && p->T > 0 &&
          p->veh_len > 0 && p->x0 > 0 && p->g_a >= 0 && p->g_b >= 0 &&
          p->alpha_i >= 0 && p->alpha_a >= 0 && p->alpha_b >= 0 &&
          p->eps_a >= 0 && p->eps_a <= 100 && p->eps_b >= 0 && p->eps_b <= 100 &&
          p->bin_seconds > 0 && p->delta == 4 && p->n_bins >= 1 &&
          (p->free_mode == 0 || p->free_mode == 1) &&
          (p->lane_change == 0 || p->lane_change == 1)))
        return OR_EINVAL;
    double bs = p->bin_seconds / (double)p->dt;
    int32_t bsi = (int32_t)llround(bs);
    if (bsi < 1 || fabs(bs - (double)bsi) > 1e-9) return OR_EINVAL;
    or_sim *s = (or_sim *)xcalloc(1, sizeof(or_sim));
    if (!s) return OR_ENOMEM;
    s->p = *p;
    s->bin_steps = bsi;
    /* entry window: a vehicle of length L plus the standstill gap s0 */
    s->W = (int32_t)ceil((double)p->veh_len + (double)p->s0);
    s->two_sqrt_ab = (float)(2.0 * sqrt((double)p->a * (double)p->b));
    s->half_dt = 0.5f * p->dt;
    *out = s;
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* network */

int or_load_network(or_sim *s, int32_t n_nodes, int32_t n_edges,
                    const int32_t *src, const int32_t *dst, const float *length,
                    const uint8_t *lanes, const float *speed) {
    if (!s || n_nodes <= 0 || n_edges <= 0) return OR_EINVAL;
    for (int32_t e = 0; e < n_edges; e++) {
        if (src[e] < 0 || src[e] >= n_nodes || dst[e] < 0 || dst[e] >= n_nodes) return OR_EINVAL;
        if (lanes[e] < 1 || lanes[e] > 8) return OR_EINVAL;
        if (!(speed[e] > 0.0f && speed[e] <= 254.0f)) return OR_EINVAL;
        if (!(length[e] > 0.0f)) return OR_EINVAL;
        double c = ceil((double)length[e]);
        if (c < (double)(s->W + 1) || c > 65535.0) return OR_EINVAL;
    }
    s->n_nodes = n_nodes;
    s->n_edges = n_edges;
    s->src = (int32_t *)xcalloc(n_edges, 4);
    s->dst = (int32_t *)xcalloc(n_edges, 4);
    s->cells = (int32_t *)xcalloc(n_edges, 4);
    s->lanes = (int32_t *)xcalloc(n_edges, 4);
    s->rank = (int32_t *)xcalloc(n_edges, 4);
    s->outdeg = (int32_t *)xcalloc(n_edges, 4);
    s->v0 = (float *)xcalloc(n_edges, 4);
    s->lane_off = (int64_t *)xcalloc(n_edges, 8);
    s->slot_off = (int64_t *)xcalloc(n_edges, 8);
    s->blocked = (uint8_t *)xcalloc(n_edges, 1);
    if (!s->src || !s->dst || !s->cells || !s->lanes || !s->rank || !s->outdeg ||
        !s->v0 || !s->lane_off || !s->slot_off || !s->blocked)
        return OR_ENOMEM;
    double vmax = 0.0;
    int64_t off = 0, slot = 0;
    for (int32_t e = 0; e < n_edges; e++) {
        s->src[e] = src[e];
        s->dst[e] = dst[e];
        s->cells[e] = (int32_t)ceil((double)length[e]);
        s->lanes[e] = lanes[e];
        s->v0[e] = speed[e];
        s->lane_off[e] = off;
        off += (int64_t)s->cells[e] * lanes[e];
        s->slot_off[e] = slot;
        slot += lanes[e];
        if ((double)speed[e] > vmax) vmax = (double)speed[e];
    }
    s->map_bytes = off;
    s->n_slots = slot;
    /* rank of each edge among the out-edges of its source node, ordered by
       edge id, and that node's out-degree (for the required-lane rule) */
    int32_t *deg = (int32_t *)xcalloc(n_nodes, 4);
    if (!deg) return OR_ENOMEM;
    for (int32_t e = 0; e < n_edges; e++) {
        s->rank[e] = deg[src[e]];
        deg[src[e]]++;
    }
    for (int32_t e = 0; e < n_edges; e++) s->outdeg[e] = deg[src[e]];
    free(deg);
    /* leader look-ahead in cells: at least the paper's 2*dt*v bound, extended
       to the IDM desired gap s0 + T*v at the network's top speed */
    double reach = 2.0 * (double)s->p.dt * vmax;
    double desired = (double)s->p.s0 + (double)s->p.T * vmax;
    s->D = (int32_t)ceil((double)s->p.veh_len + (reach > desired ? reach : desired));
    s->map = (uint8_t *)malloc((size_t)(s->map_bytes ? s->map_bytes : 1));
    if (!s->map) return OR_ENOMEM;
    memset(s->map, FREE_BYTE, (size_t)s->map_bytes);
    int64_t nb = (int64_t)n_edges * s->p.n_bins;
    s->n_exits = (int32_t *)xcalloc(n_edges, 4);
    s->tt_sum = (int64_t *)xcalloc(n_edges, 8);
    s->inflow_bin = (int32_t *)xcalloc(nb, 4);
    s->exits_bin = (int32_t *)xcalloc(nb, 4);
    s->tt_bin = (int64_t *)xcalloc(nb, 8);
    s->occ_bin = (int64_t *)xcalloc(nb, 8);
    if (!s->n_exits || !s->tt_sum || !s->inflow_bin || !s->exits_bin || !s->tt_bin || !s->occ_bin)
        return OR_ENOMEM;
    s->loaded_net = 1;
    return OR_OK;
}

int or_block_edge(or_sim *s, int32_t e, int32_t on) {
    if (!s || !s->loaded_net || e < 0 || e >= s->n_edges) return OR_EINVAL;
    s->blocked[e] = on ? 1 : 0;
    return OR_OK;
}

static void drop_signals(or_sim *s) {
    free(s->sig_nph); free(s->sig_green); free(s->sig_allred); free(s->sig_off); free(s->sig_phase);
    s->sig_nph = s->sig_green = s->sig_allred = s->sig_off = s->sig_phase = NULL;
}

/* Install a fixed-time signal plan (copied), or remove it (n_phases NULL).
 * Per node: n_phases (0 = no signal, else 1..15), green >= 1 and allred >= 0
 * steps per phase, offset in [0, cycle) with cycle = n_phases*(green+allred)
 * <= 65535.  Per edge: the phase of its downstream node it is served in,
 * -1 for none (always -1 at a node without a signal). */
int or_set_signals(or_sim *s, const int32_t *n_phases, const int32_t *green, const int32_t *allred,
                   const int32_t *offset, const int32_t *edge_phase) {
    if (!s || !s->loaded_net) return OR_EINVAL;
    if (!n_phases) {
        drop_signals(s);
        return OR_OK;
    }
    if (!green || !allred || !offset || !edge_phase) return OR_EINVAL;
    for (int32_t n = 0; n < s->n_nodes; n++) {
        if (n_phases[n] < 0 || n_phases[n] > 15) return OR_EINVAL;
        if (n_phases[n] == 0) continue;
        if (green[n] < 1 || allred[n] < 0) return OR_EINVAL;
        int64_t cyc = (int64_t)n_phases[n] * ((int64_t)green[n] + allred[n]);
        if (cyc > 65535 || offset[n] < 0 || offset[n] >= cyc) return OR_EINVAL;
    }
    for (int32_t e = 0; e < s->n_edges; e++) {
        int32_t np = n_phases[s->dst[e]];
        if (edge_phase[e] < -1 || edge_phase[e] >= (np > 0 ? np : 0)) return OR_EINVAL;
    }
    drop_signals(s);
    size_t nn = (size_t)s->n_nodes * 4, ne = (size_t)s->n_edges * 4;
    s->sig_nph = (int32_t *)xcalloc(nn, 1);
    s->sig_green = (int32_t *)xcalloc(nn, 1);
    s->sig_allred = (int32_t *)xcalloc(nn, 1);
    s->sig_off = (int32_t *)xcalloc(nn, 1);
    s->sig_phase = (int32_t *)xcalloc(ne, 1);
    if (!s->sig_nph || !s->sig_green || !s->sig_allred || !s->sig_off || !s->sig_phase) {
        drop_signals(s);
        return OR_ENOMEM;
    }
    memcpy(s->sig_nph, n_phases, nn);
    memcpy(s->sig_green, green, nn);
    memcpy(s->sig_allred, allred, nn);
    memcpy(s->sig_off, offset, nn);
    memcpy(s->sig_phase, edge_phase, ne);
    return OR_OK;
}

int32_t or_window(const or_sim *s, int32_t which) {
    return which == 0 ? s->W : which == 1 ? s->D : s->bin_steps;
}

/* ------------------------------------------------------------------------ */
/* trips */

static const int32_t *g_sort_dep; /* for qsort: single-threaded oracle */
static int cmp_dep_plain(const void *a, const void *b) {
    int64_t i = *(const int64_t *)a, j = *(const int64_t *)b;
    if (g_sort_dep[i] != g_sort_dep[j]) return g_sort_dep[i] < g_sort_dep[j] ? -1 : 1;
    return i < j ? -1 : (i > j);
}

int or_load_trips(or_sim *s, int64_t n_trips, const int32_t *depart,
                  const int64_t *route_off, const int32_t *route_edges) {
    if (!s) return OR_EINVAL;
    if (!s->loaded_net) return OR_ESTATE;
    if (n_trips < 0 || n_trips >= 0x7fffffff) return OR_EINVAL;
    if (route_off[0] != 0) return OR_EINVAL;
    for (int64_t i = 0; i < n_trips; i++) {
        if (depart[i] < 0) return OR_EINVAL;
        if (route_off[i + 1] <= route_off[i]) return OR_EINVAL;
        for (int64_t j = route_off[i]; j < route_off[i + 1]; j++) {
            int32_t e = route_edges[j];
            if (e < 0 || e >= s->n_edges) return OR_EINVAL;
            if (j > route_off[i] && s->dst[route_edges[j - 1]] != s->src[e]) return OR_EINVAL;
        }
    }
    int64_t nr = route_off[n_trips];
    free(s->depart); free(s->route_off); free(s->route); free(s->status);
    free(s->edge); free(s->lane); free(s->rp); free(s->enter_step);
    free(s->arrival_step); free(s->x); free(s->v); free(s->dep_order);
    free(s->stuck); free(s->act);
    free(s->kind); free(s->tlane); free(s->new_lane); free(s->xn); free(s->vn);
    free(s->target); free(s->cand); free(s->cand_slot); free(s->next_act);
    free(s->claim_min); free(s->touched); free(s->cand_claims); free(s->moved_edge);
    s->n_trips = n_trips;
    s->depart = (int32_t *)xcalloc(n_trips, 4);
    s->route_off = (int64_t *)xcalloc(n_trips + 1, 8);
    s->route = (int32_t *)xcalloc(nr, 4);
    s->status = (uint8_t *)xcalloc(n_trips, 1);
    s->edge = (int32_t *)xcalloc(n_trips, 4);
    s->lane = (int32_t *)xcalloc(n_trips, 4);
    s->rp = (int32_t *)xcalloc(n_trips, 4);
    s->enter_step = (int32_t *)xcalloc(n_trips, 4);
    s->arrival_step = (int32_t *)xcalloc(n_trips, 4);
    s->x = (float *)xcalloc(n_trips, 4);
    s->v = (float *)xcalloc(n_trips, 4);
    s->dep_order = (int64_t *)xcalloc(n_trips, 8);
    s->stuck = (int64_t *)xcalloc(n_trips, 8);
    s->act = (int64_t *)xcalloc(n_trips, 8);
    s->kind = (int32_t *)xcalloc(n_trips, 4);
    s->tlane = (int32_t *)xcalloc(n_trips, 4);
    s->new_lane = (int32_t *)xcalloc(n_trips, 4);
    s->xn = (float *)xcalloc(n_trips, 4);
    s->vn = (float *)xcalloc(n_trips, 4);
    s->target = (int64_t *)xcalloc(n_trips, 8);
    s->cand = (int64_t *)xcalloc(n_trips, 8);
    s->cand_slot = (int64_t *)xcalloc(n_trips, 8);
    s->next_act = (int64_t *)xcalloc(n_trips, 8);
    s->touched = (int64_t *)xcalloc(n_trips, 8);
    s->cand_claims = (uint8_t *)xcalloc(n_trips, 1);
    s->moved_edge = (uint8_t *)xcalloc(n_trips, 1);
    s->claim_min = (int64_t *)xcalloc(s->n_slots, 8);
    if (!s->depart || !s->route_off || !s->route || !s->status || !s->edge ||
        !s->lane || !s->rp || !s->enter_step || !s->arrival_step || !s->x ||
        !s->v || !s->dep_order || !s->stuck || !s->act || !s->kind ||
        !s->tlane || !s->new_lane || !s->xn || !s->vn || !s->target ||
        !s->cand || !s->cand_slot || !s->next_act || !s->touched ||
        !s->cand_claims || !s->moved_edge || !s->claim_min)
        return OR_ENOMEM;
    for (int64_t q = 0; q < s->n_slots; q++) s->claim_min[q] = INT64_MAX;
    s->n_touched = 0;
    memcpy(s->depart, depart, (size_t)n_trips * 4);
    memcpy(s->route_off, route_off, (size_t)(n_trips + 1) * 8);
    memcpy(s->route, route_edges, (size_t)nr * 4);
    for (int64_t i = 0; i < n_trips; i++) {
        s->status[i] = ST_WAIT;
        s->edge[i] = -1;
        s->arrival_step[i] = -1;
        s->enter_step[i] = -1;
        s->dep_order[i] = i;
    }
    g_sort_dep = s->depart;
    qsort(s->dep_order, (size_t)n_trips, sizeof(int64_t), cmp_dep_plain);
    s->dep_next = 0;
    s->n_stuck = 0;
    s->n_act = 0;
    memset(s->map, FREE_BYTE, (size_t)s->map_bytes);
    int64_t nb = (int64_t)s->n_edges * s->p.n_bins;
    memset(s->n_exits, 0, (size_t)s->n_edges * 4);
    memset(s->tt_sum, 0, (size_t)s->n_edges * 8);
    memset(s->inflow_bin, 0, (size_t)nb * 4);
    memset(s->exits_bin, 0, (size_t)nb * 4);
    memset(s->tt_bin, 0, (size_t)nb * 8);
    memset(s->occ_bin, 0, (size_t)nb * 8);
    memset(&s->c, 0, sizeof(s->c));
    s->k = 0;
    s->invariant_broken = 0;
    s->loaded_trips = 1;
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* small pieces, each a direct statement of one rule */

static int64_t cell_index(const or_sim *s, int32_t e, int32_t l, int32_t c) {
    return s->lane_off[e] + (int64_t)l * s->cells[e] + c;
}

/* occupancy byte for a vehicle with speed v: speed in m/s truncated, capped at 254 */
static uint8_t speed_byte(float v) {
    float c = v < 254.0f ? v : 254.0f;
    return (uint8_t)(int32_t)c;
}

static int32_t bin_of(const or_sim *s, int32_t step) {
    int32_t b = step / s->bin_steps;
    return b < s->p.n_bins - 1 ? b : s->p.n_bins - 1;
}

/* are the first W cells of lane l on edge e free in the current map? */
static int entry_free(const or_sim *s, int32_t e, int32_t l) {
    if (s->blocked[e]) return 0;
    for (int32_t c = 0; c < s->W; c++)
        if (s->map[cell_index(s, e, l, c)] != FREE_BYTE) return 0;
    return 1;
}

/* may vehicles on edge e pass its downstream signal at step k?  The node's
 * cycle runs phase 0, 1, ... each for green + allred steps, starting at step
 * -offset; edge e is served in its phase's first `green` steps. */
static int approach_green(const or_sim *s, int32_t e, int32_t k) {
    if (!s->sig_nph || s->sig_phase[e] < 0) return 1;
    int32_t n = s->dst[e];
    int64_t per = (int64_t)s->sig_green[n] + s->sig_allred[n];
    int64_t cycle = per * s->sig_nph[n];
    int64_t t = ((int64_t)k + s->sig_off[n]) % cycle;
    int64_t phase = t / per, into = t % per;
    return phase == s->sig_phase[e] && into < s->sig_green[n];
}

/* first occupied cell in cells lo..hi (inclusive) of lane l, or -1 */
static int32_t scan_forward(const or_sim *s, int32_t e, int32_t l, int32_t lo, int32_t hi) {
    for (int32_t c = lo; c <= hi; c++)
        if (s->map[cell_index(s, e, l, c)] != FREE_BYTE) return c;
    return -1;
}

/* first occupied cell going down from hi to lo (inclusive), or -1 */
static int32_t scan_backward(const or_sim *s, int32_t e, int32_t l, int32_t hi, int32_t lo) {
    for (int32_t c = hi; c >= lo; c--)
        if (s->map[cell_index(s, e, l, c)] != FREE_BYTE) return c;
    return -1;
}

/* SplitMix64 output function (Steele, Lea & Flood 2014) */
/* key of the stream of the random gap terms (an arbitrary odd constant) */
#define EPS_STREAM 0xD6E8FEB86659FD93ull

static uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

static float max0f(float t) { return t > 0.0f ? t : 0.0f; }

/*
 * IDM step against a leader at gap s with (quantised) speed vl.  Returns v' and
 * x' through pointers.  s <= 0 means standing bumper to bumper: stay, v=0.
 */
static void idm_follow(const or_sim *s, float x, float v, float v0, float gap,
                       float vl, float *xn, float *vn) {
    const or_params *p = &s->p;
    if (gap <= 0.0f) {
        *vn = 0.0f;
        *xn = x;
        return;
    }
    float dv = v - vl;
    float t = (v * p->T) + ((v * dv) / s->two_sqrt_ab);
    float ss = p->s0 + max0f(t);
    float r = v / v0;
    float r2 = r * r;
    float r4 = r2 * r2;
    float q = ss / gap;
    float q2 = q * q;
    float acc = p->a * ((1.0f - r4) - q2);
    float nv = v + acc * p->dt;
    *vn = nv > 0.0f ? nv : 0.0f;
    *xn = x + (v + *vn) * s->half_dt;
}

/* no leader: the paper's jump to the free speed, or IDM free-road acceleration */
static void free_move(const or_sim *s, float x, float v, float v0, float *xn, float *vn) {
    if (s->p.free_mode == 0) {
        *vn = v0;
        *xn = x + *vn * s->p.dt;
    } else {
        float r = v / v0;
        float r2 = r * r;
        float r4 = r2 * r2;
        float acc = s->p.a * (1.0f - r4);
        float nv = v + acc * s->p.dt;
        *vn = nv > 0.0f ? nv : 0.0f;
        *xn = x + (v + *vn) * s->half_dt;
    }
}

/* ------------------------------------------------------------------------ */
/* one time step, k -> k+1 */

enum { K_NONE = 0, K_MOVE, K_ARRIVE, K_CLAIM };

static void add_exit(or_sim *s, int32_t e, int32_t enter, int32_t exit_step) {
    int32_t tt = exit_step - enter;
    s->n_exits[e] += 1;
    s->tt_sum[e] += tt;
    int32_t b = bin_of(s, enter);
    s->exits_bin[(int64_t)e * s->p.n_bins + b] += 1;
    s->tt_bin[(int64_t)e * s->p.n_bins + b] += tt;
    for (int32_t st = enter; st < exit_step; st++)
        s->occ_bin[(int64_t)e * s->p.n_bins + bin_of(s, st)] += 1;
}

static void add_entry(or_sim *s, int32_t e, int32_t step) {
    s->inflow_bin[(int64_t)e * s->p.n_bins + bin_of(s, step)] += 1;
}

/* write every active vehicle into the (all-free) map; flag double occupancy.
   A cell is taken by an exchange that returns its previous byte, so a second
   vehicle on one cell is seen whichever vehicle is painted first (also when
   the all-cores build paints on several threads). */
static void paint_map(or_sim *s) {
    int broken = 0;
    #pragma omp parallel for schedule(static) reduction(| : broken)
    for (int64_t j = 0; j < s->n_act; j++) {
        int64_t i = s->act[j];
        int32_t c = (int32_t)floorf(s->x[i]);
        if (c < 0 || c >= s->cells[s->edge[i]] || s->lane[i] < 0 || s->lane[i] >= s->lanes[s->edge[i]]) {
            broken = 1;
            continue;
        }
        int64_t at = cell_index(s, s->edge[i], s->lane[i], c);
        uint8_t before = __atomic_exchange_n(&s->map[at], speed_byte(s->v[i]), __ATOMIC_RELAXED);
        if (before != FREE_BYTE) broken = 1;
    }
    if (broken) s->invariant_broken = 1;
}

static void erase_map(or_sim *s) {
    #pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < s->n_act; j++) {
        int64_t i = s->act[j];
        int32_t c = (int32_t)floorf(s->x[i]);
        if (c < 0 || c >= s->cells[s->edge[i]] || s->lane[i] < 0 || s->lane[i] >= s->lanes[s->edge[i]]) continue;
        __atomic_store_n(&s->map[cell_index(s, s->edge[i], s->lane[i], c)], (uint8_t)FREE_BYTE, __ATOMIC_RELAXED);
    }
}

/* record a claim on a target lane; remember touched slots to reset them */
static void claim(or_sim *s, int64_t slot, int64_t id) {
    if (s->claim_min[slot] == INT64_MAX) s->touched[s->n_touched++] = slot;
    if (id < s->claim_min[slot]) s->claim_min[slot] = id;
}

static int step_once(or_sim *s) {
    const or_params *p = &s->p;
    const int32_t k = s->k;
    const float L = p->veh_len;
    const int64_t n_act0 = s->n_act;
    int32_t *kind = s->kind, *tlane = s->tlane;
    float *xn = s->xn, *vn = s->vn;
    int64_t *target = s->target;

    /* map of step k */
    paint_map(s);

    /* --- longitudinal intent of every active vehicle (reads step k only) ---
       Each vehicle writes only its own entries of xn, vn, kind, target and
       tlane, so the loop may run on several threads (the all-cores build);
       its claims are recorded afterwards, in vehicle order. */
    #pragma omp parallel for schedule(dynamic, 2048)
    for (int64_t j = 0; j < n_act0; j++) {
        int64_t i = s->act[j];
        int32_t e = s->edge[i], l = s->lane[i];
        float x = s->x[i], v = s->v[i];
        int32_t C = s->cells[e];
        int32_t c = (int32_t)floorf(x);
        int last = (s->route_off[i] + s->rp[i] + 1 == s->route_off[i + 1]);
        int32_t hi = c + s->D < C - 1 ? c + s->D : C - 1;
        int32_t cl = scan_forward(s, e, l, c + 1, hi);
        float x2, v2;
        if (cl >= 0) {
            /* real leader: its front is at the start of cell cl, speed = byte */
            float vl = (float)s->map[cell_index(s, e, l, cl)];
            float gap = ((float)cl - x) - L;
            idm_follow(s, x, v, s->v0[e], gap, vl, &x2, &v2);
            float lim = (float)cl - L;
            if (x2 > lim) {
                x2 = x > lim ? x : lim;
                v2 = v2 < vl ? v2 : vl;
            }
        } else {
            int stop_line = 0;
            if (!last && c + s->D >= C) {
                int32_t en = s->route[s->route_off[i] + s->rp[i] + 1];
                int32_t ln = l < s->lanes[en] - 1 ? l : s->lanes[en] - 1;
                /* a red signal, or a taken entry window, stops the vehicle */
                stop_line = !approach_green(s, e, k) || !entry_free(s, en, ln);
            }
            if (stop_line) {
                /* downstream entry occupied: a standing obstacle at the stop line */
                float gap = (float)C - x;
                idm_follow(s, x, v, s->v0[e], gap, 0.0f, &x2, &v2);
                float lim = (float)(C - 1);
                if (x2 > lim) {
                    x2 = x > lim ? x : lim;
                    v2 = 0.0f;
                }
            } else {
                free_move(s, x, v, s->v0[e], &x2, &v2);
            }
        }
        xn[j] = x2;
        vn[j] = v2;
        kind[j] = K_MOVE;
        if (x2 >= (float)C) {
            if (last) {
                kind[j] = K_ARRIVE;
            } else {
                int32_t en = s->route[s->route_off[i] + s->rp[i] + 1];
                int32_t ln = l < s->lanes[en] - 1 ? l : s->lanes[en] - 1;
                kind[j] = K_CLAIM;
                target[j] = s->slot_off[en] + ln;
                tlane[j] = ln;
            }
        }
    }
    for (int64_t j = 0; j < n_act0; j++)
        if (kind[j] == K_CLAIM) claim(s, target[j], s->act[j]);

    /* --- departures whose time has come (reads step k only) --- */
    int64_t n_cand = 0;
    for (int64_t q = 0; q < s->n_stuck; q++) s->cand[n_cand++] = s->stuck[q];
    while (s->dep_next < s->n_trips && s->depart[s->dep_order[s->dep_next]] <= k) {
        int64_t i = s->dep_order[s->dep_next++];
        if (s->status[i] == ST_WAIT) s->cand[n_cand++] = i; /* placed trips skip */
    }
    /* each candidate checks its start lane on its own; claims in candidate order */
    #pragma omp parallel for schedule(dynamic, 2048)
    for (int64_t q = 0; q < n_cand; q++) {
        int64_t i = s->cand[q];
        int32_t e0 = s->route[s->route_off[i]];
        int32_t l0 = (int32_t)(i % s->lanes[e0]);
        s->cand_slot[q] = s->slot_off[e0] + l0;
        s->cand_claims[q] = (uint8_t)entry_free(s, e0, l0);
    }
    for (int64_t q = 0; q < n_cand; q++)
        if (s->cand_claims[q]) claim(s, s->cand_slot[q], s->cand[q]);

    /* the map of step k is no longer needed */
    erase_map(s);

    /* --- vehicles that stay on their edge take their new position and speed
       (each writes only its own state) --- */
    #pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n_act0; j++) {
        if (kind[j] != K_MOVE) continue;
        int64_t i = s->act[j];
        s->x[i] = xn[j];
        s->v[i] = vn[j];
    }

    /* --- resolve: the lowest id claiming a target lane enters it --- */
    int64_t n_new = 0;
    int64_t events = 0;
    for (int64_t j = 0; j < n_act0; j++) {
        int64_t i = s->act[j];
        if (kind[j] == K_ARRIVE) {
            int32_t e = s->edge[i];
            add_exit(s, e, s->enter_step[i], k + 1);
            s->status[i] = ST_DONE;
            s->arrival_step[i] = k + 1;
            s->edge[i] = -1;
            s->c.arrived++;
            events++;
            continue;
        }
        s->moved_edge[n_new] = 0;
        if (kind[j] == K_CLAIM) {
            int32_t e = s->edge[i];
            if (s->claim_min[target[j]] == i) {
                int32_t en = s->route[s->route_off[i] + s->rp[i] + 1];
                add_exit(s, e, s->enter_step[i], k + 1);
                add_entry(s, en, k + 1);
                s->edge[i] = en;
                s->lane[i] = tlane[j];
                s->x[i] = 0.0f;
                s->v[i] = vn[j];
                s->rp[i] += 1;
                s->enter_step[i] = k + 1;
                s->c.transfers++;
                events++;
                s->moved_edge[n_new] = 1;
            } else {
                /* lost the entry: wait at the last cell, stopped */
                float lim = (float)(s->cells[e] - 1);
                s->x[i] = s->x[i] > lim ? s->x[i] : lim;
                s->v[i] = 0.0f;
                s->c.claims_lost++;
            }
        }
        s->next_act[n_new++] = i;
    }
    int64_t n_stuck = 0;
    for (int64_t q = 0; q < n_cand; q++) {
        int64_t i = s->cand[q];
        if (s->cand_claims[q] && s->claim_min[s->cand_slot[q]] == i) {
            int32_t e0 = s->route[s->route_off[i]];
            s->status[i] = ST_ACTIVE;
            s->edge[i] = e0;
            s->lane[i] = (int32_t)(i % s->lanes[e0]);
            s->x[i] = 0.0f;
            s->v[i] = 0.0f;
            s->rp[i] = 0;
            s->enter_step[i] = k + 1;
            add_entry(s, e0, k + 1);
            s->c.departures++;
            events++;
            s->moved_edge[n_new] = 1;
            s->next_act[n_new++] = i;
        } else {
            if (s->cand_claims[q]) s->c.claims_lost++;
            s->stuck[n_stuck++] = i;
        }
    }
    s->n_stuck = n_stuck;
    for (int64_t q = 0; q < s->n_touched; q++) s->claim_min[s->touched[q]] = INT64_MAX;
    s->n_touched = 0;
    {
        int64_t *tmp = s->act;
        s->act = s->next_act;
        s->next_act = tmp;
    }
    s->n_act = n_new;

    /* --- lane change on the map after the longitudinal move --- */
    if (p->lane_change) {
        paint_map(s);
        int32_t *new_lane = s->new_lane;
        int64_t attempts = 0, accepts = 0;
        /* each vehicle decides on the painted map and writes only new_lane[j] */
        #pragma omp parallel for schedule(dynamic, 2048) reduction(+ : attempts, accepts)
        for (int64_t j = 0; j < n_new; j++) {
            int64_t i = s->act[j];
            new_lane[j] = s->lane[i];
            if (s->moved_edge[j]) continue;               /* entered an edge this step */
            if (s->route_off[i] + s->rp[i] + 1 >= s->route_off[i + 1]) continue; /* last edge */
            int32_t e = s->edge[i], l = s->lane[i];
            int32_t en = s->route[s->route_off[i] + s->rp[i] + 1];
            /* required lane: the lanes are split in proportion to the rank of
               the next edge among the out-edges of the intersection */
            int32_t req = (s->rank[en] * s->lanes[e]) / s->outdeg[en];
            if (req == l) continue;
            int32_t dir = req > l ? 1 : -1;
            /* even steps move toward lane 0 only, odd steps away from it */
            if ((k % 2 == 0 && dir > 0) || (k % 2 == 1 && dir < 0)) continue;
            float x = s->x[i], v = s->v[i];
            float d = (float)s->cells[e] - x;
            float prob = d >= p->x0 ? 0.0f : 1.0f - d / p->x0;
            uint64_t h = mix64(p->seed ^ (((uint64_t)i << 32) | (uint64_t)(uint32_t)k));
            if (!((float)(h >> 40) < prob * 16777216.0f)) continue;
            attempts++;
            /* random gap terms: a second stream keyed by the same (trip, step);
               the top 24 bits give eps_a, the next 24 eps_b, each uniform on
               [-eps, eps) in steps of eps * 2^-23 */
            float ea = 0.0f, eb = 0.0f;
            if (p->eps_a > 0.0f || p->eps_b > 0.0f) {
                uint64_t h2 = mix64(p->seed ^ EPS_STREAM ^ (((uint64_t)i << 32) | (uint64_t)(uint32_t)k));
                float ua = (float)(h2 >> 40), ub = (float)((h2 >> 16) & 0xffffffu);
                ea = p->eps_a * (ua * 0x1p-23f - 1.0f);
                eb = p->eps_b * (ub * 0x1p-23f - 1.0f);
            }
            int32_t lt = l + dir;
            int32_t c = (int32_t)floorf(x);
            int32_t C = s->cells[e];
            if (s->map[cell_index(s, e, lt, c)] != FREE_BYTE) continue;
            int ok = 1;
            int32_t hi = c + s->D < C - 1 ? c + s->D : C - 1;
            int32_t ca = scan_forward(s, e, lt, c + 1, hi);
            if (ca >= 0) {
                float va = (float)s->map[cell_index(s, e, lt, ca)];
                float g_lead = ((float)ca - x) - L;
                float crit = p->g_a + max0f(((p->alpha_i * v) - (p->alpha_a * va)) + ea);
                if (!(g_lead >= crit)) ok = 0;
            }
            int32_t lo = c - s->D > 0 ? c - s->D : 0;
            int32_t cb = scan_backward(s, e, lt, c - 1, lo);
            if (ok && cb >= 0) {
                float vb = (float)s->map[cell_index(s, e, lt, cb)];
                float g_lag = (x - L) - (float)(cb + 1);
                float crit = p->g_b + max0f(((p->alpha_b * vb) - (p->alpha_i * v)) + eb);
                if (!(g_lag >= crit)) ok = 0;
            }
            if (ok) {
                new_lane[j] = lt;
                accepts++;
            }
        }
        s->c.lc_attempts += attempts;
        s->c.lc_accepts += accepts;
        erase_map(s);
        #pragma omp parallel for schedule(static)
        for (int64_t j = 0; j < n_new; j++) s->lane[s->act[j]] = new_lane[j];
    }

    /* check the one-vehicle-per-cell invariant on the final map */
    paint_map(s);
    erase_map(s);

    s->c.vehicle_steps += n_act0;
    if (n_act0 > 0 && events == 0) s->c.watchdog++;
    else s->c.watchdog = 0;
    s->k = k + 1;
    return OR_OK;
}

/*
 * Test hook: put waiting trip i directly on route edge rp at (lane, x, v), as
 * if it had entered that edge at the current step.  Used to build exact
 * geometric situations (gap-acceptance thresholds, simultaneous claims).
 */
int or_place(or_sim *s, int64_t i, int32_t rp, int32_t lane, float x, float v) {
    if (!s || !s->loaded_trips) return OR_ESTATE;
    if (i < 0 || i >= s->n_trips || s->status[i] != ST_WAIT) return OR_EINVAL;
    if (rp < 0 || s->route_off[i] + rp >= s->route_off[i + 1]) return OR_EINVAL;
    int32_t e = s->route[s->route_off[i] + rp];
    if (lane < 0 || lane >= s->lanes[e] || !(x >= 0.0f) || !(x < (float)s->cells[e]) || !(v >= 0.0f))
        return OR_EINVAL;
    for (int64_t q = 0; q < s->n_stuck; q++)
        if (s->stuck[q] == i) return OR_EINVAL;
    s->status[i] = ST_ACTIVE;
    s->edge[i] = e;
    s->lane[i] = lane;
    s->x[i] = x;
    s->v[i] = v;
    s->rp[i] = rp;
    s->enter_step[i] = s->k;
    s->act[s->n_act++] = i;
    return OR_OK;
}

int or_step(or_sim *s, int32_t n_steps) {
    if (!s || n_steps < 0) return OR_EINVAL;
    if (!s->loaded_trips) return OR_ESTATE;
    for (int32_t t = 0; t < n_steps; t++) {
        int rc = step_once(s);
        if (rc) return rc;
    }
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* read-back */

int or_get_vehicles(const or_sim *s, int32_t *edge, uint8_t *lane, int32_t *cell,
                    float *x, float *v, int32_t *arrival_step, uint8_t *status) {
    if (!s || !s->loaded_trips) return OR_ESTATE;
    for (int64_t i = 0; i < s->n_trips; i++) {
        int act = s->status[i] == ST_ACTIVE;
        if (edge) edge[i] = act ? s->edge[i] : -1;
        if (lane) lane[i] = act ? (uint8_t)s->lane[i] : 0;
        if (cell) cell[i] = act ? (int32_t)floorf(s->x[i]) : -1;
        if (x) x[i] = act ? s->x[i] : 0.0f;
        if (v) v[i] = act ? s->v[i] : 0.0f;
        if (arrival_step) arrival_step[i] = s->arrival_step[i];
        if (status) status[i] = s->status[i];
    }
    return OR_OK;
}

/* per-trip route position and entry step of the current edge (-1 if not active) */
int or_get_progress(const or_sim *s, int32_t *rp, int32_t *enter_step) {
    if (!s || !s->loaded_trips) return OR_ESTATE;
    for (int64_t i = 0; i < s->n_trips; i++) {
        int act = s->status[i] == ST_ACTIVE;
        rp[i] = act ? s->rp[i] : -1;
        enter_step[i] = act ? s->enter_step[i] : -1;
    }
    return OR_OK;
}

/*
 * Edge statistics.  Vehicles still on an edge contribute occupancy for the
 * steps they have spent there so far (not their travel time).
 */
int or_edge_stats(const or_sim *s, int64_t *tt_sum, int32_t *n_exits,
                  int32_t *inflow_bin, int32_t *exits_bin, int64_t *tt_bin,
                  int64_t *occ_bin) {
    if (!s || !s->loaded_trips) return OR_ESTATE;
    int64_t nb = (int64_t)s->n_edges * s->p.n_bins;
    if (tt_sum) memcpy(tt_sum, s->tt_sum, (size_t)s->n_edges * 8);
    if (n_exits) memcpy(n_exits, s->n_exits, (size_t)s->n_edges * 4);
    if (inflow_bin) memcpy(inflow_bin, s->inflow_bin, (size_t)nb * 4);
    if (exits_bin) memcpy(exits_bin, s->exits_bin, (size_t)nb * 4);
    if (tt_bin) memcpy(tt_bin, s->tt_bin, (size_t)nb * 8);
    if (occ_bin) {
        memcpy(occ_bin, s->occ_bin, (size_t)nb * 8);
        for (int64_t j = 0; j < s->n_act; j++) {
            int64_t i = s->act[j];
            for (int32_t st = s->enter_step[i]; st < s->k; st++)
                occ_bin[(int64_t)s->edge[i] * s->p.n_bins + bin_of(s, st)] += 1;
        }
    }
    return OR_OK;
}

int or_get_counters(const or_sim *s, or_counters *out) {
    if (!s || !out) return OR_EINVAL;
    *out = s->c;
    out->step = s->k;
    out->active = s->n_act;
    int64_t waiting = 0;
    for (int64_t i = 0; i < s->n_trips; i++) waiting += s->status[i] == ST_WAIT;
    out->waiting = waiting;
    return OR_OK;
}

int32_t or_invariant_broken(const or_sim *s) { return s ? s->invariant_broken : 1; }

/* threads the per-vehicle loops run on (1 in the single-threaded build) */
int32_t or_threads(void) {
#ifdef _OPENMP
    return (int32_t)omp_get_max_threads();
#else
    return 1;
#endif
}
int64_t or_map_bytes(const or_sim *s) { return s ? s->map_bytes : 0; }
