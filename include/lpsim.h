/*
 * lpsim.h -- C ABI of the MI355X (gfx950) LPSim vehicle-propagation library.
 *
 * The library advances a regional microscopic traffic simulation one time
 * step at a time on one GPU, as described in Jiang, Sengupta, Demmel,
 * Williams, "Large Scale Multi-GPU Based Parallel Traffic Simulation for
 * Accelerated Traffic Assignment and Propagation":
 *   - inputs are a road network (per edge: lanes, length, upstream and
 *     downstream node; Section 3.1, network data) and routed demand (per trip:
 *     departure time and full route; Section 3.1, vehicle data);
 *   - every step updates all vehicles from the previous step's state only
 *     (Section 3.1, vehicle-dynamics equation; Algorithm 1): leader search on
 *     the byte-per-metre lane map, IDM car following, stop-line waiting and
 *     exclusive entry at intersections, departures, mandatory lane change with
 *     gap acceptance;
 *   - outputs are vehicle positions and speeds (Algorithm 1 output) and
 *     per-edge travel times (abstract: travel-time estimation).
 *
 * Conventions for every function:
 *   - returns LPSIM_OK (0) or a negative status; nothing throws;
 *   - on error, lpsim_last_error(ctx) holds a one-line description;
 *   - pointers documented "host" are read during the call only and remain
 *     owned by the caller; the library copies what it keeps;
 *   - a context is used by one host thread at a time;
 *   - after an LPSIM_EDEVICE error the context is poisoned: only
 *     lpsim_last_error and lpsim_destroy remain valid.
 *
 * Batches: lpsim_batch_load places several independent scenarios in one
 * context; every call below then covers all of them at once (arrays are the
 * scenarios' arrays concatenated in scenario order).  lpsim_load_network +
 * lpsim_load_trips is the batch of one.
 */
#ifndef LPSIM_H
#define LPSIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LPSIM_OK 0
#define LPSIM_EINVAL (-1)    /* bad argument or input data */
#define LPSIM_ENOMEM (-2)    /* device or host allocation failed */
#define LPSIM_EDEVICE (-3)   /* HIP runtime error; context poisoned */
#define LPSIM_ESTATE (-4)    /* call out of order (e.g. step before load) */
#define LPSIM_ECAPACITY (-5) /* instance exceeds a documented size limit */

/* Vehicle status values reported by lpsim_get_vehicles. */
#define LPSIM_WAITING 0
#define LPSIM_ACTIVE 1
#define LPSIM_ARRIVED 2

/* No leader: jump to the edge speed limit (Algorithm 1, "v <- v_free"). */
#define LPSIM_FREE_JUMP 0
/* No leader: IDM free-road acceleration a(1 - (v/v0)^4). */
#define LPSIM_FREE_IDM 1

typedef struct lpsim_ctx lpsim_ctx;

/*
 * Model constants (Section 3.1 notation table).  All lengths in metres, times
 * in seconds, speeds in m/s; the simulation state is binary32.
 *   dt        time step (the paper's T as a step size; it states no value)
 *   a, b      IDM acceleration potential and comfortable braking
 *   s0, T     IDM standstill gap and desired time headway
 *   delta     IDM exponent; only 4 is supported
 *   veh_len   vehicle length L (enters gaps; a vehicle marks one cell)
 *   x0        mandatory lane change starts x0 before the edge end
 *   g_a, g_b  desired lead / lag gaps for a lane change
 *   alpha_i, alpha_a, alpha_b  anticipation times (own, lead, lag)
 *   bin_seconds   statistics bin width; must be a whole number of steps
 *   n_bins    number of statistics bins; later events fall in the last bin
 *   seed      seed of the hashed lane-change draws
 *   free_mode LPSIM_FREE_JUMP or LPSIM_FREE_IDM
 *   lane_change   1 to enable mandatory lane changes, 0 to disable
 *   eps_a, eps_b  random components of the critical lead / lag gaps (Gap
 *             Acceptance equations; their law is not given): each is uniform
 *             on [-eps, eps), drawn per attempt from a second hashed stream
 *             of (seed, trip, step), and enters the speed term before its
 *             clamp at zero, so a critical gap stays >= g_a (g_b).  0..100;
 *             0 (the default) leaves the term out.
 */
typedef struct {
    float dt, a, b, s0, T, veh_len, x0, g_a, g_b, alpha_i, alpha_a, alpha_b;
    double bin_seconds;
    int32_t delta;
    int32_t n_bins;
    uint64_t seed;
    int32_t free_mode;
    int32_t lane_change;
    float eps_a, eps_b;
} lpsim_params;

typedef struct {
    int64_t step;          /* steps taken since lpsim_load_trips */
    int64_t active;        /* vehicles on the road now */
    int64_t waiting;       /* trips not yet departed */
    int64_t arrived;       /* trips finished */
    int64_t vehicle_steps; /* sum over steps of the vehicles active at the step's start */
    int64_t transfers;     /* edge-to-edge moves */
    int64_t departures;    /* trips that entered the network */
    int64_t claims_lost;   /* entry requests that lost to a lower trip id */
    int64_t lc_attempts;   /* lane-change draws that succeeded */
    int64_t lc_accepts;    /* lane changes carried out */
    int64_t watchdog;      /* consecutive steps with vehicles but no entry/exit */
    int64_t scan_bytes;    /* bytes the move launch reads beyond each vehicle's
                              28-byte state: lane-map cells scanned, next-edge entry
                              windows, signal words at a stop line (edge id and word,
                              12), entry requests, and the departure requests' reads */
} lpsim_counters;

/* Create a context.  `p` (host) is copied and validated: every length, time
 * and rate > 0 (gaps and alphas >= 0, eps_a and eps_b in 0..100), delta == 4,
 * bin_seconds/dt integral.
 * Errors: EINVAL, ENOMEM, EDEVICE (no usable GPU). */
int32_t lpsim_create(const lpsim_params *p, lpsim_ctx **out);

/* Release every device and host resource.  Accepts NULL. */
void lpsim_destroy(lpsim_ctx *ctx);

/* Optional: route device allocations through caller callbacks (for example a
 * framework's caching allocator).  Must be called before any load.  `alloc`
 * returns device memory of at least `bytes` bytes or NULL. */
int32_t lpsim_set_allocator(lpsim_ctx *ctx, void *(*alloc)(size_t bytes, void *user),
                            void (*release)(void *ptr, void *user), void *user);

/* Load the road network (Section 3.1, network data and lane map).
 *   n_nodes            number of intersections
 *   node_xy            host, 2*n_nodes floats (x, y) or NULL; when given, edges
 *                      are stored in recursive-coordinate-bisection order of
 *                      their upstream node (memory locality only; results do
 *                      not depend on it)
 *   n_edges            number of directed edges; edge e runs src[e] -> dst[e]
 *   length_m           host, edge length; the edge has ceil(length) one-metre cells
 *   lanes              host, 1..8 lanes per edge
 *   speed_limit_mps    host, 0 < v0 <= 254 (the lane-map byte holds the speed)
 * Each edge must have at least ceil(veh_len + s0) + 1 and at most 65535 cells;
 * a node may have at most 255 out-edges.  Replaces any loaded network and
 * discards loaded trips.  Errors: EINVAL, ENOMEM, ECAPACITY (lane map over
 * 4 GiB), EDEVICE. */
int32_t lpsim_load_network(lpsim_ctx *ctx, int32_t n_nodes, const float *node_xy,
                           int32_t n_edges, const int32_t *src, const int32_t *dst,
                           const float *length_m, const uint8_t *lanes,
                           const float *speed_limit_mps);

/* Load routed demand (Section 3.1, vehicle data).  Trip id = array index.
 *   depart_step    host, n_trips departure steps (>= 0); any order
 *   route_offsets  host, n_trips+1 offsets into route_edges, route_offsets[0] = 0
 *   route_edges    host, each trip's edges; non-empty and contiguous
 *                  (dst of one edge = src of the next)
 * Resets the clock to step 0, the lane map, the statistics and the counters.
 * Errors: ESTATE (no network), EINVAL, ENOMEM, ECAPACITY (more than 2^31-2
 * trips or 2^32-2 route entries), EDEVICE. */
int32_t lpsim_load_trips(lpsim_ctx *ctx, int64_t n_trips, const int32_t *depart_step,
                         const int64_t *route_offsets, const int32_t *route_edges);

/* Load n_scen independent scenarios into one context (batched execution).
 * Arrays are the scenarios' own arrays concatenated; node, edge and trip ids
 * inside each scenario's arrays are LOCAL to that scenario.
 *   node_off[n_scen+1], edge_off[n_scen+1], trip_off[n_scen+1]: host prefix sums
 *   node_xy        host, 2 floats per node, or NULL
 *   src, dst, length_m, lanes, speed_limit_mps: host, per edge
 *   depart_step    host, per trip
 *   route_offsets  host, per scenario trip_count+1 entries, each scenario's
 *                  starting at 0 (total n_trips + n_scen entries)
 *   route_edges    host, concatenated routes (local edge ids)
 *   seeds          host, per-scenario lane-change seed, or NULL for params.seed
 * A scenario's result equals what a context holding only that scenario
 * produces.  Errors as lpsim_load_network + lpsim_load_trips. */
int32_t lpsim_batch_load(lpsim_ctx *ctx, int32_t n_scen, const int32_t *node_off,
                         const int32_t *edge_off, const int64_t *trip_off,
                         const float *node_xy, const int32_t *src, const int32_t *dst,
                         const float *length_m, const uint8_t *lanes,
                         const float *speed_limit_mps, const int32_t *depart_step,
                         const int64_t *route_offsets, const int32_t *route_edges,
                         const uint64_t *seeds);

/* Advance n_steps time steps (Algorithm 1 per vehicle, synchronous update).
 *   hip_stream   a hipStream_t to order the work on, or NULL: then the call
 *                runs on an internal stream and returns after the work is done.
 * With a stream the call only enqueues; the caller synchronises the stream.
 * A call on a different stream than the previous call is ordered after the
 * work that call queued (an event on the old stream, waited for on the new
 * one), so the old stream must still exist at that point.
 * Errors: ESTATE (no trips loaded), EINVAL (n_steps < 0), EDEVICE. */
int32_t lpsim_step(lpsim_ctx *ctx, int32_t n_steps, void *hip_stream);

/* Capture, without running anything, the HIP graphs that a call
 * lpsim_step(ctx, n_steps, ...) made next would launch, so that the call does
 * not pay for the capture (a caller that times or repeats calls of one
 * length).  Steps are captured by the graph_steps of lpsim_set_launch; the
 * rest of a call (n_steps mod graph_steps, when above 1) runs as one shorter
 * graph, and a few such graphs are kept (the oldest replaced first).  A
 * no-op while kernel timing is on or with graph_steps 0.  Errors: ESTATE,
 * EINVAL (n_steps < 0), EDEVICE. */
int32_t lpsim_prepare_steps(lpsim_ctx *ctx, int32_t n_steps);

/* Per-edge statistics, in input edge order (host buffers, caller-owned).
 * Travel-time estimation is the simulator's stated purpose (abstract); each
 * traversal's time is its exit step minus the entry step t_start that
 * Algorithm 1 records when a vehicle enters an edge.
 *   tt_sum_steps[E]  sum over completed traversals of (exit step - entry step)
 *   n_exits[E]       number of completed traversals
 *   inflow_bin[E*B]  entries by entry bin (bin = step*dt / bin_seconds)
 *   exits_bin[E*B], tt_sum_bin[E*B]  completed traversals and their travel
 *                    times, binned by ENTRY step
 *   occ_steps_bin[E*B]  vehicle-steps spent on the edge per bin (density),
 *                    including vehicles still on it
 * Mean travel time of edge e in seconds = tt_sum_steps[e] * dt / n_exits[e].
 * Binned pointers may be NULL.  Waits for all queued work.  Errors: ESTATE,
 * EDEVICE. */
int32_t lpsim_edge_stats(lpsim_ctx *ctx, int64_t *tt_sum_steps, int32_t *n_exits,
                         int32_t *inflow_bin, int32_t *exits_bin, int64_t *tt_sum_bin,
                         int64_t *occ_steps_bin);

/* The binned statistics of lpsim_edge_stats, the same values in the same
 * [E*B] input-edge-order layout, written into DEVICE buffers (caller-owned,
 * any may be NULL) by kernels queued on `stream` (a hipStream_t, or NULL for
 * the context's own stream) after the steps already queued; nothing crosses
 * to the host and the call does not wait.  For callers that feed the
 * statistics to device work (the surrogate's features and targets).  A
 * later load of trips or of a network, and lpsim_destroy, wait for these
 * kernels.  Errors: ESTATE, EDEVICE. */
int32_t lpsim_edge_stats_device(lpsim_ctx *ctx, int32_t *inflow_bin, int32_t *exits_bin, int64_t *tt_sum_bin,
                                int64_t *occ_steps_bin, void *stream);

/* Vehicle positions and speeds: the output of Algorithm 1 (vehicle position
 * P and speed v), with the current edge and lane that Section 3.1 (vehicle
 * data) keeps per vehicle and the lane-map cell it marks.
 * Vehicle state per trip, trip order, input edge ids (host buffers of n_trips,
 * any may be NULL): edge (-1 unless active), lane, cell = floor(x) (-1 unless
 * active), x (m from the edge start) and v (m/s) (0 unless active),
 * arrival_step (-1 until arrived), status (LPSIM_WAITING/ACTIVE/ARRIVED).
 * Waits for all queued work.  Errors: ESTATE, EDEVICE. */
int32_t lpsim_get_vehicles(lpsim_ctx *ctx, int32_t *edge, uint8_t *lane, int32_t *cell,
                           float *x, float *v, int32_t *arrival_step, uint8_t *status);

/* Counters (see lpsim_counters).  Waits for all queued work. */
int32_t lpsim_get_counters(lpsim_ctx *ctx, lpsim_counters *out);

/* Test hook: a blocked edge accepts no entries, as a full downstream edge
 * (Section 3.1 Remarks, intersection modelling).  Input edge id. */
int32_t lpsim_block_edge(lpsim_ctx *ctx, int32_t edge, int32_t on);

/* Fixed-time signal plan (Algorithm 1 intersection branch: a vehicle at an
 * intersection proceeds as the node's signal allows; Section 3.3 keeps
 * signal states as local data).  The paper gives no signal model; this is a
 * fixed-time reading.  Node n runs n_phases[n] phases in turn, each
 * green[n] steps of green followed by allred[n] steps in which no phase is
 * served; at step k the cycle position is (k + offset[n]) mod cycle, with
 * cycle = n_phases[n] * (green[n] + allred[n]).  Edge e is served in phase
 * edge_phase[e] of its downstream node (-1: never stopped).  Outside its
 * green the stop line of e is a standing obstacle, as for a full entry
 * window: vehicles stop before it and make no entry request.  Departures
 * and arrivals pass no signal.
 *   n_phases, green, allred, offset   host, int32 [n_nodes]: 0..15 phases
 *       (0: no signal; the other three then ignored), green >= 1,
 *       allred >= 0, cycle <= 65535, 0 <= offset < cycle
 *   edge_phase   host, int32 [n_edges], input edge ids: -1 or a phase
 *       0..n_phases-1 of the edge's downstream node
 * Batched contexts take all scenarios' nodes and edges in input order (node
 * ids offset by node_off).  n_phases NULL removes the plan.  Arrays are
 * copied; the plan applies from the next step and survives reloads of trips
 * and state restores.  Errors: ESTATE (no network), EINVAL (the first bad
 * entry is named in lpsim_last_error), ENOMEM, EDEVICE. */
int32_t lpsim_set_signals(lpsim_ctx *ctx, const int32_t *n_phases, const int32_t *green,
                          const int32_t *allred, const int32_t *offset, const int32_t *edge_phase);

/* Launch shape: threads per block (64..1024, multiple of 64), blocks per
 * vehicle kernel (multiple of 8, up to 8192), steps captured per HIP graph
 * (>= 1; 0 launches kernels one by one).  Results do not depend on these.
 * The slots are reordered after every graph_steps steps (every 64 when
 * graph_steps is 0).  Defaults: 512 threads, 640 blocks, 64 steps per graph. */
int32_t lpsim_set_launch(lpsim_ctx *ctx, int32_t block_size, int32_t n_blocks,
                         int32_t graph_steps);

/* Autotuner: times n_steps from the current state for every pair
 * (block_sizes[i], block_counts[j]) on an internal stream with HIP events,
 * rewinding to the same state before each trial and after the last, then
 * keeps the fastest pair (graph_steps unchanged).  Results do not depend on
 * the launch shape, so only the speed changes.
 *   best_out     host, 3 int32: best block size, block count, and the trial
 *                time in microseconds per step (rounded)
 *   trial_us     host, n_bs*n_bc doubles (microseconds per step), or NULL
 * Errors: ESTATE, EINVAL (a shape outside lpsim_set_launch's limits), ENOMEM,
 * EDEVICE. */
int32_t lpsim_autotune(lpsim_ctx *ctx, int32_t n_steps, const int32_t *block_sizes, int32_t n_bs,
                       const int32_t *block_counts, int32_t n_bc, int32_t *best_out,
                       double *trial_us);

/* Kernel timing for measurement: when on, lpsim_step launches kernels one by
 * one on the work stream, each with a HIP event pair that takes the
 * dispatch's own start and end timestamps (hipExtLaunchKernel), so a phase's
 * time is its kernel's execution time; the reorder (several kernels) has an
 * event pair recorded around it.  lpsim_kernel_times then returns the summed
 * milliseconds and launch counts of the phases (0 move with the departure
 * requests, 1 resolve with the departures, 2 lane change, 3 lane-change
 * commit with the end of the step, 4 reorder).
 * Turning it on or off resets the sums. */
int32_t lpsim_set_timing(lpsim_ctx *ctx, int32_t on);
int32_t lpsim_kernel_times(lpsim_ctx *ctx, double *ms_out, int64_t *launches_out,
                           int32_t n_phases);

/* Checkpoint: size of a snapshot, save into a caller buffer, restore from it.
 * A restored context continues bit-identically.  Errors: ESTATE, EINVAL
 * (buffer too small or from another instance), EDEVICE. */
int32_t lpsim_state_size(lpsim_ctx *ctx, size_t *bytes);
int32_t lpsim_save_state(lpsim_ctx *ctx, void *host_buf, size_t bytes);
int32_t lpsim_restore_state(lpsim_ctx *ctx, const void *host_buf, size_t bytes);

/* ------------------------------------------------------------------------
 * Learned edge travel-time surrogate (the traffic-assignment use of the
 * simulator's output; the paper's title and abstract name traffic assignment
 * and travel-time estimation, it gives no surrogate): a perceptron
 *   x[32] -> 256 -> 256 -> 256 -> y[16], ReLU on the hidden layers,
 * bfloat16 operands on the matrix cores with binary32 accumulation; hidden
 * activations are rounded to bfloat16 (nearest even) after bias and ReLU.
 * All pointers are DEVICE pointers owned by the caller; `stream` is a
 * hipStream_t or NULL (the null stream); calls only enqueue work.
 * bfloat16 values are passed as uint16_t bit patterns.
 * Layer l maps in_l -> out_l with (in, out) = (32,256), (256,256), (256,256),
 * (256,16); biases [out_l] binary32, binary32 weights [out_l][in_l].
 * Fragment order: the bfloat16 matrices that the matrix cores read from
 * memory (the weight copies, the kept hidden activations, the backward's
 * gradients) are stored in the order of the MFMA operand fragments.  For a
 * matrix of R rows (the contracted index, R a multiple of 32) and C features
 * (a multiple of 16), element (r, f) sits at
 *   ((r / 32) * (C / 16) + f / 16) * 512 + (f % 16 + 16 * ((r % 32) / 8)) * 8 + r % 8,
 * so that one operand fragment is one contiguous 1 KiB read.  "wt" copy of
 * layer l: rows in_l, features out_l (read by the forward); "w" copy: rows
 * out_l padded to a multiple of 32 with zeros, features in_l (read by the
 * backward).
 * Errors: EINVAL (null pointer, negative size), EDEVICE (launch failure).
 * ------------------------------------------------------------------------ */

/* Fixed shape of the perceptron (any pointer may be NULL). */
int32_t lpsim_mlp_shape(int32_t *in_dim, int32_t *hidden, int32_t *out_dim);

/* y[n][16] = MLP(x[n][32]), x and y row-major; wt: the 4 "wt" copies.
 * h: NULL, or 3 pointers to buffers that receive the hidden activations
 * (needed by the backward) in fragment order with rows = the batch rows
 * padded to P = 64 ceil(n / 64) and 256 features, i.e. P * 256 bfloat16
 * each.  Rows n .. P-1 are written too and carry no meaning.  x and every
 * h[l] must be 16-byte aligned (EINVAL otherwise). */
int32_t lpsim_mlp_forward(const uint16_t *x, const uint16_t *const *wt, const float *const *bias, float *y,
                          uint16_t *const *h, int64_t n, void *stream);

/* Masked mean-squared-error gradient: dz_out[i] = bfloat16(2 (y[i] - t[i]) *
 * inv_count) where mask[i] (or every i if mask is NULL), else 0, over the
 * n*16 outputs; loss_sum (nullable) accumulates sum (y - t)^2 * inv_count. */
int32_t lpsim_mlp_loss_grad(const float *y, const float *target, const uint8_t *mask, int64_t n,
                            float inv_count, uint16_t *dz_out, float *loss_sum, void *stream);

/* Bytes of the `workspace` that lpsim_mlp_backward needs for n rows in
 * n_split batch slices: the data gradients and the input in fragment order,
 * then the slices' binary32 partial sums.  0 for invalid arguments (n < 0,
 * n_split outside 1..1024). */
size_t lpsim_mlp_workspace_bytes(int64_t n, int32_t n_split);

/* Backward pass of the binary32-accumulated perceptron for a batch of n rows:
 * x[n][32] and h (3 pointers) as produced by the forward, dz_out[n][16]
 * bfloat16 output gradient (row-major), w (4 pointers, the "w" copies).
 * Writes dwt (4 pointers, binary32 [out_l][in_l]) and db (4 pointers).
 * The weight gradients are summed over the rows of each of n_split
 * (1..1024) batch slices, then over the slices in order:
 * deterministic for fixed n_split.  x, dz_out, every h[l] and w[l], and
 * workspace (lpsim_mlp_workspace_bytes(n, n_split) bytes, caller-owned) must
 * be 16-byte aligned.  n = 0 writes zero gradients (kernels only, no
 * memset).  Three kernel launches. */
int32_t lpsim_mlp_backward(const uint16_t *x, const uint16_t *const *h, const uint16_t *dz_out,
                           const uint16_t *const *w, float *const *dwt, float *const *db, void *workspace,
                           int32_t n_split, int64_t n, void *stream);

/* lpsim_mlp_backward without any allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, serving loops,
 * harnesses that forbid hipMalloc): the same kernels and the same results
 * for the same n_split, with the workspace taken from a static device array
 * of the library (30.3 MiB, held by each GPU the library runs on until the
 * process ends).  Arguments as lpsim_mlp_backward without workspace.
 * Limits: n <= 8192 rows, n_split <= 32, else LPSIM_ECAPACITY.  All calls on
 * one GPU share its array, so calls that overlap on one GPU (different
 * streams, or threads) race; calls in one stream's order do not.
 * Errors: EINVAL, ECAPACITY, EDEVICE. */
int32_t lpsim_mlp_backward_noalloc(const uint16_t *x, const uint16_t *const *h, const uint16_t *dz_out,
                                   const uint16_t *const *w, float *const *dwt, float *const *db,
                                   int32_t n_split, int64_t n, void *stream);

/* Adam step (Kingma & Ba) on one binary32 matrix [rows][cols] = [out][in]
 * (a bias is rows = 1): m, v moment buffers, t = step count from 1.  Also
 * writes the bfloat16 copies in fragment order: wt_bf16 (rows cols, features
 * rows) and w_bf16 (rows `rows` padded to 32, features cols), either may be
 * NULL; the padding entries of w_bf16 are never written (the caller zeroes
 * them once). */
int32_t lpsim_mlp_adam(float *w, uint16_t *wt_bf16, uint16_t *w_bf16, const float *grad, float *m, float *v,
                       int32_t rows, int32_t cols, float lr, float beta1, float beta2, float eps, int32_t t,
                       void *stream);

/* ------------------------------------------------------------------------
 * Traffic assignment around the simulator (the paper's title names traffic
 * assignment; routes are the simulator's input,
 * Section 3.1 vehicle data).  The method of successive averages alternates
 * evaluation of edge travel times (full simulation, or the surrogate) with
 * shortest-time routing.
 * ------------------------------------------------------------------------ */

typedef struct lpsim_router lpsim_router;

/* Router over a directed graph (host arrays, copied).  n_threads <= 0 uses
 * every hardware thread.  Errors: EINVAL, ENOMEM. */
int32_t lpsim_router_create(int32_t n_nodes, int32_t n_edges, const int32_t *src, const int32_t *dst,
                            int32_t n_threads, lpsim_router **out);
void lpsim_router_destroy(lpsim_router *r);

/* Shortest-time route of every trip origin[i] -> dest[i] (host arrays) for
 * the edge costs `cost` (host, seconds, finite and > 0), by backward Dijkstra
 * per distinct destination in float64; among equally short choices the lower
 * edge id is taken.  Errors: EINVAL (bad ids, origin == destination,
 * unreachable destination, bad cost), ENOMEM. */
int32_t lpsim_router_solve(lpsim_router *r, const double *cost, int64_t n_trips, const int32_t *origin,
                           const int32_t *dest);

/* lpsim_router_solve with the trees computed on the current GPU: the same
 * fixed point dist[x] = min over out-edges e = (x -> y) of dist[y] + cost[e]
 * in float64, the same lowest-edge-id rule among equally short choices, so
 * the same routes.  Label-correcting relaxation over (destination, node)
 * pairs with 64-bit atomic minima and a near-far split of the frontier, then
 * one pass that picks each node's tree edge.  The trees stay on the device:
 * lpsim_router_fill after this call walks them there and copies the routes
 * back.  `stream` is a hipStream_t or NULL; the call returns when the solve
 * is done.  Device memory for the graph and the trees, and page-locked host
 * buffers for the routes coming back, are kept until lpsim_router_destroy.
 * Errors: as lpsim_router_solve, and EDEVICE. */
int32_t lpsim_router_solve_gpu(lpsim_router *r, const double *cost, int64_t n_trips, const int32_t *origin,
                               const int32_t *dest, void *stream);

/* The method of successive averages' deterministic switch: take[i] = 1
 * iff SplitMix64(seed ^ (i << 8) ^ n) mod (n + 1) == 0, so about 1/(n+1)
 * of the trips move to their new route at iteration n (1-based).  Host
 * buffer of n_trips.  Errors: EINVAL. */
int32_t lpsim_msa_switch(int64_t n_trips, int32_t n, uint64_t seed, uint8_t *take);

/* Routing cost of each edge from the statistics (lpsim_edge_stats): mean
 * travel time tt_sum_steps / n_exits, or tt_free_steps where nothing
 * exited, at least one step, times dt, in seconds (host arrays). */
int32_t lpsim_edge_tt(int32_t n_edges, const int64_t *tt_sum_steps, const int32_t *n_exits,
                      const double *tt_free_steps, double dt, double *out_s);

/* Mean travel time per (edge, bin) in steps, [E][B] float32: tt_sum_bin /
 * exits_bin in float64 rounded once, or the edge's tt_free_steps where no
 * traversal entered in the bin (host arrays). */
int32_t lpsim_edge_tt_bins(int32_t n_edges, int32_t n_bins, const int64_t *tt_sum_bin, const int32_t *exits_bin,
                           const double *tt_free_steps, float *out_steps);

/* lpsim_edge_tt_bins on device arrays, queued on `stream` (hipStream_t or
 * NULL): the same float64 quotient rounded once, so the same values.
 * Errors: EINVAL, EDEVICE. */
int32_t lpsim_edge_tt_bins_device(int32_t n_edges, int32_t n_bins, const int64_t *tt_sum_bin, const int32_t *exits_bin,
                                  const double *tt_free_steps, float *out_steps, void *stream);

/* Write the routes of the last solve (host buffers).  take_new (n_trips
 * flags) NULL takes every new route; otherwise trip i keeps its old route
 * (old_off / old_edges) where take_new[i] == 0.  out_off receives n_trips+1
 * offsets; out_edges (may be NULL to size the result first) the edge ids;
 * out_edges must not overlap old_edges.  After a GPU solve, a call that
 * follows a sizing call for the same take_new contents reuses its route
 * lengths instead of walking the trees again.
 * Errors: ESTATE (no solve), EINVAL (also for old offsets that decrease
 * over a kept route); after a GPU solve also ENOMEM and EDEVICE. */
int32_t lpsim_router_fill(lpsim_router *r, const int64_t *old_off, const int32_t *old_edges, const uint8_t *take_new,
                          int64_t *out_off, int32_t *out_edges);

/* Network loading for the surrogate (device arrays): each trip walks its
 * route from step depart+1, spending max(1, round(tt_steps[e][bin])) steps on
 * an edge entered in `bin`, until `horizon`.  Writes entries per entry bin
 * (inflow_bin, [E][B] int32) and vehicle-steps per bin (occ_steps_bin,
 * [E][B] int64), both zeroed first; exact integers.  route_off [n+1] int64,
 * route_edges int32 (input edge ids). */
int32_t lpsim_surrogate_load(const int64_t *route_off, const int32_t *route_edges, const int32_t *depart_step,
                             int64_t n_trips, const float *tt_steps, int32_t n_edges, int32_t n_bins,
                             int32_t bin_steps, int32_t horizon, int32_t *inflow_bin, int64_t *occ_steps_bin,
                             void *stream);

/* Perceptron inputs for every (edge, window of 12 bins), device arrays:
 * x_out [E * B/12][32] bfloat16 = log1p(inflow) x12, occupancy / (bin_steps *
 * ceil(length) * lanes) * jam_spacing x12, log(length), lanes/4, speed/22.4,
 * zeros.  n_bins must be a multiple of 12. */
int32_t lpsim_surrogate_features(int32_t n_edges, int32_t n_bins, int32_t bin_steps, float jam_spacing,
                                 const int32_t *inflow_bin, const int64_t *occ_steps_bin, const float *length_m,
                                 const uint8_t *lanes, const float *speed_mps, uint16_t *x_out, void *stream);

/* Training targets from simulator statistics (device arrays):
 * y_out [E * B/12][16] = log(tt_sum_bin / exits_bin / tt_free_steps) per bin
 * of the window, mask_out 1 where exits_bin > 0 (outputs 12..15 masked). */
int32_t lpsim_surrogate_targets(int32_t n_edges, int32_t n_bins, const int32_t *exits_bin, const int64_t *tt_sum_bin,
                                const float *tt_free_steps, float *y_out, uint8_t *mask_out, void *stream);

/* Damped travel-time update from predictions (device arrays):
 * tt_steps[e][b] <- (1-damping) tt + damping clamp(tt_free exp(y), 1, tt_max). */
int32_t lpsim_surrogate_tt(int32_t n_edges, int32_t n_bins, const float *y_pred, const float *tt_free_steps,
                           float damping, float tt_max, float *tt_steps, void *stream);

/* Anchored travel-time estimate for new routes (device arrays): the last
 * simulated travel time of each (edge, bin), anchor_tt_steps [E][B], moved by
 * the perceptron's predicted change of log travel time between the anchor's
 * loading and the new loading (y_new, y_anchor: [E * B/12][16] outputs of
 * lpsim_mlp_forward), the change clamped to [-max_shift, max_shift]:
 *   tt_steps_out[e][b] = clamp(anchor * exp(dy), 1, tt_max).
 * Errors: EINVAL (null pointer, bad sizes, max_shift < 0, tt_max < 1). */
int32_t lpsim_surrogate_shift(int32_t n_edges, int32_t n_bins, const float *y_new, const float *y_anchor,
                              const float *anchor_tt_steps, float max_shift, float tt_max, float *tt_steps_out,
                              void *stream);

/* Routing cost per edge in seconds (device arrays; edge_tt_s [E] float64):
 * the inflow-weighted mean over bins of tt_steps, or tt_free_steps where the
 * edge has no inflow, at least one step, times dt.  Errors: EINVAL. */
int32_t lpsim_surrogate_edge_tt(int32_t n_edges, int32_t n_bins, const int32_t *inflow_bin, const float *tt_steps,
                                const float *tt_free_steps, float dt, double *edge_tt_s, void *stream);

/* Derived constants: 0 -> entry window W (cells), 1 -> look-ahead D (cells)
 * of scenario 0, 2 -> steps per statistics bin. */
int32_t lpsim_query(const lpsim_ctx *ctx, int32_t which);

/* Last error text of this context ("" if none).  Accepts NULL. */
const char *lpsim_last_error(const lpsim_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* LPSIM_H */
