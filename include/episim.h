/*
 * episim: per-day hot path of the event-based epidemic framework of
 * Bauer, Engblom & Widgren, "Fast event-based epidemiological simulations on
 * national scales" (arXiv:1502.02908), on one AMD Instinct MI355X (gfx950).
 *
 * Each simulated day d (the window [d, d+1)) does, for every node and every
 * replicate trajectory:
 *   1. the stochastic step: Gillespie's direct method per node with the
 *      continuous state frozen (Sec. 3.1 eq:numstep3; Sec. 3.3, eq:sampling,
 *      eq:sampling2; Algorithm 1);
 *   2. the deterministic step: the externally defined events of day d in list
 *      order (eq:numstep4; Sec. 3.2, eq:event);
 *   3. the continuous-state update, forward Euler with dt = 1 for the
 *      environmental infectious pressure phi (eq:numstep5, eq:siminfpressure,
 *      the seasonal beta(t) of Sec. 4.1);
 *   4. the daily record (prevalence, compartment totals, SSA transitions, and
 *      snapshots of u and phi on requested days).
 *
 * Conventions shared by every entry point:
 *  - Plain C types only. Pointers named "host" are host memory; the library
 *    owns all device memory unless a workspace is passed in sim_device_opts.
 *  - Every function returns SIM_OK (0) or a negative SIM_E* code; nothing
 *    partial is ever reported as success. sim_last_error() gives the text.
 *  - Randomness: one Philox4x32-10 block (Salmon et al., SC'11) per SSA
 *    attempt with counter (k, node, day, 0) and key (seed, replicate id); the
 *    q-th individual drawn by event g uses counter (q/2, g, day, 1). Results
 *    are therefore a fixed function of the inputs, independent of launch
 *    shape, level grouping and batching.
 *  - Floating point: binary64 throughout, no contraction, fixed operation
 *    order; -log(rand) is a fixed sequence of + - * / (no libm).
 *  - A handle is not thread-safe; distinct handles are independent.
 */
#ifndef EPISIM_H
#define EPISIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SIM_OK           0
#define SIM_EINVAL      -1  /* an argument violates the contract below */
#define SIM_ENOMEM      -2  /* host or device allocation failed */
#define SIM_EDEVICE     -3  /* a HIP runtime call failed (message has hipGetErrorString) */
#define SIM_EINFEASIBLE -4  /* an event asked for more individuals than the selected compartments hold */
#define SIM_ESTATE      -5  /* run past the horizon, or a call out of order */
#define SIM_ELIMIT      -6  /* a node exceeded SIM_MAX_FIRED SSA transitions in one day (rates too large) */

#define SIM_MAX_COMP  8
#define SIM_MAX_TRANS 8
#define SIM_MAX_EVENT_N (1 << 24)   /* largest n of one event */
#define SIM_MAX_FIRED   (1 << 24)   /* largest number of SSA transitions of one node in one day */
#define SIM_MAX_REGIONS 4096        /* largest number of regions of the goal function */

/* Event kinds (Sec. 3.2: E1 = one node, E2 = two nodes). */
#define SIM_EXIT     0  /* E1: remove n individuals sampled from the selected compartments */
#define SIM_ENTER    1  /* E1: add n individuals to the single selected compartment */
#define SIM_INTERNAL 2  /* E1: move n sampled individuals within the node by the shift column */
#define SIM_EXTERNAL 3  /* E2: move n sampled individuals from node to dest (shifted if shift >= 0) */

/*
 * The problem statement (Sec. 2.1-2.3, Sec. 3.2). All pointers are host
 * memory, read only during sim_create, owned by the caller.
 *
 *  n_nodes, n_comp, n_trans   Nn, Nc (1..8), Nt (1..8).
 *  n_rep                      R >= 1 independent trajectories of the same network.
 *  n_days                     horizon D >= 0 (windows [d, d+1), d = 0..D-1).
 *  day0                       calendar day of simulation day 0; beta is taken at t = day0 + d.
 *  u0[Nn*Nc]                  initial X (Sec. 2.2), node-major: u0[c + Nc*i] >= 0.
 *  v0[Nn]                     initial phi >= 0 (Y with one row, Sec. 2.3).
 *  S[Nc*Nt]                   stoichiometry, S[c*Nt + k] (eq:vectorJSDE). Column k must hold
 *                             -1 at reactant[k] and be >= 0 elsewhere (keeps X >= 0).
 *  reactant[Nt], uses_phi[Nt] rate k = coef[r*Nt+k] * (phi if uses_phi[k]) * X[reactant[k]]
 *                             (Sec. 3.3 omega_n; eq:rate_s_to_i, eq:recovery_rates).
 *  coef[R*Nt] >= 0            per-replicate rate constants.
 *  alpha[R] >= 0, beta[R*4]   phi' = (1 - beta_q) phi + alpha I/N (eq:siminfpressure, Euler dt = 1);
 *                             beta in [0,1]; q = season of (day0+d) mod 365 per Sec. 4.1.
 *  phi_I_mask, phi_N_mask     bit c set: compartment c counts in I (infected) / in N (node size).
 *  E[Nc*n_select]             select matrix, E[c*n_select + s] in {0,1}.
 *  N[Nc*n_shift]              shift matrix: a moved individual of compartment c lands in
 *                             c + N[c*n_shift + h] (must stay in [0, Nc)).
 *  events (n_events < 2^31, sorted by day; order within a day is the semantic order):
 *    ev_day in [0,D), ev_kind SIM_*, ev_node in [0,Nn), ev_dest in [0,Nn) for EXTERNAL
 *    (ignored otherwise), 0 <= ev_n <= SIM_MAX_EVENT_N, ev_select in [0,n_select) (ENTER: exactly one
 *    compartment), ev_shift in [-1,n_shift) (-1 = none).
 *  record_days[n_record]      strictly ascending days in [0,D) whose end state is snapshotted.
 *  seed, replicate_id[R]      Philox key words; replicate_id NULL means 0..R-1.
 *  reactant2[Nt]              NULL, or per transition a second reactant in [0,Nc) or -1: a
 *                             mass-action rate is also multiplied by X[reactant2[k]] (the
 *                             bimolecular rate of the SIR example, Sec. 2.1).
 *  phi_pre_events             0: phi is updated from the state after the day's events (Algorithm
 *                             1, the default); 1: from the state after the SSA and before the
 *                             events (eq:numstep5 as written). Records are taken after the events
 *                             either way.
 *  n_regions, region[Nn]      regions of the goal function (Sec. 4.3): region[i] in [0, n_regions) or
 *                             -1; with n_regions > 0 the daily regional sums are recorded.
 */
typedef struct sim_problem {
    int32_t n_nodes, n_comp, n_trans, n_rep, n_days, day0;
    const int32_t *u0;
    const double *v0;
    const int32_t *S, *reactant, *uses_phi;
    const double *coef, *alpha, *beta;
    uint32_t phi_I_mask, phi_N_mask;
    int32_t n_select;
    const int32_t *E;
    int32_t n_shift;
    const int32_t *N;
    int64_t n_events;
    const int32_t *ev_day, *ev_kind, *ev_node, *ev_dest, *ev_n, *ev_select, *ev_shift;
    int32_t n_record;
    const int32_t *record_days;
    uint32_t seed;
    const uint32_t *replicate_id;
    const int32_t *reactant2;
    int32_t phi_pre_events;
    int32_t n_regions;
    const int32_t *region;
} sim_problem;

/* Execution of the event phase. */
#define SIM_EVENTS_LEVELS  0  /* conflict-free levels from the dependency pass (default) */
#define SIM_EVENTS_SERIAL  1  /* one event per level, in list order (validation mode) */

/* Device options. stream is a hipStream_t (NULL = the null stream). If
 * workspace is non-NULL it is device memory of at least
 * sim_workspace_bytes(p, o) bytes owned by the caller, kept alive until
 * sim_destroy; otherwise the library allocates. */
typedef struct sim_device_opts {
    void *stream;
    void *workspace;
    size_t workspace_bytes;
    int32_t events_mode;   /* SIM_EVENTS_* */
    int32_t block;         /* threads per workgroup for node kernels: 0 or 256 (the kernels are built for 256) */
    int32_t launch;        /* SIM_LAUNCH_*: how days are issued */
    int32_t group_herds;   /* with one lane per node and per-day launches, the largest herds per instance of
                              at least 8192 nodes whose chains a whole workgroup walks: 0 = default (4),
                              negative = none, at most 16 */
    int32_t small_level;   /* per-day launches: event levels of at most this many (event, replicate) tasks
                              run several per launch in one workgroup: 0 = default (512) */
    int32_t tile_nodes;    /* replicate tiles (R > 1): node positions per tile of 64 replicate lanes, which the
                              tile's four wavefronts take one at a time: 0 = default (128), else a power of two in
                              [4, 512]. With one replicate (R = 1) a nonzero value selects tiles as well: each
                              wavefront then walks one node's chain at a time with all its lanes (for networks
                              of few nodes with long chains); 0 keeps one lane per node */
    int32_t heavy_herds;   /* replicate tiles with per-day launches: the largest herds per instance (at most one per
                              64 nodes) whose every (herd, replicate) chain gets a wavefront of its own: 0 = default
                              (64), negative = none, at most 256 */
    int32_t few_chains;    /* at most this many live chains of a wavefront, one of them still expecting many
                              attempts, are walked one after another by the whole wavefront: 0 = default (4),
                              negative = never, at most 64 */
    int32_t group_min_attempts; /* one lane per node with per-day launches: a workgroup walks one herd's chain
                              while it still expects this many attempts in the day: 0 = default (4096) */
    int32_t slot_lanes;    /* slot handles: replicate lanes per slot, 8, 16, 32 or 64 (0 = 64); n_slots times
                              slot_lanes must be a multiple of 64 */
} sim_device_opts;

#define SIM_LAUNCH_KERNELS    0  /* one launch per day phase and per event level (default) */
#define SIM_LAUNCH_PERSISTENT 1  /* one cooperative launch per sim_run, grid barriers between phases */

/* Outputs, host memory owned by the caller; any pointer may be NULL.
 *   prevalence[D*R]       nodes with sum over phi_I_mask > 0 after day d's events, [d][r]
 *   transitions[D*R]      SSA transitions applied on day d, [d][r]
 *   totals[D*R*Nc]        sum over nodes of each compartment after day d, [d][r][c]
 *   snap_u[n_record*R*Nn*Nc], snap_v[n_record*R*Nn]
 *                         u and phi at the end of each record day, [k][r][i][c] / [k][r][i]
 *   regional[D*R*n_regions*Nc]
 *                         X summed over the nodes of each region after day d's events, [d][r][j][c]
 *                         (the inner sum of eq:goal for one sample trajectory)
 *   max_transitions[D*R]  the most SSA transitions one node applied on day d, [d][r]: the
 *                         length of the day's longest chain of Algorithm 1's inner loop
 * Days not yet simulated read as 0. */
typedef struct sim_output {
    int32_t *prevalence;
    int64_t *transitions;
    int64_t *totals;
    int32_t *snap_u;
    double *snap_v;
    int64_t *regional;
    int32_t *max_transitions;
} sim_output;

typedef struct sim_handle sim_handle;

/* Device bytes a handle for p with options o (NULL = defaults) needs, for a
 * caller-owned workspace. 0 if p or o is invalid. */
size_t sim_workspace_bytes(const sim_problem *p, const sim_device_opts *o);

/* Validate p, run the dependency pass over the events (conflict-free levels
 * per day, Sec. 3.4's re-arrangement of the event lists done once), copy
 * everything to the device, set the state to (u0, v0) at day 0.
 * o may be NULL (defaults). On failure *out is NULL and sim_last_error(NULL)
 * describes it (thread-local). */
int sim_create(const sim_problem *p, const sim_device_opts *o, sim_handle **out);

/* One handle for several instances of one model (the problems share n_comp,
 * n_trans, S, reactant, uses_phi, the phi masks, E, N, n_rep, n_days, day0 and
 * record_days; they differ in nodes, state, rates, events, seed and
 * replicate ids). Their nodes run in the same launches; every random stream
 * uses the instance's own node numbers, event numbers and seed, so each
 * instance follows exactly the trajectory it follows alone (the paper's
 * fitting workload of many trajectories over one event database, Sec. 4.3).
 * Records are indexed by set = instance * n_rep + replicate:
 * prevalence[D * n_problems * n_rep] etc. State, snapshots and get/set_state
 * use the instances' nodes concatenated in order: [r][node][c]. */
int sim_create_batch(const sim_problem *const *problems, int32_t n_problems, const sim_device_opts *o,
                     sim_handle **out);
size_t sim_workspace_bytes_batch(const sim_problem *const *problems, int32_t n_problems,
                                 const sim_device_opts *o);

/* Enqueue days [day, day + n_days) on the handle's stream (n_days = 0: to the
 * horizon): each day is one pass of Algorithm 1's outer loop (Sec. 3.1, the
 * splitting eq:numstep3 -> eq:numstep4 -> eq:numstep5): the SSA of every node
 * over the window, the day's events in list order, then the phi update.
 * Asynchronous: device-side errors (SIM_EINFEASIBLE) are reported by the next
 * synchronising call. SIM_ESTATE past the horizon. */
int sim_run(sim_handle *h, int32_t n_days);

/* Wait for the handle's work; returns the first device-side error, if any.
 * For SIM_EINFEASIBLE the message names the smallest event index, its
 * replicate and day. */
int sim_sync(sim_handle *h);

/* Copy the daily records (all D days) to the caller's buffers; synchronises.
 * The records are the outputs of Algorithm 1's loop read after each day's
 * events: node prevalence and compartment totals of X (Sec. 2.2), the SSA
 * transitions of the day (Sec. 3.3), snapshots of X and Y (Sec. 2.3). */
int sim_trajectory(sim_handle *h, sim_output *out);

/* Checkpoint: u[R*Nn*Nc] ([r][i][c]), v[R*Nn], and the next day to simulate.
 * The state (X, Y) at a window boundary is all Algorithm 1 carries from one
 * window to the next (the clock is redrawn in every window, Sec. 3.3), so a
 * run resumed from it is bit-identical to one that never stopped.
 * Synchronises. sim_set_state restores; the records of days >= day are
 * recomputed by later runs. */
int sim_get_state(sim_handle *h, int32_t *u, double *v, int32_t *day);
int sim_set_state(sim_handle *h, const int32_t *u, const double *v, int32_t day);

/* Statistics of the dependency pass: number of levels of day d (or the sum
 * over days if d < 0), and the largest over days in *max_levels. */
int64_t sim_levels(const sim_handle *h, int32_t d, int32_t *max_levels);

/* Kernel timing on the handle's stream. enable = 1 starts bracketing every
 * launch issued by later sim_run calls with HIP events (enable = 0 stops and
 * keeps the totals; enable = -1 clears them). The call synchronises and
 * writes, per kernel class SIM_K_DAY (per-day SSA + phi kernel),
 * SIM_K_EVENTS (one event level), SIM_K_CLOSE (the closing phi update) and
 * SIM_K_PERSIST (a whole persistent run), the summed milliseconds in ms[4]
 * and the number of launches in launches[4] (either may be NULL). */
#define SIM_K_DAY     0
#define SIM_K_EVENTS  1
#define SIM_K_CLOSE   2
#define SIM_K_PERSIST 3
int sim_kernel_times(sim_handle *h, int32_t enable, double *ms, int64_t *launches);

/* ---- Slot handles: many requests over one resident network ------------
 * The paper's fitting workload runs many trajectories, with different rate
 * parameters, over one event database (Sec. 4.3). A slot handle keeps one
 * network resident (nodes, initial state, events and their levels) and
 * n_slots slots of slot_lanes (sim_device_opts; 64 by default) replicate
 * lanes each. Every slot runs its own request
 * (its replicates, parameters and horizon) from its own day 0, while one
 * sim_slots_step advances all running slots by one day in shared launches:
 * the steps of the method (Alg. 1: SSA, then the day's events, then the phi
 * update) are those of sim_run, so a request's records are bit-identical to a
 * plain handle of the same network, replicates, parameters and replicate ids
 * run for the same number of days. Random streams are keyed by the network's
 * seed and the request's replicate ids, never by the slot.
 * The network problem's n_rep, rates and replicate ids are not used and
 * n_record must be 0; events_mode must be SIM_EVENTS_LEVELS. All calls on one
 * handle must come from one thread. */
size_t sim_slots_workspace_bytes(const sim_problem *network, int32_t n_slots, const sim_device_opts *o);
int sim_slots_create(const sim_problem *network, int32_t n_slots, const sim_device_opts *o, sim_handle **out);

/* Start a request in a slot that is not running (free, or finished and
 * fetched or abandoned): n_rep in [1, slot_lanes] replicates with rate constants
 * coef[n_rep*Nt], shedding rates alpha[n_rep], decay rates beta[n_rep*4] and
 * replicate_id[n_rep] (NULL: 0..n_rep-1), for horizon days in [1, D]. The
 * parameters are copied before the call returns; the slot's lanes are loaded
 * with (u0, v0) on the stream. Its day 0 runs in the next sim_slots_step. */
int sim_slot_start(sim_handle *h, int32_t slot, int32_t n_rep, int32_t horizon, const double *coef,
                   const double *alpha, const double *beta, const uint32_t *replicate_id);

/* Enqueue one day of every running slot (asynchronous). The slots whose
 * horizon this step completes (their last day closed) are written to
 * finished[] (room for n_slots) and counted in *n_finished; either may be
 * NULL. No running slot: nothing is enqueued. */
int sim_slots_step(sim_handle *h, int32_t *finished, int32_t *n_finished);

/* Number of enqueued steps the device has not finished (never blocks); -1 if
 * h is not a slot handle. Lets a caller bound how far it runs ahead. */
int32_t sim_slots_in_flight(sim_handle *h);

/* Enqueue the download of a finished slot's records, days [0, horizon):
 * prevalence[horizon*n_rep] and transitions[horizon*n_rep] as [d][r],
 * totals[horizon*n_rep*Nc] as [d][r][c] (any may be NULL). Host buffers from
 * hipHostMalloc keep the call asynchronous; others make it synchronous. The
 * buffers must stay valid until sim_slot_query returns other than 1. The
 * slot is free for sim_slot_start right after this call. */
int sim_slot_fetch(sim_handle *h, int32_t slot, int32_t *prevalence, int64_t *transitions, int64_t *totals);

/* Collect a fetch (never blocks): 1 while the download is in flight, then
 * SIM_OK, or the slot's own device-side error (SIM_EINFEASIBLE naming the
 * merged event index, replicate and day; SIM_ELIMIT). */
int sim_slot_query(sim_handle *h, int32_t slot);

/* The slot's current state after all enqueued work (synchronises):
 * u[n_rep*Nn*Nc] as [r][i][c], v[n_rep*Nn] as [r][i]. */
int sim_slot_state(sim_handle *h, int32_t slot, int32_t *u, double *v);

/* Goal function of the parameter-fitting study (Sec. 4.3): the R replicates of
 * `instance` are the N sample trajectories of one parameter vector and
 * reference[D*n_regions*Nc] ([d][j][c], host memory) holds the regional sums
 * of the reference trajectory. Over days [d_begin, d_end), already simulated,
 * with the integral over t taken as the sum over days:
 *   G2  = sum_d sum_j || mean_i x_ij(d) - ref_j(d) ||^2               (eq:goal)
 *   VG2 = sum_d sum_j (1/(N-1)) sum_i || x_ij(d) - mean_j(d) ||^2     (eq:goalvariance,
 *                                                                      eq:goalsigma; 0 if N = 1)
 * The per-day sums are reduced on the device, the days added in order on the
 * host. Synchronises. SIM_ESTATE without regions or for days not simulated. */
int sim_goal(sim_handle *h, int32_t instance, const int64_t *reference, int32_t d_begin, int32_t d_end,
             double *G2, double *VG2);

/* sim_goal for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same arguments, checks and results, bit for bit, but the staged reference,
 * the per-day terms and their sums live in a static array of the library in
 * each GPU's memory (8 MiB, held until the process ends), and the days are
 * added in order on the device. Nothing is allocated, on the device or by the
 * runtime on its behalf. The current device must be the one the handle was
 * created on. SIM_EINVAL if the range needs more than the array holds
 * (8 bytes per regional sum and day, plus 16 per day). Every call on one GPU
 * uses the same array and overwrites all of it that it reads: calls that
 * overlap on one GPU (other threads, other streams) race and must be
 * serialised by the caller. Synchronises the handle's stream. */
int sim_goal_noalloc(sim_handle *h, int32_t instance, const int64_t *reference, int32_t d_begin, int32_t d_end,
                     double *G2, double *VG2);

/* Release all resources. NULL is a no-op. */
void sim_destroy(sim_handle *h);

/* Text of the last error of h, or of the calling thread's last sim_create if h is NULL. */
const char *sim_last_error(const sim_handle *h);

/* Host-only dependency pass, exposed for testing without a GPU. Groups the
 * events into tasks and assigns each task a level (1-based) within its day:
 * a task is one external transfer, or a run of enter / exit / internal
 * events of one node with no external transfer touching that node between
 * them in list order; one thread applies a task's events in list order.
 * Any two events of one day that touch a common node, at least one of them
 * drawing individuals there, are in one task or in increasing levels in list
 * order, while additions to one node may share a level. level_out[n_events]
 * and task_out[n_events] (task numbers in order of their first event; may be
 * NULL). Returns SIM_OK or SIM_EINVAL. */
int sim_plan_levels(int64_t n_events, const int32_t *ev_day, const int32_t *ev_kind,
                    const int32_t *ev_node, const int32_t *ev_dest, int32_t n_nodes,
                    int32_t *level_out, int32_t *task_out);

#ifdef __cplusplus
}
#endif
#endif /* EPISIM_H */
