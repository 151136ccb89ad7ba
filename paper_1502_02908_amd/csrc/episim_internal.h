// Internal layout shared by the host side (episim_host.cpp) and the gfx950
// kernels (episim_device.hip) of the library. Not part of the public ABI.
//
// Device data layout (one handle = one network, R replicate trajectories):
//   lane l = pos * RL + r (replicate fastest), L = Np * RL lanes, where pos is
//   the node's position: nodes are reordered so that the largest herds (the
//   longest SSA chains) sit in different wavefronts, largest first;
//   node_id[pos] gives the caller's numbering (used for the random streams)
//   u[c * L + l]        int32 compartment counts, compartment-major (SoA) so
//                       that a wavefront's loads of one compartment coalesce
//   phi[l]              binary64 environmental infectious pressure
//   events              SoA in execution order (day, then level, then task,
//                       then list order), 28 bytes per event: global index g,
//                       merged index, node, dest, n, packed meta (kind,
//                       select mask, shift id), compartment map of the shift
#pragma once
#include <cstdint>

namespace episim {

constexpr int MAXC = 8;
constexpr int MAXT = 8;
constexpr unsigned long long STATUS_OK = ~0ull;  // else (g << 32) | replicate of an infeasible event
constexpr unsigned long long STATUS_LIMIT_TAG = 0xFFFFFFFEull;  // high word when a node hit SIM_MAX_FIRED

// meta word of an event: bits 0-1 kind, bits 2-9 select mask, bits 10-15 shift id + 1 (0 = none),
// bit 16 set when the event continues the task of the event before it
__host__ __device__ inline uint32_t meta_pack(int kind, uint32_t mask, int shift) {
    return (uint32_t)kind | (mask << 2) | ((uint32_t)(shift + 1) << 10);
}
constexpr int MAX_SHIFT_IDS = 63;
constexpr uint32_t kMetaCont = 1u << 16;

// Model description, passed by value (lands in the kernel-argument segment,
// read with scalar loads).
struct Model {
    int32_t nc, nt;
    int32_t pairs;              // 1: compartments [S1,I1,...], transitions S_p<->I_p (see PairRules)
    int32_t day0;
    uint32_t seed;
    uint32_t uses_phi;          // bit k: rate k proportional to phi
    uint32_t imask, nmask;      // compartments counted in I and in N
    int32_t reactant[MAXT];
    int32_t reactant2[MAXT];    // second reactant of a mass-action rate, -1 if none
    int32_t phi_pre;            // 1: phi from the state after the SSA, before the events
    int32_t S[MAXC][MAXT];      // S[c][k]
};

// One slot of a slot handle: the handle step at which the slot's day 0 runs
// (-1: never started), its replicate count (lanes W slot .. W slot + n_rep - 1
// for slots of W lanes) and its horizon in days.
struct SlotInfo {
    int32_t t0, n_rep, horizon, pad;
};

// A handle holds n_inst instances (networks) of one model, each run with the
// same number R of replicates; "set" = inst * R + r indexes everything that
// belongs to one trajectory (parameters, replicate id, records). A slot
// handle holds one network and RL / slot_lanes slots with R = RL sets; each
// slot runs its own request at its own day.
struct DevState {
    int32_t *u;                 // [nc][L]
    double *phi;                // [L]
    int64_t L;                  // Np * RL, Np = positions (nodes of all instances plus padding)
    int32_t Np, R;              // R replicates per instance
    int32_t RL;                 // lane stride per position: R, or R rounded up to 64 (lanes r >= R are idle)
    int32_t n_days;
    int32_t n_inst;
    int32_t n_nodes;            // nodes of all instances (no padding), for the snapshot layout
    const int32_t *node_id;     // [Np] node number within its instance, -1 for padding
    const int32_t *inst;        // [Np] instance of each position
    const int32_t *inst_off;    // [n_inst] first node of each instance in the concatenated numbering
    const uint32_t *seed;       // [n_inst] first Philox key word of each instance
    const double *coef;         // [sets][nt]
    const double *alpha;        // [sets]
    const double *beta;         // [sets][4]
    const uint32_t *repid;      // [sets] second Philox key word
    unsigned long long *status; // first infeasible event, or STATUS_OK ([RL / slot_lanes] in a slot handle)
    SlotInfo *slots;            // [RL / slot_lanes] slot table of a slot handle, null otherwise
    // slot handles, rewritten before every step: the slots with a day of events
    // to run and the 64-lane columns with a lane that runs, each ascending; the
    // step's launches cover only these (grid y = their count)
    const int32_t *run_slots;   // [RL / slot_lanes]
    const int32_t *run_cols;    // [RL / 64]
    // replicate tiles: the herds whose every (herd, replicate) chain gets a
    // wavefront of its own, and the units that hold only such herds
    int32_t tile_nodes;         // positions of one replicate tile (a power of two, 32 .. 512)
    int32_t slot_lanes;         // slot handles: replicate lanes of one slot (8, 16, 32 or 64)
    uint32_t few_chains;        // at most this many live chains of a wavefront are walked one after another
    double group_min_attempts;  // a workgroup walks one chain while it expects this many attempts
    int32_t n_heavy;
    const int32_t *heavy_pos;   // [n_heavy]
    const uint8_t *unit_heavy;  // [n_units], null if n_heavy == 0
    const uint8_t *unit_group;  // [n_units]: one lane per node, the unit's first herd is walked by the whole workgroup
    // daily records
    int32_t *prevalence;        // [D][sets]
    int64_t *transitions;       // [D][sets]
    int64_t *totals;            // [D][sets][nc]
    int32_t *max_fired;         // [D][sets] most SSA transitions of one node on the day
    int32_t *snap_u;            // [n_record][R][n_nodes][nc]
    double *snap_v;             // [n_record][R][n_nodes]
    const int32_t *rec_slot;    // [D] snapshot slot of day d, or -1
    int32_t n_regions;          // regions of the goal function's aggregates (0: none)
    const int32_t *pos_region;  // [Np] region of each position, -1 outside regions
    int64_t *regional;          // [D][sets][n_regions][nc] compartment sums per region
};

struct DevEvents {
    const int32_t *g;           // index of the event within its instance's list (random stream)
    const int32_t *gm;          // index in the merged list of all instances (error report)
    const int32_t *node;
    const int32_t *dest;
    const int32_t *n;
    const uint32_t *meta;
    const uint32_t *smap;       // per event: landing compartment of each source compartment, 4 bits each
    const int32_t *task_off;    // task boundaries into the arrays above (a task's events in list order)
    const int64_t *lvl_off;     // level boundaries into the tasks
    const int32_t *priv_off;    // [D * n_units + 1]: private tasks of unit u on day d are
                                // priv_off[d * n_units + u] .. priv_off[d * n_units + u + 1] - 1
    const int32_t *priv_ev_off; // [D * n_units + 1]: their events, contiguous, in the same numbering
    // days run in LDS (one lane per node): the positions their level tasks touch
    // are slot_pos[day_slot_off[d]] ..; slot_src / slot_dst give each event's
    // slot of its node / destination on such a day, -1 otherwise
    const int32_t *day_slot_off;
    const int32_t *slot_pos;
    const int32_t *unit_stage_off;  // [D * n_units + 1]: slots of day d held by unit u (one lane per node):
    const int32_t *unit_stage;      // local position | slot << 8
    int32_t *stage;                 // [kDaySlotCap * MAXC]: their counts after the day kernel, [slot][c]
    const uint32_t *slot_key;   // [3 per slot] Philox key (seed, replicate id) and set of the slot's node
    const int64_t *lvl_ev_off;  // event offsets of each level
    const int32_t *slot_src;
    const int32_t *slot_dst;
    const int32_t *lvl_ptr;     // [D+1]: levels of day d are lvl_ptr[d] .. lvl_ptr[d+1]-1
};

// Layouts of the day phase: one lane per node with workgroup sums (R == 1),
// or tiles of kTileNodes nodes x 64 replicate lanes per workgroup (R > 1,
// lane stride RL a multiple of 64).
constexpr int kTileNodes = 128;       // default positions of a replicate tile
constexpr uint32_t kFewChains = 4;     // default: at most this many live chains walked one after another
constexpr double kGroupMinAttempts = 4096.0;  // default: a workgroup walks a chain expecting this many attempts
constexpr int kLaneUnit = 256;  // positions of one workgroup with one lane per node
enum { LAYOUT_LANES = 0, LAYOUT_TILE = 1 };

// Positions per unit of the day phase (a workgroup's nodes); a private task
// (a level-1 run of one node's single-node events) runs in its node's unit
// right after the SSA.
inline int64_t unit_positions(int layout, int64_t tile) { return layout == LAYOUT_TILE ? tile : kLaneUnit; }

// Host-side launchers (episim_device.hip). Each returns a hipError_t as int.
// A day whose levels run in LDS: its levels lv0 .. lv0 + nl - 1, slots
// s0 .. s0 + ns - 1 and level events e0 .. e0 + ne - 1.
struct EventDayArgs {
    int32_t lv0, nl, s0, ns;
    int64_t e0, ne;
};
int launch_day(const Model &m, const DevState &s, const DevEvents &ev, int32_t d, int prologue, int ssa,
               int layout, void *stream);
int launch_events(const Model &m, const DevState &s, const DevEvents &ev, int32_t d, int64_t begin,
                  int64_t end, void *stream);
int launch_event_levels(const Model &m, const DevState &s, const DevEvents &ev, int32_t d, int32_t lv_begin,
                        int32_t lv_end, void *stream);
// levels of at most this many (task, replicate) pairs are grouped into one
// single-workgroup launch
constexpr int64_t kSmallLevel = 512;
// a day with one lane per node, at most kDayEventCap level events in at most
// kDayLevelCap levels and at most kDaySlotCap distinct nodes touched by them
// runs its levels in LDS
constexpr int64_t kDayEventCap = 512;
constexpr int64_t kDaySlotCap = 768;
constexpr int64_t kDayLevelCap = 64;
int launch_event_day(const Model &m, const DevState &s, const DevEvents &ev, int32_t d, const EventDayArgs &a,
                     void *stream);
// A slot handle's step: the day kernel over the n_cols columns of s.run_cols,
// and levels k .. k_end - 1 of the days of the n_run slots of s.run_slots.
int launch_slot_day(const Model &m, const DevState &s, const DevEvents &ev, int32_t step, int32_t n_cols,
                    void *stream);
int launch_slot_events(const Model &m, const DevState &s, const DevEvents &ev, int32_t step, int32_t k,
                       int32_t k_end, int64_t max_count, int32_t n_run, void *stream);
int launch_goal(const DevState &s, int32_t nc, int64_t s0, int32_t N, const int64_t *ref, int32_t d_begin,
                int32_t n_days, double *part, void *stream);
// The day terms part[0 .. n) and part[n .. 2n) added in day order into out[0]
// and out[1] (one thread; the order of the host loop of sim_goal).
int launch_goal_sum(const double *part, int32_t n, double *out, void *stream);
// Bytes of the static device array that the entry points which allocate
// nothing use for their intermediate buffers (one array per GPU, held until
// the process ends), and its address on the current device (looked up once
// per device, then cached).
constexpr size_t kScratchBytes = (size_t)8 << 20;
int scratch_address(void **out);
int launch_slot_init(const DevState &s, int32_t nc, const int32_t *u0, const double *v0, int32_t slot,
                     const SlotInfo &info, void *stream);
int launch_persistent(const Model &m, const DevState &s, const DevEvents &ev, int32_t d_begin,
                      int32_t d_end, int layout, void *stream, char *why, int why_len);

}  // namespace episim
