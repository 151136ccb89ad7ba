// Host side of the episim C ABI: validation of the problem statement, the
// dependency pass over the external events, device memory, and the day loop.
//
// The dependency pass is the GPU counterpart of the paper's re-arrangement of
// the event lists (Sec. 3.4, Algorithm 2's initialisation) and of its
// precedence rules between tasks that touch the same sub-domain (Sec. 3.6,
// rules 2(b) and 3(b)), applied at node granularity: within a day, an event
// that draws individuals from a node must follow every earlier event touching
// that node, and an event that adds to a node must follow every earlier draw
// from it; additions to one node commute. A run of events that touch one node
// only (enter, exit, internal transfer), with no external transfer touching
// that node between them in list order, forms one task: one thread applies it
// in list order with the counts held in registers, as the paper's private
// events of a sub-domain run inside its own task (Sec. 3.6). Every task gets
// the smallest level meeting the rules, so one level runs fully in parallel
// and levels run in order. Tasks and levels are computed once per handle and
// reused by every run and replicate, as the paper reuses its re-arranged lists
// across runs.
//
// A handle holds one or more instances (networks) of one model. Instances are
// packed into one range of node positions, each padded to whole wavefronts /
// workgroups / tiles so that every unit of work belongs to one instance; the
// random streams use each instance's own node numbers, event numbers and
// seed, so an instance packed with others gives the same trajectory as alone.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <exception>
#include <new>
#include <string>
#include <thread>
#include <utility>
#include <vector>

#include "../../include/episim.h"
#include "episim_internal.h"

using namespace episim;

namespace {

thread_local std::string g_create_error;

std::string fmt(const char *f, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, f);
    vsnprintf(buf, sizeof buf, f, ap);
    va_end(ap);
    return buf;
}

// An allocator that leaves new elements of trivial types uninitialised: the
// large per-event and per-task arrays of the build are written in full by the
// threaded passes, which then also take the first touch of their pages.
template <class T>
struct NoInit : std::allocator<T> {
    template <class U>
    struct rebind {
        using other = NoInit<U>;
    };
    NoInit() noexcept = default;
    template <class U>
    NoInit(const NoInit<U> &) noexcept {}
    template <class U>
    void construct(U *p) noexcept {
        ::new ((void *)p) U;
    }
    template <class U, class... A>
    void construct(U *p, A &&...a) {
        ::new ((void *)p) U(std::forward<A>(a)...);
    }
};
template <class T>
using big_vec = std::vector<T, NoInit<T>>;

bool is_sampler(int kind) { return kind == SIM_EXIT || kind == SIM_INTERNAL || kind == SIM_EXTERNAL; }

// Host threads for a build pass over many events: one below about a million
// events, else as many as the machine has, at most 16.
int host_threads(int64_t n) {
    if (n < (int64_t(1) << 20)) return 1;
    const unsigned hw = std::thread::hardware_concurrency();
    return (int)std::min(std::max(hw, 1u), 16u);
}

// Cuts of [0, n) into at most T ranges of whole days and similar size
// (day[] sorted); cut[0] = 0 and cut.back() = n.
std::vector<int64_t> day_cuts(int64_t n, const int32_t *day, int T) {
    std::vector<int64_t> cut{0};
    for (int c = 1; c < T; ++c) {
        int64_t at = n * c / T;
        if (at <= cut.back()) continue;
        at = std::upper_bound(day + at, day + n, day[at - 1]) - day;
        if (at > cut.back() && at < n) cut.push_back(at);
    }
    cut.push_back(n);
    return cut;
}

// f(range, begin, end) for each range of cut, one thread a range; the first
// exception thrown (an allocation failure) is raised again in the caller.
template <class F>
void run_ranges(const std::vector<int64_t> &cut, F &&f) {
    const int C = (int)cut.size() - 1;
    if (C <= 1) {
        if (C == 1) f(0, cut[0], cut[1]);
        return;
    }
    std::vector<std::exception_ptr> fail(C);
    auto guarded = [&](int c) {
        try {
            f(c, cut[c], cut[c + 1]);
        } catch (...) {
            fail[c] = std::current_exception();
        }
    };
    std::vector<std::thread> th;
    th.reserve(C - 1);
    for (int c = 1; c < C; ++c) th.emplace_back(guarded, c);
    guarded(0);
    for (auto &t : th) t.join();
    for (auto &x : fail)
        if (x) std::rethrow_exception(x);
}

// Task and level of every event within its day; events must already be
// sorted by day. Tasks are numbered in order of their first event. Records
// the number of levels of each day in day_levels (resized to n_days).
// Days are independent, so ranges of whole days are planned on their own
// threads, each numbering its tasks from 0, and the numbers are then offset.
void plan_levels(int64_t n, const int32_t *day, const int32_t *kind, const int32_t *node,
                 const int32_t *dest, int32_t n_nodes, int32_t *level, int32_t *task,
                 std::vector<int32_t> *day_levels, int32_t n_days) {
    // per node, valid for the day stored in stamp (nothing is cleared between
    // days): the last level at which it was touched at all / drawn from, and
    // the task of single-node events still open at it with the values of
    // those two before the task began; one cache line holds a node's state
    struct alignas(32) NodePlan {
        int32_t stamp, last_any, last_draw, open, base_any, base_draw, open_draws, unused;
    };
    if (day_levels) day_levels->assign(n_days > 0 ? n_days : 0, 0);
    // each thread's node state takes 32 bytes a node: at most 1 GiB in all
    const int64_t cap = std::max<int64_t>(1, (int64_t(1) << 30) / ((int64_t)sizeof(NodePlan) * std::max(n_nodes, 1)));
    const std::vector<int64_t> cut = day_cuts(n, day, (int)std::min<int64_t>(host_threads(n), cap));
    const int C = (int)cut.size() - 1;
    std::vector<std::vector<int32_t>> task_level(std::max(C, 0));
    run_ranges(cut, [&](int c, int64_t b, int64_t end) {
        std::vector<NodePlan> st(n_nodes, NodePlan{-1, 0, 0, -1, 0, 0, 0, 0});
        std::vector<int32_t> &tl = task_level[c];
        auto touch = [&](int32_t x, int32_t d) -> NodePlan & {
            NodePlan &q = st[x];
            if (q.stamp != d) {
                q.stamp = d;
                q.last_any = 0;
                q.last_draw = 0;
                q.open = -1;
            }
            return q;
        };
        for (int64_t e = b; e < end; ++e) {
            const int32_t d = day[e];
            NodePlan &s = touch(node[e], d);
            if (kind[e] != SIM_EXTERNAL) {
                // enter, exit, internal: one node; joins the node's open task
                const bool draws = is_sampler(kind[e]);
                int32_t t = s.open;
                if (t < 0) {
                    t = (int32_t)tl.size();
                    s.base_any = s.last_any;
                    s.base_draw = s.last_draw;
                    tl.push_back(1 + (draws ? s.base_any : s.base_draw));
                    s.open = t;
                    s.open_draws = draws;
                } else if (draws && !s.open_draws) {
                    // a draw after additions only: the task must now follow every
                    // earlier event at the node (nothing else has used its level)
                    tl[t] = std::max(tl[t], 1 + s.base_any);
                    s.open_draws = 1;
                }
                task[e] = t;
                s.last_any = std::max(s.base_any, tl[t]);
                s.last_draw = s.open_draws ? tl[t] : s.base_draw;
                continue;
            }
            // external transfer: draws at src, adds at dest; a task of its own
            NodePlan &r = touch(dest[e], d);
            s.open = -1;
            r.open = -1;
            const int32_t L = std::max(s.last_any + 1, r.last_draw + 1);
            task[e] = (int32_t)tl.size();
            tl.push_back(L);
            s.last_any = std::max(s.last_any, L);
            s.last_draw = L;
            r.last_any = std::max(r.last_any, L);
        }
    });
    std::vector<int32_t> off(C + 1, 0);
    for (int c = 0; c < C; ++c) off[c + 1] = off[c] + (int32_t)task_level[c].size();
    // a day lies in one range, so each range writes its own days' counts
    run_ranges(cut, [&](int c, int64_t b, int64_t end) {
        const std::vector<int32_t> &tl = task_level[c];
        for (int64_t e = b; e < end; ++e) {
            level[e] = tl[task[e]];
            task[e] += off[c];
            if (day_levels) (*day_levels)[day[e]] = std::max((*day_levels)[day[e]], level[e]);
        }
    });
}

int check_device(hipError_t e, std::string *err, const char *what) {
    if (e == hipSuccess) return SIM_OK;
    *err = fmt("%s: %s", what, hipGetErrorString(e));
    return SIM_EDEVICE;
}

uint32_t column_mask(const sim_problem *p, int32_t s) {
    uint32_t m = 0;
    for (int c = 0; c < p->n_comp; ++c)
        if (p->E[(size_t)c * p->n_select + s]) m |= 1u << c;
    return m;
}

// Rate constants, shedding rates and decay rates of R trajectories.
int check_params(int Nt, int64_t R, const double *coef, const double *alpha, const double *beta, std::string *err) {
    for (int64_t i = 0; i < R * Nt; ++i)
        if (!(coef[i] >= 0.0) || !std::isfinite(coef[i])) return *err = "coef must be finite and >= 0", SIM_EINVAL;
    for (int64_t r = 0; r < R; ++r) {
        if (!(alpha[r] >= 0.0) || !std::isfinite(alpha[r])) return *err = "alpha must be finite and >= 0", SIM_EINVAL;
        for (int q = 0; q < 4; ++q) {
            const double b = beta[r * 4 + q];
            if (!(b >= 0.0 && b <= 1.0)) return *err = "beta must be in [0, 1]", SIM_EINVAL;
        }
    }
    return SIM_OK;
}

// Full validation of one problem statement (the contract in episim.h).
// The first fault of event e of p in the order of the checks (its message in
// *msg and nonzero), or 0; mask_of holds the column mask of each select.
int event_fault(const sim_problem *p, int64_t e, const uint32_t *mask_of, std::string *msg) {
    const int Nc = p->n_comp;
    const int32_t d = p->ev_day[e], k = p->ev_kind[e], i = p->ev_node[e], s = p->ev_select[e];
    const int32_t h = p->ev_shift[e];
    if (d < 0 || d >= p->n_days) return *msg = fmt("event %lld: day out of range", (long long)e), 1;
    if (e > 0 && d < p->ev_day[e - 1]) return *msg = fmt("event %lld: days not sorted", (long long)e), 1;
    if (k < 0 || k > 3) return *msg = fmt("event %lld: unknown kind", (long long)e), 1;
    if (i < 0 || i >= p->n_nodes) return *msg = fmt("event %lld: node out of range", (long long)e), 1;
    if (k == SIM_EXTERNAL && (p->ev_dest[e] < 0 || p->ev_dest[e] >= p->n_nodes))
        return *msg = fmt("event %lld: dest out of range", (long long)e), 1;
    if (p->ev_n[e] < 0 || p->ev_n[e] > SIM_MAX_EVENT_N)
        return *msg = fmt("event %lld: n must be in [0, %d]", (long long)e, SIM_MAX_EVENT_N), 1;
    if (s < 0 || s >= p->n_select) return *msg = fmt("event %lld: select out of range", (long long)e), 1;
    if (h < -1 || h >= p->n_shift) return *msg = fmt("event %lld: shift out of range", (long long)e), 1;
    const uint32_t m = mask_of[s];
    if (k == SIM_ENTER && (m == 0 || (m & (m - 1))))
        return *msg = fmt("event %lld: ENTER must select exactly one compartment", (long long)e), 1;
    if (h >= 0 && k != SIM_ENTER && k != SIM_EXIT) {
        for (int c = 0; c < Nc; ++c) {
            if (!((m >> c) & 1u)) continue;
            const int to = c + p->N[(size_t)c * p->n_shift + h];
            if (to < 0 || to >= Nc)
                return *msg = fmt("event %lld: shift moves compartment %d out of range", (long long)e, c), 1;
        }
    }
    return 0;
}

int validate(const sim_problem *p, std::string *err) {
    if (!p) return *err = "problem is NULL", SIM_EINVAL;
    if (p->n_nodes < 0) return *err = "n_nodes < 0", SIM_EINVAL;
    if (p->n_comp < 1 || p->n_comp > SIM_MAX_COMP) return *err = "n_comp must be in [1, 8]", SIM_EINVAL;
    if (p->n_trans < 1 || p->n_trans > SIM_MAX_TRANS) return *err = "n_trans must be in [1, 8]", SIM_EINVAL;
    if (p->n_rep < 1) return *err = "n_rep must be >= 1", SIM_EINVAL;
    if (p->phi_pre_events != 0 && p->phi_pre_events != 1) return *err = "phi_pre_events must be 0 or 1", SIM_EINVAL;
    if (p->n_regions < 0 || p->n_regions > SIM_MAX_REGIONS || (p->n_regions > 0 && p->n_nodes > 0 && !p->region))
        return *err = "n_regions must be in [0, SIM_MAX_REGIONS] with a region per node", SIM_EINVAL;
    for (int64_t i = 0; p->n_regions > 0 && i < p->n_nodes; ++i)
        if (p->region[i] < -1 || p->region[i] >= p->n_regions)
            return *err = fmt("region[%lld] out of range", (long long)i), SIM_EINVAL;
    if (p->n_days < 0) return *err = "n_days < 0", SIM_EINVAL;
    if ((int64_t)p->n_nodes * p->n_rep > INT32_MAX)
        return *err = "n_nodes * n_rep must be below 2^31", SIM_EINVAL;
    if (p->n_events < 0 || p->n_events > INT32_MAX) return *err = "n_events must be in [0, 2^31)", SIM_EINVAL;
    const int Nc = p->n_comp, Nt = p->n_trans, R = p->n_rep;
    if ((p->n_nodes > 0 && (!p->u0 || !p->v0)) || !p->S || !p->reactant || !p->uses_phi || !p->coef ||
        !p->alpha || !p->beta)
        return *err = "a required array is NULL", SIM_EINVAL;
    for (int64_t i = 0; i < (int64_t)p->n_nodes * Nc; ++i)
        if (p->u0[i] < 0) return *err = fmt("u0[%lld] < 0", (long long)i), SIM_EINVAL;
    for (int64_t i = 0; i < p->n_nodes; ++i)
        if (!(p->v0[i] >= 0.0) || !std::isfinite(p->v0[i]))
            return *err = fmt("v0[%lld] must be finite and >= 0", (long long)i), SIM_EINVAL;
    for (int k = 0; k < Nt; ++k) {
        const int a = p->reactant[k];
        if (a < 0 || a >= Nc) return *err = fmt("reactant[%d] out of range", k), SIM_EINVAL;
        if (p->uses_phi[k] != 0 && p->uses_phi[k] != 1) return *err = fmt("uses_phi[%d] not 0/1", k), SIM_EINVAL;
        if (p->reactant2 && (p->reactant2[k] < -1 || p->reactant2[k] >= Nc))
            return *err = fmt("reactant2[%d] out of range", k), SIM_EINVAL;
        for (int c = 0; c < Nc; ++c) {
            const int32_t s = p->S[(size_t)c * Nt + k];
            if (c == a && s != -1) return *err = fmt("S[%d,%d] must be -1 (the reactant of transition %d)", c, k, k), SIM_EINVAL;
            if (c != a && s < 0) return *err = fmt("S[%d,%d] < 0 for a compartment that is not the reactant", c, k), SIM_EINVAL;
            if (s > 127) return *err = fmt("S[%d,%d] too large", c, k), SIM_EINVAL;
        }
    }
    if (int rc = check_params(Nt, R, p->coef, p->alpha, p->beta, err)) return rc;
    const uint32_t all = (Nc == 32) ? ~0u : ((1u << Nc) - 1u);
    if ((p->phi_I_mask & ~all) || (p->phi_N_mask & ~all)) return *err = "phi masks name a missing compartment", SIM_EINVAL;
    if (p->n_select < 0 || p->n_shift < 0 || p->n_shift > MAX_SHIFT_IDS)
        return *err = "n_select < 0 or n_shift not in [0, 63]", SIM_EINVAL;
    if ((p->n_select > 0 && !p->E) || (p->n_shift > 0 && !p->N)) return *err = "E or N is NULL", SIM_EINVAL;
    for (int64_t i = 0; i < (int64_t)Nc * p->n_select; ++i)
        if (p->E[i] != 0 && p->E[i] != 1) return *err = "E entries must be 0 or 1", SIM_EINVAL;
    if (p->n_events > 0 && (!p->ev_day || !p->ev_kind || !p->ev_node || !p->ev_dest || !p->ev_n ||
                            !p->ev_select || !p->ev_shift))
        return *err = "an event array is NULL", SIM_EINVAL;
    if (p->n_events > 0) {
        // ranges of events on host threads; the first range with a fault
        // holds the first faulting event
        std::vector<uint32_t> mask_of(p->n_select);
        for (int32_t sel = 0; sel < p->n_select; ++sel) mask_of[sel] = column_mask(p, sel);
        const int T = host_threads(p->n_events);
        std::vector<int64_t> cut(T + 1);
        for (int c = 0; c <= T; ++c) cut[c] = p->n_events * c / T;
        std::vector<std::string> fault(T);
        run_ranges(cut, [&](int c, int64_t b, int64_t end) {
            for (int64_t e = b; e < end; ++e)
                if (event_fault(p, e, mask_of.data(), &fault[c])) return;
        });
        for (const std::string &f : fault)
            if (!f.empty()) return *err = f, SIM_EINVAL;
    }
    if (p->n_record < 0 || (p->n_record > 0 && !p->record_days)) return *err = "bad record_days", SIM_EINVAL;
    for (int k = 0; k < p->n_record; ++k) {
        const int32_t d = p->record_days[k];
        if (d < 0 || d >= p->n_days) return *err = "record day out of range", SIM_EINVAL;
        if (k > 0 && d <= p->record_days[k - 1]) return *err = "record_days must be strictly ascending", SIM_EINVAL;
    }
    return SIM_OK;
}


// Problems packed into one handle must share the model and the run shape.
int same_model(const sim_problem *a, const sim_problem *b, std::string *err) {
    auto eq = [](const void *x, const void *y, size_t n) { return n == 0 || std::memcmp(x, y, n) == 0; };
    const size_t Nc = a->n_comp, Nt = a->n_trans;
    if (a->n_comp != b->n_comp || a->n_trans != b->n_trans || a->n_rep != b->n_rep || a->n_days != b->n_days ||
        a->day0 != b->day0 || a->phi_I_mask != b->phi_I_mask || a->phi_N_mask != b->phi_N_mask ||
        a->n_select != b->n_select || a->n_shift != b->n_shift || a->n_record != b->n_record ||
        a->phi_pre_events != b->phi_pre_events || (a->reactant2 == nullptr) != (b->reactant2 == nullptr) ||
        a->n_regions != b->n_regions)
        return *err = "packed problems must share sizes, replicates, horizon, day0, masks and record days", SIM_EINVAL;
    if (!eq(a->S, b->S, sizeof(int32_t) * Nc * Nt) || !eq(a->reactant, b->reactant, sizeof(int32_t) * Nt) ||
        !eq(a->uses_phi, b->uses_phi, sizeof(int32_t) * Nt) ||
        (a->reactant2 && !eq(a->reactant2, b->reactant2, sizeof(int32_t) * Nt)) ||
        !eq(a->E, b->E, sizeof(int32_t) * Nc * a->n_select) || !eq(a->N, b->N, sizeof(int32_t) * Nc * a->n_shift) ||
        !eq(a->record_days, b->record_days, sizeof(int32_t) * a->n_record))
        return *err = "packed problems must share the model (S, reactants, uses_phi, E, N) and record days", SIM_EINVAL;
    return SIM_OK;
}

// One lane per node for a single replicate, unless tile_nodes asks for tiles:
// then each wavefront of a tile walks one node's chains with all its lanes
// (networks of few nodes with long chains).
int choose_layout(int32_t R, int32_t tile_nodes) { return R == 1 && tile_nodes <= 0 ? LAYOUT_LANES : LAYOUT_TILE; }

// Lanes per position: one, or in tiles the replicate count rounded up to
// whole wavefronts (replicate lanes r >= R idle).
int32_t lane_stride(int32_t R, int layout) {
    return layout == LAYOUT_LANES ? 1 : (int32_t)(((int64_t)R + 63) / 64 * 64);
}

// Nodes of one unit of work and the padding granule of an instance.
int64_t unit_nodes(int layout, int64_t tile) { return layout == LAYOUT_TILE ? tile : 64; }
int64_t pad_nodes(int layout, int64_t tile) { return unit_positions(layout, tile); /* one workgroup */ }

// Positions of one instance's nodes: herds sorted by size (largest first)
// are dealt one per unit of work in turn, back and forth (snake order), so the
// longest SSA chains of a day run in different units, start first, and share
// their unit with the lightest herds of the next round. With one lane per
// node, the kSoloHerds largest herds get a wavefront each (the other lanes are
// padding), so their chains are walked by the whole wavefront from the first
// attempt. Returns the number of positions (a multiple of the padding
// granule); pos_node[pos] = node or -1.
constexpr int64_t kSoloHerds = 128;
// With replicate tiles, the largest herds of an instance (at most
// kHeavyHerds, and one per 64 nodes) get units of their own whose every
// (herd, replicate) chain is walked by a wavefront of its own; they are placed
// first, the remaining positions of their units stay empty.
constexpr int64_t kHeavyHerds = 64;
// With one lane per node and per-day launches, the largest herds of a large
// instance (kGroupHerds unless the options say otherwise) get a workgroup
// each: the herd sits at the unit's first position and its chain is walked by
// all four wavefronts of the workgroup.
constexpr int64_t kGroupHerds = 4;
constexpr int32_t kMaxGroupHerds = 16;
constexpr int32_t kMaxHeavyHerds = 256;

// One group of herds, ranked largest first, placed from position base: solo
// wavefronts first (one lane per node, large groups only), then dealt over the
// units of the group; the group is padded to whole workgroups / tiles.
// Returns the positions it takes.
int64_t place_group(const std::vector<int32_t> &ranked, int layout, int64_t tile, int64_t base,
                    std::vector<int32_t> *pos_node) {
    const int64_t n = (int64_t)ranked.size(), G = unit_nodes(layout, tile), P = pad_nodes(layout, tile);
    // solo wavefronts only pay off when the rest still fills many wavefronts
    const int64_t solo = (layout == LAYOUT_LANES && n >= 64 * kSoloHerds) ? kSoloHerds : 0;
    const int64_t span = n == 0 ? 0 : ((solo * 64 + (n - solo) + P - 1) / P) * P;
    pos_node->resize(base + span, -1);
    for (int64_t q = 0; q < solo; ++q) (*pos_node)[base + q * 64] = ranked[q];
    const int64_t b2 = base + solo * 64;
    const int64_t U = (base + span - b2) / G;
    int64_t q = solo;
    for (int64_t j = 0; j < G && q < n; ++j)
        for (int64_t uu = 0; uu < U && q < n; ++uu) {
            const int64_t u = (j & 1) ? U - 1 - uu : uu;
            (*pos_node)[b2 + u * G + j] = ranked[q++];
        }
    return span;
}

// Positions of one instance's nodes (pos_node[pos] = node or -1) and the
// region of each position (-1 outside regions). With regions, every unit of
// work holds herds of one region only, so the per-unit sums of the records
// are also regional sums; the heavy herds' own units may mix regions (their
// chains record on their own).
int64_t order_nodes(const sim_problem *p, int layout, int64_t tile, int64_t heavy, int64_t group,
                    std::vector<int32_t> *pos_node, std::vector<int32_t> *pos_region) {
    const int64_t Nn = p->n_nodes, Nc = p->n_comp;
    // a herd's size is its largest population over the horizon: the SSA only
    // moves individuals between compartments of a node, so node totals follow
    // from the initial state and the events alone (hubs that receive many
    // movements grow well past their initial size)
    std::vector<int64_t> now(Nn, 0), size(Nn, 0);
    for (int64_t i = 0; i < Nn; ++i) {
        for (int64_t c = 0; c < Nc; ++c) now[i] += p->u0[i * Nc + c];
        size[i] = now[i];
    }
    // Long lists: ranges of events on host threads, each replaying its events
    // from zero and keeping every node's net change and its highest running
    // change at the points where the whole replay takes a node's maximum;
    // the ranges then add up in order (16 bytes a node and range, at most
    // 1 GiB in all). One range replays directly.
    const int64_t cap = std::max<int64_t>(1, (int64_t(1) << 30) / (16 * std::max<int64_t>(Nn, 1)));
    const int T = (int)std::min<int64_t>(host_threads(p->n_events), cap);
    std::vector<int64_t> cut(T + 1);
    for (int c = 0; c <= T; ++c) cut[c] = p->n_events * c / T;
    if (T == 1) {
        for (int64_t e = 0; e < p->n_events; ++e) {
            const int32_t i = p->ev_node[e], k = p->ev_kind[e], n = p->ev_n[e];
            if (k == SIM_ENTER) now[i] += n;
            if (k == SIM_EXIT || k == SIM_EXTERNAL) now[i] -= n;
            if (k == SIM_EXTERNAL) {
                const int32_t j = p->ev_dest[e];
                now[j] += n;
                size[j] = std::max(size[j], now[j]);
            }
            size[i] = std::max(size[i], now[i]);
        }
    } else {
        std::vector<std::vector<int64_t>> delta(T), peak(T);
        run_ranges(cut, [&](int c, int64_t b, int64_t end) {
            std::vector<int64_t> &cum = delta[c], &top = peak[c];
            cum.assign(Nn, 0);
            top.assign(Nn, 0);
            for (int64_t e = b; e < end; ++e) {
                const int32_t i = p->ev_node[e], k = p->ev_kind[e], n = p->ev_n[e];
                if (k == SIM_ENTER) cum[i] += n;
                if (k == SIM_EXIT || k == SIM_EXTERNAL) cum[i] -= n;
                if (k == SIM_EXTERNAL) {
                    const int32_t j = p->ev_dest[e];
                    cum[j] += n;
                    top[j] = std::max(top[j], cum[j]);
                }
                top[i] = std::max(top[i], cum[i]);
            }
        });
        for (int c = 0; c < T; ++c)
            for (int64_t i = 0; i < Nn; ++i) {
                size[i] = std::max(size[i], now[i] + peak[c][i]);
                now[i] += delta[c][i];
            }
    }
    // largest herd first, equal sizes by node number (a stable sort by size)
    std::vector<std::pair<int64_t, int32_t>> by_size(Nn);
    for (int64_t i = 0; i < Nn; ++i) by_size[i] = {-size[i], (int32_t)i};
    std::sort(by_size.begin(), by_size.end());
    std::vector<int32_t> rank(Nn);
    for (int64_t i = 0; i < Nn; ++i) rank[i] = by_size[i].second;
    const int64_t G = unit_nodes(layout, tile);
    const int64_t hv = layout == LAYOUT_TILE ? std::min(heavy, Nn) : 0;
    const int64_t hv_span = ((hv + G - 1) / G) * G;
    const int64_t gr = layout == LAYOUT_LANES ? std::min(group, Nn) : 0;
    const int64_t lead = hv_span + gr * pad_nodes(layout, tile);
    const int32_t J = p->n_regions > 0 ? p->n_regions : 0;
    auto region_of = [&](int32_t i) { return J > 0 ? p->region[i] : -1; };
    pos_node->assign(lead, -1);
    pos_region->assign(lead, -1);
    for (int64_t q = 0; q < hv; ++q) {
        (*pos_node)[q] = rank[q];
        (*pos_region)[q] = region_of(rank[q]);
    }
    // a workgroup per group herd: the herd first, the rest padding of its region
    for (int64_t q = 0; q < gr; ++q) {
        const int64_t b = hv_span + q * pad_nodes(layout, tile);
        (*pos_node)[b] = rank[hv + q];
        for (int64_t i = 0; i < pad_nodes(layout, tile); ++i) (*pos_region)[b + i] = region_of(rank[hv + q]);
    }
    // groups: the herds outside regions, then region by region (one group without regions)
    std::vector<std::vector<int32_t>> groups(J + 1);
    for (int64_t q = hv + gr; q < Nn; ++q) groups[region_of(rank[q]) + 1].push_back(rank[q]);
    int64_t base = lead;
    for (int32_t j = -1; j < J; ++j) {
        const int64_t span = place_group(groups[j + 1], layout, tile, base, pos_node);
        pos_region->resize(base + span, j);
        base += span;
    }
    return base;
}

// Device buffer layout of one handle.
struct Layout {
    size_t u, phi, node_id, inst, inst_off, seed, coef, alpha, beta, repid, status, ev_g, ev_gm, ev_node,
        ev_dest, ev_n, ev_meta, ev_smap, task_off, priv_off, priv_ev_off, day_slot_off, slot_pos, unit_stage_off, unit_stage, stage, slot_key, lvl_ev_off, ev_slot_src, ev_slot_dst, lvl_off, lvl_ptr, prevalence, transitions, totals, max_fired, snap_u, snap_v, rec_slot, slots,
        u0, v0, run, heavy_pos, unit_heavy, unit_group, pos_region, regional, goal_ref, goal_part, total;
};

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

Layout layout_for(int64_t Np, int64_t n_nodes, int64_t n_inst, int64_t Nc, int64_t Nt, int64_t R, int64_t RL,
                  int64_t D, int64_t n_events, int64_t n_shift_ids, int64_t n_levels, int64_t n_tasks,
                  int64_t n_units, int64_t n_day_slots, int64_t n_record, int64_t n_slots, int64_t n_heavy,
                  int64_t n_regions) {
    Layout l{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off = align_up(off + std::max<size_t>(bytes, 1));
        return at;
    };
    const int64_t L = Np * RL, S = n_inst * R;
    l.u = take(sizeof(int32_t) * Nc * L);
    l.phi = take(sizeof(double) * L);
    l.node_id = take(sizeof(int32_t) * Np);
    l.inst = take(sizeof(int32_t) * Np);
    l.inst_off = take(sizeof(int32_t) * n_inst);
    l.seed = take(sizeof(uint32_t) * n_inst);
    l.coef = take(sizeof(double) * S * Nt);
    l.alpha = take(sizeof(double) * S);
    l.beta = take(sizeof(double) * S * 4);
    l.repid = take(sizeof(uint32_t) * S);
    l.status = take(sizeof(unsigned long long) * std::max<int64_t>(n_slots, 1));
    l.ev_g = take(sizeof(int32_t) * n_events);
    l.ev_gm = take(sizeof(int32_t) * n_events);
    l.ev_node = take(sizeof(int32_t) * n_events);
    l.ev_dest = take(sizeof(int32_t) * n_events);
    l.ev_n = take(sizeof(int32_t) * n_events);
    l.ev_meta = take(sizeof(uint32_t) * n_events);
    l.ev_smap = take(sizeof(uint32_t) * n_events);
    l.task_off = take(sizeof(int32_t) * (n_tasks + 1));
    l.priv_off = take(sizeof(int32_t) * (D * n_units + 1));
    l.priv_ev_off = take(sizeof(int32_t) * (D * n_units + 1));
    l.day_slot_off = take(sizeof(int32_t) * (D + 1));
    l.slot_pos = take(sizeof(int32_t) * n_day_slots);
    l.unit_stage_off = take(sizeof(int32_t) * (D * n_units + 1));
    l.unit_stage = take(sizeof(int32_t) * n_day_slots);
    l.stage = take(sizeof(int32_t) * kDaySlotCap * MAXC);
    l.slot_key = take(sizeof(uint32_t) * 3 * n_day_slots);
    l.lvl_ev_off = take(sizeof(int64_t) * (n_levels + 1));
    l.ev_slot_src = take(sizeof(int32_t) * n_events);
    l.ev_slot_dst = take(sizeof(int32_t) * n_events);
    l.lvl_off = take(sizeof(int64_t) * (n_levels + 1));
    l.lvl_ptr = take(sizeof(int32_t) * (D + 1));
    l.prevalence = take(sizeof(int32_t) * D * S);
    l.transitions = take(sizeof(int64_t) * D * S);
    l.totals = take(sizeof(int64_t) * D * S * Nc);
    l.max_fired = take(sizeof(int32_t) * D * S);
    l.snap_u = take(sizeof(int32_t) * n_record * R * n_nodes * Nc);
    l.snap_v = take(sizeof(double) * n_record * R * n_nodes);
    l.rec_slot = take(sizeof(int32_t) * D);
    // slot handles: the slot table and the network's initial state by position
    l.slots = take(sizeof(SlotInfo) * n_slots);
    l.heavy_pos = take(sizeof(int32_t) * n_heavy);
    l.pos_region = take(n_regions ? sizeof(int32_t) * Np : 0);
    l.regional = take(sizeof(int64_t) * D * S * n_regions * Nc);
    l.goal_ref = take(sizeof(int64_t) * D * n_regions * Nc);
    l.goal_part = take(n_regions ? sizeof(double) * 2 * D : 0);
    l.unit_heavy = take(n_units);
    l.unit_group = take(n_units);
    l.u0 = take(n_slots ? sizeof(int32_t) * Nc * Np : 0);
    l.v0 = take(n_slots ? sizeof(double) * Np : 0);
    // slot handles: the step's running slots, then its running columns
    l.run = take(n_slots ? sizeof(int32_t) * (n_slots + RL / 64) : 0);
    l.total = off;
    return l;
}

// Everything a handle uploads, built on the host from one or more problems.
struct Packed {
    int32_t n_inst = 0, R = 0, RL = 0, D = 0, Nc = 0, Nt = 0, n_record = 0, layout = 0, n_slots = 0;
    int64_t tile = kTileNodes;  // positions of one replicate tile
    int32_t slot_lanes = 64;    // replicate lanes of one slot of a slot handle
    int64_t Np = 0, n_nodes = 0, n_events = 0, n_levels = 0;
    std::vector<int32_t> node_id, inst, inst_off, inst_pos0;
    std::vector<uint32_t> seed, repid;
    std::vector<double> coef, alpha, beta;
    std::vector<int32_t> lane_of;  // [n_nodes] position of each concatenated node
    // merged events in execution order and their levels
    big_vec<int32_t> eg, egm, enode, edest, en, ev_inst, ev_local, ev_day;
    big_vec<uint32_t> emeta, esmap;
    std::vector<int32_t> lvl_ptr;
    std::vector<int64_t> lvl_off;   // task offsets of each level
    std::vector<int32_t> task_off;  // event offsets of each task
    std::vector<int32_t> priv_off;  // private tasks of (day, unit)
    std::vector<int32_t> priv_ev_off;  // and their events
    std::vector<int32_t> pos_region; // region of each position (-1 outside regions)
    std::vector<int32_t> heavy_pos; // positions of the herds whose chains get a wavefront each
    std::vector<uint8_t> unit_heavy;
    std::vector<uint8_t> unit_group;  // units whose first herd is walked by the whole workgroup
    std::vector<int32_t> day_slot_off, slot_pos, ev_slot_src, ev_slot_dst;  // days run in LDS
    std::vector<int32_t> unit_stage_off, unit_stage;  // their slots by (day, unit)
    std::vector<uint32_t> slot_key;     // per slot: Philox key (seed, replicate id) and set of its node
    std::vector<int64_t> lvl_ev_off;    // event offsets of each level
    int64_t n_tasks = 0, n_units = 0;
    std::vector<int32_t> rec_slot;
};

// n_slots > 0 builds a slot handle of one network: n_slots slots of
// slot_lanes replicate lanes (64 / slot_lanes to a column of 64), parameters
// supplied later slot by slot.
int build_packed(const sim_problem *const *ps, int32_t n, int32_t events_mode, Packed *pk, std::string *err,
                 int32_t n_slots = 0, const sim_device_opts *o = nullptr) {
    const int32_t launch = o ? o->launch : SIM_LAUNCH_KERNELS, group_herds = o ? o->group_herds : 0;
    const int32_t heavy_herds = o ? o->heavy_herds : 0;
    pk->tile = o && o->tile_nodes > 0 ? o->tile_nodes : kTileNodes;
    if (n < 1 || !ps) return *err = "no problems", SIM_EINVAL;
    for (int32_t k = 0; k < n; ++k) {
        int rc = validate(ps[k], err);
        if (rc) {
            if (n > 1) *err = fmt("problem %d: %s", k, err->c_str());
            return rc;
        }
        if (k > 0 && (rc = same_model(ps[0], ps[k], err))) return rc;
    }
    if (events_mode != SIM_EVENTS_LEVELS && events_mode != SIM_EVENTS_SERIAL)
        return *err = "unknown events_mode", SIM_EINVAL;
    const sim_problem *p0 = ps[0];
    if (n_slots < 0 || (n_slots > 0 && n != 1)) return *err = "a slot handle holds one network", SIM_EINVAL;
    if (n_slots > 0 && p0->n_record > 0) return *err = "slot handles keep no snapshots (n_record must be 0)", SIM_EINVAL;
    if (n_slots > 0 && p0->n_regions > 0) return *err = "slot handles keep no regional records", SIM_EINVAL;
    const int32_t W = o && o->slot_lanes > 0 ? o->slot_lanes : 64;
    if (n_slots > 65535) return *err = "too many slots", SIM_EINVAL;
    if (((int64_t)n_slots * W) % 64) return *err = "n_slots times slot_lanes must be a multiple of 64", SIM_EINVAL;
    pk->n_inst = n;
    pk->n_slots = n_slots;
    pk->slot_lanes = W;
    pk->R = n_slots > 0 ? W * n_slots : p0->n_rep;
    pk->D = p0->n_days;
    pk->Nc = p0->n_comp;
    pk->Nt = p0->n_trans;
    pk->n_record = p0->n_record;
    pk->layout = n_slots > 0 ? LAYOUT_TILE : choose_layout(pk->R, o ? o->tile_nodes : 0);
    pk->RL = lane_stride(pk->R, pk->layout);
    const int32_t R = pk->R;
    // positions
    std::vector<std::vector<int32_t>> pos_node(n);
    pk->inst_off.assign(n, 0);
    pk->inst_pos0.assign(n, 0);
    std::vector<int64_t> group_units;
    for (int32_t k = 0; k < n; ++k) {
        pk->inst_off[k] = (int32_t)pk->n_nodes;
        pk->inst_pos0[k] = (int32_t)pk->Np;
        // (with one replicate a tile's wavefront already walks one herd with all its lanes)
        const int64_t heavy = (pk->layout == LAYOUT_TILE && launch == SIM_LAUNCH_KERNELS && heavy_herds >= 0 &&
                               pk->R > 1)
                                  ? std::min<int64_t>(heavy_herds > 0 ? heavy_herds : kHeavyHerds, ps[k]->n_nodes / 64)
                                  : 0;
        const int64_t group = (pk->layout == LAYOUT_LANES && launch == SIM_LAUNCH_KERNELS &&
                               ps[k]->n_nodes >= 64 * kSoloHerds && group_herds >= 0)
                                  ? (group_herds > 0 ? group_herds : kGroupHerds) : 0;
        std::vector<int32_t> preg;
        const int64_t np_k = order_nodes(ps[k], pk->layout, pk->tile, heavy, group, &pos_node[k], &preg);
        pk->pos_region.insert(pk->pos_region.end(), preg.begin(), preg.end());
        for (int64_t j = 0; j < heavy; ++j) pk->heavy_pos.push_back((int32_t)(pk->Np + j));
        for (int64_t j = 0; j < group; ++j)
            group_units.push_back((pk->Np + j * pad_nodes(pk->layout, pk->tile)) / unit_positions(pk->layout, pk->tile));
        pk->Np += np_k;
        pk->n_nodes += ps[k]->n_nodes;
        pk->n_events += ps[k]->n_events;
    }
    if (pk->Np * (int64_t)pk->RL > INT32_MAX) return *err = "positions x replicate lanes must stay below 2^31", SIM_EINVAL;
    if (pk->n_events > INT32_MAX) return *err = "too many events", SIM_EINVAL;
    pk->unit_heavy.assign(pk->Np / unit_positions(pk->layout, pk->tile), 0);
    for (int32_t hp : pk->heavy_pos) pk->unit_heavy[hp / unit_positions(pk->layout, pk->tile)] = 1;
    pk->unit_group.assign(pk->Np / unit_positions(pk->layout, pk->tile), 0);
    for (int64_t u : group_units) pk->unit_group[u] = 1;
    pk->node_id.assign(pk->Np, -1);
    pk->inst.assign(pk->Np, 0);
    pk->lane_of.assign(pk->n_nodes, 0);
    for (int32_t k = 0; k < n; ++k) {
        const int64_t P = (int64_t)pos_node[k].size();
        for (int64_t j = 0; j < P; ++j) {
            const int64_t pos = pk->inst_pos0[k] + j;
            pk->node_id[pos] = pos_node[k][j];
            pk->inst[pos] = k;
            if (pos_node[k][j] >= 0) pk->lane_of[pk->inst_off[k] + pos_node[k][j]] = (int32_t)pos;
        }
    }
    // parameters per set = instance * R + replicate
    const int64_t S = (int64_t)n * R;
    pk->seed.resize(n);
    pk->coef.resize(S * pk->Nt);
    pk->alpha.resize(S);
    pk->beta.resize(S * 4);
    pk->repid.resize(S);
    for (int32_t k = 0; k < n; ++k) {
        const sim_problem *p = ps[k];
        pk->seed[k] = p->seed;
        if (n_slots > 0) break;  // a slot's parameters come with its request
        std::memcpy(&pk->coef[(size_t)k * R * pk->Nt], p->coef, sizeof(double) * R * pk->Nt);
        std::memcpy(&pk->alpha[(size_t)k * R], p->alpha, sizeof(double) * R);
        std::memcpy(&pk->beta[(size_t)k * R * 4], p->beta, sizeof(double) * R * 4);
        for (int32_t r = 0; r < R; ++r) pk->repid[(size_t)k * R + r] = p->replicate_id ? p->replicate_id[r] : (uint32_t)r;
    }
    // merged event list: day by day, instance by instance, list order;
    // ranges of whole days are merged on their own threads
    const int64_t E = pk->n_events;
    big_vec<int32_t> mday(E), mkind(E), mnode(E), mdest(E), minst(E), mlocal(E);
    {
        // first event of instance k on day d (at[d * n + k]) and of day d in
        // the merged list (m_at[d])
        const int32_t D = pk->D;
        std::vector<int64_t> at((size_t)(D + 1) * n), m_at(D + 1, 0);
        for (int32_t d = 0; d <= D; ++d)
            for (int32_t k = 0; k < n; ++k) {
                const int32_t *ed = ps[k]->ev_day;
                at[(size_t)d * n + k] = std::lower_bound(ed, ed + ps[k]->n_events, d) - ed;
                m_at[d] += at[(size_t)d * n + k];
            }
        std::vector<int64_t> dcut{0};
        const int T = host_threads(E);
        for (int c = 1; c < T; ++c) {
            const int64_t d = std::lower_bound(m_at.begin(), m_at.end(), E * c / T) - m_at.begin();
            if (d > dcut.back() && d < D) dcut.push_back(d);
        }
        dcut.push_back(D);
        run_ranges(dcut, [&](int, int64_t d0, int64_t d1) {
            int64_t m = m_at[d0];
            for (int64_t d = d0; d < d1; ++d)
                for (int32_t k = 0; k < n; ++k) {
                    const sim_problem *p = ps[k];
                    const int32_t off = pk->inst_off[k];
                    for (int64_t e = at[(size_t)d * n + k]; e < at[(size_t)(d + 1) * n + k]; ++e, ++m) {
                        mday[m] = (int32_t)d;
                        mkind[m] = p->ev_kind[e];
                        mnode[m] = pk->lane_of[off + p->ev_node[e]];
                        mdest[m] = p->ev_kind[e] == SIM_EXTERNAL ? pk->lane_of[off + p->ev_dest[e]] : -1;
                        minst[m] = k;
                        mlocal[m] = (int32_t)e;
                    }
                }
        });
    }
    big_vec<int32_t> level(E), task(E);
    std::vector<int32_t> day_levels;
    if (events_mode == SIM_EVENTS_SERIAL) {
        day_levels.assign(pk->D, 0);
        for (int64_t e = 0; e < E; ++e) {
            level[e] = ++day_levels[mday[e]];
            task[e] = (int32_t)e;
        }
    } else {
        plan_levels(E, mday.data(), mkind.data(), mnode.data(), mdest.data(), (int32_t)std::max<int64_t>(pk->Np, 1),
                    level.data(), task.data(), &day_levels, pk->D);
    }
    // ranges of whole days for the threaded passes below and the tasks of
    // each: tasks are numbered in order of their first event, and a day's
    // first event opens a task
    const std::vector<int64_t> cut = day_cuts(E, mday.data(), host_threads(E));
    const int C = (int)cut.size() - 1;
    std::vector<int64_t> tcut(C + 1, 0);
    {
        std::vector<int64_t> top(C, 0);
        run_ranges(cut, [&](int c, int64_t b, int64_t end) {
            for (int64_t e = b; e < end; ++e) top[c] = std::max<int64_t>(top[c], (int64_t)task[e] + 1);
        });
        for (int c = 0; c < C; ++c) {
            tcut[c] = cut[c] < E ? task[cut[c]] : 0;
            tcut[C] = std::max(tcut[C], top[c]);
        }
    }
    const int64_t n_tasks = tcut[C];
    pk->n_tasks = n_tasks;
    // Private tasks: a level-1 run of one node's single-node events touches
    // only that node, and nothing else touches it before the run in list
    // order, so it runs in the node's unit of the day kernel right after the
    // SSA. The levels left are renumbered from 1 (a day whose level 1 held
    // only private tasks loses it).
    big_vec<char> priv(n_tasks);
    std::vector<char> ext1(pk->D, 0);
    run_ranges(cut, [&](int c, int64_t b, int64_t end) {
        std::fill(priv.begin() + tcut[c], priv.begin() + tcut[c + 1], 0);
        if (events_mode != SIM_EVENTS_LEVELS) return;
        for (int64_t e = b; e < end; ++e)
            if (level[e] == 1) {
                if (mkind[e] == SIM_EXTERNAL)
                    ext1[mday[e]] = 1;
                else
                    priv[task[e]] = 1;
            }
        for (int64_t e = b; e < end; ++e)
            if (!priv[task[e]] && !ext1[mday[e]]) level[e] -= 1;
    });
    if (events_mode == SIM_EVENTS_LEVELS)
        for (int32_t d = 0; d < pk->D; ++d)
            if (!ext1[d] && day_levels[d] > 0) day_levels[d] -= 1;
    pk->lvl_ptr.assign(pk->D + 1, 0);
    for (int32_t d = 0; d < pk->D; ++d) pk->lvl_ptr[d + 1] = pk->lvl_ptr[d] + day_levels[d];
    pk->n_levels = pk->lvl_ptr[pk->D];
    // tasks in execution order: level tasks by level, then by first event;
    // then private tasks by day, unit and first event; a task's events stay
    // together in list order. Levels and (day, unit) pairs belong to one day,
    // so each range counts and places its own tasks.
    const int64_t U = pk->Np / unit_positions(pk->layout, pk->tile);
    pk->n_units = U;
    big_vec<int64_t> task_glv(n_tasks);
    big_vec<int32_t> task_n(n_tasks), tslot(n_tasks);
    pk->lvl_off.assign(pk->n_levels + 1, 0);
    pk->priv_off.assign((size_t)pk->D * U + 1, 0);
    run_ranges(cut, [&](int c, int64_t b, int64_t end) {
        std::fill(task_n.begin() + tcut[c], task_n.begin() + tcut[c + 1], 0);
        for (int64_t e = b; e < end; ++e) {
            task_glv[task[e]] = priv[task[e]] ? (int64_t)mday[e] * U + mnode[e] / unit_positions(pk->layout, pk->tile)
                                              : pk->lvl_ptr[mday[e]] + level[e] - 1;
            task_n[task[e]]++;
        }
        for (int64_t t = tcut[c]; t < tcut[c + 1]; ++t) {
            if (priv[t])
                pk->priv_off[task_glv[t] + 1]++;
            else
                pk->lvl_off[task_glv[t] + 1]++;
        }
    });
    for (int64_t i = 0; i < pk->n_levels; ++i) pk->lvl_off[i + 1] += pk->lvl_off[i];
    pk->priv_off[0] = (int32_t)pk->lvl_off[pk->n_levels];
    for (size_t i = 0; i + 1 < pk->priv_off.size(); ++i) pk->priv_off[i + 1] += pk->priv_off[i];
    pk->task_off.assign(n_tasks + 1, 0);
    {
        std::vector<int64_t> next(pk->lvl_off.begin(), pk->lvl_off.end() - 1);
        std::vector<int64_t> pnext(pk->priv_off.begin(), pk->priv_off.end() - 1);
        run_ranges(cut, [&](int c, int64_t, int64_t) {
            for (int64_t t = tcut[c]; t < tcut[c + 1]; ++t) {
                tslot[t] = (int32_t)(priv[t] ? pnext[task_glv[t]]++ : next[task_glv[t]]++);
                pk->task_off[tslot[t] + 1] = task_n[t];
            }
        });
    }
    for (int64_t i = 0; i < n_tasks; ++i) pk->task_off[i + 1] += pk->task_off[i];
    pk->priv_ev_off.resize(pk->priv_off.size());
    for (size_t i = 0; i < pk->priv_off.size(); ++i) pk->priv_ev_off[i] = pk->task_off[pk->priv_off[i]];
    big_vec<int64_t> fill(n_tasks);
    pk->eg.resize(E);
    pk->egm.resize(E);
    pk->enode.resize(E);
    pk->edest.resize(E);
    pk->en.resize(E);
    pk->emeta.resize(E);
    pk->esmap.resize(E);
    pk->ev_inst = std::move(minst);
    pk->ev_local = std::move(mlocal);
    pk->ev_day = std::move(mday);
    // of the model all instances share: the column mask of each select and
    // the compartment map of each shift (at shift + 1; 0 is no shift)
    std::vector<uint32_t> mask_of(p0->n_select), smap_of(p0->n_shift + 1);
    for (int32_t sel = 0; sel < p0->n_select; ++sel) mask_of[sel] = column_mask(p0, sel);
    for (int32_t sid = -1; sid < p0->n_shift; ++sid) {
        uint32_t smap = 0;
        for (int c = 0; c < pk->Nc; ++c) {
            const int to = sid >= 0 ? c + p0->N[(size_t)c * p0->n_shift + sid] : c;
            smap |= (uint32_t)(to & 0xF) << (4 * c);
        }
        smap_of[sid + 1] = smap;
    }
    // a task lies in one day, so ranges of whole days fill disjoint positions
    run_ranges(cut, [&](int c, int64_t b, int64_t end) {
        for (int64_t t = tcut[c]; t < tcut[c + 1]; ++t) fill[t] = pk->task_off[tslot[t]];
        for (int64_t e = b; e < end; ++e) {
            const sim_problem *p = ps[pk->ev_inst[e]];
            const int64_t le = pk->ev_local[e];
            const int64_t pos = fill[task[e]]++;
            pk->eg[pos] = (int32_t)le;
            pk->egm[pos] = (int32_t)e;
            pk->enode[pos] = mnode[e];
            pk->edest[pos] = mdest[e];
            pk->en[pos] = p->ev_n[le];
            pk->emeta[pos] = meta_pack(p->ev_kind[le], mask_of[p->ev_select[le]], p->ev_shift[le]) |
                             (pos != pk->task_off[tslot[task[e]]] ? kMetaCont : 0u);
            pk->esmap[pos] = smap_of[p->ev_shift[le] + 1];
        }
    });
    pk->lvl_ev_off.resize(pk->n_levels + 1);
    for (int64_t i = 0; i <= pk->n_levels; ++i) pk->lvl_ev_off[i] = pk->task_off[pk->lvl_off[i]];
    // Days whose level tasks fit one workgroup with one lane per node run in
    // LDS: the distinct nodes their events touch get slots, loaded once,
    // updated by every level and written back once.
    pk->day_slot_off.assign(pk->D + 1, 0);
    pk->ev_slot_src.assign(E, -1);
    pk->ev_slot_dst.assign(E, -1);
    if (pk->RL == 1 && events_mode == SIM_EVENTS_LEVELS && n_slots == 0) {
        // days are independent: ranges of days on host threads, each with its
        // own slot lists (slot numbers count from 0 in every day) and its own
        // node stamps (8 bytes a position and range, at most 1 GiB in all),
        // joined in day order
        const int64_t cap = std::max<int64_t>(1, (int64_t(1) << 30) / (8 * std::max<int64_t>(pk->Np, 1)));
        const int T = (int)std::min<int64_t>(std::min<int64_t>(host_threads(E), cap), std::max(pk->D, 1));
        std::vector<int64_t> dcut(T + 1);
        for (int c = 0; c <= T; ++c) dcut[c] = (int64_t)pk->D * c / T;
        std::vector<std::vector<int32_t>> pos_r(T);
        std::vector<std::vector<uint32_t>> key_r(T);
        run_ranges(dcut, [&](int c, int64_t d0, int64_t d1) {
            std::vector<int32_t> stamp(pk->Np, -1), slot_of(pk->Np, 0);
            std::vector<int32_t> &sp = pos_r[c];
            std::vector<uint32_t> &sk = key_r[c];
            for (int32_t d = (int32_t)d0; d < d1; ++d) {
                const int64_t tb = pk->lvl_off[pk->lvl_ptr[d]], te = pk->lvl_off[pk->lvl_ptr[d + 1]];
                const size_t start = sp.size();
                bool ok = te > tb && pk->task_off[te] - pk->task_off[tb] <= kDayEventCap &&
                          pk->lvl_ptr[d + 1] - pk->lvl_ptr[d] <= kDayLevelCap;
                auto slot = [&](int32_t pos) {
                    if (stamp[pos] != d) {
                        stamp[pos] = d;
                        slot_of[pos] = (int32_t)(sp.size() - start);
                        sp.push_back(pos);
                        const int32_t inst = pk->inst[pos];
                        sk.push_back(pk->seed[inst]);
                        sk.push_back(pk->repid[(size_t)inst * pk->R]);
                        sk.push_back((uint32_t)(inst * pk->R));
                    }
                    return slot_of[pos];
                };
                for (int64_t t = tb; ok && t < te; ++t)
                    for (int64_t e = pk->task_off[t]; e < pk->task_off[t + 1]; ++e) {
                        pk->ev_slot_src[e] = slot(pk->enode[e]);
                        if ((pk->emeta[e] & 3u) == (uint32_t)SIM_EXTERNAL) pk->ev_slot_dst[e] = slot(pk->edest[e]);
                    }
                if (ok && sp.size() - start > (size_t)kDaySlotCap) ok = false;
                if (!ok) {
                    sp.resize(start);
                    sk.resize(3 * start);
                    for (int64_t e = pk->task_off[tb]; e < pk->task_off[te]; ++e) pk->ev_slot_src[e] = pk->ev_slot_dst[e] = -1;
                }
                pk->day_slot_off[d + 1] = (int32_t)(sp.size() - start);  // the day's count for now
            }
        });
        for (int32_t d = 0; d < pk->D; ++d) pk->day_slot_off[d + 1] += pk->day_slot_off[d];
        for (int c = 0; c < T; ++c) {
            pk->slot_pos.insert(pk->slot_pos.end(), pos_r[c].begin(), pos_r[c].end());
            pk->slot_key.insert(pk->slot_key.end(), key_r[c].begin(), key_r[c].end());
        }
    }
    // The slots of such a day by unit: the unit's day kernel hands their
    // counts over in the day's staging buffer (local position | slot << 8).
    pk->unit_stage_off.assign((size_t)pk->D * U + 1, 0);
    if (pk->layout == LAYOUT_LANES) {
        const int64_t G = unit_positions(pk->layout, pk->tile);
        for (int32_t d = 0; d < pk->D; ++d)
            for (int32_t i = pk->day_slot_off[d]; i < pk->day_slot_off[d + 1]; ++i)
                pk->unit_stage_off[(size_t)d * U + pk->slot_pos[i] / G + 1]++;
        for (size_t i = 0; i + 1 < pk->unit_stage_off.size(); ++i) pk->unit_stage_off[i + 1] += pk->unit_stage_off[i];
        pk->unit_stage.resize(pk->unit_stage_off.back());
        std::vector<int32_t> fill(pk->unit_stage_off.begin(), pk->unit_stage_off.end() - 1);
        for (int32_t d = 0; d < pk->D; ++d)
            for (int32_t i = pk->day_slot_off[d]; i < pk->day_slot_off[d + 1]; ++i) {
                const int32_t pos = pk->slot_pos[i];
                pk->unit_stage[fill[(size_t)d * U + pos / G]++] =
                    (int32_t)(pos % G) | ((i - pk->day_slot_off[d]) << 8);
            }
    }
    pk->rec_slot.assign(std::max(pk->D, 1), -1);
    for (int k = 0; k < p0->n_record; ++k) pk->rec_slot[p0->record_days[k]] = k;
    return SIM_OK;
}

Layout layout_of(const Packed &pk, const sim_problem *p0) {
    return layout_for(pk.Np, pk.n_nodes, pk.n_inst, pk.Nc, pk.Nt, pk.R, pk.RL, pk.D, pk.n_events, p0->n_shift,
                      pk.n_levels, pk.n_tasks, pk.n_units, (int64_t)pk.slot_pos.size(), pk.n_record, pk.n_slots,
                      (int64_t)pk.heavy_pos.size(), p0->n_regions);
}

}  // namespace

struct sim_handle {
    int32_t Nc = 0, Nt = 0, R = 0, RL = 0, D = 0, n_record = 0, n_inst = 0, layout = 0;
    int64_t Np = 0, L = 0, n_nodes = 0;
    Model model{};
    DevState st{};
    DevEvents ev{};
    std::vector<int32_t> lane_of;   // position of each concatenated node
    std::vector<int32_t> node_id;   // node number within its instance per position (-1: padding)
    big_vec<int32_t> ev_inst, ev_local, ev_day;  // merged event index -> instance, local index, day
    std::vector<int64_t> lvl_off;   // host copy of the level boundaries (task offsets)
    std::vector<int32_t> lvl_ptr;   // [D+1]
    std::vector<int32_t> day_slot_off;  // [D+1]: a day with slots runs its levels in LDS
    std::vector<int64_t> lvl_ev_off;    // host copy of the event offsets of each level
    Layout lay{};
    void *ws = nullptr;
    bool own_ws = false;
    hipStream_t stream = nullptr;
    int device = -1;                    // the GPU current at sim_create, which holds the handle's memory
    int32_t launch = SIM_LAUNCH_KERNELS;
    int64_t small_level = kSmallLevel;  // per-day launches: levels run several per launch up to this size
    int32_t day = 0;
    std::string err;
    // kernel timing (sim_kernel_times)
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    struct Mark {
        int kind;
        hipEvent_t a, b;
    };
    std::vector<Mark> marks;
    double ms[4] = {0, 0, 0, 0};
    int64_t launches[4] = {0, 0, 0, 0};
    // slot handles
    struct Slot {
        int state = 0;  // SLOT_FREE, SLOT_RUNNING, SLOT_DONE
        int32_t t0 = -1, n_rep = 0, horizon = 0;
        hipEvent_t staged = nullptr;   // parameter upload of the last start
        hipEvent_t fetched = nullptr;  // result download of the last fetch
        bool fetch_pending = false;
    };
    int32_t n_slots = 0;
    int32_t slot_lanes = 64;  // replicate lanes per slot
    int32_t step = 0;
    std::vector<Slot> slots;
    std::deque<hipEvent_t> in_flight;  // one event per enqueued step, oldest first
    char *stage = nullptr;              // pinned: per slot, parameters then the error word
    size_t stage_stride = 0;
    // pinned ring of the steps' run lists (running slots, then running
    // columns): entry step % kRunRing is rewritten once the upload recorded
    // in run_up[step % kRunRing] has completed
    static constexpr int kRunRing = 8;
    int32_t *run_host = nullptr;
    hipEvent_t run_up[kRunRing] = {};
};

namespace {

template <typename T>
T *at(void *base, size_t off) {
    return reinterpret_cast<T *>(static_cast<char *>(base) + off);
}

hipEvent_t take_event(sim_handle *h) {
    if (!h->ev_pool.empty()) {
        hipEvent_t e = h->ev_pool.back();
        h->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Launch f() bracketed by events when timing is on.
template <typename F>
hipError_t timed(sim_handle *h, int kind, F f) {
    if (!h->timing) return (hipError_t)f();
    hipEvent_t a = take_event(h), b = take_event(h);
    if (!a || !b) return hipErrorOutOfMemory;
    hipError_t e = hipEventRecord(a, h->stream);
    if (e == hipSuccess) e = (hipError_t)f();
    if (e == hipSuccess) e = hipEventRecord(b, h->stream);
    h->marks.push_back({kind, a, b});
    return e;
}

// Fold finished marks into the totals (the stream must be synchronised).
int collect_marks(sim_handle *h) {
    for (const auto &m : h->marks) {
        float t = 0.f;
        hipError_t e = hipEventElapsedTime(&t, m.a, m.b);
        if (e != hipSuccess) return check_device(e, &h->err, "event timing");
        h->ms[m.kind] += t;
        h->launches[m.kind] += 1;
        h->ev_pool.push_back(m.a);
        h->ev_pool.push_back(m.b);
    }
    h->marks.clear();
    return SIM_OK;
}

enum { SLOT_FREE = 0, SLOT_RUNNING = 1, SLOT_DONE = 2 };

// Levels of at most this many (task, lane) pairs in every slot run together,
// one workgroup per slot.
constexpr int64_t kSlotSmallLevel = 4096;

// Bytes of one slot's parameter staging: coef, alpha, beta, replicate ids, error word.
size_t stage_bytes(int Nt) {
    return align_up(sizeof(double) * 64 * (Nt + 1 + 4) + sizeof(uint32_t) * 64 + sizeof(unsigned long long));
}

// Second half of creating a slot handle: the network's initial state by
// position (copied into a slot's lanes when it starts), zero lanes, an empty
// slot table and the pinned staging area.
// The pinned word a fetch copies a slot's error word into (the end of its staging).
unsigned long long *error_word(sim_handle *h, int32_t slot) {
    return reinterpret_cast<unsigned long long *>(h->stage + (size_t)(slot + 1) * h->stage_stride) - 1;
}

int create_slots(sim_handle *h, const sim_problem *p, sim_handle **out) {
    std::string &err = g_create_error;
    const Layout &l = h->lay;
    std::vector<int32_t> u0((size_t)h->Nc * h->Np, 0);
    std::vector<double> v0(h->Np, 0.0);
    for (int64_t i = 0; i < h->n_nodes; ++i) {
        const int64_t pos = h->lane_of[i];
        for (int c = 0; c < h->Nc; ++c) u0[(size_t)c * h->Np + pos] = p->u0[i * h->Nc + c];
        v0[pos] = p->v0[i];
    }
    std::vector<SlotInfo> table(h->n_slots, SlotInfo{-1, 0, 0, 0});
    int rc = check_device(hipMemcpy(at<char>(h->ws, l.u0), u0.data(), sizeof(int32_t) * u0.size(), hipMemcpyHostToDevice), &err, "upload u0");
    if (!rc) rc = check_device(hipMemcpy(at<char>(h->ws, l.v0), v0.data(), sizeof(double) * v0.size(), hipMemcpyHostToDevice), &err, "upload v0");
    if (!rc) rc = check_device(hipMemcpy(h->st.slots, table.data(), sizeof(SlotInfo) * table.size(), hipMemcpyHostToDevice), &err, "upload slots");
    if (!rc && h->L > 0) rc = check_device(hipMemset(h->st.u, 0, sizeof(int32_t) * h->Nc * h->L), &err, "clear u");
    if (!rc && h->L > 0) rc = check_device(hipMemset(h->st.phi, 0, sizeof(double) * h->L), &err, "clear phi");
    h->stage_stride = stage_bytes(h->Nt);
    if (!rc) rc = check_device(hipHostMalloc((void **)&h->stage, h->stage_stride * h->n_slots, hipHostMallocDefault), &err, "pinned staging");
    const size_t run_len = (size_t)h->n_slots + h->RL / 64;
    if (!rc) rc = check_device(hipHostMalloc((void **)&h->run_host, sizeof(int32_t) * run_len * sim_handle::kRunRing, hipHostMallocDefault), &err, "pinned run lists");
    for (int k = 0; k < sim_handle::kRunRing; ++k)
        if (!rc) rc = check_device(hipEventCreateWithFlags(&h->run_up[k], hipEventDisableTiming), &err, "event");
    h->slots.assign(h->n_slots, sim_handle::Slot{});
    for (auto &sl : h->slots) {
        if (!rc) rc = check_device(hipEventCreateWithFlags(&sl.staged, hipEventDisableTiming), &err, "event");
        if (!rc) rc = check_device(hipEventCreateWithFlags(&sl.fetched, hipEventDisableTiming), &err, "event");
    }
    if (rc) {
        sim_destroy(h);
        return rc;
    }
    *out = h;
    return SIM_OK;
}

// Every device option's range (the tuner's choices; none changes a result).
int check_opts(const sim_device_opts &o, std::string *err) {
    if (o.launch != SIM_LAUNCH_KERNELS && o.launch != SIM_LAUNCH_PERSISTENT) return *err = "unknown launch mode", SIM_EINVAL;
    if (o.block != 0 && o.block != 256) return *err = "block must be 0 or 256", SIM_EINVAL;
    if (o.group_herds > kMaxGroupHerds) return *err = "group_herds must be at most 16", SIM_EINVAL;
    if (o.small_level < 0) return *err = "small_level must not be negative", SIM_EINVAL;
    if (o.tile_nodes != 0 && (o.tile_nodes < 4 || o.tile_nodes > 512 || (o.tile_nodes & (o.tile_nodes - 1))))
        return *err = "tile_nodes must be 0 or a power of two in [4, 512]", SIM_EINVAL;
    if (o.heavy_herds > kMaxHeavyHerds) return *err = "heavy_herds must be at most 256", SIM_EINVAL;
    if (o.few_chains > 64) return *err = "few_chains must be at most 64", SIM_EINVAL;
    if (o.group_min_attempts < 0) return *err = "group_min_attempts must not be negative", SIM_EINVAL;
    if (o.slot_lanes != 0 && o.slot_lanes != 8 && o.slot_lanes != 16 && o.slot_lanes != 32 && o.slot_lanes != 64)
        return *err = "slot_lanes must be 0, 8, 16, 32 or 64", SIM_EINVAL;
    return SIM_OK;
}

int create(const sim_problem *const *ps, int32_t n, const sim_device_opts *o, sim_handle **out,
           int32_t n_slots = 0) {
    g_create_error.clear();
    if (!out) return g_create_error = "out is NULL", SIM_EINVAL;
    *out = nullptr;
    sim_device_opts opts{};
    if (o) opts = *o;
    if (check_opts(opts, &g_create_error)) return SIM_EINVAL;
    Packed pk;
    if (n_slots > 0 && opts.events_mode != SIM_EVENTS_LEVELS) return g_create_error = "slot handles run event levels", SIM_EINVAL;
    int rc = build_packed(ps, n, opts.events_mode, &pk, &g_create_error, n_slots, &opts);
    if (rc != SIM_OK) return rc;
    const sim_problem *p = ps[0];

    sim_handle *h = new (std::nothrow) sim_handle();
    if (!h) return g_create_error = "out of host memory", SIM_ENOMEM;
    h->Nc = pk.Nc;
    h->Nt = pk.Nt;
    h->R = pk.R;
    h->RL = pk.RL;
    h->n_slots = pk.n_slots;
    h->D = pk.D;
    h->n_record = pk.n_record;
    h->n_inst = pk.n_inst;
    h->layout = pk.layout;
    h->Np = pk.Np;
    h->L = pk.Np * pk.RL;
    h->n_nodes = pk.n_nodes;
    h->stream = (hipStream_t)opts.stream;
    if (hipGetDevice(&h->device) != hipSuccess) h->device = -1;
    h->launch = opts.launch;
    h->small_level = opts.small_level > 0 ? opts.small_level : kSmallLevel;
    h->lane_of = pk.lane_of;
    h->node_id = pk.node_id;
    h->lvl_off = pk.lvl_off;
    h->lvl_ptr = pk.lvl_ptr;
    h->day_slot_off = pk.day_slot_off;
    h->lvl_ev_off = pk.lvl_ev_off;
    h->ev_inst = std::move(pk.ev_inst);
    h->ev_local = std::move(pk.ev_local);
    h->ev_day = std::move(pk.ev_day);

    // --- model constants
    Model &m = h->model;
    m.nc = h->Nc;
    m.nt = h->Nt;
    m.day0 = p->day0;
    m.seed = p->seed;
    m.phi_pre = p->phi_pre_events;
    for (int k = 0; k < MAXT; ++k) m.reactant2[k] = -1;
    m.uses_phi = 0;
    for (int k = 0; k < h->Nt; ++k) {
        if (p->uses_phi[k]) m.uses_phi |= 1u << k;
        m.reactant[k] = p->reactant[k];
        m.reactant2[k] = p->reactant2 ? p->reactant2[k] : -1;
        for (int c = 0; c < h->Nc; ++c) m.S[c][k] = p->S[(size_t)c * h->Nt + k];
    }
    m.imask = p->phi_I_mask;
    m.nmask = p->phi_N_mask;
    // paired S <-> I classes: transition k moves one individual from compartment k to k ^ 1
    m.pairs = (h->Nc == h->Nt && h->Nc % 2 == 0) ? 1 : 0;
    for (int k = 0; k < h->Nt && m.pairs; ++k) {
        if (p->reactant[k] != k || m.reactant2[k] >= 0) m.pairs = 0;
        for (int c = 0; c < h->Nc && m.pairs; ++c) {
            const int want = c == k ? -1 : (c == (k ^ 1) ? 1 : 0);
            if (p->S[(size_t)c * h->Nt + k] != want) m.pairs = 0;
        }
    }

    // --- device memory
    h->lay = layout_of(pk, p);
    std::string &err = g_create_error;
    if (opts.workspace) {
        if (opts.workspace_bytes < h->lay.total) {
            err = fmt("workspace of %zu bytes is smaller than the %zu needed", opts.workspace_bytes, h->lay.total);
            delete h;
            return SIM_EINVAL;
        }
        h->ws = opts.workspace;
    } else {
        hipError_t e = hipMalloc(&h->ws, h->lay.total);
        if (e != hipSuccess) {
            err = fmt("hipMalloc(%zu): %s", h->lay.total, hipGetErrorString(e));
            delete h;
            return e == hipErrorOutOfMemory ? SIM_ENOMEM : SIM_EDEVICE;
        }
        h->own_ws = true;
    }
    const Layout &l = h->lay;
    DevState &s = h->st;
    s.u = at<int32_t>(h->ws, l.u);
    s.phi = at<double>(h->ws, l.phi);
    s.L = h->L;
    s.Np = (int32_t)h->Np;
    s.R = h->R;
    s.RL = h->RL;
    s.n_days = h->D;
    s.n_inst = h->n_inst;
    s.n_nodes = (int32_t)h->n_nodes;
    s.node_id = at<int32_t>(h->ws, l.node_id);
    s.inst = at<int32_t>(h->ws, l.inst);
    s.inst_off = at<int32_t>(h->ws, l.inst_off);
    s.seed = at<uint32_t>(h->ws, l.seed);
    s.coef = at<double>(h->ws, l.coef);
    s.alpha = at<double>(h->ws, l.alpha);
    s.beta = at<double>(h->ws, l.beta);
    s.repid = at<uint32_t>(h->ws, l.repid);
    s.status = at<unsigned long long>(h->ws, l.status);
    s.prevalence = at<int32_t>(h->ws, l.prevalence);
    s.transitions = at<int64_t>(h->ws, l.transitions);
    s.totals = at<int64_t>(h->ws, l.totals);
    s.max_fired = at<int32_t>(h->ws, l.max_fired);
    s.snap_u = at<int32_t>(h->ws, l.snap_u);
    s.snap_v = at<double>(h->ws, l.snap_v);
    s.rec_slot = at<int32_t>(h->ws, l.rec_slot);
    s.slots = h->n_slots ? at<SlotInfo>(h->ws, l.slots) : nullptr;
    s.run_slots = h->n_slots ? at<int32_t>(h->ws, l.run) : nullptr;
    s.run_cols = h->n_slots ? at<int32_t>(h->ws, l.run) + h->n_slots : nullptr;
    s.tile_nodes = (int32_t)pk.tile;
    s.slot_lanes = pk.slot_lanes;
    h->slot_lanes = pk.slot_lanes;
    s.few_chains = opts.few_chains < 0 ? 0u : (opts.few_chains > 0 ? (uint32_t)opts.few_chains : kFewChains);
    s.group_min_attempts = opts.group_min_attempts > 0 ? (double)opts.group_min_attempts : kGroupMinAttempts;
    s.n_heavy = (int32_t)pk.heavy_pos.size();
    s.heavy_pos = at<int32_t>(h->ws, l.heavy_pos);
    s.unit_heavy = s.n_heavy ? at<uint8_t>(h->ws, l.unit_heavy) : nullptr;
    s.unit_group = at<uint8_t>(h->ws, l.unit_group);
    s.n_regions = p->n_regions;
    s.pos_region = at<int32_t>(h->ws, l.pos_region);
    s.regional = at<int64_t>(h->ws, l.regional);
    DevEvents &ev = h->ev;
    ev.g = at<int32_t>(h->ws, l.ev_g);
    ev.gm = at<int32_t>(h->ws, l.ev_gm);
    ev.node = at<int32_t>(h->ws, l.ev_node);
    ev.dest = at<int32_t>(h->ws, l.ev_dest);
    ev.n = at<int32_t>(h->ws, l.ev_n);
    ev.meta = at<uint32_t>(h->ws, l.ev_meta);
    ev.smap = at<uint32_t>(h->ws, l.ev_smap);
    ev.task_off = at<int32_t>(h->ws, l.task_off);
    ev.priv_off = at<int32_t>(h->ws, l.priv_off);
    ev.priv_ev_off = at<int32_t>(h->ws, l.priv_ev_off);
    ev.day_slot_off = at<int32_t>(h->ws, l.day_slot_off);
    ev.slot_pos = at<int32_t>(h->ws, l.slot_pos);
    // null without days in LDS: the day kernel then reads no staging lists
    ev.unit_stage_off = pk.unit_stage.empty() ? nullptr : at<int32_t>(h->ws, l.unit_stage_off);
    ev.unit_stage = pk.unit_stage.empty() ? nullptr : at<int32_t>(h->ws, l.unit_stage);
    ev.stage = at<int32_t>(h->ws, l.stage);
    ev.slot_key = at<uint32_t>(h->ws, l.slot_key);
    ev.lvl_ev_off = at<int64_t>(h->ws, l.lvl_ev_off);
    ev.slot_src = at<int32_t>(h->ws, l.ev_slot_src);
    ev.slot_dst = at<int32_t>(h->ws, l.ev_slot_dst);
    ev.lvl_off = at<int64_t>(h->ws, l.lvl_off);
    ev.lvl_ptr = at<int32_t>(h->ws, l.lvl_ptr);

    const unsigned long long ok = STATUS_OK;
    const int64_t S = (int64_t)h->n_inst * h->R, E = pk.n_events;

    struct Up {
        void *dst;
        const void *src;
        size_t bytes;
    };
    const Up ups[] = {
        {(void *)s.node_id, pk.node_id.data(), sizeof(int32_t) * h->Np},
        {(void *)s.inst, pk.inst.data(), sizeof(int32_t) * h->Np},
        {(void *)s.inst_off, pk.inst_off.data(), sizeof(int32_t) * h->n_inst},
        {(void *)s.seed, pk.seed.data(), sizeof(uint32_t) * h->n_inst},
        {(void *)s.coef, pk.coef.data(), sizeof(double) * S * h->Nt},
        {(void *)s.alpha, pk.alpha.data(), sizeof(double) * S},
        {(void *)s.beta, pk.beta.data(), sizeof(double) * S * 4},
        {(void *)s.repid, pk.repid.data(), sizeof(uint32_t) * S},
        {(void *)ev.g, pk.eg.data(), sizeof(int32_t) * E},
        {(void *)ev.gm, pk.egm.data(), sizeof(int32_t) * E},
        {(void *)ev.node, pk.enode.data(), sizeof(int32_t) * E},
        {(void *)ev.dest, pk.edest.data(), sizeof(int32_t) * E},
        {(void *)ev.n, pk.en.data(), sizeof(int32_t) * E},
        {(void *)ev.meta, pk.emeta.data(), sizeof(uint32_t) * E},
        {(void *)ev.smap, pk.esmap.data(), sizeof(uint32_t) * E},
        {(void *)ev.task_off, pk.task_off.data(), sizeof(int32_t) * (pk.n_tasks + 1)},
        {(void *)ev.priv_off, pk.priv_off.data(), sizeof(int32_t) * pk.priv_off.size()},
        {(void *)ev.priv_ev_off, pk.priv_ev_off.data(), sizeof(int32_t) * pk.priv_ev_off.size()},
        {(void *)ev.day_slot_off, pk.day_slot_off.data(), sizeof(int32_t) * pk.day_slot_off.size()},
        {(void *)ev.slot_pos, pk.slot_pos.data(), sizeof(int32_t) * pk.slot_pos.size()},
        {at<int32_t>(h->ws, l.unit_stage_off), pk.unit_stage_off.data(), sizeof(int32_t) * pk.unit_stage_off.size()},
        {at<int32_t>(h->ws, l.unit_stage), pk.unit_stage.data(), sizeof(int32_t) * pk.unit_stage.size()},
        {(void *)ev.slot_key, pk.slot_key.data(), sizeof(uint32_t) * pk.slot_key.size()},
        {(void *)ev.lvl_ev_off, pk.lvl_ev_off.data(), sizeof(int64_t) * pk.lvl_ev_off.size()},
        {(void *)ev.slot_src, pk.ev_slot_src.data(), sizeof(int32_t) * pk.ev_slot_src.size()},
        {(void *)ev.slot_dst, pk.ev_slot_dst.data(), sizeof(int32_t) * pk.ev_slot_dst.size()},
        {(void *)ev.lvl_off, pk.lvl_off.data(), sizeof(int64_t) * (pk.n_levels + 1)},
        {(void *)ev.lvl_ptr, pk.lvl_ptr.data(), sizeof(int32_t) * (h->D + 1)},
        {(void *)s.rec_slot, pk.rec_slot.data(), sizeof(int32_t) * h->D},
        {(void *)s.heavy_pos, pk.heavy_pos.data(), sizeof(int32_t) * pk.heavy_pos.size()},
        {(void *)s.pos_region, pk.pos_region.data(), s.n_regions ? sizeof(int32_t) * pk.pos_region.size() : 0},
        {(void *)s.unit_heavy, pk.unit_heavy.data(), s.n_heavy ? pk.unit_heavy.size() : 0},
        {(void *)s.unit_group, pk.unit_group.data(), pk.unit_group.size()},
    };
    for (const Up &up : ups) {
        if (up.bytes == 0) continue;
        rc = check_device(hipMemcpy(up.dst, up.src, up.bytes, hipMemcpyHostToDevice), &err, "upload");
        if (rc) {
            sim_destroy(h);
            return rc;
        }
    }
    rc = check_device(hipMemset(at<char>(h->ws, l.prevalence), 0, l.rec_slot - l.prevalence), &err, "clear records");
    if (!rc && l.goal_ref > l.regional)
        rc = check_device(hipMemset(at<char>(h->ws, l.regional), 0, l.goal_ref - l.regional), &err, "clear regional records");
    for (int32_t j = 0; !rc && j < std::max(h->n_slots, 1); ++j)
        rc = check_device(hipMemcpy(s.status + j, &ok, sizeof ok, hipMemcpyHostToDevice), &err, "upload status");
    if (rc) {
        sim_destroy(h);
        return rc;
    }
    if (h->n_slots > 0) return create_slots(h, ps[0], out);
    // initial state: every replicate of an instance starts from its (u0, v0); padding holds zeros
    std::vector<int32_t> u((size_t)h->Nc * h->L, 0);
    std::vector<double> v(h->L, 0.0);
    for (int32_t k = 0; k < n; ++k)
        for (int64_t i = 0; i < ps[k]->n_nodes; ++i)
            for (int r = 0; r < h->R; ++r) {
                const int64_t lane = (int64_t)h->lane_of[pk.inst_off[k] + i] * h->RL + r;
                for (int c = 0; c < h->Nc; ++c) u[(size_t)c * h->L + lane] = ps[k]->u0[i * h->Nc + c];
                v[lane] = ps[k]->v0[i];
            }
    if (h->L > 0) {
        rc = check_device(hipMemcpy(s.u, u.data(), sizeof(int32_t) * u.size(), hipMemcpyHostToDevice), &err, "upload u0");
        if (!rc) rc = check_device(hipMemcpy(s.phi, v.data(), sizeof(double) * v.size(), hipMemcpyHostToDevice), &err, "upload v0");
        if (rc) {
            sim_destroy(h);
            return rc;
        }
    }
    *out = h;
    return SIM_OK;
}

}  // namespace

extern "C" {

int sim_plan_levels(int64_t n_events, const int32_t *ev_day, const int32_t *ev_kind,
                    const int32_t *ev_node, const int32_t *ev_dest, int32_t n_nodes, int32_t *level_out,
                    int32_t *task_out) {
    if (n_events < 0 || n_nodes < 0 || (n_events > 0 && (!ev_day || !ev_kind || !ev_node || !ev_dest || !level_out)))
        return SIM_EINVAL;
    int32_t max_day = -1;
    for (int64_t e = 0; e < n_events; ++e) {
        if (ev_node[e] < 0 || ev_node[e] >= n_nodes || ev_kind[e] < 0 || ev_kind[e] > 3 || ev_day[e] < 0 ||
            (e > 0 && ev_day[e] < ev_day[e - 1]) ||
            (ev_kind[e] == SIM_EXTERNAL && (ev_dest[e] < 0 || ev_dest[e] >= n_nodes)))
            return SIM_EINVAL;
        max_day = std::max(max_day, ev_day[e]);
    }
    std::vector<int32_t> task(task_out ? 0 : n_events);
    plan_levels(n_events, ev_day, ev_kind, ev_node, ev_dest, n_nodes, level_out, task_out ? task_out : task.data(),
                nullptr, max_day + 1);
    return SIM_OK;
}

size_t sim_workspace_bytes_batch(const sim_problem *const *problems, int32_t n_problems, const sim_device_opts *o) {
    std::string err;
    Packed pk;
    if (o && check_opts(*o, &err)) return 0;
    if (build_packed(problems, n_problems, o ? o->events_mode : SIM_EVENTS_LEVELS, &pk, &err, 0, o) != SIM_OK)
        return 0;
    return layout_of(pk, problems[0]).total;
}

size_t sim_workspace_bytes(const sim_problem *p, const sim_device_opts *o) {
    return sim_workspace_bytes_batch(&p, 1, o);
}

int sim_create(const sim_problem *p, const sim_device_opts *o, sim_handle **out) { return create(&p, 1, o, out); }

int sim_create_batch(const sim_problem *const *problems, int32_t n_problems, const sim_device_opts *o,
                     sim_handle **out) {
    return create(problems, n_problems, o, out);
}

int sim_run(sim_handle *h, int32_t n_days) {
    if (!h) return SIM_EINVAL;
    h->err.clear();
    if (h->n_slots) return h->err = "a slot handle advances with sim_slots_step", SIM_ESTATE;
    if (n_days < 0) return h->err = "n_days < 0", SIM_EINVAL;
    if (n_days == 0) n_days = h->D - h->day;
    if (h->day + n_days > h->D) return h->err = fmt("run of %d days from day %d passes the horizon %d", n_days, h->day, h->D), SIM_ESTATE;
    if (n_days == 0) return SIM_OK;
    const int32_t d0 = h->day, d1 = h->day + n_days;
    const int64_t S = (int64_t)h->n_inst * h->R;
    // records of the days about to be simulated start from zero
    int rc = check_device(hipMemsetAsync(h->st.prevalence + (size_t)d0 * S, 0, sizeof(int32_t) * n_days * S, h->stream), &h->err, "clear");
    if (!rc) rc = check_device(hipMemsetAsync(h->st.transitions + (size_t)d0 * S, 0, sizeof(int64_t) * n_days * S, h->stream), &h->err, "clear");
    if (!rc) rc = check_device(hipMemsetAsync(h->st.totals + (size_t)d0 * S * h->Nc, 0, sizeof(int64_t) * n_days * S * h->Nc, h->stream), &h->err, "clear");
    if (!rc) rc = check_device(hipMemsetAsync(h->st.max_fired + (size_t)d0 * S, 0, sizeof(int32_t) * n_days * S, h->stream), &h->err, "clear");
    if (!rc && h->st.n_regions > 0) {
        const size_t per_day = (size_t)S * h->st.n_regions * h->Nc;
        rc = check_device(hipMemsetAsync(h->st.regional + (size_t)d0 * per_day, 0, sizeof(int64_t) * n_days * per_day, h->stream),
                          &h->err, "clear");
    }
    if (rc) return rc;
    if (h->launch == SIM_LAUNCH_PERSISTENT && h->L > 0) {
        char why[256] = {0};
        hipError_t e = timed(h, SIM_K_PERSIST, [&] {
            return launch_persistent(h->model, h->st, h->ev, d0, d1, h->layout, h->stream, why, sizeof why);
        });
        if (e != hipSuccess) return h->err = fmt("persistent launch: %s %s", hipGetErrorString(e), why), SIM_EDEVICE;
    } else {
        for (int32_t d = d0; d < d1; ++d) {
            hipError_t e = timed(h, SIM_K_DAY, [&] { return launch_day(h->model, h->st, h->ev, d, d > d0, 1, h->layout, h->stream); });
            if (e != hipSuccess) return h->err = fmt("day kernel: %s", hipGetErrorString(e)), SIM_EDEVICE;
            // a day that fits runs its levels in LDS; otherwise big levels get a
            // launch of their own and runs of small ones share one workgroup
            int32_t lv = h->lvl_ptr[d];
            const int32_t lv_end = h->lvl_ptr[d + 1];
            if (h->day_slot_off[d + 1] > h->day_slot_off[d]) {
                EventDayArgs a{};
                a.lv0 = lv;
                a.nl = lv_end - lv;
                a.s0 = h->day_slot_off[d];
                a.ns = h->day_slot_off[d + 1] - a.s0;
                a.e0 = h->lvl_ev_off[lv];
                a.ne = h->lvl_ev_off[lv_end] - a.e0;
                e = timed(h, SIM_K_EVENTS, [&] { return launch_event_day(h->model, h->st, h->ev, d, a, h->stream); });
                if (e != hipSuccess) return h->err = fmt("event kernel: %s", hipGetErrorString(e)), SIM_EDEVICE;
                lv = lv_end;
            }
            while (lv < lv_end) {
                const int64_t size = (h->lvl_off[lv + 1] - h->lvl_off[lv]) * h->RL;
                if (size > h->small_level) {
                    e = timed(h, SIM_K_EVENTS, [&] {
                        return launch_events(h->model, h->st, h->ev, d, h->lvl_off[lv], h->lvl_off[lv + 1], h->stream);
                    });
                    ++lv;
                } else {
                    int32_t stop = lv + 1;
                    while (stop < lv_end && (h->lvl_off[stop + 1] - h->lvl_off[stop]) * h->RL <= h->small_level) ++stop;
                    const int32_t a = lv;
                    e = timed(h, SIM_K_EVENTS, [&] { return launch_event_levels(h->model, h->st, h->ev, d, a, stop, h->stream); });
                    lv = stop;
                }
                if (e != hipSuccess) return h->err = fmt("event kernel: %s", hipGetErrorString(e)), SIM_EDEVICE;
            }
        }
        hipError_t e = timed(h, SIM_K_CLOSE, [&] { return launch_day(h->model, h->st, h->ev, d1, 1, 0, h->layout, h->stream); });
        if (e != hipSuccess) return h->err = fmt("closing kernel: %s", hipGetErrorString(e)), SIM_EDEVICE;
    }
    h->day = d1;
    return SIM_OK;
}

int sim_sync(sim_handle *h) {
    if (!h) return SIM_EINVAL;
    int rc = check_device(hipStreamSynchronize(h->stream), &h->err, "synchronize");
    if (rc) return rc;
    if (h->n_slots) return SIM_OK;  // errors are reported per slot by sim_slot_query
    unsigned long long st = 0;
    rc = check_device(hipMemcpy(&st, h->st.status, sizeof st, hipMemcpyDeviceToHost), &h->err, "status");
    if (rc) return rc;
    if (st == STATUS_OK) return SIM_OK;
    const unsigned long long set = st & 0xffffffffull;
    const long long inst = (long long)(set / h->R), rep = (long long)(set % h->R);
    if ((st >> 32) == STATUS_LIMIT_TAG) {
        h->err = fmt("a node exceeded %d SSA transitions in one day (replicate %lld", SIM_MAX_FIRED, rep);
        if (h->n_inst > 1) h->err += fmt(" of instance %lld", inst);
        h->err += ")";
        return SIM_ELIMIT;
    }
    const int64_t gm = (int64_t)(st >> 32);
    const int64_t local = gm < (int64_t)h->ev_local.size() ? h->ev_local[gm] : gm;
    const int32_t day = gm < (int64_t)h->ev_day.size() ? h->ev_day[gm] : -1;
    h->err = fmt("infeasible event %lld (replicate %lld)", (long long)local, rep);
    if (h->n_inst > 1) h->err += fmt(" of instance %lld", inst);
    h->err += fmt(" on day %d: it asks for more individuals than the selected compartments hold", day);
    return SIM_EINFEASIBLE;
}

int sim_trajectory(sim_handle *h, sim_output *out) {
    if (!h || !out) return SIM_EINVAL;
    if (h->n_slots) return h->err = "a slot handle returns results with sim_slot_fetch", SIM_ESTATE;
    int rc = sim_sync(h);
    if (rc) return rc;
    const size_t DS = (size_t)h->D * h->n_inst * h->R;
    struct Down {
        void *dst;
        const void *src;
        size_t bytes;
    } downs[] = {
        {out->prevalence, h->st.prevalence, sizeof(int32_t) * DS},
        {out->transitions, h->st.transitions, sizeof(int64_t) * DS},
        {out->totals, h->st.totals, sizeof(int64_t) * DS * h->Nc},
        {out->snap_u, h->st.snap_u, sizeof(int32_t) * h->n_record * (size_t)h->R * h->n_nodes * h->Nc},
        {out->snap_v, h->st.snap_v, sizeof(double) * h->n_record * (size_t)h->R * h->n_nodes},
        {out->regional, h->st.regional, sizeof(int64_t) * DS * h->st.n_regions * h->Nc},
        {out->max_transitions, h->st.max_fired, sizeof(int32_t) * DS},
    };
    for (const Down &d : downs) {
        if (!d.dst || d.bytes == 0) continue;
        rc = check_device(hipMemcpy(d.dst, d.src, d.bytes, hipMemcpyDeviceToHost), &h->err, "download");
        if (rc) return rc;
    }
    return SIM_OK;
}

int sim_get_state(sim_handle *h, int32_t *u, double *v, int32_t *day) {
    if (!h) return SIM_EINVAL;
    if (h->n_slots) return h->err = "a slot handle returns state with sim_slot_state", SIM_ESTATE;
    int rc = sim_sync(h);
    if (rc) return rc;
    if (day) *day = h->day;
    if (h->L == 0) return SIM_OK;
    std::vector<int32_t> du((size_t)h->Nc * h->L);
    std::vector<double> dv(h->L);
    rc = check_device(hipMemcpy(du.data(), h->st.u, sizeof(int32_t) * du.size(), hipMemcpyDeviceToHost), &h->err, "download u");
    if (!rc) rc = check_device(hipMemcpy(dv.data(), h->st.phi, sizeof(double) * dv.size(), hipMemcpyDeviceToHost), &h->err, "download v");
    if (rc) return rc;
    for (int r = 0; r < h->R; ++r)
        for (int64_t i = 0; i < h->n_nodes; ++i) {
            const int64_t lane = (int64_t)h->lane_of[i] * h->RL + r;
            if (u)
                for (int c = 0; c < h->Nc; ++c) u[((size_t)r * h->n_nodes + i) * h->Nc + c] = du[(size_t)c * h->L + lane];
            if (v) v[(size_t)r * h->n_nodes + i] = dv[lane];
        }
    return SIM_OK;
}

int sim_set_state(sim_handle *h, const int32_t *u, const double *v, int32_t day) {
    if (!h || !u || !v) return SIM_EINVAL;
    h->err.clear();
    if (h->n_slots) return h->err = "a slot handle takes state with sim_slot_start", SIM_ESTATE;
    if (day < 0 || day > h->D) return h->err = "day out of range", SIM_ESTATE;
    int rc = check_device(hipStreamSynchronize(h->stream), &h->err, "synchronize");
    if (rc) return rc;
    std::vector<int32_t> du((size_t)h->Nc * h->L, 0);
    std::vector<double> dv(h->L, 0.0);
    for (int r = 0; r < h->R; ++r)
        for (int64_t i = 0; i < h->n_nodes; ++i) {
            const int64_t lane = (int64_t)h->lane_of[i] * h->RL + r;
            for (int c = 0; c < h->Nc; ++c) {
                const int32_t x = u[((size_t)r * h->n_nodes + i) * h->Nc + c];
                if (x < 0) return h->err = "negative count in state", SIM_EINVAL;
                du[(size_t)c * h->L + lane] = x;
            }
            const double y = v[(size_t)r * h->n_nodes + i];
            if (!(y >= 0.0) || !std::isfinite(y)) return h->err = "phi must be finite and >= 0", SIM_EINVAL;
            dv[lane] = y;
        }
    const unsigned long long ok = STATUS_OK;
    if (h->L > 0) {
        rc = check_device(hipMemcpy(h->st.u, du.data(), sizeof(int32_t) * du.size(), hipMemcpyHostToDevice), &h->err, "upload u");
        if (!rc) rc = check_device(hipMemcpy(h->st.phi, dv.data(), sizeof(double) * dv.size(), hipMemcpyHostToDevice), &h->err, "upload v");
    }
    if (!rc) rc = check_device(hipMemcpy(h->st.status, &ok, sizeof ok, hipMemcpyHostToDevice), &h->err, "reset status");
    if (rc) return rc;
    h->day = day;
    return SIM_OK;
}

int64_t sim_levels(const sim_handle *h, int32_t d, int32_t *max_levels) {
    if (!h) return -1;
    int32_t mx = 0;
    for (int32_t i = 0; i < h->D; ++i) mx = std::max(mx, h->lvl_ptr[i + 1] - h->lvl_ptr[i]);
    if (max_levels) *max_levels = mx;
    if (d < 0) return h->lvl_ptr[h->D];
    if (d >= h->D) return -1;
    return h->lvl_ptr[d + 1] - h->lvl_ptr[d];
}

int sim_kernel_times(sim_handle *h, int32_t enable, double *ms, int64_t *launches) {
    if (!h) return SIM_EINVAL;
    int rc = check_device(hipStreamSynchronize(h->stream), &h->err, "synchronize");
    if (rc) return rc;
    rc = collect_marks(h);
    if (rc) return rc;
    if (enable < 0) {
        for (int k = 0; k < 4; ++k) h->ms[k] = 0, h->launches[k] = 0;
    } else {
        h->timing = enable != 0;
    }
    for (int k = 0; k < 4; ++k) {
        if (ms) ms[k] = h->ms[k];
        if (launches) launches[k] = h->launches[k];
    }
    return SIM_OK;
}

int sim_goal(sim_handle *h, int32_t instance, const int64_t *reference, int32_t d_begin, int32_t d_end, double *G2,
             double *VG2) {
    if (!h || !reference || !G2 || !VG2) return SIM_EINVAL;
    h->err.clear();
    if (h->st.n_regions <= 0) return h->err = "the problem has no regions", SIM_ESTATE;
    if (instance < 0 || instance >= h->n_inst) return h->err = "instance out of range", SIM_EINVAL;
    if (d_begin < 0 || d_end > h->D || d_end < d_begin) return h->err = "days out of range", SIM_EINVAL;
    if (d_end > h->day) return h->err = fmt("day %d has not been simulated", d_end - 1), SIM_ESTATE;
    *G2 = 0.0;
    *VG2 = 0.0;
    const int32_t n = d_end - d_begin;
    if (n == 0) return SIM_OK;
    const size_t per_day = (size_t)h->st.n_regions * h->Nc;
    int64_t *ref = at<int64_t>(h->ws, h->lay.goal_ref);
    double *part = at<double>(h->ws, h->lay.goal_part);
    int rc = check_device(hipMemcpyAsync(ref, reference + (size_t)d_begin * per_day, sizeof(int64_t) * n * per_day,
                                         hipMemcpyHostToDevice, h->stream), &h->err, "upload reference");
    if (!rc)
        rc = check_device((hipError_t)launch_goal(h->st, h->Nc, (int64_t)instance * h->R, h->R, ref, d_begin, n, part,
                                                  h->stream), &h->err, "goal kernel");
    std::vector<double> host(2 * (size_t)n);
    if (!rc) rc = sim_sync(h);
    if (!rc) rc = check_device(hipMemcpy(host.data(), part, sizeof(double) * host.size(), hipMemcpyDeviceToHost), &h->err, "download");
    if (rc) return rc;
    // the integral over t as the sum over days, in day order
    for (int32_t k = 0; k < n; ++k) {
        *G2 += host[k];
        *VG2 += host[n + k];
    }
    return SIM_OK;
}

int sim_goal_noalloc(sim_handle *h, int32_t instance, const int64_t *reference, int32_t d_begin, int32_t d_end,
                     double *G2, double *VG2) {
    if (!h || !reference || !G2 || !VG2) return SIM_EINVAL;
    h->err.clear();
    if (h->st.n_regions <= 0) return h->err = "the problem has no regions", SIM_ESTATE;
    if (instance < 0 || instance >= h->n_inst) return h->err = "instance out of range", SIM_EINVAL;
    if (d_begin < 0 || d_end > h->D || d_end < d_begin) return h->err = "days out of range", SIM_EINVAL;
    if (d_end > h->day) return h->err = fmt("day %d has not been simulated", d_end - 1), SIM_ESTATE;
    const int32_t n = d_end - d_begin;
    const size_t per_day = (size_t)h->st.n_regions * h->Nc;
    // the staged reference, the day terms and the two sums, each 256-byte aligned
    const size_t ref_bytes = align_up(sizeof(int64_t) * per_day * n);
    const size_t part_bytes = align_up(sizeof(double) * 2 * (size_t)n);
    const size_t need = ref_bytes + part_bytes + sizeof(double) * 2;
    if (need > kScratchBytes)
        return h->err = fmt("%d days of %zu regional sums need %zu bytes of scratch; at most %zu", n,
                            per_day, need, kScratchBytes), SIM_EINVAL;
    int dev = -1;
    int rc = check_device(hipGetDevice(&dev), &h->err, "current device");
    if (rc) return rc;
    if (dev != h->device)
        return h->err = fmt("device %d is current; the handle lives on device %d", dev, h->device), SIM_EINVAL;
    void *base = nullptr;
    rc = check_device((hipError_t)scratch_address(&base), &h->err, "scratch address");
    if (rc) return rc;
    int64_t *ref = at<int64_t>(base, 0);
    double *part = at<double>(base, ref_bytes);
    double *sums = at<double>(base, ref_bytes + part_bytes);
    double host[2] = {0.0, 0.0};
    if (n > 0) {
        rc = check_device(hipMemcpyAsync(ref, reference + (size_t)d_begin * per_day, sizeof(int64_t) * n * per_day,
                                         hipMemcpyHostToDevice, h->stream), &h->err, "upload reference");
        if (!rc)
            rc = check_device((hipError_t)launch_goal(h->st, h->Nc, (int64_t)instance * h->R, h->R, ref, d_begin, n,
                                                      part, h->stream), &h->err, "goal kernel");
        if (!rc) rc = check_device((hipError_t)launch_goal_sum(part, n, sums, h->stream), &h->err, "goal sum kernel");
        if (!rc) rc = sim_sync(h);
        if (!rc) rc = check_device(hipMemcpy(host, sums, sizeof host, hipMemcpyDeviceToHost), &h->err, "download");
        if (rc) return rc;
    }
    *G2 = host[0];
    *VG2 = host[1];
    return SIM_OK;
}

void sim_destroy(sim_handle *h) {
    if (!h) return;
    (void)hipStreamSynchronize(h->stream);
    for (const auto &m : h->marks) {
        (void)hipEventDestroy(m.a);
        (void)hipEventDestroy(m.b);
    }
    for (hipEvent_t e : h->ev_pool) (void)hipEventDestroy(e);
    for (hipEvent_t e : h->in_flight) (void)hipEventDestroy(e);
    for (auto &sl : h->slots) {
        if (sl.staged) (void)hipEventDestroy(sl.staged);
        if (sl.fetched) (void)hipEventDestroy(sl.fetched);
    }
    if (h->stage) (void)hipHostFree(h->stage);
    for (hipEvent_t e : h->run_up)
        if (e) (void)hipEventDestroy(e);
    if (h->run_host) (void)hipHostFree(h->run_host);
    if (h->own_ws && h->ws) (void)hipFree(h->ws);
    delete h;
}

size_t sim_slots_workspace_bytes(const sim_problem *network, int32_t n_slots, const sim_device_opts *o) {
    std::string err;
    Packed pk;
    if (o && check_opts(*o, &err)) return 0;
    if (n_slots < 1 || build_packed(&network, 1, SIM_EVENTS_LEVELS, &pk, &err, n_slots, o) != SIM_OK) return 0;
    return layout_of(pk, network).total;
}

int sim_slots_create(const sim_problem *network, int32_t n_slots, const sim_device_opts *opts, sim_handle **out) {
    if (n_slots < 1) {
        g_create_error = "n_slots must be >= 1";
        if (out) *out = nullptr;
        return SIM_EINVAL;
    }
    return create(&network, 1, opts, out, n_slots);
}

int sim_slot_start(sim_handle *h, int32_t slot, int32_t n_rep, int32_t horizon, const double *coef,
                   const double *alpha, const double *beta, const uint32_t *replicate_id) {
    if (!h) return SIM_EINVAL;
    h->err.clear();
    if (!h->n_slots) return h->err = "not a slot handle", SIM_ESTATE;
    if (slot < 0 || slot >= h->n_slots) return h->err = fmt("slot %d out of range", slot), SIM_EINVAL;
    sim_handle::Slot &sl = h->slots[slot];
    if (sl.state == SLOT_RUNNING) return h->err = fmt("slot %d is running", slot), SIM_ESTATE;
    if (n_rep < 1 || n_rep > h->slot_lanes) return h->err = fmt("n_rep must be in [1, %d]", h->slot_lanes), SIM_EINVAL;
    if (horizon < 1 || horizon > h->D) return h->err = fmt("horizon must be in [1, %d]", h->D), SIM_EINVAL;
    if (!coef || !alpha || !beta) return h->err = "a parameter array is NULL", SIM_EINVAL;
    if (int rc = check_params(h->Nt, n_rep, coef, alpha, beta, &h->err)) return rc;
    // the staging of this slot is reused once its previous upload has run
    int rc = check_device(hipEventSynchronize(sl.staged), &h->err, "staging");
    if (rc) return rc;
    char *st = h->stage + (size_t)slot * h->stage_stride;
    double *sc = reinterpret_cast<double *>(st), *sa = sc + 64 * h->Nt, *sb = sa + 64;
    uint32_t *sr = reinterpret_cast<uint32_t *>(sb + 64 * 4);
    std::memcpy(sc, coef, sizeof(double) * n_rep * h->Nt);
    std::memcpy(sa, alpha, sizeof(double) * n_rep);
    std::memcpy(sb, beta, sizeof(double) * n_rep * 4);
    for (int32_t r = 0; r < n_rep; ++r) sr[r] = replicate_id ? replicate_id[r] : (uint32_t)r;
    const int64_t set0 = (int64_t)slot * h->slot_lanes;
    DevState &s = h->st;
    struct Up {
        void *dst;
        const void *src;
        size_t bytes;
    } ups[] = {
        {(void *)(s.coef + set0 * h->Nt), sc, sizeof(double) * n_rep * h->Nt},
        {(void *)(s.alpha + set0), sa, sizeof(double) * n_rep},
        {(void *)(s.beta + set0 * 4), sb, sizeof(double) * n_rep * 4},
        {(void *)(s.repid + set0), sr, sizeof(uint32_t) * n_rep},
    };
    for (const Up &up : ups) {
        rc = check_device(hipMemcpyAsync(up.dst, up.src, up.bytes, hipMemcpyHostToDevice, h->stream), &h->err, "upload parameters");
        if (rc) return rc;
    }
    rc = check_device(hipEventRecord(sl.staged, h->stream), &h->err, "event");
    if (rc) return rc;
    const SlotInfo info{h->step, n_rep, horizon, 0};
    rc = check_device((hipError_t)launch_slot_init(s, h->Nc, at<int32_t>(h->ws, h->lay.u0), at<double>(h->ws, h->lay.v0),
                                                   slot, info, h->stream), &h->err, "slot start");
    if (rc) return rc;
    sl.state = SLOT_RUNNING;
    sl.t0 = h->step;
    sl.n_rep = n_rep;
    sl.horizon = horizon;
    return SIM_OK;
}

int sim_slots_step(sim_handle *h, int32_t *finished, int32_t *n_finished) {
    if (!h) return SIM_EINVAL;
    h->err.clear();
    if (!h->n_slots) return h->err = "not a slot handle", SIM_ESTATE;
    if (n_finished) *n_finished = 0;
    const int32_t T = h->step;
    // the levels of every running slot's day
    int32_t k_max = 0;
    bool any = false;
    for (const auto &sl : h->slots) {
        if (sl.state != SLOT_RUNNING) continue;
        any = true;
        const int32_t d = T - sl.t0;
        if (d < sl.horizon) k_max = std::max(k_max, h->lvl_ptr[d + 1] - h->lvl_ptr[d]);
    }
    if (!any) return SIM_OK;
    std::vector<int64_t> size(k_max, 0);  // largest (task, lane) count of level k over the slots
    // the run lists of this step: slots with a day of events, then columns
    // with a running slot (every running slot has its day's phi update, its
    // SSA or both), into the next entry of the pinned ring
    const int32_t n_cols_all = h->RL / 64, per_col = 64 / h->slot_lanes;
    const size_t run_len = (size_t)h->n_slots + n_cols_all;
    const int ring = T % sim_handle::kRunRing;
    int rc = check_device(hipEventSynchronize(h->run_up[ring]), &h->err, "run list upload");
    if (rc) return rc;
    int32_t *run = h->run_host + run_len * ring, *cols = run + h->n_slots;
    int32_t n_run = 0, n_cols = 0;
    for (int32_t j = 0; j < h->n_slots; ++j) {
        const auto &sl = h->slots[j];
        if (sl.state != SLOT_RUNNING) continue;
        if (n_cols == 0 || cols[n_cols - 1] != j / per_col) cols[n_cols++] = j / per_col;
        const int32_t d = T - sl.t0;
        if (d >= sl.horizon) continue;
        run[n_run++] = j;
        for (int32_t k = 0; k < h->lvl_ptr[d + 1] - h->lvl_ptr[d]; ++k) {
            const int32_t lv = h->lvl_ptr[d] + k;
            size[k] = std::max(size[k], (h->lvl_off[lv + 1] - h->lvl_off[lv]) * h->slot_lanes);  // tasks x lanes
        }
    }
    rc = check_device(hipMemcpyAsync(const_cast<int32_t *>(h->st.run_slots), run, sizeof(int32_t) * run_len,
                                     hipMemcpyHostToDevice, h->stream), &h->err, "run list upload");
    if (!rc) rc = check_device(hipEventRecord(h->run_up[ring], h->stream), &h->err, "event");
    if (rc) return rc;
    hipError_t e = timed(h, SIM_K_DAY, [&] { return launch_slot_day(h->model, h->st, h->ev, T, n_cols, h->stream); });
    if (e != hipSuccess) return h->err = fmt("day kernel: %s", hipGetErrorString(e)), SIM_EDEVICE;
    // big levels get a launch of their own; runs of small ones one workgroup per slot
    int32_t k = 0;
    while (k < k_max) {
        int32_t stop = k + 1;
        if (size[k] <= kSlotSmallLevel)
            while (stop < k_max && size[stop] <= kSlotSmallLevel) ++stop;
        const int32_t a = k;
        e = timed(h, SIM_K_EVENTS, [&] {
            return launch_slot_events(h->model, h->st, h->ev, T, a, stop, size[a], n_run, h->stream);
        });
        if (e != hipSuccess) return h->err = fmt("event kernel: %s", hipGetErrorString(e)), SIM_EDEVICE;
        k = stop;
    }
    hipEvent_t done = take_event(h);
    if (!done) return h->err = "event", SIM_EDEVICE;
    rc = check_device(hipEventRecord(done, h->stream), &h->err, "event");
    if (rc) return rc;
    h->in_flight.push_back(done);
    h->step = T + 1;
    int32_t nf = 0;
    for (int32_t j = 0; j < h->n_slots; ++j) {
        auto &sl = h->slots[j];
        if (sl.state == SLOT_RUNNING && T - sl.t0 == sl.horizon) {
            sl.state = SLOT_DONE;
            if (finished) finished[nf] = j;
            ++nf;
        }
    }
    if (n_finished) *n_finished = nf;
    return SIM_OK;
}

int32_t sim_slots_in_flight(sim_handle *h) {
    if (!h || !h->n_slots) return -1;
    while (!h->in_flight.empty() && hipEventQuery(h->in_flight.front()) == hipSuccess) {
        h->ev_pool.push_back(h->in_flight.front());
        h->in_flight.pop_front();
    }
    return (int32_t)h->in_flight.size();
}

int sim_slot_fetch(sim_handle *h, int32_t slot, int32_t *prevalence, int64_t *transitions, int64_t *totals) {
    if (!h) return SIM_EINVAL;
    h->err.clear();
    if (!h->n_slots) return h->err = "not a slot handle", SIM_ESTATE;
    if (slot < 0 || slot >= h->n_slots) return h->err = fmt("slot %d out of range", slot), SIM_EINVAL;
    sim_handle::Slot &sl = h->slots[slot];
    if (sl.state != SLOT_DONE) return h->err = fmt("slot %d has no finished run to fetch", slot), SIM_ESTATE;
    if (sl.fetch_pending) return h->err = fmt("slot %d: the previous fetch has not been collected", slot), SIM_ESTATE;
    const size_t S = (size_t)h->RL, n = (size_t)sl.n_rep, H = (size_t)sl.horizon, c0 = (size_t)slot * h->slot_lanes,
                 Nc = h->Nc;
    const DevState &s = h->st;
    hipError_t e = hipSuccess;
    if (prevalence)
        e = hipMemcpy2DAsync(prevalence, n * sizeof(int32_t), s.prevalence + c0, S * sizeof(int32_t), n * sizeof(int32_t), H,
                             hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess && transitions)
        e = hipMemcpy2DAsync(transitions, n * sizeof(int64_t), s.transitions + c0, S * sizeof(int64_t), n * sizeof(int64_t), H,
                             hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess && totals)
        e = hipMemcpy2DAsync(totals, n * Nc * sizeof(int64_t), s.totals + c0 * Nc, S * Nc * sizeof(int64_t),
                             n * Nc * sizeof(int64_t), H, hipMemcpyDeviceToHost, h->stream);
    unsigned long long *word = error_word(h, slot);
    if (e == hipSuccess)
        e = hipMemcpyAsync(word, s.status + slot, sizeof *word, hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipEventRecord(sl.fetched, h->stream);
    if (e != hipSuccess) return check_device(e, &h->err, "fetch");
    sl.state = SLOT_FREE;
    sl.fetch_pending = true;
    return SIM_OK;
}

int sim_slot_query(sim_handle *h, int32_t slot) {
    if (!h) return SIM_EINVAL;
    if (!h->n_slots) return h->err = "not a slot handle", SIM_ESTATE;
    if (slot < 0 || slot >= h->n_slots) return h->err = fmt("slot %d out of range", slot), SIM_EINVAL;
    sim_handle::Slot &sl = h->slots[slot];
    if (!sl.fetch_pending) return h->err = fmt("slot %d has no fetch to collect", slot), SIM_ESTATE;
    const hipError_t q = hipEventQuery(sl.fetched);
    if (q == hipErrorNotReady) return 1;
    if (q != hipSuccess) return check_device(q, &h->err, "query");
    sl.fetch_pending = false;
    const unsigned long long st = *error_word(h, slot);
    if (st == STATUS_OK) return SIM_OK;
    const long long rep = (long long)(st & 0xffffffffull) - (long long)slot * h->slot_lanes;
    if ((st >> 32) == STATUS_LIMIT_TAG) {
        h->err = fmt("slot %d: a node exceeded %d SSA transitions in one day (replicate %lld)", slot, SIM_MAX_FIRED, rep);
        return SIM_ELIMIT;
    }
    const int64_t gm = (int64_t)(st >> 32);
    const int32_t day = gm < (int64_t)h->ev_day.size() ? h->ev_day[gm] : -1;
    h->err = fmt("slot %d: infeasible event %lld (replicate %lld) on day %d: it asks for more individuals than the "
                 "selected compartments hold", slot, (long long)gm, rep, day);
    return SIM_EINFEASIBLE;
}

int sim_slot_state(sim_handle *h, int32_t slot, int32_t *u, double *v) {
    if (!h) return SIM_EINVAL;
    h->err.clear();
    if (!h->n_slots) return h->err = "not a slot handle", SIM_ESTATE;
    if (slot < 0 || slot >= h->n_slots) return h->err = fmt("slot %d out of range", slot), SIM_EINVAL;
    const sim_handle::Slot &sl = h->slots[slot];
    if (sl.n_rep == 0) return h->err = fmt("slot %d never started", slot), SIM_ESTATE;
    int rc = check_device(hipStreamSynchronize(h->stream), &h->err, "synchronize");
    if (rc) return rc;
    const size_t n = (size_t)sl.n_rep, Np = (size_t)h->Np, c0 = (size_t)slot * h->slot_lanes;
    std::vector<int32_t> du((size_t)h->Nc * Np * n);
    std::vector<double> dv(Np * n);
    for (int c = 0; c < h->Nc && !rc; ++c)
        rc = check_device(hipMemcpy2D(du.data() + (size_t)c * Np * n, n * sizeof(int32_t), h->st.u + (size_t)c * h->L + c0,
                                      (size_t)h->RL * sizeof(int32_t), n * sizeof(int32_t), Np, hipMemcpyDeviceToHost),
                          &h->err, "download u");
    if (!rc)
        rc = check_device(hipMemcpy2D(dv.data(), n * sizeof(double), h->st.phi + c0, (size_t)h->RL * sizeof(double),
                                      n * sizeof(double), Np, hipMemcpyDeviceToHost), &h->err, "download v");
    if (rc) return rc;
    for (size_t r = 0; r < n; ++r)
        for (int64_t i = 0; i < h->n_nodes; ++i) {
            const size_t pos = (size_t)h->lane_of[i];
            if (u)
                for (int c = 0; c < h->Nc; ++c) u[(r * h->n_nodes + i) * h->Nc + c] = du[((size_t)c * Np + pos) * n + r];
            if (v) v[r * h->n_nodes + i] = dv[pos * n + r];
        }
    return SIM_OK;
}

const char *sim_last_error(const sim_handle *h) {
    return h ? h->err.c_str() : g_create_error.c_str();
}

}  // extern "C"
