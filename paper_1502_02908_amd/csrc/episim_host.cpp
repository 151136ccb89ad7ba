// Host side of the episim C ABI: validation of the problem statement, the
// dependency pass over the external events, device memory, and the day loop.
//
// The dependency pass is the GPU counterpart of the paper's re-arrangement of
// the event lists (Sec. 3.4, Algorithm 2's initialisation) and of its
// precedence rules between tasks that touch the same sub-domain (Sec. 3.6,
// rules 2(b) and 3(b)), applied at node granularity: within a day, an event
// that draws individuals from a node must follow every earlier event touching
// that node, and an event that adds to a node must follow every earlier draw
// from it; additions to one node commute. Each event gets the smallest level
// meeting these rules, so one level runs fully in parallel and levels run in
// order. The levels are computed once per handle and reused by every run and
// replicate, as the paper reuses its re-arranged lists across runs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
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

bool is_sampler(int kind) { return kind == SIM_EXIT || kind == SIM_INTERNAL || kind == SIM_EXTERNAL; }

// Level of every event within its day; events must already be sorted by day.
// Returns the number of levels of each day in day_levels (resized to n_days).
void plan_levels(int64_t n, const int32_t *day, const int32_t *kind, const int32_t *node,
                 const int32_t *dest, int32_t n_nodes, int32_t *level,
                 std::vector<int32_t> *day_levels, int32_t n_days) {
    // last level at which a node was touched at all / drawn from, valid for
    // the day stored in stamp (so nothing is cleared between days)
    std::vector<int32_t> stamp(n_nodes, -1), last_any(n_nodes, 0), last_draw(n_nodes, 0);
    if (day_levels) day_levels->assign(n_days > 0 ? n_days : 0, 0);
    auto get = [&](std::vector<int32_t> &a, int32_t x, int32_t d) {
        if (stamp[x] != d) {
            stamp[x] = d;
            last_any[x] = 0;
            last_draw[x] = 0;
        }
        return a[x];
    };
    for (int64_t e = 0; e < n; ++e) {
        const int32_t d = day[e];
        int32_t L = 1;
        const int32_t src = node[e];
        const bool draws = is_sampler(kind[e]);
        // the node an event adds to: ENTER adds at its node, EXTERNAL at dest
        const int32_t add = kind[e] == SIM_ENTER ? src : (kind[e] == SIM_EXTERNAL ? dest[e] : -1);
        if (draws) L = std::max(L, get(last_any, src, d) + 1);
        if (add >= 0) L = std::max(L, get(last_draw, add, d) + 1);
        level[e] = L;
        if (draws) {
            get(last_any, src, d);
            last_any[src] = std::max(last_any[src], L);
            last_draw[src] = L;
        }
        if (add >= 0) {
            get(last_any, add, d);
            last_any[add] = std::max(last_any[add], L);
        }
        if (day_levels) (*day_levels)[d] = std::max((*day_levels)[d], L);
    }
}

int check_device(hipError_t e, std::string *err, const char *what) {
    if (e == hipSuccess) return SIM_OK;
    *err = fmt("%s: %s", what, hipGetErrorString(e));
    return SIM_EDEVICE;
}

// Device buffer layout of one handle.
struct Layout {
    size_t u, phi, node_id, coef, alpha, beta, repid, shift, status, ev_g, ev_node, ev_dest, ev_n, ev_meta,
        lvl_off, lvl_ptr, prevalence, transitions, totals, snap_u, snap_v, rec_slot, total;
};

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

Layout layout_for(int64_t Nn, int64_t Nc, int64_t Nt, int64_t R, int64_t D, int64_t n_events,
                  int64_t n_shift_ids, int64_t n_levels, int64_t n_record) {
    Layout l{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off = align_up(off + std::max<size_t>(bytes, 1));
        return at;
    };
    const int64_t L = Nn * R;
    l.u = take(sizeof(int32_t) * Nc * L);
    l.phi = take(sizeof(double) * L);
    l.node_id = take(sizeof(int32_t) * Nn);
    l.coef = take(sizeof(double) * R * Nt);
    l.alpha = take(sizeof(double) * R);
    l.beta = take(sizeof(double) * R * 4);
    l.repid = take(sizeof(uint32_t) * R);
    l.shift = take(sizeof(int32_t) * MAXC * std::max<int64_t>(n_shift_ids, 1));
    l.status = take(sizeof(unsigned long long));
    l.ev_g = take(sizeof(int32_t) * n_events);
    l.ev_node = take(sizeof(int32_t) * n_events);
    l.ev_dest = take(sizeof(int32_t) * n_events);
    l.ev_n = take(sizeof(int32_t) * n_events);
    l.ev_meta = take(sizeof(uint32_t) * n_events);
    l.lvl_off = take(sizeof(int64_t) * (n_levels + 1));
    l.lvl_ptr = take(sizeof(int32_t) * (D + 1));
    l.prevalence = take(sizeof(int32_t) * D * R);
    l.transitions = take(sizeof(int64_t) * D * R);
    l.totals = take(sizeof(int64_t) * D * R * Nc);
    l.snap_u = take(sizeof(int32_t) * n_record * R * Nn * Nc);
    l.snap_v = take(sizeof(double) * n_record * R * Nn);
    l.rec_slot = take(sizeof(int32_t) * D);
    l.total = off;
    return l;
}

// Position of every node: herds sorted by size (largest first) are dealt out
// one per wavefront in turn, back and forth (snake order), so that the
// longest SSA chains of a day run in different wavefronts, start first, and
// share their wavefront with the lightest herds of the next round.
// perm[pos] = node, inv[node] = pos.
void order_nodes(const sim_problem *p, std::vector<int32_t> *perm, std::vector<int32_t> *inv) {
    const int64_t Nn = p->n_nodes, Nc = p->n_comp;
    std::vector<int64_t> size(Nn, 0);
    for (int64_t i = 0; i < Nn; ++i)
        for (int64_t c = 0; c < Nc; ++c) size[i] += p->u0[i * Nc + c];
    std::vector<int32_t> rank(Nn);
    for (int64_t i = 0; i < Nn; ++i) rank[i] = (int32_t)i;
    std::stable_sort(rank.begin(), rank.end(), [&](int32_t a, int32_t b) { return size[a] > size[b]; });
    const int64_t G = std::max<int64_t>(1, 64 / p->n_rep);  // nodes per wavefront
    const int64_t W = (Nn + G - 1) / G;                     // wavefronts
    perm->assign(Nn, 0);
    inv->assign(Nn, 0);
    int64_t q = 0;
    for (int64_t j = 0; j < G; ++j)
        for (int64_t ww = 0; ww < W; ++ww) {
            const int64_t w = (j & 1) ? W - 1 - ww : ww;
            const int64_t pos = w * G + j;
            if (pos >= Nn) continue;
            const int32_t node = rank[q++];
            (*perm)[pos] = node;
            (*inv)[node] = (int32_t)pos;
        }
}

uint32_t column_mask(const sim_problem *p, int32_t s) {
    uint32_t m = 0;
    for (int c = 0; c < p->n_comp; ++c)
        if (p->E[(size_t)c * p->n_select + s]) m |= 1u << c;
    return m;
}

// Full validation of the problem statement (the contract in episim.h).
int validate(const sim_problem *p, std::string *err) {
    if (!p) return *err = "problem is NULL", SIM_EINVAL;
    if (p->n_nodes < 0) return *err = "n_nodes < 0", SIM_EINVAL;
    if (p->n_comp < 1 || p->n_comp > SIM_MAX_COMP) return *err = "n_comp must be in [1, 8]", SIM_EINVAL;
    if (p->n_trans < 1 || p->n_trans > SIM_MAX_TRANS) return *err = "n_trans must be in [1, 8]", SIM_EINVAL;
    if (p->n_rep < 1) return *err = "n_rep must be >= 1", SIM_EINVAL;
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
        for (int c = 0; c < Nc; ++c) {
            const int32_t s = p->S[(size_t)c * Nt + k];
            if (c == a && s != -1) return *err = fmt("S[%d,%d] must be -1 (the reactant of transition %d)", c, k, k), SIM_EINVAL;
            if (c != a && s < 0) return *err = fmt("S[%d,%d] < 0 for a compartment that is not the reactant", c, k), SIM_EINVAL;
            if (s > 127) return *err = fmt("S[%d,%d] too large", c, k), SIM_EINVAL;
        }
    }
    for (int64_t i = 0; i < (int64_t)R * Nt; ++i)
        if (!(p->coef[i] >= 0.0) || !std::isfinite(p->coef[i])) return *err = "coef must be finite and >= 0", SIM_EINVAL;
    for (int r = 0; r < R; ++r) {
        if (!(p->alpha[r] >= 0.0) || !std::isfinite(p->alpha[r])) return *err = "alpha must be finite and >= 0", SIM_EINVAL;
        for (int q = 0; q < 4; ++q) {
            const double b = p->beta[r * 4 + q];
            if (!(b >= 0.0 && b <= 1.0)) return *err = "beta must be in [0, 1]", SIM_EINVAL;
        }
    }
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
    for (int64_t e = 0; e < p->n_events; ++e) {
        const int32_t d = p->ev_day[e], k = p->ev_kind[e], i = p->ev_node[e], s = p->ev_select[e];
        const int32_t h = p->ev_shift[e];
        if (d < 0 || d >= p->n_days) return *err = fmt("event %lld: day out of range", (long long)e), SIM_EINVAL;
        if (e > 0 && d < p->ev_day[e - 1]) return *err = fmt("event %lld: days not sorted", (long long)e), SIM_EINVAL;
        if (k < 0 || k > 3) return *err = fmt("event %lld: unknown kind", (long long)e), SIM_EINVAL;
        if (i < 0 || i >= p->n_nodes) return *err = fmt("event %lld: node out of range", (long long)e), SIM_EINVAL;
        if (k == SIM_EXTERNAL && (p->ev_dest[e] < 0 || p->ev_dest[e] >= p->n_nodes))
            return *err = fmt("event %lld: dest out of range", (long long)e), SIM_EINVAL;
        if (p->ev_n[e] < 0 || p->ev_n[e] > SIM_MAX_EVENT_N)
            return *err = fmt("event %lld: n must be in [0, %d]", (long long)e, SIM_MAX_EVENT_N), SIM_EINVAL;
        if (s < 0 || s >= p->n_select) return *err = fmt("event %lld: select out of range", (long long)e), SIM_EINVAL;
        if (h < -1 || h >= p->n_shift) return *err = fmt("event %lld: shift out of range", (long long)e), SIM_EINVAL;
        const uint32_t m = column_mask(p, s);
        if (k == SIM_ENTER && (m == 0 || (m & (m - 1))))
            return *err = fmt("event %lld: ENTER must select exactly one compartment", (long long)e), SIM_EINVAL;
        if (h >= 0 && k != SIM_ENTER && k != SIM_EXIT) {
            for (int c = 0; c < Nc; ++c) {
                if (!((m >> c) & 1u)) continue;
                const int to = c + p->N[(size_t)c * p->n_shift + h];
                if (to < 0 || to >= Nc)
                    return *err = fmt("event %lld: shift moves compartment %d out of range", (long long)e, c), SIM_EINVAL;
            }
        }
    }
    if (p->n_record < 0 || (p->n_record > 0 && !p->record_days)) return *err = "bad record_days", SIM_EINVAL;
    for (int k = 0; k < p->n_record; ++k) {
        const int32_t d = p->record_days[k];
        if (d < 0 || d >= p->n_days) return *err = "record day out of range", SIM_EINVAL;
        if (k > 0 && d <= p->record_days[k - 1]) return *err = "record_days must be strictly ascending", SIM_EINVAL;
    }
    return SIM_OK;
}

}  // namespace

struct sim_handle {
    int32_t Nn = 0, Nc = 0, Nt = 0, R = 0, D = 0, n_record = 0;
    int64_t L = 0;
    Model model{};
    DevState st{};
    DevEvents ev{};
    std::vector<int32_t> perm, inv;  // position -> node, node -> position
    std::vector<int64_t> lvl_off;   // host copy of the level boundaries
    std::vector<int32_t> lvl_ptr;   // [D+1]
    Layout lay{};
    void *ws = nullptr;
    bool own_ws = false;
    hipStream_t stream = nullptr;
    int32_t launch = SIM_LAUNCH_KERNELS;
    int32_t block = 256;
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
};

namespace {

template <typename T>
T *at(void *base, size_t off) {
    return reinterpret_cast<T *>(static_cast<char *>(base) + off);
}

int64_t count_shift_ids(const sim_problem *p) { return p->n_shift; }

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

}  // namespace

extern "C" {

int sim_plan_levels(int64_t n_events, const int32_t *ev_day, const int32_t *ev_kind,
                    const int32_t *ev_node, const int32_t *ev_dest, int32_t n_nodes, int32_t *level_out) {
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
    plan_levels(n_events, ev_day, ev_kind, ev_node, ev_dest, n_nodes, level_out, nullptr, max_day + 1);
    return SIM_OK;
}

size_t sim_workspace_bytes(const sim_problem *p, const sim_device_opts *o) {
    std::string err;
    if (validate(p, &err) != SIM_OK) return 0;
    const int32_t mode = o ? o->events_mode : SIM_EVENTS_LEVELS;
    int64_t n_levels = 0;
    if (mode == SIM_EVENTS_SERIAL) {
        n_levels = p->n_events;
    } else if (mode == SIM_EVENTS_LEVELS) {
        std::vector<int32_t> level(p->n_events);
        std::vector<int32_t> day_levels;
        plan_levels(p->n_events, p->ev_day, p->ev_kind, p->ev_node, p->ev_dest, p->n_nodes, level.data(),
                    &day_levels, p->n_days);
        for (int32_t v : day_levels) n_levels += v;
    } else {
        return 0;
    }
    return layout_for(p->n_nodes, p->n_comp, p->n_trans, p->n_rep, p->n_days, p->n_events,
                      count_shift_ids(p), n_levels, p->n_record).total;
}

int sim_create(const sim_problem *p, const sim_device_opts *o, sim_handle **out) {
    g_create_error.clear();
    if (!out) return g_create_error = "out is NULL", SIM_EINVAL;
    *out = nullptr;
    int rc = validate(p, &g_create_error);
    if (rc != SIM_OK) return rc;
    sim_device_opts opts{};
    if (o) opts = *o;
    if (opts.events_mode != SIM_EVENTS_LEVELS && opts.events_mode != SIM_EVENTS_SERIAL)
        return g_create_error = "unknown events_mode", SIM_EINVAL;
    if (opts.launch != SIM_LAUNCH_KERNELS && opts.launch != SIM_LAUNCH_PERSISTENT)
        return g_create_error = "unknown launch mode", SIM_EINVAL;

    sim_handle *h = new (std::nothrow) sim_handle();
    if (!h) return g_create_error = "out of host memory", SIM_ENOMEM;
    h->Nn = p->n_nodes;
    h->Nc = p->n_comp;
    h->Nt = p->n_trans;
    h->R = p->n_rep;
    h->D = p->n_days;
    h->n_record = p->n_record;
    h->L = (int64_t)p->n_nodes * p->n_rep;
    h->stream = (hipStream_t)opts.stream;
    h->launch = opts.launch;
    h->block = opts.block > 0 ? opts.block : 256;
    const int64_t n = p->n_events;
    order_nodes(p, &h->perm, &h->inv);

    // --- dependency pass and execution order (stable by day, level, list order)
    std::vector<int32_t> level(n);
    std::vector<int32_t> day_levels;
    if (opts.events_mode == SIM_EVENTS_SERIAL) {
        day_levels.assign(h->D, 0);
        for (int64_t e = 0; e < n; ++e) level[e] = ++day_levels[p->ev_day[e]];
    } else {
        plan_levels(n, p->ev_day, p->ev_kind, p->ev_node, p->ev_dest, p->n_nodes, level.data(), &day_levels,
                    h->D);
    }
    h->lvl_ptr.assign(h->D + 1, 0);
    for (int32_t d = 0; d < h->D; ++d) h->lvl_ptr[d + 1] = h->lvl_ptr[d] + day_levels[d];
    const int64_t n_levels = h->lvl_ptr[h->D];
    h->lvl_off.assign(n_levels + 1, 0);
    for (int64_t e = 0; e < n; ++e) h->lvl_off[h->lvl_ptr[p->ev_day[e]] + level[e]]++;  // count into slot+1
    for (int64_t i = 0; i < n_levels; ++i) h->lvl_off[i + 1] += h->lvl_off[i];
    std::vector<int64_t> fill(h->lvl_off.begin(), h->lvl_off.end() - 1);
    std::vector<int32_t> eg(n), enode(n), edest(n), en(n);
    std::vector<uint32_t> emeta(n);
    for (int64_t e = 0; e < n; ++e) {
        const int64_t pos = fill[h->lvl_ptr[p->ev_day[e]] + level[e] - 1]++;
        eg[pos] = (int32_t)e;
        enode[pos] = h->inv[p->ev_node[e]];
        edest[pos] = p->ev_kind[e] == SIM_EXTERNAL ? h->inv[p->ev_dest[e]] : -1;
        en[pos] = p->ev_n[e];
        emeta[pos] = meta_pack(p->ev_kind[e], column_mask(p, p->ev_select[e]), p->ev_shift[e]);
    }

    // --- model constants
    Model &m = h->model;
    m.nc = h->Nc;
    m.nt = h->Nt;
    m.day0 = p->day0;
    m.seed = p->seed;
    m.uses_phi = 0;
    for (int k = 0; k < h->Nt; ++k) {
        if (p->uses_phi[k]) m.uses_phi |= 1u << k;
        m.reactant[k] = p->reactant[k];
        for (int c = 0; c < h->Nc; ++c) m.S[c][k] = p->S[(size_t)c * h->Nt + k];
    }
    m.imask = p->phi_I_mask;
    m.nmask = p->phi_N_mask;
    // paired S <-> I classes: transition k moves one individual from compartment k to k ^ 1
    m.pairs = (h->Nc == h->Nt && h->Nc % 2 == 0) ? 1 : 0;
    for (int k = 0; k < h->Nt && m.pairs; ++k) {
        if (p->reactant[k] != k) m.pairs = 0;
        for (int c = 0; c < h->Nc && m.pairs; ++c) {
            const int want = c == k ? -1 : (c == (k ^ 1) ? 1 : 0);
            if (p->S[(size_t)c * h->Nt + k] != want) m.pairs = 0;
        }
    }

    // --- device memory
    h->lay = layout_for(h->Nn, h->Nc, h->Nt, h->R, h->D, n, count_shift_ids(p), n_levels, h->n_record);
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
    s.node_id = at<int32_t>(h->ws, l.node_id);
    s.L = h->L;
    s.Nn = h->Nn;
    s.R = h->R;
    s.n_days = h->D;
    s.coef = at<double>(h->ws, l.coef);
    s.alpha = at<double>(h->ws, l.alpha);
    s.beta = at<double>(h->ws, l.beta);
    s.repid = at<uint32_t>(h->ws, l.repid);
    s.shift = at<int32_t>(h->ws, l.shift);
    s.status = at<unsigned long long>(h->ws, l.status);
    s.prevalence = at<int32_t>(h->ws, l.prevalence);
    s.transitions = at<int64_t>(h->ws, l.transitions);
    s.totals = at<int64_t>(h->ws, l.totals);
    s.snap_u = at<int32_t>(h->ws, l.snap_u);
    s.snap_v = at<double>(h->ws, l.snap_v);
    s.rec_slot = at<int32_t>(h->ws, l.rec_slot);
    DevEvents &ev = h->ev;
    ev.g = at<int32_t>(h->ws, l.ev_g);
    ev.node = at<int32_t>(h->ws, l.ev_node);
    ev.dest = at<int32_t>(h->ws, l.ev_dest);
    ev.n = at<int32_t>(h->ws, l.ev_n);
    ev.meta = at<uint32_t>(h->ws, l.ev_meta);
    ev.lvl_off = at<int64_t>(h->ws, l.lvl_off);
    ev.lvl_ptr = at<int32_t>(h->ws, l.lvl_ptr);

    // --- host staging of everything that is uploaded
    std::vector<uint32_t> repid(h->R);
    for (int r = 0; r < h->R; ++r) repid[r] = p->replicate_id ? p->replicate_id[r] : (uint32_t)r;
    std::vector<int32_t> shift(MAXC * std::max<int64_t>(p->n_shift, 1), 0);
    for (int hh = 0; hh < p->n_shift; ++hh)
        for (int c = 0; c < h->Nc; ++c) shift[hh * MAXC + c] = p->N[(size_t)c * p->n_shift + hh];
    std::vector<int32_t> rec_slot(std::max(h->D, 1), -1);
    for (int k = 0; k < p->n_record; ++k) rec_slot[p->record_days[k]] = k;
    const unsigned long long ok = STATUS_OK;

    struct Up {
        void *dst;
        const void *src;
        size_t bytes;
    };
    const Up ups[] = {
        {(void *)s.coef, p->coef, sizeof(double) * h->R * h->Nt},
        {(void *)s.alpha, p->alpha, sizeof(double) * h->R},
        {(void *)s.beta, p->beta, sizeof(double) * h->R * 4},
        {(void *)s.repid, repid.data(), sizeof(uint32_t) * h->R},
        {(void *)s.shift, shift.data(), sizeof(int32_t) * shift.size()},
        {(void *)s.status, &ok, sizeof ok},
        {(void *)ev.g, eg.data(), sizeof(int32_t) * n},
        {(void *)ev.node, enode.data(), sizeof(int32_t) * n},
        {(void *)ev.dest, edest.data(), sizeof(int32_t) * n},
        {(void *)ev.n, en.data(), sizeof(int32_t) * n},
        {(void *)ev.meta, emeta.data(), sizeof(uint32_t) * n},
        {(void *)ev.lvl_off, h->lvl_off.data(), sizeof(int64_t) * (n_levels + 1)},
        {(void *)ev.lvl_ptr, h->lvl_ptr.data(), sizeof(int32_t) * (h->D + 1)},
        {(void *)s.rec_slot, rec_slot.data(), sizeof(int32_t) * h->D},
        {(void *)s.node_id, h->perm.data(), sizeof(int32_t) * h->Nn},
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
    if (rc) {
        sim_destroy(h);
        return rc;
    }
    // initial state: every replicate starts from (u0, v0)
    std::vector<int32_t> u((size_t)h->Nc * h->L);
    std::vector<double> v(h->L);
    for (int64_t i = 0; i < h->Nn; ++i)
        for (int r = 0; r < h->R; ++r) {
            const int64_t lane = (int64_t)h->inv[i] * h->R + r;
            for (int c = 0; c < h->Nc; ++c) u[(size_t)c * h->L + lane] = p->u0[i * h->Nc + c];
            v[lane] = p->v0[i];
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

int sim_run(sim_handle *h, int32_t n_days) {
    if (!h) return SIM_EINVAL;
    h->err.clear();
    if (n_days < 0) return h->err = "n_days < 0", SIM_EINVAL;
    if (n_days == 0) n_days = h->D - h->day;
    if (h->day + n_days > h->D) return h->err = fmt("run of %d days from day %d passes the horizon %d", n_days, h->day, h->D), SIM_ESTATE;
    if (n_days == 0) return SIM_OK;
    const int32_t d0 = h->day, d1 = h->day + n_days;
    const Layout &l = h->lay;
    // records of the days about to be simulated start from zero
    int rc = SIM_OK;
    rc = check_device(hipMemsetAsync(h->st.prevalence + (size_t)d0 * h->R, 0, sizeof(int32_t) * n_days * h->R, h->stream), &h->err, "clear");
    if (!rc) rc = check_device(hipMemsetAsync(h->st.transitions + (size_t)d0 * h->R, 0, sizeof(int64_t) * n_days * h->R, h->stream), &h->err, "clear");
    if (!rc) rc = check_device(hipMemsetAsync(h->st.totals + (size_t)d0 * h->R * h->Nc, 0, sizeof(int64_t) * n_days * h->R * h->Nc, h->stream), &h->err, "clear");
    (void)l;
    if (rc) return rc;
    if (h->launch == SIM_LAUNCH_PERSISTENT && h->L > 0) {
        char why[256] = {0};
        hipError_t e = timed(h, SIM_K_PERSIST, [&] {
            return launch_persistent(h->model, h->st, h->ev, d0, d1, h->block, h->stream, why, sizeof why);
        });
        if (e != hipSuccess) return h->err = fmt("persistent launch: %s %s", hipGetErrorString(e), why), SIM_EDEVICE;
    } else {
        for (int32_t d = d0; d < d1; ++d) {
            hipError_t e = timed(h, SIM_K_DAY, [&] { return launch_day(h->model, h->st, d, d > d0, 1, h->block, h->stream); });
            if (e != hipSuccess) return h->err = fmt("day kernel: %s", hipGetErrorString(e)), SIM_EDEVICE;
            // big levels get a launch of their own; runs of small ones share one workgroup
            int32_t lv = h->lvl_ptr[d];
            const int32_t lv_end = h->lvl_ptr[d + 1];
            while (lv < lv_end) {
                const int64_t size = (h->lvl_off[lv + 1] - h->lvl_off[lv]) * h->R;
                if (size > kSmallLevel) {
                    e = timed(h, SIM_K_EVENTS, [&] {
                        return launch_events(h->model, h->st, h->ev, d, h->lvl_off[lv], h->lvl_off[lv + 1], h->stream);
                    });
                    ++lv;
                } else {
                    int32_t stop = lv + 1;
                    while (stop < lv_end && (h->lvl_off[stop + 1] - h->lvl_off[stop]) * h->R <= kSmallLevel) ++stop;
                    const int32_t a = lv;
                    e = timed(h, SIM_K_EVENTS, [&] { return launch_event_levels(h->model, h->st, h->ev, d, a, stop, h->stream); });
                    lv = stop;
                }
                if (e != hipSuccess) return h->err = fmt("event kernel: %s", hipGetErrorString(e)), SIM_EDEVICE;
            }
        }
        hipError_t e = timed(h, SIM_K_CLOSE, [&] { return launch_day(h->model, h->st, d1, 1, 0, h->block, h->stream); });
        if (e != hipSuccess) return h->err = fmt("closing kernel: %s", hipGetErrorString(e)), SIM_EDEVICE;
    }
    h->day = d1;
    return SIM_OK;
}

int sim_sync(sim_handle *h) {
    if (!h) return SIM_EINVAL;
    int rc = check_device(hipStreamSynchronize(h->stream), &h->err, "synchronize");
    if (rc) return rc;
    unsigned long long st = 0;
    rc = check_device(hipMemcpy(&st, h->st.status, sizeof st, hipMemcpyDeviceToHost), &h->err, "status");
    if (rc) return rc;
    if (st != STATUS_OK && (st >> 32) == STATUS_LIMIT_TAG) {
        return h->err = fmt("a node of replicate %llu exceeded %d SSA transitions in one day", st & 0xffffffffull,
                            SIM_MAX_FIRED),
               SIM_ELIMIT;
    }
    if (st != STATUS_OK) {
        return h->err = fmt("infeasible event %llu (replicate %llu): it asks for more individuals than the "
                            "selected compartments hold", st >> 32, st & 0xffffffffull),
               SIM_EINFEASIBLE;
    }
    return SIM_OK;
}

int sim_trajectory(sim_handle *h, sim_output *out) {
    if (!h || !out) return SIM_EINVAL;
    int rc = sim_sync(h);
    if (rc) return rc;
    const size_t DR = (size_t)h->D * h->R;
    struct Down {
        void *dst;
        const void *src;
        size_t bytes;
    } downs[] = {
        {out->prevalence, h->st.prevalence, sizeof(int32_t) * DR},
        {out->transitions, h->st.transitions, sizeof(int64_t) * DR},
        {out->totals, h->st.totals, sizeof(int64_t) * DR * h->Nc},
        {out->snap_u, h->st.snap_u, sizeof(int32_t) * h->n_record * (size_t)h->R * h->Nn * h->Nc},
        {out->snap_v, h->st.snap_v, sizeof(double) * h->n_record * (size_t)h->R * h->Nn},
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
        for (int64_t i = 0; i < h->Nn; ++i) {
            const int64_t lane = (int64_t)h->inv[i] * h->R + r;
            if (u)
                for (int c = 0; c < h->Nc; ++c) u[((size_t)r * h->Nn + i) * h->Nc + c] = du[(size_t)c * h->L + lane];
            if (v) v[(size_t)r * h->Nn + i] = dv[lane];
        }
    return SIM_OK;
}

int sim_set_state(sim_handle *h, const int32_t *u, const double *v, int32_t day) {
    if (!h || !u || !v) return SIM_EINVAL;
    h->err.clear();
    if (day < 0 || day > h->D) return h->err = "day out of range", SIM_ESTATE;
    int rc = check_device(hipStreamSynchronize(h->stream), &h->err, "synchronize");
    if (rc) return rc;
    std::vector<int32_t> du((size_t)h->Nc * h->L);
    std::vector<double> dv(h->L);
    for (int r = 0; r < h->R; ++r)
        for (int64_t i = 0; i < h->Nn; ++i) {
            const int64_t lane = (int64_t)h->inv[i] * h->R + r;
            for (int c = 0; c < h->Nc; ++c) {
                const int32_t x = u[((size_t)r * h->Nn + i) * h->Nc + c];
                if (x < 0) return h->err = "negative count in state", SIM_EINVAL;
                du[(size_t)c * h->L + lane] = x;
            }
            const double y = v[(size_t)r * h->Nn + i];
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

void sim_destroy(sim_handle *h) {
    if (!h) return;
    (void)hipStreamSynchronize(h->stream);
    for (const auto &m : h->marks) {
        (void)hipEventDestroy(m.a);
        (void)hipEventDestroy(m.b);
    }
    for (hipEvent_t e : h->ev_pool) (void)hipEventDestroy(e);
    if (h->own_ws && h->ws) (void)hipFree(h->ws);
    delete h;
}

const char *sim_last_error(const sim_handle *h) {
    return h ? h->err.c_str() : g_create_error.c_str();
}

}  // extern "C"
