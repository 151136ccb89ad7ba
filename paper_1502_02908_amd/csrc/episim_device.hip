// gfx950 kernels of the per-day step (Bauer, Engblom & Widgren,
// arXiv:1502.02908, Sec. 3.1-3.3 and Algorithm 1):
//   k_day      for every lane (node, replicate): the continuous-state update
//              closing the previous day (eq:numstep5 with eq:siminfpressure)
//              and that day's record, then the direct-method SSA over the
//              window [d, d+1) with phi frozen (eq:numstep3, eq:sampling,
//              eq:sampling2);
//   k_events   one conflict-free level of day d's external events
//              (eq:numstep4, Sec. 3.2): a thread per (event, replicate);
//   k_persist  the same phases for a run of days in one cooperative launch,
//              with grid barriers between phases.
// All binary64 arithmetic is written in a fixed order with contraction off,
// so results are a fixed function of the inputs.
#include <hip/hip_runtime.h>
#include <hip/hip_cooperative_groups.h>

#include <cstdio>

#include "../../include/episim.h"
#include "episim_internal.h"

#pragma clang fp contract(off)

namespace episim {
namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
constexpr int kEvKindMask = 3;

// ---------------------------------------------------------------------------
// Counter-based random numbers: Philox4x32-10 (Salmon et al., SC'11).
// ---------------------------------------------------------------------------
struct Word4 {
    uint32_t a, b, c, d;
};

__device__ __forceinline__ Word4 philox4x32_10(Word4 x, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        const uint32_t lo_a = 0xD2511F53u * x.a;
        const uint32_t hi_a = __umulhi(0xD2511F53u, x.a);
        const uint32_t lo_c = 0xCD9E8D57u * x.c;
        const uint32_t hi_c = __umulhi(0xCD9E8D57u, x.c);
        x = Word4{hi_c ^ x.b ^ k0, lo_c, hi_a ^ x.d ^ k1, lo_a};
        k0 += 0x9E3779B9u;  // Weyl increments of the key between rounds
        k1 += 0xBB67AE85u;
    }
    return x;
}

// rand in (0,1) of eq:sampling: the odd multiple of 2^-53 whose upper 52 bits
// are the top 52 bits of hi:lo.
__device__ __forceinline__ double unit_open(uint32_t lo, uint32_t hi) {
    const uint64_t x = ((uint64_t)hi << 32) | (uint64_t)lo;
    return (double)((x >> 11) | 1ull) * 0x1p-53;
}

// -log(u), u in (0,1): fold u = m 2^e with m in (sqrt2/2, sqrt2], then
// log m = 2 atanh(s), s = (m-1)/(m+1), with the series to s^23 and ln 2 split
// into a 32-bit head and a tail.
__device__ __forceinline__ double minus_log(double u) {
    const double kSqrt2 = 0x1.6a09e667f3bcdp+0;
    const double kLn2Head = 0x1.62e42ff000000p-1;
    const double kLn2Tail = -0x1.718432a1b0e26p-35;
    const long long bits = __double_as_longlong(u);
    int ex = (int)((bits >> 52) & 0x7ff) - 1023;
    double m = __longlong_as_double((bits & 0x000fffffffffffffLL) | 0x3ff0000000000000LL);
    if (m > kSqrt2) {
        m = m * 0.5;
        ex = ex + 1;
    }
    const double f = m - 1.0;
    const double s = f / (2.0 + f);
    const double z = s * s;
    double q = 1.0 / 23.0;
    q = 1.0 / 21.0 + z * q;
    q = 1.0 / 19.0 + z * q;
    q = 1.0 / 17.0 + z * q;
    q = 1.0 / 15.0 + z * q;
    q = 1.0 / 13.0 + z * q;
    q = 1.0 / 11.0 + z * q;
    q = 1.0 / 9.0 + z * q;
    q = 1.0 / 7.0 + z * q;
    q = 1.0 / 5.0 + z * q;
    q = 1.0 / 3.0 + z * q;
    const double zq = z * q;
    const double t = s + s * zq;
    const double lm = t + t;
    const double e = (double)ex;
    return -(e * kLn2Head + (lm + e * kLn2Tail));
}

// Season of beta(t) (Sec. 4.1).
__device__ __forceinline__ int season(int64_t t) {
    int64_t y = t % 365;
    if (y < 0) y += 365;
    return y <= 91 ? 0 : (y <= 182 ? 1 : (y <= 273 ? 2 : 3));
}

template <int NC>
__device__ __forceinline__ bool comp_on(const Model &m, int c) {
    return NC != MAXC || c < m.nc;
}
template <int NT>
__device__ __forceinline__ bool trans_on(const Model &m, int k) {
    return NT != MAXT || k < m.nt;
}

// omega_k = cphi_k * X[reactant_k], where cphi_k is the rate constant times
// phi for the transitions that use phi (the product (c * phi) * X of Sec. 3.3,
// eq:rate_s_to_i); lambda and the running sums cum_k in transition order.
template <int NC, int NT>
__device__ __forceinline__ double propensities(const Model &m, const double (&cphi)[NT],
                                               const int32_t (&x)[NC], double (&w)[NT],
                                               double (&cum)[NT]) {
    double lam = 0.0;
#pragma unroll
    for (int k = 0; k < NT; ++k) {
        w[k] = 0.0;
        cum[k] = lam;
        if (!trans_on<NT>(m, k)) continue;
        int32_t xr = 0;
#pragma unroll
        for (int cc = 0; cc < NC; ++cc)
            if (m.reactant[k] == cc) xr = x[cc];
        w[k] = cphi[k] * (double)xr;
        lam = lam + w[k];
        cum[k] = lam;
    }
    return lam;
}

// Inversion of eq:sampling2: the first transition with a positive rate whose
// running sum reaches target (the last positive one if rounding leaves none).
template <int NT>
__device__ __forceinline__ int choose(const Model &m, const double (&w)[NT], const double (&cum)[NT],
                                      double target) {
    int j = -1, last = -1;
#pragma unroll
    for (int k = 0; k < NT; ++k) {
        if (!trans_on<NT>(m, k)) continue;
        if (w[k] > 0.0) {
            last = k;
            if (j < 0 && cum[k] >= target) j = k;
        }
    }
    return j < 0 ? last : j;
}

template <int NC, int NT>
__device__ __forceinline__ void apply_transition(const Model &m, int j, int32_t (&x)[NC]) {
#pragma unroll
    for (int k = 0; k < NT; ++k) {
        if (k == j) {
#pragma unroll
            for (int cc = 0; cc < NC; ++cc) x[cc] += m.S[cc][k];
        }
    }
}

__device__ __forceinline__ double lane_f64(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, lane);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), lane);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Per-lane direct method over the window [d, d+1) (Algorithm 1's inner loop):
// attempt k draws one Philox block (k, node, d, 0); x is updated in place.
template <int NC, int NT>
__device__ __forceinline__ int32_t ssa_lane(const Model &m, const double (&cphi)[NT], int32_t (&x)[NC],
                                            uint32_t node, uint32_t day, uint32_t key1,
                                            unsigned long long *status, int32_t r) {
    double w[NT], cum[NT];
    double lam = propensities<NC, NT>(m, cphi, x, w, cum);
    double clock = 0.0;
    uint32_t draw = 0;
    int32_t fired = 0;
    while (lam > 0.0) {
        const Word4 o = philox4x32_10(Word4{draw, node, day, 0u}, m.seed, key1);
        draw = draw + 1;
        const double tau = minus_log(unit_open(o.a, o.b)) / lam;
        if (!(clock + tau < 1.0)) break;
        clock = clock + tau;
        const int j = choose<NT>(m, w, cum, unit_open(o.c, o.d) * lam);
        apply_transition<NC, NT>(m, j, x);
        fired = fired + 1;
        if (fired >= SIM_MAX_FIRED) {  // bounded work per lane: report instead of running on
            atomicMin(status, (STATUS_LIMIT_TAG << 32) | (unsigned long long)(uint32_t)r);
            break;
        }
        lam = propensities<NC, NT>(m, cphi, x, w, cum);
    }
    return fired;
}

// The same chain for one heavy lane h, run by the whole wavefront: the draws
// do not depend on the state, so lane i computes Philox block k0 + i and its
// -log(rand) in parallel; the state-dependent part (division, comparison,
// inversion, update) then walks those 64 draws in order with every lane
// holding the same values. Returns the transitions and leaves the new counts
// in x (identical in all lanes).
template <int NC, int NT>
__device__ __forceinline__ int32_t ssa_wave(const Model &m, const double (&cphi)[NT], int32_t (&x)[NC],
                                            uint32_t node, uint32_t day, uint32_t key1,
                                            unsigned long long *status, int32_t r) {
    const uint32_t lane = threadIdx.x & 63u;
    double w[NT], cum[NT];
    double lam = propensities<NC, NT>(m, cphi, x, w, cum);
    double clock = 0.0;
    int32_t fired = 0;
    bool go = lam > 0.0;
    for (uint32_t k0 = 0; go; k0 += 64) {
        const Word4 o = philox4x32_10(Word4{k0 + lane, node, day, 0u}, m.seed, key1);
        const double e_mine = minus_log(unit_open(o.a, o.b));
        const double u_mine = unit_open(o.c, o.d);
        for (int i = 0; i < 64; ++i) {
            const double tau = lane_f64(e_mine, i) / lam;
            if (!(clock + tau < 1.0)) {
                go = false;
                break;
            }
            clock = clock + tau;
            const int j = choose<NT>(m, w, cum, lane_f64(u_mine, i) * lam);
            apply_transition<NC, NT>(m, j, x);
            fired = fired + 1;
            if (fired >= SIM_MAX_FIRED) {
                if (lane == 0) atomicMin(status, (STATUS_LIMIT_TAG << 32) | (unsigned long long)(uint32_t)r);
                go = false;
                break;
            }
            lam = propensities<NC, NT>(m, cphi, x, w, cum);
            if (!(lam > 0.0)) {
                go = false;
                break;
            }
        }
    }
    return fired;
}

__device__ __forceinline__ long long wave_sum(long long v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Per-lane contributions to the daily records of one phase.
template <int NC>
struct Tally {
    long long prev, trans;
    long long tot[NC];
};

// Sum tallies over the workgroup (R == 1) and add them to the day's records.
template <int NC>
__device__ void flush_block(const Model &m, const DevState &s, const Tally<NC> &t, int32_t d_rec,
                            int32_t d_ssa) {
    __shared__ long long part[kWaves][2 + NC];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    long long v[2 + NC];
    v[0] = t.prev;
    v[1] = t.trans;
#pragma unroll
    for (int c = 0; c < NC; ++c) v[2 + c] = t.tot[c];
#pragma unroll
    for (int i = 0; i < 2 + NC; ++i) {
        const long long w = wave_sum(v[i]);
        if (lane == 0) part[wave][i] = w;
    }
    __syncthreads();
    if (threadIdx.x < 2 + NC) {
        const int i = threadIdx.x;
        long long sum = 0;
#pragma unroll
        for (int q = 0; q < kWaves; ++q) sum += part[q][i];
        if (i == 0 && d_rec >= 0) {
            if (sum) atomicAdd(&s.prevalence[d_rec], (int32_t)sum);
        } else if (i == 1 && d_ssa >= 0) {
            if (sum) atomicAdd((unsigned long long *)&s.transitions[d_ssa], (unsigned long long)sum);
        } else if (i >= 2 && d_rec >= 0 && comp_on<NC>(m, i - 2)) {
            if (sum) atomicAdd((unsigned long long *)&s.totals[(int64_t)d_rec * m.nc + (i - 2)],
                               (unsigned long long)sum);
        }
    }
    __syncthreads();
}

// Per-lane records when lanes of a workgroup belong to different replicates.
template <int NC>
__device__ __forceinline__ void flush_lane(const Model &m, const DevState &s, const Tally<NC> &t,
                                           int r, int32_t d_rec, int32_t d_ssa) {
    if (d_rec >= 0) {
        const int64_t row = (int64_t)d_rec * s.R + r;
        if (t.prev) atomicAdd(&s.prevalence[row], (int32_t)t.prev);
#pragma unroll
        for (int c = 0; c < NC; ++c)
            if (comp_on<NC>(m, c) && t.tot[c])
                atomicAdd((unsigned long long *)&s.totals[row * m.nc + c], (unsigned long long)t.tot[c]);
    }
    if (d_ssa >= 0 && t.trans)
        atomicAdd((unsigned long long *)&s.transitions[(int64_t)d_ssa * s.R + r],
                  (unsigned long long)t.trans);
}

// Lanes whose total rate at the start of the window is at least kHeavy run
// their chain cooperatively (ssa_wave) when a wavefront holds at most
// kWaveChains of them; everything else runs per lane. Both paths perform the
// same arithmetic on the same draws.
constexpr double kHeavy = 12.0;
constexpr int kWaveChains = 4;

// The day phase for the lane l of a wavefront (every lane of the wavefront
// must call it; lanes with l >= L take part in the wavefront-level steps
// only): close day d-1 (phi update + record) if prologue, then run the SSA of
// day d if ssa. Adds the lane's counts to t.
template <int NC, int NT>
__device__ __forceinline__ void day_wave(const Model &m, const DevState &s, int64_t l, int32_t d,
                                         bool prologue, bool ssa, Tally<NC> &t) {
    const bool active = l < s.L;
    const int32_t R = s.R;
    const int32_t r = !active || R == 1 ? 0 : (int32_t)(l % R);
    const int32_t pos = !active ? 0 : (R == 1 ? (int32_t)l : (int32_t)(l / R));
    int32_t x[NC];
    double phi = 0.0;
    uint32_t node = 0;
#pragma unroll
    for (int c = 0; c < NC; ++c) x[c] = 0;
    if (active) {
#pragma unroll
        for (int c = 0; c < NC; ++c) x[c] = comp_on<NC>(m, c) ? s.u[(int64_t)c * s.L + l] : 0;
        phi = s.phi[l];
        node = (uint32_t)s.node_id[pos];
    }
    if (active && prologue) {
        const double phi_in = phi;
        const int32_t dp = d - 1;
        long long I = 0, N = 0;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            if ((m.imask >> c) & 1u) I += x[c];
            if ((m.nmask >> c) & 1u) N += x[c];
        }
        const int q = season((int64_t)m.day0 + dp);
        const double a = 1.0 - s.beta[r * 4 + q];
        const double b = a * phi;
        const double shed = N > 0 ? s.alpha[r] * ((double)I / (double)N) : 0.0;
        phi = b + shed;
        t.prev += I > 0 ? 1 : 0;
#pragma unroll
        for (int c = 0; c < NC; ++c) t.tot[c] += x[c];
        const int32_t slot = s.rec_slot[dp];
        if (slot >= 0) {
            const int64_t base = (((int64_t)slot * R + r) * s.Nn + node);
#pragma unroll
            for (int c = 0; c < NC; ++c)
                if (comp_on<NC>(m, c)) s.snap_u[base * m.nc + c] = x[c];
            s.snap_v[base] = phi;
        }
        if (__double_as_longlong(phi) != __double_as_longlong(phi_in)) s.phi[l] = phi;
    }
    if (!ssa) return;
    double cphi[NT];
    const uint32_t key1 = active ? s.repid[r] : 0u;
#pragma unroll
    for (int k = 0; k < NT; ++k) {
        double c = active && trans_on<NT>(m, k) ? s.coef[r * m.nt + k] : 0.0;
        if ((m.uses_phi >> k) & 1u) c = c * phi;
        cphi[k] = c;
    }
    double w0[NT], cum0[NT];
    const double lam0 = propensities<NC, NT>(m, cphi, x, w0, cum0);
    const bool heavy = active && lam0 >= kHeavy;
    const unsigned long long hmask = __ballot(heavy);
    const int n_heavy = __popcll(hmask);
    const bool wave_path = n_heavy >= 1 && n_heavy <= kWaveChains;
    int32_t fired = 0;
    if (active && !(wave_path && heavy))
        fired = ssa_lane<NC, NT>(m, cphi, x, node, (uint32_t)d, key1, s.status, r);
    if (wave_path) {
        unsigned long long todo = hmask;
        while (todo) {
            const int h = __ffsll((long long)todo) - 1;
            todo &= todo - 1;
            int32_t xh[NC];
            double ch[NT];
#pragma unroll
            for (int c = 0; c < NC; ++c) xh[c] = __builtin_amdgcn_readlane(x[c], h);
#pragma unroll
            for (int k = 0; k < NT; ++k) ch[k] = lane_f64(cphi[k], h);
            const uint32_t nh = (uint32_t)__builtin_amdgcn_readlane((int)node, h);
            const uint32_t kh = (uint32_t)__builtin_amdgcn_readlane((int)key1, h);
            const int32_t rh = __builtin_amdgcn_readlane(r, h);
            const int32_t fh = ssa_wave<NC, NT>(m, ch, xh, nh, (uint32_t)d, kh, s.status, rh);
            if ((int)(threadIdx.x & 63u) == h) {
                fired = fh;
#pragma unroll
                for (int c = 0; c < NC; ++c) x[c] = xh[c];
            }
        }
    }
    t.trans += fired;
    if (active && fired) {
#pragma unroll
        for (int c = 0; c < NC; ++c)
            if (comp_on<NC>(m, c)) s.u[(int64_t)c * s.L + l] = x[c];
    }
}

template <int NC, int NT>
__global__ __launch_bounds__(kBlock) void k_day(Model m, DevState s, int32_t d, int32_t prologue,
                                                int32_t ssa) {
    if (*(volatile unsigned long long *)s.status != STATUS_OK) return;  // uniform early exit
    const int64_t l = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    Tally<NC> t{};
    day_wave<NC, NT>(m, s, l, d, prologue != 0, ssa != 0, t);
    const int32_t d_rec = prologue ? d - 1 : -1;
    const int32_t d_ssa = ssa ? d : -1;
    if (s.R == 1) {
        flush_block<NC>(m, s, t, d_rec, d_ssa);
    } else if (l < s.L) {
        flush_lane<NC>(m, s, t, (int32_t)(l % s.R), d_rec, d_ssa);
    }
}

// ---------------------------------------------------------------------------
// Events (Sec. 3.2): one thread per (event, replicate) of a conflict-free
// level. Within a level a node is either drawn from by exactly one event or
// only added to, so draws use plain loads/stores and additions commute
// (integer atomics).
// ---------------------------------------------------------------------------
template <int NC>
__device__ __forceinline__ void event_one(const Model &m, const DevState &s, const DevEvents &ev,
                                          int64_t e, int32_t r, int32_t d) {
    const uint32_t meta = ev.meta[e];
    const int kind = (int)(meta & kEvKindMask);
    const uint32_t mask = (meta >> 2) & 0xffu;
    const int sid = (int)((meta >> 10) & 0x3fu) - 1;
    const int32_t node = ev.node[e];
    const int32_t n = ev.n[e];
    const int64_t ls = (int64_t)node * s.R + r;
    if (kind == SIM_ENTER) {
#pragma unroll
        for (int c = 0; c < NC; ++c)
            if ((mask >> c) & 1u) atomicAdd(&s.u[(int64_t)c * s.L + ls], n);
        return;
    }
    int32_t x[NC];
    long long tot = 0;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        x[c] = 0;
        if ((mask >> c) & 1u) {
            x[c] = s.u[(int64_t)c * s.L + ls];
            tot += x[c];
        }
    }
    const uint32_t g = (uint32_t)ev.g[e];
    if ((long long)n > tot) {
        atomicMin(s.status, ((unsigned long long)g << 32) | (unsigned long long)(uint32_t)r);
        return;
    }
    int32_t take[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) take[c] = 0;
    const uint32_t key1 = s.repid[r];
    Word4 o{0, 0, 0, 0};
    for (int32_t q = 0; q < n; ++q) {
        uint64_t bits;
        if ((q & 1) == 0) {
            o = philox4x32_10(Word4{(uint32_t)q >> 1, g, (uint32_t)d, 1u}, m.seed, key1);
            bits = ((uint64_t)o.b << 32) | o.a;
        } else {
            bits = ((uint64_t)o.d << 32) | o.c;
        }
        uint64_t pick = __umul64hi(bits, (uint64_t)tot);  // uniform on [0, tot)
        int chosen = -1;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            if (chosen < 0 && ((mask >> c) & 1u)) {
                if (pick < (uint64_t)x[c]) {
                    chosen = c;
                } else {
                    pick -= (uint64_t)x[c];
                }
            }
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            if (c == chosen) {
                x[c] -= 1;
                take[c] += 1;
            }
        }
        tot -= 1;
    }
    if (kind == SIM_INTERNAL) {
        int32_t y[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) y[c] = ((mask >> c) & 1u) ? x[c] : 0;
        uint32_t touched = mask;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            if (take[c]) {
                const int to = sid >= 0 ? c + s.shift[sid * MAXC + c] : c;
#pragma unroll
                for (int cc = 0; cc < NC; ++cc) {
                    if (cc == to) {
                        if (!((touched >> cc) & 1u)) {
                            y[cc] = s.u[(int64_t)cc * s.L + ls];
                            touched |= 1u << cc;
                        }
                        y[cc] += take[c];
                    }
                }
            }
        }
#pragma unroll
        for (int c = 0; c < NC; ++c)
            if ((touched >> c) & 1u) s.u[(int64_t)c * s.L + ls] = y[c];
        return;
    }
#pragma unroll
    for (int c = 0; c < NC; ++c)
        if ((mask >> c) & 1u) s.u[(int64_t)c * s.L + ls] = x[c];
    if (kind == SIM_EXTERNAL) {
        const int64_t ld = (int64_t)ev.dest[e] * s.R + r;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            if (take[c]) {
                const int to = sid >= 0 ? c + s.shift[sid * MAXC + c] : c;
                atomicAdd(&s.u[(int64_t)to * s.L + ld], take[c]);
            }
        }
    }
}

template <int NC>
__global__ __launch_bounds__(kBlock) void k_events(Model m, DevState s, DevEvents ev, int32_t d,
                                                   int64_t begin, int64_t end) {
    if (*(volatile unsigned long long *)s.status != STATUS_OK) return;
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t count = (end - begin) * s.R;
    if (t >= count) return;
    const int64_t e = begin + (s.R == 1 ? t : t / s.R);
    const int32_t r = s.R == 1 ? 0 : (int32_t)(t % s.R);
    event_one<NC>(m, s, ev, e, r, d);
}

// ---------------------------------------------------------------------------
// A run of days in one cooperative launch: phases separated by grid barriers.
// ---------------------------------------------------------------------------
template <int NC, int NT>
__global__ __launch_bounds__(kBlock) void k_persist(Model m, DevState s, DevEvents ev, int32_t d_begin,
                                                    int32_t d_end) {
    namespace cg = cooperative_groups;
    cg::grid_group grid = cg::this_grid();
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    const int64_t first = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    for (int32_t d = d_begin; d <= d_end; ++d) {
        const bool prologue = d > d_begin;
        const bool ssa = d < d_end;
        if (*(volatile unsigned long long *)s.status == STATUS_OK) {
            Tally<NC> t{};
            const int64_t span = ((s.L + kBlock - 1) / kBlock) * kBlock;  // whole workgroups
            for (int64_t l = first; l < span; l += stride) {
                if (s.R == 1) {
                    day_wave<NC, NT>(m, s, l, d, prologue, ssa, t);
                } else {
                    Tally<NC> one{};
                    day_wave<NC, NT>(m, s, l, d, prologue, ssa, one);
                    if (l < s.L)
                        flush_lane<NC>(m, s, one, (int32_t)(l % s.R), prologue ? d - 1 : -1, ssa ? d : -1);
                }
            }
            if (s.R == 1) flush_block<NC>(m, s, t, prologue ? d - 1 : -1, ssa ? d : -1);
        }
        if (!ssa) break;
        grid.sync();
        for (int32_t lv = ev.lvl_ptr[d]; lv < ev.lvl_ptr[d + 1]; ++lv) {
            const int64_t begin = ev.lvl_off[lv], end = ev.lvl_off[lv + 1];
            const int64_t count = (end - begin) * s.R;
            if (*(volatile unsigned long long *)s.status == STATUS_OK) {
                for (int64_t t = first; t < count; t += stride) {
                    const int64_t e = begin + (s.R == 1 ? t : t / s.R);
                    event_one<NC>(m, s, ev, e, s.R == 1 ? 0 : (int32_t)(t % s.R), d);
                }
            }
            grid.sync();
        }
    }
}

template <int NC, int NT>
struct Kernels {
    static void *day() { return (void *)&k_day<NC, NT>; }
    static void *events() { return (void *)&k_events<NC>; }
    static void *persist() { return (void *)&k_persist<NC, NT>; }
};

struct Table {
    void *day, *events, *persist;
};

Table pick(int nc, int nt) {
    if (nc == 2 && nt == 2) return {Kernels<2, 2>::day(), Kernels<2, 2>::events(), Kernels<2, 2>::persist()};
    if (nc == 6 && nt == 6) return {Kernels<6, 6>::day(), Kernels<6, 6>::events(), Kernels<6, 6>::persist()};
    return {Kernels<MAXC, MAXT>::day(), Kernels<MAXC, MAXT>::events(), Kernels<MAXC, MAXT>::persist()};
}

}  // namespace

int launch_day(const Model &m, const DevState &s, int32_t d, int prologue, int ssa, int block,
               void *stream) {
    (void)block;
    if (s.L == 0) return hipSuccess;
    const Table t = pick(m.nc, m.nt);
    const unsigned grid = (unsigned)((s.L + kBlock - 1) / kBlock);
    Model mm = m;
    DevState ss = s;
    int32_t dd = d, pro = prologue, sa = ssa;
    void *args[] = {&mm, &ss, &dd, &pro, &sa};
    return (int)hipLaunchKernel(t.day, dim3(grid), dim3(kBlock), args, 0, (hipStream_t)stream);
}

int launch_events(const Model &m, const DevState &s, const DevEvents &ev, int32_t d, int64_t begin,
                  int64_t end, void *stream) {
    const int64_t count = (end - begin) * s.R;
    if (count <= 0) return hipSuccess;
    const Table t = pick(m.nc, m.nt);
    const unsigned grid = (unsigned)((count + kBlock - 1) / kBlock);
    Model mm = m;
    DevState ss = s;
    DevEvents ee = ev;
    int32_t dd = d;
    int64_t b = begin, e = end;
    void *args[] = {&mm, &ss, &ee, &dd, &b, &e};
    return (int)hipLaunchKernel(t.events, dim3(grid), dim3(kBlock), args, 0, (hipStream_t)stream);
}

int launch_persistent(const Model &m, const DevState &s, const DevEvents &ev, int32_t d_begin,
                      int32_t d_end, int block, void *stream, char *why, int why_len) {
    (void)block;
    const Table t = pick(m.nc, m.nt);
    int dev = 0;
    hipError_t err = hipGetDevice(&dev);
    if (err != hipSuccess) return (int)err;
    int cus = 0, per_cu = 0;
    err = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (err != hipSuccess) return (int)err;
    err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, t.persist, kBlock, 0);
    if (err != hipSuccess) return (int)err;
    if (per_cu < 1) {
        snprintf(why, why_len, "persistent kernel cannot be resident (occupancy 0)");
        return (int)hipErrorInvalidConfiguration;
    }
    const int64_t want = (s.L + kBlock - 1) / kBlock;
    int64_t grid = (int64_t)cus * per_cu;
    if (want < grid) grid = want > 0 ? want : 1;
    Model mm = m;
    DevState ss = s;
    DevEvents ee = ev;
    int32_t a = d_begin, b = d_end;
    void *args[] = {&mm, &ss, &ee, &a, &b};
    return (int)hipLaunchCooperativeKernel(t.persist, dim3((unsigned)grid), dim3(kBlock), args, 0,
                                           (hipStream_t)stream);
}

}  // namespace episim
