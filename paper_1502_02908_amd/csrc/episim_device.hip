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

#include <algorithm>
#include <cstdio>
#include <mutex>

#include "../../include/episim.h"
#include "episim_internal.h"

#pragma clang fp contract(off)

// Intermediate buffers of the entry points that allocate nothing (the goal
// function's staged reference and day terms): a fixed array in every GPU's
// memory, kept until the process ends. Calls on one GPU share it.
static __device__ __align__(256) unsigned char scratch[episim::kScratchBytes];

namespace episim {
namespace {

constexpr int kBlock = 256;
static_assert(kBlock == kLaneUnit, "a workgroup of one-lane-per-node kernels is one unit");
constexpr int kMaxScratchDevices = 64;
constexpr int kWaves = kBlock / 64;
constexpr int kEvKindMask = 3;
constexpr int kEvBlock = 1024;  // workgroup that runs a group of small event levels

// ---------------------------------------------------------------------------
// Counter-based random numbers: Philox4x32-10 (Salmon et al., SC'11).
// ---------------------------------------------------------------------------
struct Word4 {
    uint32_t a, b, c, d;
};

__device__ __forceinline__ Word4 philox4x32_10(Word4 x, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        const uint64_t pa = (uint64_t)0xD2511F53u * (uint64_t)x.a;  // one 32x32->64 multiply each
        const uint64_t pc = (uint64_t)0xCD9E8D57u * (uint64_t)x.c;
        x = Word4{(uint32_t)(pc >> 32) ^ x.b ^ k0, (uint32_t)pc, (uint32_t)(pa >> 32) ^ x.d ^ k1, (uint32_t)pa};
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

// Loads of the state in the event phase are plain loads, so that the
// compartments of one node are fetched together. They see the last writes
// because a launch starts with clean caches, and because every kernel that
// runs several levels, or events after the SSA, follows its barrier with
// fresh_l1(): additions are device-scope atomics done in L2, which the CU's
// L1 does not see, so the acquire drops the L1 lines before the next level.
__device__ __forceinline__ int32_t load_state(const int32_t *p) { return *p; }

__device__ __forceinline__ void fresh_l1() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }

template <int NC>
__device__ __forceinline__ bool comp_on(const Model &m, int c) {
    return NC != MAXC || c < m.nc;
}
template <int NT>
__device__ __forceinline__ bool trans_on(const Model &m, int k) {
    return NT != MAXT || k < m.nt;
}

// ---------------------------------------------------------------------------
// The stochastic step (Sec. 3.3, Algorithm 1's inner loop; eq:sampling and
// eq:sampling2). A lane's chain keeps its counts as exact binary64 values
// (counts stay far below 2^53), so omega_k = cphi_k * X[reactant_k] is the
// same product (c * phi) * (double)X in the same order as the plain method;
// cphi_k is the rate constant times phi for the transitions that use phi.
// lambda and the running sums cum_k are summed in transition order.
// ---------------------------------------------------------------------------
template <int NC_, int NT_>
struct Chain {
    static constexpr int NC = NC_, NT = NT_;
    double xd[NC_];
    double cphi[NT_];
    double cum[NT_];
    double lam, clock;
    int32_t fired;
};

// Any stoichiometry (column k: -1 at reactant k, non-negative elsewhere).
template <int NC_, int NT_>
struct GenericRules {
    static constexpr int NC = NC_, NT = NT_;
    static constexpr int kPairs = 0;
    static constexpr int kTileWaves = 2;  // waves per SIMD the replicate-tile kernel is built for
    using State = Chain<NC, NT>;
    __device__ static __forceinline__ double rate(const Model &m, const State &c, int k) {
        double xr = 0.0, xr2 = 0.0;
#pragma unroll
        for (int cc = 0; cc < NC; ++cc) {
            if (m.reactant[k] == cc) xr = c.xd[cc];
            if (m.reactant2[k] == cc) xr2 = c.xd[cc];
        }
        const double w = c.cphi[k] * xr;
        // a mass-action rate is also proportional to its second reactant
        return m.reactant2[k] >= 0 ? w * xr2 : w;
    }
    __device__ static __forceinline__ void rates(const Model &m, State &c) {
        double lam = 0.0;
#pragma unroll
        for (int k = 0; k < NT; ++k) {
            if (trans_on<NT>(m, k)) lam = lam + rate(m, c, k);
            c.cum[k] = lam;
        }
        c.lam = lam;
    }
    __device__ static __forceinline__ void apply(const Model &m, int j, State &c) {
#pragma unroll
        for (int k = 0; k < NT; ++k) {
            if (k == j) {
#pragma unroll
                for (int cc = 0; cc < NC; ++cc) c.xd[cc] = c.xd[cc] + (double)m.S[cc][k];
            }
        }
    }
    // j is the same in every lane: apply it and recompute all rates
    __device__ static __forceinline__ void apply_uniform(const Model &m, int j, State &c) {
        apply(m, j, c);
        rates(m, c);
    }
};

// Paired classes: compartments [S_1, I_1, ..., S_P, I_P] and transitions
// 2p: S_p -> I_p, 2p+1: I_p -> S_p, each with its own compartment as reactant
// (eq:vectorJSDE for eq:vtectrans; P = 1 is the plain SIS model). The host
// selects these rules only when S and the reactants have exactly this form.
template <int NP>
struct PairRules {
    static constexpr int NC = 2 * NP, NT = 2 * NP;
    static constexpr int kPairs = NP;
    // replicate tiles of paired classes are built for three waves per SIMD
    // (at most 168 VGPRs, with a 16-byte spill): the third wave hides the
    // latency of the chains' dependent binary64 arithmetic and of the state
    // loads (12 % faster on the batched workload than the two waves 185
    // VGPRs allow; bit-identical)
    static constexpr int kTileWaves = 3;
    using State = Chain<NC, NT>;
    __device__ static __forceinline__ double rate(const Model &, const State &c, int k) {
        return c.cphi[k] * c.xd[k];
    }
    __device__ static __forceinline__ void rates(const Model &m, State &c) {
        double lam = 0.0;
#pragma unroll
        for (int k = 0; k < NT; ++k) {
            lam = lam + rate(m, c, k);
            c.cum[k] = lam;
        }
        c.lam = lam;
    }
    __device__ static __forceinline__ void apply(const Model &, int j, State &c) {
        const int p = j >> 1;
        const double dS = (j & 1) ? 1.0 : -1.0;  // infection takes an S, recovery returns one
#pragma unroll
        for (int q = 0; q < NP; ++q) {
            const double dq = q == p ? dS : 0.0;
            c.xd[2 * q] = c.xd[2 * q] + dq;
            c.xd[2 * q + 1] = c.xd[2 * q + 1] - dq;
        }
    }
    // j is the same in every lane (a scalar): only class j/2 changes, so only
    // the running sums from its first transition on are recomputed (the
    // earlier ones are unchanged, so the values equal a full recomputation).
    __device__ static __forceinline__ void apply_uniform(const Model &m, int j, State &c) {
        const int p = j >> 1;
        const double dS = (j & 1) ? 1.0 : -1.0;
#pragma unroll
        for (int q = 0; q < NP; ++q) {
            if (q == p) {
                c.xd[2 * q] = c.xd[2 * q] + dS;
                c.xd[2 * q + 1] = c.xd[2 * q + 1] - dS;
                double lam = q == 0 ? 0.0 : c.cum[2 * q - 1];
#pragma unroll
                for (int k = 2 * q; k < NT; ++k) {
                    lam = lam + rate(m, c, k);
                    c.cum[k] = lam;
                }
                c.lam = lam;
            }
        }
    }
};

// The single-chain walk for paired classes (defined below).
template <int NP, bool FED = false>
__device__ __forceinline__ void pairs_walk_block(const Model &m, Chain<2 * NP, 2 * NP> &c, uint32_t kbase,
                                                 uint32_t node, uint32_t day, uint32_t key0, uint32_t key1,
                                                 unsigned long long *status, int32_t r);

// Inversion of eq:sampling2: the first transition with a positive rate whose
// running sum reaches target. With target > 0 that is the number of running
// sums below target (they never decrease, and a transition with rate 0 cannot
// be the first to reach a positive target); target can be 0 only if U*lambda
// underflows, and then it is the first positive rate.
template <class Rules>
__device__ __forceinline__ int invert(const Model &m, const typename Rules::State &c, double target) {
    constexpr int NT = Rules::NT;
    int j = 0;
#pragma unroll
    for (int k = 0; k < NT; ++k) j += c.cum[k] < target ? 1 : 0;
    if (__builtin_expect(!(target > 0.0), 0)) {
        j = NT;
#pragma unroll
        for (int k = NT - 1; k >= 0; --k)
            if (trans_on<NT>(m, k) && Rules::rate(m, c, k) > 0.0) j = k;
    }
    return j;
}

template <int NP>
__device__ __forceinline__ void pairs_rates_full(Chain<2 * NP, 2 * NP> &c) {
    double lam = 0.0;
#pragma unroll
    for (int k = 0; k < 2 * NP; ++k) {
        lam = lam + c.cphi[k] * c.xd[k];
        c.cum[k] = lam;
    }
    c.lam = lam;
}

// One attempt of the direct method with the draw (E, U) = (-log rand_1,
// rand_2): tau = E / lambda; the transition fires only if it lands inside the
// window. Returns whether the chain goes on.
template <class Rules>
__device__ __forceinline__ bool chain_step(const Model &m, typename Rules::State &c, double E, double U,
                                           unsigned long long *status, int32_t r) {
    const double tau = E / c.lam;
    const double t1 = c.clock + tau;
    const int j = invert<Rules>(m, c, U * c.lam);
    if (!(t1 < 1.0)) return false;
    c.clock = t1;
    Rules::apply(m, j, c);
    c.fired = c.fired + 1;
    Rules::rates(m, c);
    if (c.fired >= SIM_MAX_FIRED) {  // bounded work per lane: report instead of running on
        atomicMin(status, (STATUS_LIMIT_TAG << 32) | (unsigned long long)(uint32_t)r);
        return false;
    }
    return c.lam > 0.0;
}

__device__ __forceinline__ double lane_f64(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, lane);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), lane);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Inclusive prefix sum over the 64 lanes of a wavefront: shifts by 1, 2, 4, 8
// within rows of 16 lanes, then lane 15's sum into rows 1 and 3 and lane 31's
// into rows 2 and 3 (lanes without a source add +0).
template <int Ctrl, int RowMask>
__device__ __forceinline__ double dpp_f64(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, Ctrl, RowMask, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), Ctrl, RowMask, 0xf, false);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

__device__ __forceinline__ double wave_prefix_sum(double v) {
    v = v + dpp_f64<0x111, 0xf>(v);  // row_shr:1
    v = v + dpp_f64<0x112, 0xf>(v);  // row_shr:2
    v = v + dpp_f64<0x114, 0xf>(v);  // row_shr:4
    v = v + dpp_f64<0x118, 0xf>(v);  // row_shr:8
    v = v + dpp_f64<0x142, 0xa>(v);  // row_bcast:15
    v = v + dpp_f64<0x143, 0xc>(v);  // row_bcast:31
    return v;
}

// The clock of a round without the attempt-by-attempt sum. While the running
// clock stays in one binade [2^e, 2^(e+1)) every partial sum is an integer
// multiple of its spacing h = 2^(e-52), and adding a waiting time rounds to
// the nearest multiple: s + tau -> (s/h + rn(tau/h)) h. Those integers add
// exactly (each partial sum that matters stays below 2^53), so one prefix sum
// over the lanes gives every partial sum of the round bit for bit. A sum that
// reaches 2^(e+1) leaves the binade: for e = -1 that is the window end (the
// attempt does not fire, whatever the rounding above 1); otherwise the round
// has to be summed attempt by attempt, and so has a round in which a waiting
// time lies exactly half-way between two multiples (ties round to even, which
// depends on the partial sum) or whose clock is 0. Returns the number of
// attempts that fire (-1: sum attempt by attempt) and their clock.
__device__ __forceinline__ int clock_by_scan(double clock, double tau, double *clock_out) {
    const long long cb = __double_as_longlong(clock);
    const int e = (int)((cb >> 52) & 0x7ff) - 1023;
    if (!(clock > 0.0) || e < -960 || e > -1) return -1;
    const double up = __longlong_as_double((long long)(1023 + 52 - e) << 52);    // 2^(52-e)
    const double down = __longlong_as_double((long long)(1023 - 52 + e) << 52);  // 2^(e-52)
    const double S0 = clock * up;                                                // in [2^52, 2^53)
    const double T = 0x1p53 - S0;
    const double v = tau * up;
    const double fl = floor(v);
    const double fr = v - fl;
    const double P = wave_prefix_sum(fr > 0.5 ? fl + 1.0 : fl);
    const int A = (int)__popcll(__ballot(P < T));
    const unsigned long long upto = A >= 63 ? ~0ull : ((2ull << A) - 1ull);
    if ((__ballot(fr == 0.5) & upto) != 0ull) return -1;
    if (A < 64 && e != -1) return -1;
    *clock_out = A > 0 ? (S0 + lane_f64(P, A - 1)) * down : clock;
    return A;
}

// Value v[idx / 64] of lane idx % 64 (idx uniform over the wavefront).
template <int W>
__device__ __forceinline__ double part_at(const double (&v)[W], int idx) {
    double out = 0.0;
#pragma unroll
    for (int w = 0; w < W; ++w)
        if (idx / 64 == w) out = lane_f64(v[w], idx % 64);
    return out;
}

// The clock of a round of the workgroup walk without the attempt-by-attempt
// sum (the rule of clock_by_scan, carried past ties and binade ends). While the running
// clock s stays in one binade [2^e, 2^(e+1)) every partial sum is an integer
// multiple of its spacing h = 2^(e-52), and adding a waiting time rounds to
// the nearest multiple: s + tau -> (s/h + rn(tau/h)) h. Those integers add
// exactly (each partial sum that matters stays below 2^53), so prefix sums
// over the round's attempts (attempt w * 64 + lane in tau[w]) give the
// partial sums bit for bit up to the first attempt that either reaches
// 2^(e+1) or lies exactly half-way between two multiples (ties round to even,
// which depends on the partial sum). That attempt is added as the
// attempt-by-attempt walk adds it, and the scan goes on from the next one in
// the binade of the new sum; so does an attempt added to a clock of 0. The
// first attempt whose sum is not below 1 ends the round. Returns the number of
// attempts that fire and their clock, or -1 for a clock too small to scale
// (the caller sums attempt by attempt). Every lane of the wavefront calls it.
template <int W>
__device__ __forceinline__ int clock_exact_scan(double clock, const double (&tau)[W], double *clock_out) {
    const int lane = threadIdx.x & 63;
    constexpr int N = 64 * W;
    int done = 0;  // attempts before done fire; s is the clock after them
    double s = clock;
    for (int iter = 0; iter <= N; ++iter) {
        if (done == N) break;
        if (!(s > 0.0)) {
            const double t0 = part_at<W>(tau, done);  // 0 + tau is tau
            if (!(t0 < 1.0)) break;
            s = t0;
            ++done;
            continue;
        }
        const long long cb = __double_as_longlong(s);
        const int e = (int)((cb >> 52) & 0x7ff) - 1023;
        if (e < -960) return -1;
        const double up = __longlong_as_double((long long)(1023 + 52 - e) << 52);    // 2^(52-e)
        const double down = __longlong_as_double((long long)(1023 - 52 + e) << 52);  // 2^(e-52)
        const double S0 = s * up;                                                    // in [2^52, 2^53)
        const double T = 0x1p53 - S0;
        double P[W];
        int special = N;  // first attempt past the binade or on a tie
        double carry = 0.0;
#pragma unroll
        for (int w = 0; w < W; ++w) {
            const bool live = 64 * w + lane >= done;
            const double v = tau[w] * up;
            const double fl = floor(v);
            const double fr = v - fl;
            P[w] = wave_prefix_sum(live ? (fr > 0.5 ? fl + 1.0 : fl) : 0.0) + carry;
            carry = lane_f64(P[w], 63);
            const unsigned long long odd = __ballot(live && (fr == 0.5 || !(P[w] < T)));
            if (special == N && odd != 0ull) special = 64 * w + __ffsll((long long)odd) - 1;
        }
        const double before = special > done ? (S0 + part_at<W>(P, special - 1)) * down : s;
        if (special == N) {
            s = before;
            done = N;
            break;
        }
        const double s2 = before + part_at<W>(tau, special);
        if (!(s2 < 1.0)) {
            s = before;
            done = special;
            break;
        }
        s = s2;
        done = special + 1;
    }
    *clock_out = s;
    return done;
}

// One chain walked by the whole wavefront, 64 attempts per round, for paired
// classes. Attempt kbase + i belongs to lane i; its draws do not depend on the
// state, but the transition it picks (eq:sampling2) and its waiting time
// (eq:sampling) depend on the state the attempts before it leave. Each lane
// first assumes the round's starting state, then recomputes its state from the
// transitions the lanes below it picked (a ballot per transition and a count of
// the set bits below the lane) and its own pick from that state, until no pick
// changes. Lane i is settled after i + 1 passes whatever the guesses were, so
// the result is the one attempt-by-attempt walk gives; with many individuals
// the rates barely move and one or two passes settle every lane (and only the
// lanes up to the first attempt surely past the window end need to). The
// waiting times then follow in parallel, and the clock's partial sums, which
// binary64 addition rounds one by one, come from an exact integer prefix sum
// (clock_by_scan) or, where that does not apply, attempt by attempt. The
// attempts whose sum stays below the window end fire; they form a prefix of
// the lanes because the clock never decreases. Every lane holds the same
// chain state.
// Counts are exact integers in binary64 and the rates, running sums, targets
// and waiting times are the same functions of the same state as in a walk
// attempt by attempt, so the bits agree.
// With FED, every thread of a workgroup calls it: wavefront 0 walks the chain
// while wavefront 1 computes the next round's draws (Philox, -log rand, rand)
// into LDS, one round ahead, with a workgroup barrier per round; the draws do
// not depend on the state, so the walk is the same.
template <int NP, bool FED>
__device__ __forceinline__ void pairs_walk_block(const Model &m, Chain<2 * NP, 2 * NP> &c, uint32_t kbase,
                                                 uint32_t node, uint32_t day, uint32_t key0, uint32_t key1,
                                                 unsigned long long *status, int32_t r) {
    constexpr int NT = 2 * NP;
    __shared__ double sh_tau[kWaves][64];
    __shared__ double sh_draw[2][2][64];  // fed walk: [buffer][E, U][attempt of the round]
    __shared__ int sh_go;                 // fed walk: 0 once wavefront 0 has ended the chain
    const uint32_t lane = threadIdx.x & 63u;
    const int wave = threadIdx.x >> 6;
    const unsigned long long below = (1ull << lane) - 1ull;
    [[maybe_unused]] int rnd = 0;
    if constexpr (FED) {
        auto produce = [&](uint32_t kb, int b) {
            const Word4 o = philox4x32_10(Word4{kb + lane, node, day, 0u}, key0, key1);
            sh_draw[b][0][lane] = minus_log(unit_open(o.a, o.b));
            sh_draw[b][1][lane] = unit_open(o.c, o.d);
        };
        if (wave == 1) produce(kbase, 0);
        if (threadIdx.x == 0) sh_go = 1;
        __syncthreads();
        if (wave != 0) {
            // the producer (and two idle wavefronts): one barrier per round of
            // wavefront 0, which clears sh_go before the barrier of its last
            for (;; ++rnd) {
                if (wave == 1) produce(kbase + 64u * (uint32_t)(rnd + 1), (rnd + 1) & 1);
                __syncthreads();
                if (!sh_go) return;
            }
        }
    }
    for (;; ++rnd) {
        double E, U;
        if constexpr (FED) {
            E = sh_draw[rnd & 1][0][lane];
            U = sh_draw[rnd & 1][1][lane];
        } else {
            const Word4 o = philox4x32_10(Word4{kbase + lane, node, day, 0u}, key0, key1);
            E = minus_log(unit_open(o.a, o.b));
            U = unit_open(o.c, o.d);
        }
        // guess: every attempt sees the round's starting state
        int j = 0;
        {
            const double target = U * c.lam;
#pragma unroll
            for (int k = 0; k < NT; ++k) j += c.cum[k] < target ? 1 : 0;
        }
        double lam = c.lam;
        int settle = 63;  // the attempts 0 .. settle need their final picks
        for (int pass = 0; pass < 64; ++pass) {
            double x[NT];
#pragma unroll
            for (int q = 0; q < NP; ++q) {
                const int inf = __popcll(__ballot(j == 2 * q) & below);
                const int rec = __popcll(__ballot(j == 2 * q + 1) & below);
                const double dS = (double)(rec - inf);
                x[2 * q] = c.xd[2 * q] + dS;
                x[2 * q + 1] = c.xd[2 * q + 1] - dS;
            }
            double cum[NT];
            double l = 0.0;
#pragma unroll
            for (int k = 0; k < NT; ++k) {
                l = l + c.cphi[k] * x[k];
                cum[k] = l;
            }
            // target > 0 whenever the attempt can fire: target = 0 needs
            // lambda < 2^-1021, and then tau = E/lambda > 1 since E >= 2^-53
            const double target = U * l;
            int jn = 0;
#pragma unroll
            for (int k = 0; k < NT; ++k) jn += cum[k] < target ? 1 : 0;
            const unsigned long long moved = __ballot(jn != j);
            j = jn;
            lam = l;
            if (moved == 0ull) break;
            if (pass == 0) continue;  // large herds settle in one or two passes without it
            // An attempt whose clock surely lands past the window end stops
            // the chain, so only the picks up to it have to settle. If none of
            // them moved in this pass, they and their waiting times are those
            // of the attempt-by-attempt walk (each was computed from the
            // unchanged picks below it); the clock bound then comes from exact
            // waiting times, and its margin is far above the rounding of the
            // approximate prefix sum.
            const double reach = c.clock + wave_prefix_sum(l > 0.0 ? E / l : __builtin_inf());
            const unsigned long long over = __ballot(!(reach < 1.0 + 0x1p-30));
            if (over != 0ull) {
                const int a = __ffsll((long long)over) - 1;
                if ((moved & (a >= 63 ? ~0ull : ((2ull << a) - 1ull))) == 0ull) {
                    settle = a;
                    break;
                }
            }
        }
        // lambda = 0: tau = inf, never fires; attempts past `settle` do not
        // fire and may hold unsettled picks
        const double tau = (int)lane > settle ? __builtin_inf() : E / lam;
        double clock;
        int A = clock_by_scan(c.clock, tau, &clock);
        if (A < 0) {
            // the clock, attempt by attempt. The waiting times go through LDS
            // and come back as broadcast reads, which issue ahead of the
            // dependent additions.
            sh_tau[wave][lane] = tau;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            double t = c.clock;
#pragma unroll 16
            for (int i = 0; i < 64; ++i) t = t + sh_tau[wave][i];
            A = 64;
            clock = t;
            if (!(t < 1.0)) {
                double s = c.clock, mine = 0.0;
#pragma unroll 16
                for (int i = 0; i < 64; ++i) {
                    s = s + sh_tau[wave][i];
                    if ((int)lane == i) mine = s;
                }
                A = __popcll(__ballot(mine < 1.0));
                clock = A > 0 ? lane_f64(mine, A - 1) : c.clock;
            }
            __builtin_amdgcn_wave_barrier();  // the next round rewrites sh_tau
        }
        bool limit = false;
        if (c.fired + A >= SIM_MAX_FIRED) {
            A = SIM_MAX_FIRED - c.fired;
            limit = true;
        }
        const unsigned long long fired = A >= 64 ? ~0ull : ((1ull << A) - 1ull);
#pragma unroll
        for (int q = 0; q < NP; ++q) {
            const int inf = __popcll(__ballot(j == 2 * q) & fired);
            const int rec = __popcll(__ballot(j == 2 * q + 1) & fired);
            const double dS = (double)(rec - inf);
            c.xd[2 * q] = c.xd[2 * q] + dS;
            c.xd[2 * q + 1] = c.xd[2 * q + 1] - dS;
        }
        if (A > 0 && !limit) c.clock = clock;
        c.fired = c.fired + A;
        pairs_rates_full<NP>(c);
        if (limit && lane == 0) atomicMin(status, (STATUS_LIMIT_TAG << 32) | (unsigned long long)(uint32_t)r);
        const bool done = limit || A < 64 || !(c.lam > 0.0);
        if constexpr (FED) {
            if (done && lane == 0) sh_go = 0;
            __syncthreads();  // the producer's next round is in LDS; with sh_go = 0 the others leave
        }
        if (done) return;
        kbase = kbase + 64;
    }
}

// One chain walked by the four wavefronts of a workgroup, 256 attempts per
// round (attempt kbase + t for thread t), for paired classes: the scheme of
// pairs_walk_block, with the picks of each wavefront (one ballot per
// transition) shared in LDS so that an attempt counts the picks of every
// attempt below it, and the clock of the 256 waiting times decided by
// wavefront 0. Every thread of the workgroup calls it with the same state and
// ends with the same state. It pays off for long chains only: a round starts
// only while the window still expects min_attempts attempts
// (lambda (1 - clock)), and a round whose picks do not settle within
// kGroupPasses passes is dropped. Returns whether the chain is done; if not,
// the caller continues with the single-wavefront walk from attempt kbase and
// state c, which are those at the start of a round.
constexpr int kGroupPasses = 8;

template <int NP>
__device__ bool pairs_walk_group(Chain<2 * NP, 2 * NP> &c, uint32_t &kbase, uint32_t node, uint32_t day,
                                 uint32_t key0, uint32_t key1, unsigned long long *status, int32_t r,
                                 double min_attempts) {
    constexpr int NT = 2 * NP;
    constexpr int kRound = kBlock;
    __shared__ unsigned long long sh_b[2][kWaves][NT];  // picks of each wavefront and pass, per transition
    __shared__ int sh_moved[2][kWaves];
    __shared__ double sh_tau[kRound];
    __shared__ double sh_clock;
    __shared__ int sh_fired;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const unsigned long long below = (1ull << lane) - 1ull;
    int buf = 0;
    for (;;) {
        if (c.lam * (1.0 - c.clock) < min_attempts) return false;  // the same in every thread
        const Word4 o = philox4x32_10(Word4{kbase + (uint32_t)t, node, day, 0u}, key0, key1);
        const double E = minus_log(unit_open(o.a, o.b));
        const double U = unit_open(o.c, o.d);
        int j = 0;
        {
            const double target = U * c.lam;
#pragma unroll
            for (int k = 0; k < NT; ++k) j += c.cum[k] < target ? 1 : 0;
        }
        double lam = c.lam;
        bool settled = false;
        for (int pass = 0; pass < kGroupPasses; ++pass) {
            unsigned long long bk[NT];
#pragma unroll
            for (int k = 0; k < NT; ++k) bk[k] = __ballot(j == k);
            if (lane == 0) {
#pragma unroll
                for (int k = 0; k < NT; ++k) sh_b[buf][wave][k] = bk[k];
            }
            __syncthreads();
            double l = 0.0, cum[NT];
#pragma unroll
            for (int q = 0; q < NP; ++q) {
                int inf = (int)__popcll(bk[2 * q] & below), rec = (int)__popcll(bk[2 * q + 1] & below);
                for (int w = 0; w < wave; ++w) {
                    inf += (int)__popcll(sh_b[buf][w][2 * q]);
                    rec += (int)__popcll(sh_b[buf][w][2 * q + 1]);
                }
                const double dS = (double)(rec - inf);
                l = l + c.cphi[2 * q] * (c.xd[2 * q] + dS);
                cum[2 * q] = l;
                l = l + c.cphi[2 * q + 1] * (c.xd[2 * q + 1] - dS);
                cum[2 * q + 1] = l;
            }
            const double target = U * l;
            int jn = 0;
#pragma unroll
            for (int k = 0; k < NT; ++k) jn += cum[k] < target ? 1 : 0;
            const bool moved = __ballot(jn != j) != 0ull;
            j = jn;
            lam = l;
            if (lane == 0) sh_moved[buf][wave] = moved ? 1 : 0;
            __syncthreads();
            bool any = false;
#pragma unroll
            for (int w = 0; w < kWaves; ++w) any = any || sh_moved[buf][w] != 0;
            buf ^= 1;
            if (!any) {
                settled = true;
                break;
            }
        }
        if (!settled) return false;  // the same in every thread; nothing of this round applied
        const int last = buf ^ 1;  // the final picks' ballots
        sh_tau[t] = E / lam;       // lambda = 0: tau = inf, never fires
        __syncthreads();
        if (wave == 0) {
            double tw[kWaves];
#pragma unroll
            for (int w = 0; w < kWaves; ++w) tw[w] = sh_tau[64 * w + lane];
            double clock;
            int A = clock_exact_scan<kWaves>(c.clock, tw, &clock);
            if (A < 0) {
                // attempt by attempt, in order
                double s = c.clock, mine[kWaves];
#pragma unroll
                for (int w = 0; w < kWaves; ++w) {
                    mine[w] = 0.0;
#pragma unroll 16
                    for (int i = 0; i < 64; ++i) {
                        s = s + sh_tau[64 * w + i];
                        if (lane == i) mine[w] = s;
                    }
                }
                A = 0;
#pragma unroll
                for (int w = 0; w < kWaves; ++w) A += (int)__popcll(__ballot(mine[w] < 1.0));
                clock = c.clock;
#pragma unroll
                for (int w = 0; w < kWaves; ++w)
                    if (A > 0 && (A - 1) / 64 == w) clock = lane_f64(mine[w], (A - 1) % 64);
            }
            if (lane == 0) {
                sh_clock = clock;
                sh_fired = A;
            }
        }
        __syncthreads();
        int A = sh_fired;
        const double clock = sh_clock;
        bool limit = false;
        if (c.fired + A >= SIM_MAX_FIRED) {
            A = SIM_MAX_FIRED - c.fired;
            limit = true;
        }
#pragma unroll
        for (int q = 0; q < NP; ++q) {
            int inf = 0, rec = 0;
#pragma unroll
            for (int w = 0; w < kWaves; ++w) {
                const int nw = A - 64 * w;
                const unsigned long long fired = nw >= 64 ? ~0ull : (nw > 0 ? ((1ull << nw) - 1ull) : 0ull);
                inf += (int)__popcll(sh_b[last][w][2 * q] & fired);
                rec += (int)__popcll(sh_b[last][w][2 * q + 1] & fired);
            }
            const double d = (double)(rec - inf);
            c.xd[2 * q] = c.xd[2 * q] + d;
            c.xd[2 * q + 1] = c.xd[2 * q + 1] - d;
        }
        if (A > 0 && !limit) c.clock = clock;
        c.fired = c.fired + A;
        pairs_rates_full<NP>(c);
        if (limit) {
            if (t == 0) atomicMin(status, (STATUS_LIMIT_TAG << 32) | (unsigned long long)(uint32_t)r);
            return true;
        }
        if (A < kRound || !(c.lam > 0.0)) return true;
        kbase = kbase + kRound;
    }
}

// A single live chain, run by the whole wavefront with every lane holding
// the same state: lane i computes attempt kbase + i, and the attempts are
// walked in order with the chosen transition held in a scalar register.
template <class Rules>
__device__ __forceinline__ void chain_uniform(const Model &m, typename Rules::State &c, uint32_t kbase,
                                              uint32_t node, uint32_t day, uint32_t key0, uint32_t key1,
                                              unsigned long long *status, int32_t r) {
    const uint32_t lane = threadIdx.x & 63u;
    for (;;) {
        const Word4 o = philox4x32_10(Word4{kbase + lane, node, day, 0u}, key0, key1);
        const double e_mine = minus_log(unit_open(o.a, o.b));
        const double u_mine = unit_open(o.c, o.d);
        for (int i = 0; i < 64; ++i) {
            const double tau = lane_f64(e_mine, i) / c.lam;
            const double t1 = c.clock + tau;
            const int j = __builtin_amdgcn_readfirstlane(invert<Rules>(m, c, lane_f64(u_mine, i) * c.lam));
            if (!(t1 < 1.0)) return;
            c.clock = t1;
            Rules::apply_uniform(m, j, c);
            c.fired = c.fired + 1;
            if (c.fired >= SIM_MAX_FIRED) {
                if (lane == 0) atomicMin(status, (STATUS_LIMIT_TAG << 32) | (unsigned long long)(uint32_t)r);
                return;
            }
            if (!(c.lam > 0.0)) return;
        }
        kbase = kbase + 64;
    }
}

// Every chain of a wavefront to the end of the window. Attempt k of a chain
// uses Philox block (k, node, day, 0); the blocks do not depend on the state,
// so while m < 64 chains are live the wavefront computes 64/m blocks per
// chain in parallel (their -log rand and rand), parks them in LDS, and each
// live lane then walks its own in order. With all 64 lanes live each lane
// draws its own block; with one chain left, or at most `few` of which one
// still expects many attempts, the whole wavefront walks them one after
// another (pairs_walk_block). Node, day and key are each lane's own (lanes of
// a slot handle may be at different days). Every lane of the wavefront must
// call this.
template <class Rules>
__device__ __forceinline__ void run_chains(const Model &m, typename Rules::State &c, bool live, uint32_t node,
                                           uint32_t day, uint32_t key0, uint32_t key1,
                                           unsigned long long *status, int32_t r, uint32_t few_chains) {
    __shared__ double sh_e[kWaves][64], sh_u[kWaves][64];
    __shared__ uint32_t sh_node[kWaves][64], sh_key[kWaves][64], sh_seed[kWaves][64], sh_k[kWaves][64];
    __shared__ uint32_t sh_day[kWaves][64];
    const int wave = threadIdx.x >> 6;
    const uint32_t lane = threadIdx.x & 63u;
    uint32_t kbase = 0;  // next attempt index of this lane's chain
    live = live && c.lam > 0.0;
    for (;;) {
        const unsigned long long mask = __ballot(live);
        if (mask == 0ull) break;
        if (mask == ~0ull) {
            const Word4 o = philox4x32_10(Word4{kbase, node, day, 0u}, key0, key1);
            kbase = kbase + 1;
            live = chain_step<Rules>(m, c, minus_log(unit_open(o.a, o.b)), unit_open(o.c, o.d), status, r);
            continue;
        }
        const uint32_t nlive = (uint32_t)__popcll(mask);
        // One chain left, or a few of which one still expects many attempts in
        // the window (lambda (1 - clock)): the whole wavefront walks them one
        // after another, 64 attempts at a time, instead of a lane each.
        const bool few = nlive <= few_chains &&
                         (nlive == 1 || __ballot(live && c.lam * (1.0 - c.clock) > 10.0 * (double)nlive) != 0ull);
        for (unsigned long long left = few ? mask : 0ull; left != 0ull; left &= left - 1ull) {
            const int h = __ffsll((long long)left) - 1;
            typename Rules::State u;
#pragma unroll
            for (int k = 0; k < Rules::NC; ++k) u.xd[k] = lane_f64(c.xd[k], h);
#pragma unroll
            for (int k = 0; k < Rules::NT; ++k) {
                u.cphi[k] = lane_f64(c.cphi[k], h);
                u.cum[k] = lane_f64(c.cum[k], h);
            }
            u.lam = lane_f64(c.lam, h);
            u.clock = lane_f64(c.clock, h);
            u.fired = __builtin_amdgcn_readlane(c.fired, h);
            const uint32_t kb = (uint32_t)__builtin_amdgcn_readlane((int)kbase, h);
            const uint32_t nh = (uint32_t)__builtin_amdgcn_readlane((int)node, h);
            const uint32_t dh = (uint32_t)__builtin_amdgcn_readlane((int)day, h);
            const uint64_t st = (uint64_t)status;
            unsigned long long *sth = (unsigned long long *)(((uint64_t)(uint32_t)__builtin_amdgcn_readlane(
                                                                  (int)(uint32_t)(st >> 32), h) << 32) |
                                                              (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)st, h));
            const uint32_t k0 = (uint32_t)__builtin_amdgcn_readlane((int)key0, h);
            const uint32_t k1 = (uint32_t)__builtin_amdgcn_readlane((int)key1, h);
            const int32_t rh = __builtin_amdgcn_readlane(r, h);
            if constexpr (Rules::kPairs > 0) {
                pairs_walk_block<Rules::kPairs>(m, u, kb, nh, dh, k0, k1, sth, rh);
            } else {
                chain_uniform<Rules>(m, u, kb, nh, dh, k0, k1, sth, rh);
            }
            if ((int)lane == h) c = u;
        }
        if (few) break;
        const uint32_t per = 64u / nlive;
        const uint32_t rank = (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
        if (live) {
            sh_node[wave][rank] = node;
            sh_day[wave][rank] = day;
            sh_key[wave][rank] = key1;
            sh_seed[wave][rank] = key0;
            sh_k[wave][rank] = kbase;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (lane < nlive * per) {
            const uint32_t ch = lane % nlive, t = lane / nlive;
            const Word4 o = philox4x32_10(Word4{sh_k[wave][ch] + t, sh_node[wave][ch], sh_day[wave][ch], 0u},
                                          sh_seed[wave][ch], sh_key[wave][ch]);
            sh_e[wave][ch * per + t] = minus_log(unit_open(o.a, o.b));
            sh_u[wave][ch * per + t] = unit_open(o.c, o.d);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (live) {
            for (uint32_t t = 0; t < per; ++t) {
                live = chain_step<Rules>(m, c, sh_e[wave][rank * per + t], sh_u[wave][rank * per + t], status, r);
                if (!live) break;
            }
            kbase = kbase + per;
        }
        __builtin_amdgcn_wave_barrier();  // the next round rewrites the LDS slots
    }
}

// Whether no error has been recorded, read once per workgroup so that every
// thread takes the same branch (another wavefront of the workgroup may record
// an error while this one is still starting). Every thread must call it.
__device__ __forceinline__ bool block_ok(const unsigned long long *status) {
    __shared__ int ok;
    __syncthreads();
    if (threadIdx.x == 0) ok = *(volatile const unsigned long long *)status == STATUS_OK;
    __syncthreads();
    return ok != 0;
}

// block_ok for a kernel that checks once per launch: thread 0 reads the
// status word right away, alongside the loads the workgroup has already
// issued, and one barrier publishes it (no earlier reader of the flag to wait
// for), so the check adds no round trip of its own.
__device__ __forceinline__ bool block_ok_once(const unsigned long long *status) {
    __shared__ int ok;
    if (threadIdx.x == 0) ok = *(volatile const unsigned long long *)status == STATUS_OK;
    __syncthreads();
    return ok != 0;
}

// Wavefront reductions with DPP lane moves, which run in the vector ALU:
// pairs and quads (quad permutes), rows of 8 and 16 lanes (half-row and row
// mirrors), then row 0 into row 1 and row 2 into row 3 (broadcast of lane 15),
// then rows 0-1 into rows 2-3 (broadcast of lane 31); lane 63 ends with the
// whole wavefront, read back as a uniform value. Every lane must be active.
// (A shuffle butterfly would wait on an LDS crossbar round trip per step.)
template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ int32_t dpp_move(int32_t v) {
    // lanes of rows outside ROWS read 0
    return __builtin_amdgcn_update_dpp(0, v, CTRL, ROWS, 0xf, false);
}

template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ long long dpp_move64(long long v) {
    const uint32_t lo = (uint32_t)dpp_move<CTRL, ROWS>((int32_t)(uint32_t)v);
    const uint32_t hi = (uint32_t)dpp_move<CTRL, ROWS>((int32_t)(uint32_t)((unsigned long long)v >> 32));
    return (long long)(((unsigned long long)hi << 32) | lo);
}

constexpr int kDppXor1 = 0xb1, kDppXor2 = 0x4e, kDppHalfMirror = 0x141, kDppMirror = 0x140,
              kDppBcast15 = 0x142, kDppBcast31 = 0x143;

__device__ __forceinline__ long long wave_sum(long long v) {
    v += dpp_move64<kDppXor1>(v);
    v += dpp_move64<kDppXor2>(v);
    v += dpp_move64<kDppHalfMirror>(v);
    v += dpp_move64<kDppMirror>(v);
    v += dpp_move64<kDppBcast15, 0xa>(v);
    v += dpp_move64<kDppBcast31, 0xc>(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int32_t)(uint32_t)v, 63);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int32_t)(uint32_t)((unsigned long long)v >> 32), 63);
    return (long long)(((unsigned long long)hi << 32) | lo);
}

// Per-lane contributions to the daily records of one phase.
template <int NC>
struct Tally {
    long long prev, trans;
    long long tot[NC];
    int32_t most;  // most SSA transitions of one lane's chain (the day's straggler)
};

// (for values >= 0: rows outside a broadcast's mask read 0)
__device__ __forceinline__ int32_t wave_max(int32_t v) {
    v = max(v, dpp_move<kDppXor1>(v));
    v = max(v, dpp_move<kDppXor2>(v));
    v = max(v, dpp_move<kDppHalfMirror>(v));
    v = max(v, dpp_move<kDppMirror>(v));
    v = max(v, dpp_move<kDppBcast15, 0xa>(v));
    v = max(v, dpp_move<kDppBcast31, 0xc>(v));
    return __builtin_amdgcn_readlane(v, 63);
}

// Sum tallies over the workgroup and add them to the records of one set
// (every lane of the workgroup belongs to the same trajectory).
template <int NC>
__device__ void flush_block(const Model &m, const DevState &s, const Tally<NC> &t, int32_t set, int32_t d_rec,
                            int32_t d_ssa, int32_t region) {
    __shared__ long long part[kWaves][2 + NC];
    __shared__ int32_t part_most[kWaves];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t S = (int64_t)s.n_inst * s.R;
    const int32_t most = wave_max(t.most);
    if (lane == 0) part_most[wave] = most;
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
            if (sum) atomicAdd(&s.prevalence[d_rec * S + set], (int32_t)sum);
        } else if (i == 1 && d_ssa >= 0) {
            if (sum) {
                atomicAdd((unsigned long long *)&s.transitions[d_ssa * S + set], (unsigned long long)sum);
                int32_t m_all = 0;
#pragma unroll
                for (int q = 0; q < kWaves; ++q) m_all = max(m_all, part_most[q]);
                atomicMax(&s.max_fired[d_ssa * S + set], m_all);
            }
        } else if (i >= 2 && d_rec >= 0 && comp_on<NC>(m, i - 2)) {
            if (sum) atomicAdd((unsigned long long *)&s.totals[(d_rec * S + set) * m.nc + (i - 2)],
                               (unsigned long long)sum);
            if (sum && region >= 0)
                atomicAdd((unsigned long long *)&s.regional[((d_rec * S + set) * s.n_regions + region) * m.nc + (i - 2)],
                          (unsigned long long)sum);
        }
    }
    __syncthreads();
}

// Sum tallies over the wavefronts of a replicate tile (lane = replicate) and
// add them to the records of the lane's set.
template <int NC>
__device__ void flush_tile(const Model &m, const DevState &s, const Tally<NC> &t, int32_t set, int32_t d_rec,
                           int32_t d_ssa, int32_t region) {
    __shared__ long long part[kWaves][64][2 + NC];
    __shared__ int32_t part_most[kWaves][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t S = (int64_t)s.n_inst * s.R;
    part[wave][lane][0] = t.prev;
    part[wave][lane][1] = t.trans;
    part_most[wave][lane] = t.most;
#pragma unroll
    for (int c = 0; c < NC; ++c) part[wave][lane][2 + c] = t.tot[c];
    __syncthreads();
    if (wave == 0 && set >= 0) {
        long long v[2 + NC];
#pragma unroll
        for (int i = 0; i < 2 + NC; ++i) {
            v[i] = 0;
#pragma unroll
            for (int q = 0; q < kWaves; ++q) v[i] += part[q][lane][i];
        }
        if (d_rec >= 0) {
            if (v[0]) atomicAdd(&s.prevalence[d_rec * S + set], (int32_t)v[0]);
#pragma unroll
            for (int c = 0; c < NC; ++c)
                if (comp_on<NC>(m, c) && v[2 + c]) {
                    atomicAdd((unsigned long long *)&s.totals[(d_rec * S + set) * m.nc + c], (unsigned long long)v[2 + c]);
                    if (region >= 0)
                        atomicAdd((unsigned long long *)&s.regional[((d_rec * S + set) * s.n_regions + region) * m.nc + c],
                                  (unsigned long long)v[2 + c]);
                }
        }
        if (d_ssa >= 0 && v[1]) {
            atomicAdd((unsigned long long *)&s.transitions[d_ssa * S + set], (unsigned long long)v[1]);
            int32_t m_all = 0;
#pragma unroll
            for (int q = 0; q < kWaves; ++q) m_all = max(m_all, part_most[q][lane]);
            atomicMax(&s.max_fired[d_ssa * S + set], m_all);
        }
    }
    __syncthreads();
}

// The SSA of a workgroup whose only herd sits in thread 0 (one lane per node):
// with paired classes its chain is walked by all four wavefronts, otherwise
// as anywhere else. Every thread of the workgroup calls it.
template <class Rules>
__device__ void group_chain(const Model &m, typename Rules::State &c, bool live, uint32_t node, uint32_t day,
                            uint32_t key0, uint32_t key1, unsigned long long *status, int32_t r,
                            uint32_t few_chains, double min_attempts) {
    if constexpr (Rules::kPairs == 0) {
        run_chains<Rules>(m, c, live, node, day, key0, key1, status, r, few_chains);
    } else {
        constexpr int NT = Rules::NT;
        __shared__ double sh_x[NT], sh_cphi[NT], sh_cum[NT], sh_lam;
        __shared__ uint32_t sh_key[4];
        __shared__ int sh_go;
        if (threadIdx.x == 0) {
#pragma unroll
            for (int k = 0; k < NT; ++k) {
                sh_x[k] = c.xd[k];
                sh_cphi[k] = c.cphi[k];
                sh_cum[k] = c.cum[k];
            }
            sh_lam = c.lam;
            sh_key[0] = node;
            sh_key[1] = key0;
            sh_key[2] = key1;
            sh_key[3] = (uint32_t)r;
            sh_go = live && c.lam > 0.0 ? 1 : 0;
        }
        __syncthreads();
        if (!sh_go) return;  // the same in every thread
        // the day's critical chain: its wavefronts issue ahead of the other
        // waves on their SIMDs while it is walked
        __builtin_amdgcn_s_setprio(3);
        typename Rules::State u;
#pragma unroll
        for (int k = 0; k < NT; ++k) {
            u.xd[k] = sh_x[k];
            u.cphi[k] = sh_cphi[k];
            u.cum[k] = sh_cum[k];
        }
        u.lam = sh_lam;
        u.clock = 0.0;
        u.fired = 0;
        uint32_t kb = 0;
        // a short chain, or the end of a long one, is walked by wavefront 0
        // (thread 0 is in it) while wavefront 1 draws one round ahead
        if (!pairs_walk_group<Rules::kPairs>(u, kb, sh_key[0], day, sh_key[1], sh_key[2], status, (int32_t)sh_key[3],
                                             min_attempts))
            pairs_walk_block<Rules::kPairs, true>(m, u, kb, sh_key[0], day, sh_key[1], sh_key[2], status,
                                                  (int32_t)sh_key[3]);
        __builtin_amdgcn_s_setprio(0);
        if (threadIdx.x == 0) c = u;
    }
}

// Per-lane parameters of a replicate tile, staged in LDS once per tile (every
// position of a tile belongs to one instance, so lane r has the same set):
// rate constants, shedding and decay rates and the Philox key.
struct TileParams {
    double (*coef)[64];   // [MAXT][64]
    double *alpha;        // [64]
    double (*beta)[64];   // [4][64]
    uint32_t *key0, *key1;
};

// Draw n of the tot individuals in the compartments of mask from x without
// replacement (Sec. 3.2): draw q picks the individual at a uniform position
// in [0, remaining) of the selected compartments in ascending order, from the
// Philox block (q / 2, g, d, 1). Removes them from x and counts them in take.
// pre, when given, holds the first kPreDraws draws (computed ahead in parallel);
// an event that needs no more than those (every movement of up to five
// animals) has all its picks multiplied out at once, since draw q picks among
// tot - q individuals whatever the earlier picks were, and only the walk over
// the compartments stays serial.
constexpr int kPreDraws = 6;

template <int NC>
__device__ __forceinline__ void draw_individuals(int32_t *x, int32_t *take, uint32_t mask, int32_t n, long long tot,
                                                 uint32_t g, int32_t d, uint32_t key0, uint32_t key1,
                                                 const uint64_t *pre = nullptr) {
    long long cum[NC];  // running sums of the selected compartments, ascending
    long long run = 0;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        take[c] = 0;
        run += ((mask >> c) & 1u) ? x[c] : 0;
        cum[c] = run;
    }
    if (pre && n <= kPreDraws && tot <= 0x7fffffffLL) {
        // the running sums and picks fit 32 bits (the same comparisons)
        uint32_t pick[kPreDraws], cum32[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) cum32[c] = (uint32_t)cum[c];
#pragma unroll
        for (int q = 0; q < kPreDraws; ++q)
            pick[q] = q < n ? (uint32_t)__umul64hi(pre[q], (uint64_t)(tot - q)) : 0u;
#pragma unroll
        for (int q = 0; q < kPreDraws; ++q) {
            if (q >= n) break;
            int chosen = 0;
#pragma unroll
            for (int c = 0; c < NC; ++c) chosen += cum32[c] <= pick[q] ? 1 : 0;
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const int hit = c == chosen ? 1 : 0;
                x[c] -= hit;
                take[c] += hit;
                cum32[c] -= c >= chosen ? 1u : 0u;
            }
        }
        return;
    }
    Word4 o{0, 0, 0, 0};
    for (int32_t q = 0; q < n; ++q) {
        uint64_t bits;
        if (pre && q < kPreDraws) {
            bits = pre[q];
        } else if ((q & 1) == 0) {
            o = philox4x32_10(Word4{(uint32_t)q >> 1, g, (uint32_t)d, 1u}, key0, key1);
            bits = ((uint64_t)o.b << 32) | o.a;
        } else {
            bits = ((uint64_t)o.d << 32) | o.c;
        }
        const uint64_t pick = __umul64hi(bits, (uint64_t)tot);  // uniform on [0, tot)
        // the compartment holding individual `pick` in ascending order is the
        // number of running sums at or below it (a compartment outside the
        // mask, or empty, repeats the sum before it and is passed over)
        int chosen = 0;
#pragma unroll
        for (int c = 0; c < NC; ++c) chosen += (uint64_t)cum[c] <= pick ? 1 : 0;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const int hit = c == chosen ? 1 : 0;
            x[c] -= hit;
            take[c] += hit;
            cum[c] -= c >= chosen ? 1 : 0;
        }
        tot -= 1;
    }
}

// Compartment that an individual drawn from compartment c lands in (internal
// and external transfers): 4 bits per source compartment of the event's map.
__device__ __forceinline__ int shifted(uint32_t smap, int c) { return (int)((smap >> (4 * c)) & 0xFu); }

// The loads day_wave starts from: the lane's position's node and instance, its
// counts and phi (zeros for a lane past the end).
template <int NC>
struct LaneLoad {
    int32_t x[NC];
    double phi;
    int32_t nid, inst;
};

template <int NC>
__device__ __forceinline__ LaneLoad<NC> lane_load(const Model &m, const DevState &s, int64_t l) {
    LaneLoad<NC> q;
    q.nid = -1;
    q.inst = 0;
    q.phi = 0.0;
#pragma unroll
    for (int c = 0; c < NC; ++c) q.x[c] = 0;
    if (l < s.L) {
        const int64_t pos = s.RL == 1 ? l : l / s.RL;
        q.nid = s.node_id[pos];
        q.inst = s.inst[pos];
#pragma unroll
        for (int c = 0; c < NC; ++c) q.x[c] = comp_on<NC>(m, c) ? s.u[(int64_t)c * s.L + l] : 0;
        q.phi = s.phi[l];
    }
    return q;
}

// What a kernel may add to day_wave: after_prologue() runs on every lane once
// the previous day is closed, before the SSA; after_ssa(state, active) sees the
// lane's chain state after the SSA and returns whether day_wave stores it.
struct NoHooks {
    __device__ void after_prologue() const {}
    template <class St>
    __device__ bool after_ssa(const St &, bool) const { return true; }
};

// The day phase for the lane l of a wavefront (every lane of the wavefront
// must call it; lanes with l >= L or replicate lane r >= r_end take part in
// the wavefront-level steps only): close day d-1 (phi update + record) if
// prologue, then run the SSA of day d if ssa. Adds the lane's counts to t.
// uniform_set >= 0 is the set of every lane (a workgroup of one instance and
// one replicate), so that its parameters are read without waiting for the
// lane's instance. Every load that does not depend on another is issued
// first (padding positions hold zeros).
template <class Rules, class Hooks = NoHooks>
__device__ __forceinline__ void day_wave(const Model &m, const DevState &s, int64_t l, int32_t d,
                                         bool prologue, bool ssa, Tally<Rules::NC> &t, int32_t r_end,
                                         unsigned long long *status, const TileParams *tp = nullptr,
                                         const Hooks &hooks = Hooks{}, int32_t uniform_set = -1,
                                         bool group_walk = false, bool lane_on = true) {
    constexpr int NC = Rules::NC, NT = Rules::NT;
    const int32_t R = s.R, RL = s.RL;
    const bool in_range = l < s.L;
    const int32_t r = !in_range || RL == 1 ? 0 : (int32_t)(l % RL);
    const int32_t rec = prologue ? s.rec_slot[d - 1] : -1;
    const LaneLoad<NC> q = lane_load<NC>(m, s, l);
    int32_t x[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) x[c] = q.x[c];
    double phi = q.phi;
    int32_t nid = q.nid, inst = q.inst;
    // padding positions and idle lanes take part in the wavefront steps only
    const bool active = lane_on && r < r_end && nid >= 0;
    if (!active) {
        inst = 0;
        phi = 0.0;
#pragma unroll
        for (int c = 0; c < NC; ++c) x[c] = 0;
    }
    const int32_t set = uniform_set >= 0 ? uniform_set : inst * R + r;
    const uint32_t node = active ? (uint32_t)nid : 0u;
    // phi_{d+1} = (1 - beta(day0 + d)) phi_d + alpha I/N (eq:siminfpressure, Euler step)
    auto phi_next = [&](const int32_t *y, int32_t dd, double ph, long long *Iout) {
        long long I = 0, N = 0;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            if ((m.imask >> c) & 1u) I += y[c];
            if ((m.nmask >> c) & 1u) N += y[c];
        }
        *Iout = I;
        const int q = season((int64_t)m.day0 + dd);
        const int lane = threadIdx.x & 63;
        const double a = 1.0 - (tp ? tp->beta[q][lane] : s.beta[set * 4 + q]);
        const double b = a * ph;
        const double shed = N > 0 ? (tp ? tp->alpha[lane] : s.alpha[set]) * ((double)I / (double)N) : 0.0;
        return b + shed;
    };
    if (active && prologue) {
        const double phi_in = phi;
        const int32_t dp = d - 1;
        long long I = 0;
        if (m.phi_pre) {
            // phi was already fed by the state before the events of day dp
#pragma unroll
            for (int c = 0; c < NC; ++c)
                if ((m.imask >> c) & 1u) I += x[c];
        } else {
            phi = phi_next(x, dp, phi, &I);
        }
        t.prev += I > 0 ? 1 : 0;
#pragma unroll
        for (int c = 0; c < NC; ++c) t.tot[c] += x[c];
        const int32_t slot = rec;
        if (slot >= 0) {
            const int64_t base = (((int64_t)slot * R + r) * s.n_nodes + s.inst_off[inst] + node);
#pragma unroll
            for (int c = 0; c < NC; ++c)
                if (comp_on<NC>(m, c)) s.snap_u[base * m.nc + c] = x[c];
            s.snap_v[base] = phi;
        }
        if (__double_as_longlong(phi) != __double_as_longlong(phi_in)) s.phi[l] = phi;
    }
    hooks.after_prologue();
    // d, prologue and ssa may differ between the lanes of a slot handle's
    // wavefront: a lane without the SSA today takes part with no live chain
    if (__ballot(ssa) == 0ull) return;
    const bool walks = active && ssa;
    typename Rules::State ch;
    const int lane_t = threadIdx.x & 63;
    const uint32_t key0 = active ? (tp ? tp->key0[lane_t] : s.seed[inst]) : 0u;
    const uint32_t key1 = active ? (tp ? tp->key1[lane_t] : s.repid[set]) : 0u;
#pragma unroll
    for (int k = 0; k < NT; ++k) {
        double c = active && trans_on<NT>(m, k) ? (tp ? tp->coef[k][lane_t] : s.coef[set * m.nt + k]) : 0.0;
        if ((m.uses_phi >> k) & 1u) c = c * phi;
        ch.cphi[k] = c;
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) ch.xd[c] = (double)x[c];
    ch.clock = 0.0;
    ch.fired = 0;
    Rules::rates(m, ch);
    if (group_walk)
        group_chain<Rules>(m, ch, walks, node, (uint32_t)d, key0, key1, status, set, s.few_chains,
                           s.group_min_attempts);
    else
        run_chains<Rules>(m, ch, walks, node, (uint32_t)d, key0, key1, status, set, s.few_chains);
    t.trans += ch.fired;
    t.most = max(t.most, (int32_t)ch.fired);
    if (hooks.after_ssa(ch, walks) && walks && ch.fired) {
#pragma unroll
        for (int c = 0; c < NC; ++c)
            if (comp_on<NC>(m, c)) s.u[(int64_t)c * s.L + l] = (int32_t)ch.xd[c];
    }
    if (walks && m.phi_pre) {
        // eq:numstep5 as written: phi from the state after the SSA, before the events
        int32_t y[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) y[c] = (int32_t)ch.xd[c];
        long long I = 0;
        const double phi2 = phi_next(y, d, phi, &I);
        if (__double_as_longlong(phi2) != __double_as_longlong(phi)) s.phi[l] = phi2;
    }
}

template <int NC>
__device__ __forceinline__ void event_task(const Model &m, const DevState &s, const DevEvents &ev, int64_t t,
                                           int32_t r, int32_t d, unsigned long long *status);

// The private tasks of one unit (a workgroup's positions) on day d, right after
// its SSA: lane_of_pair maps the pairs (task, lane) of the workgroup, nl lanes
// per position starting at r0, lanes r >= r_end idle. The SSA results of the
// unit must be visible to the whole workgroup (a workgroup barrier first).
template <int NC>
__device__ __forceinline__ void private_tasks(const Model &m, const DevState &s, const DevEvents &ev, int32_t d,
                                              int64_t unit, int64_t n_units, int32_t r0, int32_t nl, int32_t r_end,
                                              unsigned long long *status) {
    fresh_l1();
    const int64_t k = (int64_t)d * n_units + unit;
    const int64_t t0 = ev.priv_off[k], t1 = ev.priv_off[k + 1];
    const int64_t count = (t1 - t0) * nl;
    for (int64_t i = threadIdx.x; i < count; i += kBlock) {
        const int64_t t = t0 + (nl == 1 ? i : i / nl);
        const int32_t r = r0 + (nl == 1 ? 0 : (int32_t)(i % nl));
        if (r < r_end) event_task<NC>(m, s, ev, t, r, d, status);
    }
}

// One private event of a workgroup's day, staged in LDS.
struct PrivEv {
    uint32_t meta, smap;
    int32_t n, g, gm, node;
};

// A unit's private events in LDS (one lane per node): the event a thread
// fetched at the start is parked once the prologue is done, and the counts
// each lane holds after the SSA are handed over instead of being stored.
template <int NC>
struct LdsPrivHooks {
    PrivEv *pe;
    int32_t (*x)[kBlock];
    int32_t *touch;
    const PrivEv *mine;
    bool has, lds;
    __device__ void after_prologue() const {
        if (has) pe[threadIdx.x] = *mine;
    }
    template <class St>
    __device__ bool after_ssa(const St &ch, bool active) const {
        if (!lds) return true;
#pragma unroll
        for (int c = 0; c < NC; ++c) x[c][threadIdx.x] = active ? (int32_t)ch.xd[c] : 0;
        touch[threadIdx.x] = active && ch.fired ? 1 : 0;
        return false;
    }
};

// One private task (a run of one node's single-node events, i the first)
// applied to the counts in LDS, with the arithmetic of event_task. A run that
// draws has the node to itself; runs of additions only may share it and add
// atomically.
template <int NC>
__device__ void private_task_lds(const PrivEv *pe, int i, int n_ev, int32_t (*xs)[kBlock], int32_t *touch,
                                 int32_t base, int32_t d, uint32_t key0, uint32_t key1, int32_t set,
                                 unsigned long long *status) {
    const int loc = pe[i].node - base;
    int end = i + 1;
    while (end < n_ev && (pe[end].meta & kMetaCont)) ++end;
    bool draws = false;
    for (int j = i; j < end; ++j) draws = draws || (int)(pe[j].meta & kEvKindMask) != SIM_ENTER;
    touch[loc] = 1;
    if (!draws) {
        for (int j = i; j < end; ++j) {
            const uint32_t mask = (pe[j].meta >> 2) & 0xffu;
#pragma unroll
            for (int c = 0; c < NC; ++c)
                if ((mask >> c) & 1u) atomicAdd(&xs[c][loc], pe[j].n);
        }
        return;
    }
    int32_t x[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) x[c] = xs[c][loc];
    for (int j = i; j < end; ++j) {
        const uint32_t meta = pe[j].meta;
        const int kind = (int)(meta & kEvKindMask);
        const uint32_t mask = (meta >> 2) & 0xffu;
        const int32_t n = pe[j].n;
        if (kind == SIM_ENTER) {
#pragma unroll
            for (int c = 0; c < NC; ++c)
                if ((mask >> c) & 1u) x[c] += n;
            continue;
        }
        long long tot = 0;
#pragma unroll
        for (int c = 0; c < NC; ++c)
            if ((mask >> c) & 1u) tot += x[c];
        if ((long long)n > tot) {
            atomicMin(status, ((unsigned long long)(uint32_t)pe[j].gm << 32) | (unsigned long long)(uint32_t)set);
            break;
        }
        int32_t take[NC];
        draw_individuals<NC>(x, take, mask, n, tot, (uint32_t)pe[j].g, d, key0, key1);
        if (kind == SIM_INTERNAL) {
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                if (take[c]) {
                    const int to = shifted(pe[j].smap, c);
#pragma unroll
                    for (int cc = 0; cc < NC; ++cc)
                        if (cc == to) x[cc] += take[c];
                }
            }
        }
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) xs[c][loc] = x[c];
}

// The LDS of a day whose levels run in LDS: the touched nodes' counts (slots),
// their Philox keys and sets, the day's events, the level bounds and the first
// draws of every event.
template <int NC>
struct EventDayShared {
    int32_t u[kDaySlotCap * NC];
    uint32_t k0[kDaySlotCap], k1[kDaySlotCap];
    int32_t set[kDaySlotCap], pos[kDaySlotCap];
    int32_t n[kDayEventCap], g[kDayEventCap];
    uint32_t meta[kDayEventCap], smap[kDayEventCap];
    int16_t ss[kDayEventCap], sd[kDayEventCap];
    int32_t lv[kDayLevelCap + 1];
    uint64_t pre[kDayEventCap * kPreDraws];
};

template <class Rules>
__global__ __launch_bounds__(kBlock) void k_day(Model m, DevState s, DevEvents ev, int32_t d, int32_t prologue,
                                                int32_t ssa) {
    constexpr int NC = Rules::NC;
    __shared__ PrivEv sh_pe[kBlock];
    __shared__ int32_t sh_x[NC][kBlock];
    __shared__ int32_t sh_touch[kBlock];
    const int64_t l = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    // The unit's private events of the day. With at most one per thread they
    // are fetched now, alongside the state, and applied to the counts in LDS
    // right after the SSA; each node is then stored once. Otherwise the SSA
    // stores its counts and the tasks run on global memory. Their bounds and
    // the workgroup's set (one lane per node; instances are padded to whole
    // workgroups) are read before the status check, which waits for them.
    const int64_t k = (int64_t)d * (s.Np / kLaneUnit) + blockIdx.x;
    const int32_t pe0 = ssa ? ev.priv_ev_off[k] : 0;
    const int32_t npe = ssa ? ev.priv_ev_off[k + 1] - pe0 : 0;
    const int32_t set = s.inst[(int64_t)blockIdx.x * kBlock];
    const bool group = s.unit_group[blockIdx.x] != 0;
    // the unit's nodes among the slots of a day whose remaining events run in
    // LDS: their final counts go to the day's staging buffer (one per thread)
    const bool staged = ssa && ev.unit_stage_off;
    const int32_t st0 = staged ? ev.unit_stage_off[k] : 0;
    const int32_t nst = staged ? ev.unit_stage_off[k + 1] - st0 : 0;
    if (!block_ok_once(s.status)) return;
    const uint32_t key0 = s.seed[set], key1 = s.repid[set];
    const bool lds = npe <= kBlock;
    const bool has = lds && (int)threadIdx.x < npe;
    const int32_t stage_entry = (int)threadIdx.x < nst ? ev.unit_stage[st0 + threadIdx.x] : -1;
    PrivEv mine{0u, 0u, 0, 0, 0, 0};
    if (has) {
        const int64_t e = pe0 + threadIdx.x;
        mine = PrivEv{ev.meta[e], ev.smap[e], ev.n[e], ev.g[e], ev.gm[e], ev.node[e]};
    }
    const LdsPrivHooks<NC> hooks{sh_pe, sh_x, sh_touch, &mine, has, lds && ssa};
    Tally<NC> t{};
    day_wave<Rules>(m, s, l, d, prologue != 0, ssa != 0, t, s.R, s.status, nullptr, hooks, set, group);
    const int32_t d_rec = prologue ? d - 1 : -1;
    const int32_t d_ssa = ssa ? d : -1;
    flush_block<NC>(m, s, t, set, d_rec, d_ssa, s.n_regions ? s.pos_region[(int64_t)blockIdx.x * kBlock] : -1);
    if (!ssa) return;
    if (!lds) {
        private_tasks<NC>(m, s, ev, d, blockIdx.x, s.Np / kLaneUnit, 0, 1, 1, s.status);
        if (nst > 0) {
            __syncthreads();
            fresh_l1();
            if (stage_entry >= 0) {
                const int64_t ls = (int64_t)blockIdx.x * kBlock + (stage_entry & 0xff);
#pragma unroll
                for (int c = 0; c < NC; ++c)
                    ev.stage[(stage_entry >> 8) * NC + c] = comp_on<NC>(m, c) ? load_state(&s.u[(int64_t)c * s.L + ls]) : 0;
            }
        }
    } else {
        // flush_block's barriers make the parked events and counts visible
        if (has && !(sh_pe[threadIdx.x].meta & kMetaCont))
            private_task_lds<NC>(sh_pe, threadIdx.x, npe, sh_x, sh_touch, (int32_t)(blockIdx.x * kBlock), d, key0,
                                 key1, set, s.status);
        __syncthreads();
        if (sh_touch[threadIdx.x]) {
#pragma unroll
            for (int c = 0; c < NC; ++c)
                if (comp_on<NC>(m, c)) s.u[(int64_t)c * s.L + l] = sh_x[c][threadIdx.x];
        }
        if (stage_entry >= 0) {
#pragma unroll
            for (int c = 0; c < NC; ++c)
                ev.stage[(stage_entry >> 8) * NC + c] = comp_on<NC>(m, c) ? sh_x[c][stage_entry & 0xff] : 0;
        }
    }
}

// Replicate tiles (replicate lanes in columns of 64): a tile workgroup takes
// positions [x * tile_nodes, (x + 1) * tile_nodes) and the replicate lanes
// [64 y, 64 y + 64) of column y; its wavefronts take the positions one at a
// time, and a lane always holds the same replicate, so its counts add up in
// registers. In a slot handle the columns are those of the step's run list,
// each holding 64 / slot_lanes slots: d is the handle's step, a slot's own
// day is d - t0, and its lanes past its replicate count are idle.
//
// Past the regular tiles, workgroups of four wavefronts take the heavy herds:
// each wavefront one (herd, replicate) chain, walked with the whole wavefront
// (kHeavyBlocks workgroups cover the 64 replicate lanes of a column), then the
// herd's private task for that replicate; the units holding heavy herds are
// skipped by the regular tiles.
constexpr int kHeavyBlocks = 64 / kWaves;

template <class Rules>
__device__ __forceinline__ void heavy_chain(const Model &m, const DevState &s, const DevEvents &ev, int64_t hb,
                                            int32_t r, int32_t d, bool prologue, bool ssa, bool on,
                                            unsigned long long *status) {
    constexpr int NC = Rules::NC;
    const int lane = threadIdx.x & 63;
    const int32_t pos = s.heavy_pos[hb / kHeavyBlocks];
    if (!on) return;  // the same in every lane of the wavefront
    Tally<NC> t{};
    day_wave<Rules>(m, s, lane == 0 ? (int64_t)pos * s.RL + r : s.L, d, prologue, ssa, t, s.RL, status);
    const int32_t inst = s.inst[pos];
    const int64_t S = (int64_t)s.n_inst * s.R;
    const int64_t set = (int64_t)inst * s.R + r;
    if (lane == 0) {
        if (prologue) {
            if (t.prev) atomicAdd(&s.prevalence[(d - 1) * S + set], (int32_t)t.prev);
            const int32_t region = s.n_regions ? s.pos_region[pos] : -1;
#pragma unroll
            for (int c = 0; c < NC; ++c)
                if (comp_on<NC>(m, c) && t.tot[c]) {
                    atomicAdd((unsigned long long *)&s.totals[((d - 1) * S + set) * m.nc + c], (unsigned long long)t.tot[c]);
                    if (region >= 0)
                        atomicAdd((unsigned long long *)&s.regional[(((d - 1) * S + set) * s.n_regions + region) * m.nc + c],
                                  (unsigned long long)t.tot[c]);
                }
        }
        if (ssa && t.trans) {
            atomicAdd((unsigned long long *)&s.transitions[d * S + set], (unsigned long long)t.trans);
            atomicMax(&s.max_fired[d * S + set], t.most);
        }
    }
    if (!ssa) return;
    // the herd's private task of the day (at most one per node and day), run
    // by another lane of this wavefront: lane 0's stores first, then fresh lines
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    fresh_l1();
    const int64_t k = (int64_t)d * (s.Np / s.tile_nodes) + pos / s.tile_nodes;
    const int64_t t0 = ev.priv_off[k], t1 = ev.priv_off[k + 1];
    for (int64_t tk = t0 + lane; tk < t1; tk += 64)
        if (ev.node[ev.task_off[tk]] == pos) event_task<NC>(m, s, ev, tk, r, d, status);
}

// A lane r of a slot handle: its slot (slot_lanes lanes each), whether the
// slot runs at handle step d, the slot's own day and its error word. A slot
// whose request failed stops.
struct SlotLane {
    int32_t day, n_live;
    bool on, prologue, ssa;
    unsigned long long *status;
};

__device__ __forceinline__ SlotLane slot_lane(const DevState &s, int32_t d, int32_t r) {
    const int32_t slot = r / s.slot_lanes;
    const SlotInfo si = s.slots[slot];
    SlotLane q;
    q.day = d - si.t0;
    q.n_live = si.n_rep;
    q.status = s.status + slot;
    q.on = si.t0 >= 0 && q.day >= 0 && q.day <= si.horizon && r - slot * s.slot_lanes < si.n_rep &&
           *q.status == STATUS_OK;
    q.prologue = q.on && q.day > 0;
    q.ssa = q.on && q.day < si.horizon;
    return q;
}

// With SLOTS (a slot handle), grid row y runs the column s.run_cols[y] and
// lane r belongs to slot r / slot_lanes, which runs its own request from its
// own day 0: every lane takes its day, its phases
// and its error word from its slot, and a failed slot stops without stopping
// the others.
template <class Rules, bool SLOTS>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(Rules::kTileWaves, 8))) void k_day_tile(
    Model m, DevState s, DevEvents ev, int32_t d, int32_t prologue, int32_t ssa) {
    constexpr int NC = Rules::NC;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t nx = s.Np / s.tile_nodes;
    // Dispatch order (workgroups start in linear order): the tiles of every
    // column first, then the heavy-herd chains, largest herd first with all
    // its columns, so that the short chains of the smaller heavy herds fill
    // the compute units that the last tiles leave free. bx is the tile (or
    // nx + heavy block) and by the grid row of the workgroup.
    const int64_t lin = (int64_t)blockIdx.x + (int64_t)gridDim.x * blockIdx.y;
    const int64_t n_tiles = nx * gridDim.y;
    const bool heavy = lin >= n_tiles;
    const int64_t bx = heavy ? nx + (lin - n_tiles) / gridDim.y : lin % nx;
    const int64_t by = heavy ? (lin - n_tiles) % gridDim.y : lin / nx;
    if (s.n_heavy && bx < nx && s.unit_heavy[bx]) return;  // uniform over the workgroup
    if constexpr (!SLOTS) {
        if (!block_ok_once(s.status)) return;
    }
    // the column of 64 replicate lanes (a slot handle launches only the
    // columns that run this step)
    const int32_t col = SLOTS ? s.run_cols[by] : (int32_t)by;
    if (heavy) {
        const int64_t hb = bx - nx;
        const int32_t rh = col * 64 + (int32_t)(hb % kHeavyBlocks) * kWaves + wave;
        if constexpr (SLOTS) {
            const SlotLane q = slot_lane(s, d, rh);
            heavy_chain<Rules>(m, s, ev, hb, rh, q.day, q.prologue, q.ssa, q.on, q.status);
        } else {
            heavy_chain<Rules>(m, s, ev, hb, rh, d, prologue != 0, ssa != 0, rh < s.R, s.status);
        }
        return;
    }
    const int64_t pos0 = bx * s.tile_nodes;
    const int32_t r = col * 64 + lane;
    bool on = r < s.R, pro = prologue != 0, walk = ssa != 0;
    int32_t day = d;
    unsigned long long *status = s.status;
    if constexpr (SLOTS) {
        const SlotLane q = slot_lane(s, d, r);
        on = q.on;
        pro = q.prologue;
        walk = q.ssa;
        day = q.day;
        status = q.status;
        if (!__syncthreads_or(on ? 1 : 0)) return;  // no lane of the column runs
    }
    __shared__ double sh_coef[Rules::NT][64], sh_alpha[64], sh_beta[4][64];
    __shared__ uint32_t sh_k0[64], sh_k1[64];
    __shared__ int32_t sh_next;  // the next position of the tile that no wavefront has taken
    if (threadIdx.x == 0) sh_next = kWaves;
    if (wave == 0 && on) {
        const int32_t inst = s.inst[pos0];  // every position of a tile belongs to one instance
        const int64_t set = (int64_t)inst * s.R + r;
#pragma unroll
        for (int k = 0; k < Rules::NT; ++k) sh_coef[k][lane] = trans_on<Rules::NT>(m, k) ? s.coef[set * m.nt + k] : 0.0;
        sh_alpha[lane] = s.alpha[set];
#pragma unroll
        for (int q = 0; q < 4; ++q) sh_beta[q][lane] = s.beta[set * 4 + q];
        sh_k0[lane] = s.seed[inst];
        sh_k1[lane] = s.repid[set];
    }
    __syncthreads();
    const TileParams tp{sh_coef, sh_alpha, sh_beta, sh_k0, sh_k1};
    Tally<NC> t{};
    // positions are taken one at a time as wavefronts come free: a herd with
    // a long chain holds up only its own wavefront, the others take the
    // remaining positions (nodes are independent within the day, and the
    // tallies are integer sums and maxima, so the order changes no result)
    for (int j = wave; j < s.tile_nodes;) {
        const int64_t pos = pos0 + j;
        if (pos >= s.Np) break;
        day_wave<Rules>(m, s, pos * s.RL + r, day, pro, walk, t, s.RL, status, &tp, NoHooks{}, -1, false, on);
        int32_t next = 0;
        if (lane == 0) next = atomicAdd(&sh_next, 1);
        j = __shfl(next, 0);
    }
    // instances are padded to whole tiles: one instance per workgroup
    flush_tile<NC>(m, s, t, on ? s.inst[pos0] * s.R + r : -1, pro ? day - 1 : -1, walk ? day : -1,
                   s.n_regions ? s.pos_region[pos0] : -1);
    if constexpr (SLOTS) {
        // each slot of the column at its own day (flush_tile's barriers publish the SSA results)
        for (int32_t g = 0; g < 64 / s.slot_lanes; ++g) {
            const int32_t r0 = col * 64 + g * s.slot_lanes;
            const SlotLane q = slot_lane(s, d, r0);  // the same in every thread
            if (q.ssa)
                private_tasks<NC>(m, s, ev, q.day, bx, nx, r0, s.slot_lanes, r0 + q.n_live, q.status);
        }
    } else {
        if (ssa) private_tasks<NC>(m, s, ev, d, bx, nx, col * 64, 64, s.R, s.status);
    }
}

// ---------------------------------------------------------------------------
// Events (Sec. 3.2): one thread per (event, replicate) of a conflict-free
// level. Within a level a node is either drawn from by exactly one event or
// only added to, so draws use plain loads/stores and additions commute
// (integer atomics).
// ---------------------------------------------------------------------------


// What one event needs besides the state: its packed kind / mask / shift,
// node, destination, count, Philox counter word g, merged index gm (error
// report) and the instance of its node.
struct EvDesc {
    uint32_t meta, smap;
    int32_t node, dest, n, g, gm, inst;
};

__device__ __forceinline__ EvDesc load_desc(const DevState &s, const DevEvents &ev, int64_t e) {
    EvDesc q;
    q.meta = ev.meta[e];
    q.smap = ev.smap[e];
    q.node = ev.node[e];
    q.dest = ev.dest[e];
    q.n = ev.n[e];
    q.g = ev.g[e];
    q.gm = ev.gm[e];
    q.inst = s.inst[q.node];
    return q;
}

template <int NC>
__device__ __forceinline__ void event_apply(const Model &m, const DevState &s, const EvDesc &q, int32_t r, int32_t d,
                                            unsigned long long *status) {
    const uint32_t meta = q.meta;
    const int kind = (int)(meta & kEvKindMask);
    const uint32_t mask = (meta >> 2) & 0xffu;
    const int32_t node = q.node;
    const int32_t n = q.n;
    const int64_t ls = (int64_t)node * s.RL + r;
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
            x[c] = load_state(&s.u[(int64_t)c * s.L + ls]);
            tot += x[c];
        }
    }
    const uint32_t g = (uint32_t)q.g;
    const int32_t inst = q.inst;
    const int32_t set = inst * s.R + r;
    if ((long long)n > tot) {
        atomicMin(status, ((unsigned long long)(uint32_t)q.gm << 32) | (unsigned long long)(uint32_t)set);
        return;
    }
    int32_t take[NC];
    draw_individuals<NC>(x, take, mask, n, tot, g, d, s.seed[inst], s.repid[set]);
    if (kind == SIM_INTERNAL) {
        int32_t y[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) y[c] = ((mask >> c) & 1u) ? x[c] : 0;
        uint32_t touched = mask;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            if (take[c]) {
                const int to = shifted(q.smap, c);
#pragma unroll
                for (int cc = 0; cc < NC; ++cc) {
                    if (cc == to) {
                        if (!((touched >> cc) & 1u)) {
                            y[cc] = load_state(&s.u[(int64_t)cc * s.L + ls]);
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
        const int64_t ld = (int64_t)q.dest * s.RL + r;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            if (take[c]) {
                const int to = shifted(q.smap, c);
                atomicAdd(&s.u[(int64_t)to * s.L + ld], take[c]);
            }
        }
    }
}

template <int NC>
__device__ __forceinline__ void event_one(const Model &m, const DevState &s, const DevEvents &ev,
                                          int64_t e, int32_t r, int32_t d, unsigned long long *status) {
    event_apply<NC>(m, s, load_desc(s, ev, e), r, d, status);
}

// One task (replicate lane r): a single event, or a run of one node's enter /
// exit / internal events in list order. A run that draws has its node to
// itself within its level (every other event touching the node is in another
// level), so its counts stay in registers from the first event to the last;
// a run of additions only may share the node with other additions and adds
// atomically, event by event.
template <int NC>
__device__ __forceinline__ void event_task(const Model &m, const DevState &s, const DevEvents &ev, int64_t t,
                                           int32_t r, int32_t d, unsigned long long *status) {
    const int64_t e0 = ev.task_off[t], e1 = ev.task_off[t + 1];
    bool draws = false;
    if (e1 - e0 > 1)
        for (int64_t e = e0; e < e1; ++e) draws = draws || (int)(ev.meta[e] & kEvKindMask) != SIM_ENTER;
    if (!draws) {
        for (int64_t e = e0; e < e1; ++e) event_one<NC>(m, s, ev, e, r, d, status);
        return;
    }
    const int32_t node = ev.node[e0];
    const int64_t ls = (int64_t)node * s.RL + r;
    int32_t x[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) x[c] = comp_on<NC>(m, c) ? load_state(&s.u[(int64_t)c * s.L + ls]) : 0;
    const int32_t inst = s.inst[node];
    const int32_t set = inst * s.R + r;
    const uint32_t key0 = s.seed[inst], key1 = s.repid[set];
    uint32_t touched = 0;
    for (int64_t e = e0; e < e1; ++e) {
        const uint32_t meta = ev.meta[e];
        const int kind = (int)(meta & kEvKindMask);
        const uint32_t mask = (meta >> 2) & 0xffu;
        const int32_t n = ev.n[e];
        touched |= mask;
        if (kind == SIM_ENTER) {
#pragma unroll
            for (int c = 0; c < NC; ++c)
                if ((mask >> c) & 1u) x[c] += n;
            continue;
        }
        long long tot = 0;
#pragma unroll
        for (int c = 0; c < NC; ++c)
            if ((mask >> c) & 1u) tot += x[c];
        if ((long long)n > tot) {
            atomicMin(status, ((unsigned long long)(uint32_t)ev.gm[e] << 32) | (unsigned long long)(uint32_t)set);
            break;
        }
        int32_t take[NC];
        draw_individuals<NC>(x, take, mask, n, tot, (uint32_t)ev.g[e], d, key0, key1);
        if (kind == SIM_INTERNAL) {
            const uint32_t smap = ev.smap[e];
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                if (take[c]) {
                    const int to = shifted(smap, c);
#pragma unroll
                    for (int cc = 0; cc < NC; ++cc)
                        if (cc == to) x[cc] += take[c];
                    touched |= 1u << to;
                }
            }
        }
    }
#pragma unroll
    for (int c = 0; c < NC; ++c)
        if ((touched >> c) & 1u) s.u[(int64_t)c * s.L + ls] = x[c];
}

template <int NC>
__global__ __launch_bounds__(kBlock) void k_events(Model m, DevState s, DevEvents ev, int32_t d,
                                                   int64_t begin, int64_t end) {
    if (*(volatile unsigned long long *)s.status != STATUS_OK) return;
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t count = (end - begin) * s.RL;
    if (t >= count) return;
    const int64_t e = begin + (s.RL == 1 ? t : t / s.RL);
    const int32_t r = s.RL == 1 ? 0 : (int32_t)(t % s.RL);
    if (r < s.R) event_task<NC>(m, s, ev, e, r, d, s.status);
}

// A run of small levels [lv_begin, lv_end) of day d in one workgroup, with a
// workgroup barrier between levels (the levels' order is all that links them).
// The descriptors of all its tasks (contiguous in execution order) are staged
// in LDS first, so each level then waits on one round trip for the state
// only; a task of several events keeps to its own loads.
constexpr int kGroupCap = 1024;

template <int NC>
__global__ __launch_bounds__(kEvBlock) void k_event_levels(Model m, DevState s, DevEvents ev, int32_t d,
                                                           int32_t lv_begin, int32_t lv_end) {
    if (!block_ok_once(s.status)) return;
    __shared__ EvDesc sh_desc[kGroupCap];
    __shared__ int32_t sh_multi[kGroupCap];
    const int64_t tb = ev.lvl_off[lv_begin], te = ev.lvl_off[lv_end];
    const bool staged = te - tb <= kGroupCap;
    if (staged) {
        for (int64_t i = threadIdx.x; i < te - tb; i += kEvBlock) {
            const int64_t e0 = ev.task_off[tb + i], e1 = ev.task_off[tb + i + 1];
            sh_multi[i] = e1 - e0 > 1;
            if (e1 - e0 == 1) sh_desc[i] = load_desc(s, ev, e0);
        }
        __syncthreads();
    }
    for (int32_t lv = lv_begin; lv < lv_end; ++lv) {
        const int64_t begin = ev.lvl_off[lv], end = ev.lvl_off[lv + 1];
        const int64_t count = (end - begin) * s.RL;
        for (int64_t t = threadIdx.x; t < count; t += kEvBlock) {
            const int64_t k = begin + (s.RL == 1 ? t : t / s.RL);
            const int32_t r = s.RL == 1 ? 0 : (int32_t)(t % s.RL);
            if (r >= s.R) continue;
            if (staged && !sh_multi[k - tb])
                event_apply<NC>(m, s, sh_desc[k - tb], r, d, s.status);
            else
                event_task<NC>(m, s, ev, k, r, d, s.status);
        }
        __syncthreads();
        fresh_l1();
    }
}

// A day's levels in LDS (one lane per node): the nodes its level tasks touch
// are loaded into slots once, every level updates the slots (draws with plain
// LDS loads and stores, since a node drawn from is alone in its level;
// additions with LDS atomics, which commute), and the slots are written back
// once. Same draws and order as the global-memory path.
template <int NC>
__device__ __forceinline__ void slot_event(const Model &m, const DevState &s, const DevEvents &ev, uint32_t meta,
                                           uint32_t smap, int32_t n, uint32_t g, int32_t e, int32_t *xs, int32_t *xd,
                                           uint32_t key0, uint32_t key1, int32_t set, int32_t d,
                                           unsigned long long *status, const uint64_t *pre) {
    const int kind = (int)(meta & kEvKindMask);
    const uint32_t mask = (meta >> 2) & 0xffu;
    // A selection of one or two compartments c0 < c1 with its draws computed
    // ahead (every column of the farm model, every movement of up to six
    // animals): the running sums of the walk below are 0 before c0, x[c0]
    // from c0 to c1 and the total from c1 on, so a pick below the count left
    // in c0 takes from c0 and any other from c1 (the same picks, counts and
    // write order as the walk over all compartments).
    const uint32_t rest = mask & (mask - 1u);
    if (mask != 0u && (rest & (rest - 1u)) == 0u && n <= kPreDraws && (kind != SIM_ENTER || rest == 0u)) {
        const int c0 = __builtin_ctz(mask);
        const int c1 = rest ? __builtin_ctz(rest) : c0;
        if (kind == SIM_ENTER) {
            __hip_atomic_fetch_add(&xs[c0], n, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            return;
        }
        const int32_t x0 = xs[c0], x1 = rest ? xs[c1] : 0;
        const long long tot = (long long)x0 + (long long)x1;
        if ((long long)n > tot) {
            atomicMin(status, ((unsigned long long)(uint32_t)ev.gm[e] << 32) | (unsigned long long)(uint32_t)set);
            return;
        }
        if (tot <= 0x7fffffffLL) {
            int32_t t0 = 0, t1 = 0;
            uint32_t left0 = (uint32_t)x0;
#pragma unroll
            for (int q = 0; q < kPreDraws; ++q) {
                if (q >= n) break;
                const uint32_t pick = (uint32_t)__umul64hi(pre[q], (uint64_t)(tot - q));
                const int in0 = pick < left0 ? 1 : 0;
                left0 -= (uint32_t)in0;
                t0 += in0;
                t1 += 1 - in0;
            }
            xs[c0] = x0 - t0;
            if (rest) xs[c1] = x1 - t1;
            if (kind == SIM_INTERNAL) {
                if (t0) xs[shifted(smap, c0)] += t0;
                if (t1) xs[shifted(smap, c1)] += t1;
            } else if (kind == SIM_EXTERNAL) {
                if (t0) __hip_atomic_fetch_add(&xd[shifted(smap, c0)], t0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                if (t1) __hip_atomic_fetch_add(&xd[shifted(smap, c1)], t1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
            return;
        }
    }
    if (kind == SIM_ENTER) {
#pragma unroll
        for (int c = 0; c < NC; ++c)
            if ((mask >> c) & 1u) __hip_atomic_fetch_add(&xs[c], n, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        return;
    }
    int32_t x[NC];
    long long tot = 0;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        x[c] = ((mask >> c) & 1u) ? xs[c] : 0;
        tot += x[c];
    }
    if ((long long)n > tot) {
        atomicMin(status, ((unsigned long long)(uint32_t)ev.gm[e] << 32) | (unsigned long long)(uint32_t)set);
        return;
    }
    int32_t take[NC];
    draw_individuals<NC>(x, take, mask, n, tot, g, d, key0, key1, pre);
    if (kind == SIM_INTERNAL) {
#pragma unroll
        for (int c = 0; c < NC; ++c)
            if ((mask >> c) & 1u) xs[c] = x[c];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            if (take[c]) {
                const int to = shifted(smap, c);
                xs[to] += take[c];
            }
        }
        return;
    }
#pragma unroll
    for (int c = 0; c < NC; ++c)
        if ((mask >> c) & 1u) xs[c] = x[c];
    if (kind == SIM_EXTERNAL) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            if (take[c]) {
                const int to = shifted(smap, c);
                __hip_atomic_fetch_add(&xd[to], take[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        }
    }
}

// The day's level events are contiguous (e0 .. e0 + ne - 1, by level, then
// task); the launch carries the day's offsets, and the day kernel has staged
// the slots' counts in slot order, so that staging is one round trip for the
// event fields, slot keys, level bounds and counts. Every thread of the
// workgroup calls it (any workgroup size).
template <int NC>
__device__ void event_day_levels(const Model &m, const DevState &s, const DevEvents &ev, const EventDayArgs &a,
                                 int32_t d, EventDayShared<NC> &sh) {
    const int nth = (int)blockDim.x;
    const int32_t nl = a.nl, ns = a.ns, ne = (int32_t)a.ne, s0 = a.s0;
    const int64_t e0 = a.e0;
    for (int i = threadIdx.x; i <= nl; i += nth) sh.lv[i] = (int32_t)(ev.lvl_ev_off[a.lv0 + i] - e0);
    for (int i = threadIdx.x; i < ne; i += nth) {
        sh.meta[i] = ev.meta[e0 + i];
        sh.smap[i] = ev.smap[e0 + i];
        sh.n[i] = ev.n[e0 + i];
        sh.g[i] = ev.g[e0 + i];
        sh.ss[i] = (int16_t)ev.slot_src[e0 + i];
        sh.sd[i] = (int16_t)ev.slot_dst[e0 + i];
    }
    // the slots' counts, staged by the day kernel (no wait for slot_pos)
    for (int i = threadIdx.x; i < ns; i += nth) {
        sh.k0[i] = ev.slot_key[3 * (s0 + i)];
        sh.k1[i] = ev.slot_key[3 * (s0 + i) + 1];
        sh.set[i] = (int32_t)ev.slot_key[3 * (s0 + i) + 2];
        sh.pos[i] = ev.slot_pos[s0 + i];
#pragma unroll
        for (int c = 0; c < NC; ++c) sh.u[i * NC + c] = ev.stage[i * NC + c];
    }
    if (!block_ok_once(s.status)) return;  // its barrier also publishes the staged fields
    // the first draws of every event do not depend on the state: all at once
    for (int i = threadIdx.x; i < ne * (kPreDraws / 2); i += nth) {
        const int j = i / (kPreDraws / 2), b = i % (kPreDraws / 2);
        if ((int)(sh.meta[j] & kEvKindMask) == SIM_ENTER || 2 * b >= sh.n[j]) continue;
        const int32_t ss = sh.ss[j];
        const Word4 o = philox4x32_10(Word4{(uint32_t)b, (uint32_t)sh.g[j], (uint32_t)d, 1u}, sh.k0[ss], sh.k1[ss]);
        sh.pre[j * kPreDraws + 2 * b] = ((uint64_t)o.b << 32) | o.a;
        sh.pre[j * kPreDraws + 2 * b + 1] = ((uint64_t)o.d << 32) | o.c;
    }
    __syncthreads();
    for (int32_t k = 0; k < nl; ++k) {
        for (int32_t i = sh.lv[k] + threadIdx.x; i < sh.lv[k + 1]; i += nth) {
            if (sh.meta[i] & kMetaCont) continue;  // applied with its task's first event
            const int32_t ss = sh.ss[i];
            int32_t *xs = &sh.u[ss * NC];
            int32_t *xd = sh.sd[i] >= 0 ? &sh.u[sh.sd[i] * NC] : xs;
            // one event, or a run of one node's events in list order
            int32_t j = i;
            do {
                slot_event<NC>(m, s, ev, sh.meta[j], sh.smap[j], sh.n[j], (uint32_t)sh.g[j], (int32_t)(e0 + j), xs, xd,
                               sh.k0[ss], sh.k1[ss], sh.set[ss], d, s.status, &sh.pre[j * kPreDraws]);
                ++j;
            } while (j < sh.lv[k + 1] && (sh.meta[j] & kMetaCont));
        }
        __syncthreads();
    }
    for (int i = threadIdx.x; i < ns; i += nth) {
        const int32_t pos = sh.pos[i];
#pragma unroll
        for (int c = 0; c < NC; ++c)
            if (comp_on<NC>(m, c)) s.u[(int64_t)c * s.L + pos] = sh.u[i * NC + c];
    }
}

// A day's levels in LDS, launched on its own after the day kernel.
template <int NC>
__global__ __launch_bounds__(kEvBlock) void k_event_day(Model m, DevState s, DevEvents ev, int32_t d,
                                                        EventDayArgs a) {
    __shared__ EventDayShared<NC> sh;
    event_day_levels<NC>(m, s, ev, a, d, sh);
}

// Slot handles: level k of each slot's own day, one grid row per slot of
// s.run_slots (the slots with a day of events this step). With
// k_end > k + 1 the grid is one workgroup per slot and runs the levels
// k .. k_end-1 with a workgroup barrier between them.
template <int NC>
__global__ __launch_bounds__(kEvBlock) void k_slot_events(Model m, DevState s, DevEvents ev, int32_t step,
                                                          int32_t k, int32_t k_end) {
    const int32_t slot = s.run_slots[blockIdx.y];
    const SlotInfo si = s.slots[slot];
    const int32_t d = step - si.t0;
    if (si.t0 < 0 || d < 0 || d >= si.horizon) return;  // uniform over the workgroup
    unsigned long long *status = s.status + slot;
    if (!block_ok_once(status)) return;
    const int32_t W = s.slot_lanes;
    const int32_t lv0 = ev.lvl_ptr[d], lv_day_end = ev.lvl_ptr[d + 1];
    const int64_t stride = (int64_t)gridDim.x * kEvBlock;
    for (int32_t kk = k; kk < k_end && lv0 + kk < lv_day_end; ++kk) {
        const int64_t begin = ev.lvl_off[lv0 + kk], end = ev.lvl_off[lv0 + kk + 1];
        const int64_t count = (end - begin) * W;
        for (int64_t t = (int64_t)blockIdx.x * kEvBlock + threadIdx.x; t < count; t += stride) {
            const int32_t rr = (int32_t)(t % W);
            if (rr < si.n_rep) event_task<NC>(m, s, ev, begin + t / W, slot * W + rr, d, status);
        }
        if (k_end > k + 1) {
            __syncthreads();
            fresh_l1();
        }
    }
}

// Goal function of the fitting study (Sec. 4.3, eq:goal, eq:goalvariance): for
// day d = d_begin + blockIdx.x, with the N = R trajectories of one instance
// (sets s0 .. s0 + N - 1) and the reference's regional sums of that day
// ref[blockIdx.x][j][c], part[blockIdx.x] gets
// sum_j ||mean_i x_ij - ref_j||^2 and part[gridDim.x + blockIdx.x] gets
// sum_j sum_i ||x_ij - mean_j||^2 / (N - 1). One workgroup per day; the
// (region, compartment) terms are summed in a fixed order.
__global__ __launch_bounds__(kBlock) void k_goal(DevState s, int32_t nc, int64_t s0, int32_t N, const int64_t *ref,
                                                 int32_t d_begin, double *part) {
    __shared__ double sh_g[kBlock], sh_v[kBlock];
    const int32_t d = d_begin + (int32_t)blockIdx.x;
    const int64_t S = (int64_t)s.n_inst * s.R;
    const int32_t J = s.n_regions;
    double g = 0.0, v = 0.0;
    for (int32_t q = threadIdx.x; q < J * nc; q += kBlock) {
        const int32_t j = q / nc, c = q % nc;
        long long sum = 0;
        for (int32_t i = 0; i < N; ++i) sum += s.regional[(((int64_t)d * S + s0 + i) * J + j) * nc + c];
        const double mean = (double)sum / (double)N;
        const double diff = mean - (double)ref[((int64_t)blockIdx.x * J + j) * nc + c];
        g += diff * diff;
        double ss = 0.0;
        for (int32_t i = 0; i < N; ++i) {
            const double e = (double)s.regional[(((int64_t)d * S + s0 + i) * J + j) * nc + c] - mean;
            ss += e * e;
        }
        v += N > 1 ? ss / (double)(N - 1) : 0.0;
    }
    sh_g[threadIdx.x] = g;
    sh_v[threadIdx.x] = v;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sh_g[threadIdx.x] += sh_g[threadIdx.x + w];
            sh_v[threadIdx.x] += sh_v[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[blockIdx.x] = sh_g[0];
        part[gridDim.x + blockIdx.x] = sh_v[0];
    }
}

// The per-day terms of k_goal added in day order, as sim_goal adds them on the
// host: out[0] = (((0 + part[0]) + part[1]) + ...), out[1] likewise over
// part[n .. 2n). One thread.
__global__ __launch_bounds__(64) void k_goal_sum(const double *part, int32_t n, double *out) {
    if (threadIdx.x != 0) return;
    double g = 0.0, v = 0.0;
    for (int32_t k = 0; k < n; ++k) {
        g = g + part[k];
        v = v + part[n + k];
    }
    out[0] = g;
    out[1] = v;
}

// Start a slot: write its table entry, clear its error word and its records,
// and load every replicate lane of it with the network's initial state.
__global__ __launch_bounds__(kBlock) void k_slot_init(DevState s, int32_t nc, const int32_t *u0, const double *v0,
                                                      int32_t slot, SlotInfo info) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    if (t == 0) {
        s.slots[slot] = info;
        s.status[slot] = STATUS_OK;
    }
    const int64_t S = s.RL, W = s.slot_lanes;
    for (int64_t i = t; i < s.Np * W; i += stride) {
        const int64_t pos = i / W;
        const int32_t rr = (int32_t)(i % W);
        const int64_t l = pos * s.RL + (int64_t)slot * W + rr;
        const bool live = rr < info.n_rep;
        for (int c = 0; c < nc; ++c) s.u[(int64_t)c * s.L + l] = live ? u0[(int64_t)c * s.Np + pos] : 0;
        s.phi[l] = live ? v0[pos] : 0.0;
    }
    for (int64_t i = t; i < (int64_t)s.n_days * W; i += stride) {
        const int64_t row = (i / W) * S + (int64_t)slot * W + (i % W);
        s.prevalence[row] = 0;
        s.transitions[row] = 0;
        s.max_fired[row] = 0;
        for (int c = 0; c < nc; ++c) s.totals[row * nc + c] = 0;
    }
}

// ---------------------------------------------------------------------------
// A run of days in one cooperative launch: phases separated by grid barriers.
// ---------------------------------------------------------------------------
template <class Rules>
__global__ __launch_bounds__(kBlock) void k_persist(Model m, DevState s, DevEvents ev, int32_t d_begin,
                                                    int32_t d_end, int32_t layout) {
    constexpr int NC = Rules::NC;
    namespace cg = cooperative_groups;
    cg::grid_group grid = cg::this_grid();
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    const int64_t first = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    for (int32_t d = d_begin; d <= d_end; ++d) {
        const bool prologue = d > d_begin;
        const bool ssa = d < d_end;
        const int32_t d_rec = prologue ? d - 1 : -1, d_ssa = ssa ? d : -1;
        if (block_ok(s.status)) {
            if (layout == LAYOUT_TILE) {
                const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
                const int64_t nx = (s.Np + s.tile_nodes - 1) / s.tile_nodes;
                const int64_t n_tiles = nx * (s.RL / 64);
                for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
                    const int64_t pos0 = (tile % nx) * s.tile_nodes;
                    const int32_t r = (int32_t)(tile / nx) * 64 + lane;
                    Tally<NC> t{};
                    for (int j = wave; j < s.tile_nodes; j += kWaves) {
                        const int64_t pos = pos0 + j;
                        if (pos >= s.Np) break;
                        day_wave<Rules>(m, s, pos * s.RL + r, d, prologue, ssa, t, s.R, s.status);
                    }
                    flush_tile<NC>(m, s, t, r < s.R ? s.inst[pos0] * s.R + r : -1, d_rec, d_ssa,
                                   s.n_regions ? s.pos_region[pos0] : -1);
                    if (ssa)
                        private_tasks<NC>(m, s, ev, d, tile % nx, nx, (int32_t)(tile / nx) * 64, 64, s.R, s.status);
                }
            } else {
                const int64_t chunks = (s.L + kBlock - 1) / kBlock;
                for (int64_t chunk = blockIdx.x; chunk < chunks; chunk += gridDim.x) {
                    const int64_t l = chunk * kBlock + threadIdx.x;
                    Tally<NC> t{};
                    day_wave<Rules>(m, s, l, d, prologue, ssa, t, s.R, s.status);
                    flush_block<NC>(m, s, t, s.inst[chunk * kBlock], d_rec, d_ssa,
                                    s.n_regions ? s.pos_region[chunk * kBlock] : -1);
                    if (ssa) private_tasks<NC>(m, s, ev, d, chunk, s.Np / kLaneUnit, 0, 1, 1, s.status);
                }
            }
        }
        if (!ssa) break;
        grid.sync();
        fresh_l1();
        // big levels are spread over the grid; a run of small levels is done
        // by workgroup 0 alone; one grid barrier follows either
        int32_t lv = ev.lvl_ptr[d];
        const int32_t lv_end = ev.lvl_ptr[d + 1];
        while (lv < lv_end) {
            const int64_t size = (ev.lvl_off[lv + 1] - ev.lvl_off[lv]) * s.RL;
            if (size > kSmallLevel) {
                const int64_t begin = ev.lvl_off[lv];
                if (*(volatile unsigned long long *)s.status == STATUS_OK) {
                    for (int64_t t = first; t < size; t += stride) {
                        const int64_t e = begin + (s.RL == 1 ? t : t / s.RL);
                        const int32_t r = s.RL == 1 ? 0 : (int32_t)(t % s.RL);
                        if (r < s.R) event_task<NC>(m, s, ev, e, r, d, s.status);
                    }
                }
                ++lv;
            } else {
                int32_t stop = lv + 1;
                while (stop < lv_end && (ev.lvl_off[stop + 1] - ev.lvl_off[stop]) * s.RL <= kSmallLevel) ++stop;
                if (blockIdx.x == 0) {
                    for (int32_t k = lv; k < stop; ++k) {
                        const int64_t begin = ev.lvl_off[k];
                        const int64_t count = (ev.lvl_off[k + 1] - begin) * s.RL;
                        for (int64_t t = threadIdx.x; t < count; t += kBlock) {
                            const int64_t e = begin + (s.RL == 1 ? t : t / s.RL);
                            const int32_t r = s.RL == 1 ? 0 : (int32_t)(t % s.RL);
                            if (r < s.R) event_task<NC>(m, s, ev, e, r, d, s.status);
                        }
                        __syncthreads();
                        fresh_l1();
                    }
                }
                lv = stop;
            }
            grid.sync();
            fresh_l1();
        }
    }
}

template <class Rules>
struct Kernels {
    static void *day() { return (void *)&k_day<Rules>; }
    static void *tile() { return (void *)&k_day_tile<Rules, false>; }
    static void *tile_slots() { return (void *)&k_day_tile<Rules, true>; }
    static void *events() { return (void *)&k_events<Rules::NC>; }
    static void *levels() { return (void *)&k_event_levels<Rules::NC>; }
    static void *persist() { return (void *)&k_persist<Rules>; }
    static void *slot_events() { return (void *)&k_slot_events<Rules::NC>; }
    static void *event_day() { return (void *)&k_event_day<Rules::NC>; }
};

struct Table {
    void *day, *events, *persist, *levels, *tile, *slot_events, *event_day, *tile_slots;
};

template <class Rules>
Table table() {
    return {Kernels<Rules>::day(),    Kernels<Rules>::events(), Kernels<Rules>::persist(),
            Kernels<Rules>::levels(), Kernels<Rules>::tile(),   Kernels<Rules>::slot_events(),
            Kernels<Rules>::event_day(), Kernels<Rules>::tile_slots()};
}

Table pick(const Model &m) {
    if (m.pairs && m.nc == 2) return table<PairRules<1>>();
    if (m.pairs && m.nc == 6) return table<PairRules<3>>();
    return table<GenericRules<MAXC, MAXT>>();
}

}  // namespace

int launch_day(const Model &m, const DevState &s, const DevEvents &ev, int32_t d, int prologue, int ssa,
               int layout, void *stream) {
    if (s.L == 0) return hipSuccess;
    const Table t = pick(m);
    Model mm = m;
    DevState ss = s;
    DevEvents ee = ev;
    int32_t dd = d, pro = prologue, sa = ssa;
    void *args[] = {&mm, &ss, &ee, &dd, &pro, &sa};
    if (layout == LAYOUT_TILE) {
        if (s.slots) return hipErrorInvalidValue;  // a slot handle's day runs through launch_slot_day
        const unsigned nx = (unsigned)((s.Np + s.tile_nodes - 1) / s.tile_nodes + (int64_t)s.n_heavy * kHeavyBlocks);
        return (int)hipLaunchKernel(t.tile, dim3(nx, (unsigned)(s.RL / 64)), dim3(kBlock), args, 0, (hipStream_t)stream);
    }
    const unsigned grid = (unsigned)((s.L + kBlock - 1) / kBlock);
    return (int)hipLaunchKernel(t.day, dim3(grid), dim3(kBlock), args, 0, (hipStream_t)stream);
}

int launch_events(const Model &m, const DevState &s, const DevEvents &ev, int32_t d, int64_t begin,
                  int64_t end, void *stream) {
    const int64_t count = (end - begin) * s.RL;
    if (count <= 0) return hipSuccess;
    const Table t = pick(m);
    const unsigned grid = (unsigned)((count + kBlock - 1) / kBlock);
    Model mm = m;
    DevState ss = s;
    DevEvents ee = ev;
    int32_t dd = d;
    int64_t b = begin, e = end;
    void *args[] = {&mm, &ss, &ee, &dd, &b, &e};
    return (int)hipLaunchKernel(t.events, dim3(grid), dim3(kBlock), args, 0, (hipStream_t)stream);
}

int launch_event_levels(const Model &m, const DevState &s, const DevEvents &ev, int32_t d, int32_t lv_begin,
                        int32_t lv_end, void *stream) {
    if (lv_end <= lv_begin) return hipSuccess;
    const Table t = pick(m);
    Model mm = m;
    DevState ss = s;
    DevEvents ee = ev;
    int32_t dd = d, a = lv_begin, b = lv_end;
    void *args[] = {&mm, &ss, &ee, &dd, &a, &b};
    return (int)hipLaunchKernel(t.levels, dim3(1), dim3(kEvBlock), args, 0, (hipStream_t)stream);
}

int launch_persistent(const Model &m, const DevState &s, const DevEvents &ev, int32_t d_begin,
                      int32_t d_end, int layout, void *stream, char *why, int why_len) {
    const Table t = pick(m);
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
    const int64_t want = layout == LAYOUT_TILE ? ((s.Np + s.tile_nodes - 1) / s.tile_nodes) * (s.RL / 64)
                                               : (s.L + kBlock - 1) / kBlock;
    int64_t grid = (int64_t)cus * per_cu;
    if (want < grid) grid = want > 0 ? want : 1;
    Model mm = m;
    DevState ss = s;
    DevEvents ee = ev;
    int32_t a = d_begin, b = d_end, lay = layout;
    void *args[] = {&mm, &ss, &ee, &a, &b, &lay};
    return (int)hipLaunchCooperativeKernel(t.persist, dim3((unsigned)grid), dim3(kBlock), args, 0,
                                           (hipStream_t)stream);
}

int launch_slot_day(const Model &m, const DevState &s, const DevEvents &ev, int32_t step, int32_t n_cols,
                    void *stream) {
    if (s.L == 0 || n_cols <= 0) return hipSuccess;
    if (!s.slots || n_cols > s.RL / 64) return hipErrorInvalidValue;
    const Table t = pick(m);
    Model mm = m;
    DevState ss = s;
    DevEvents ee = ev;
    int32_t dd = step, pro = 1, sa = 1;
    void *args[] = {&mm, &ss, &ee, &dd, &pro, &sa};
    const unsigned nx = (unsigned)((s.Np + s.tile_nodes - 1) / s.tile_nodes + (int64_t)s.n_heavy * kHeavyBlocks);
    return (int)hipLaunchKernel(t.tile_slots, dim3(nx, (unsigned)n_cols), dim3(kBlock), args, 0, (hipStream_t)stream);
}

int launch_slot_events(const Model &m, const DevState &s, const DevEvents &ev, int32_t step, int32_t k,
                       int32_t k_end, int64_t max_count, int32_t n_run, void *stream) {
    if (k_end <= k || max_count <= 0 || n_run <= 0) return hipSuccess;
    if (n_run > s.RL / s.slot_lanes) return hipErrorInvalidValue;
    const Table t = pick(m);
    const int64_t want = k_end > k + 1 ? 1 : (max_count + kEvBlock - 1) / kEvBlock;
    const unsigned gx = (unsigned)std::min<int64_t>(want, 4096);
    Model mm = m;
    DevState ss = s;
    DevEvents ee = ev;
    int32_t a = step, b = k, c = k_end;
    void *args[] = {&mm, &ss, &ee, &a, &b, &c};
    return (int)hipLaunchKernel(t.slot_events, dim3(gx, (unsigned)n_run), dim3(kEvBlock), args, 0, (hipStream_t)stream);
}

int launch_event_day(const Model &m, const DevState &s, const DevEvents &ev, int32_t d, const EventDayArgs &a,
                     void *stream) {
    const Table t = pick(m);
    Model mm = m;
    DevState ss = s;
    DevEvents ee = ev;
    int32_t dd = d;
    EventDayArgs aa = a;
    void *args[] = {&mm, &ss, &ee, &dd, &aa};
    return (int)hipLaunchKernel(t.event_day, dim3(1), dim3(kEvBlock), args, 0, (hipStream_t)stream);
}

int launch_slot_init(const DevState &s, int32_t nc, const int32_t *u0, const double *v0, int32_t slot,
                     const SlotInfo &info, void *stream) {
    const int64_t work = std::max<int64_t>(s.Np * s.slot_lanes, (int64_t)s.n_days * s.slot_lanes);
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((work + kBlock - 1) / kBlock, 8192));
    DevState ss = s;
    int32_t n = nc, sl = slot;
    const int32_t *a = u0;
    const double *b = v0;
    SlotInfo in = info;
    void *args[] = {&ss, &n, &a, &b, &sl, &in};
    return (int)hipLaunchKernel((void *)&k_slot_init, dim3(grid), dim3(kBlock), args, 0, (hipStream_t)stream);
}

int launch_goal_sum(const double *part, int32_t n, double *out, void *stream) {
    const double *pp = part;
    int32_t nn = n;
    double *o = out;
    void *args[] = {&pp, &nn, &o};
    return (int)hipLaunchKernel((void *)&k_goal_sum, dim3(1), dim3(64), args, 0, (hipStream_t)stream);
}

int scratch_address(void **out) {
    static std::mutex lock;
    static void *cached[kMaxScratchDevices] = {};
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return (int)e;
    if (dev < 0 || dev >= kMaxScratchDevices) return (int)hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(lock);
    if (!cached[dev]) {
        // the array's name is a host-side stand-in: its device address on this
        // GPU comes from the runtime, and only that address is ever used
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return (int)e;
        cached[dev] = ptr;
    }
    *out = cached[dev];
    return (int)hipSuccess;
}

int launch_goal(const DevState &s, int32_t nc, int64_t s0, int32_t N, const int64_t *ref, int32_t d_begin,
                int32_t n_days, double *part, void *stream) {
    if (n_days <= 0) return hipSuccess;
    DevState ss = s;
    int32_t a = nc, n = N, db = d_begin;
    int64_t b = s0;
    const int64_t *r = ref;
    double *pp = part;
    void *args[] = {&ss, &a, &b, &n, &r, &db, &pp};
    return (int)hipLaunchKernel((void *)&k_goal, dim3((unsigned)n_days), dim3(kBlock), args, 0, (hipStream_t)stream);
}

}  // namespace episim
