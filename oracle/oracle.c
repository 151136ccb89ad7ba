/*
 * Reference oracle for the per-day step of the event-based epidemic model of
 * Bauer, Engblom & Widgren, "Fast event-based epidemiological simulations on
 * national scales" (arXiv:1502.02908).
 *
 * TEST INFRASTRUCTURE ONLY. This file is the plain, slow, sequential CPU
 * statement of what the GPU path must compute. Only the test-suite, the smoke
 * check and the benchmark's CPU-baseline leg may load it. It shares no code,
 * header or constant generator with the GPU library.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fopenmp -shared -fPIC
 * (no fast-math: every floating-point operation below is an IEEE-754 binary64
 * operation, rounded to nearest, in exactly the order written).
 *
 * What is computed (Sec. 3.1, the splitting eq:numstep3-5, and Algorithm 1):
 * for each replicate r and each day d of the horizon
 *   1. stochastic step: a Gillespie direct-method SSA per node over the
 *      window [d, d+1) with the continuous state phi frozen (eq:numstep3;
 *      Sec. 3.3 "Sequential simulation algorithm", eq:sampling, eq:sampling2);
 *   2. deterministic step: the externally defined events of day d, in list
 *      order (eq:numstep4; Sec. 3.2 eq:event);
 *   3. continuous-state update: forward Euler with dt = 1 for the
 *      environmental infectious pressure phi (eq:numstep5 with the right-hand
 *      side of eq:siminfpressure and the seasonal beta(t) of Sec. 4.1);
 *   4. daily record (prevalence, compartment totals, transition counts, and
 *      snapshots of u and phi on the requested days).
 *
 * Readings where the paper is silent or garbled (stated once here; every
 * function below follows them):
 *   - Random numbers: one Philox4x32-10 block (Salmon, Moraes, Dror & Shaw,
 *     SC'11) per SSA attempt, counter (k, node, d, 0) and key (seed,
 *     replicate id); event sampling uses counter (q/2, g, d, 1) for draw q of
 *     event g (its index in the day-sorted event list).
 *   - rand in (0,1) (eq:sampling) is U53 of two 32-bit words, never 0 or 1.
 *   - The clock is redrawn at every window start (memorylessness); a draw
 *     whose time lands on or past the window end is discarded.
 *   - phi is updated from the state after the day's events (Algorithm 1
 *     orders the events before the continuous update, and Algorithm 2 runs
 *     that update at the start of the next window), with beta taken at the
 *     left end of the integrated window, t = day0 + d.
 *   - A node with no animals sheds nothing (the shedding term is 0).
 *   - Removals sample individuals without replacement from the selected
 *     compartments; asking for more than are present is an error, never
 *     clamped (Sec. 2.1 only warns that removals need care).
 *   - The inversion of eq:sampling2 picks the first transition whose rate is
 *     positive and whose cumulative sum reaches lambda*rand.
 */
#include <stdint.h>
#include <stddef.h>
#include <string.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_MAXC 8
#define OR_MAXT 8

enum { EV_EXIT = 0, EV_ENTER = 1, EV_INTERNAL = 2, EV_EXTERNAL = 3 };

enum {
    OR_OK = 0,
    OR_EINVAL = -1,
    OR_ENOMEM = -2,
    OR_EINFEASIBLE = -4
};

/* Problem statement (Sec. 2 and Sec. 3.2). All arrays are read-only. */
typedef struct oracle_problem {
    int32_t Nn;              /* nodes */
    int32_t Nc;              /* compartments (<= 8) */
    int32_t Nt;              /* stochastic transitions (<= 8) */
    int32_t R;               /* replicates */
    int32_t day0;            /* calendar day of simulation day 0 (for beta(t)) */
    const int32_t *S;        /* stoichiometry, S[c*Nt + k] */
    const int32_t *reactant; /* [Nt] compartment whose count scales rate k */
    const int32_t *uses_phi; /* [Nt] 1 if rate k is proportional to phi */
    const double *coef;      /* [R*Nt] per-replicate rate constants */
    const double *alpha;     /* [R] shedding rate */
    const double *beta;      /* [R*4] quarterly decay rates */
    uint32_t phi_I_mask;     /* compartments counted as infected */
    uint32_t phi_N_mask;     /* compartments counted in the node size */
    int32_t n_select;
    const int32_t *E;        /* select matrix, E[c*n_select + s] in {0,1} */
    int32_t n_shift;
    const int32_t *Nsh;      /* shift matrix, Nsh[c*n_shift + h] */
    int64_t n_events;        /* events sorted by day (stable = list order) */
    const int32_t *ev_day, *ev_kind, *ev_node, *ev_dest, *ev_n, *ev_select, *ev_shift;
    uint32_t seed;
    const uint32_t *replicate_id; /* [R] */
    const int32_t *reactant2;     /* [Nt] second reactant of a mass-action rate, -1 if none; NULL: none */
    int32_t phi_pre_events;       /* 1: phi from the state after the SSA, before the events */
    int32_t n_regions;            /* regions for the aggregates of the goal function (Sec. 4.3) */
    const int32_t *region;        /* [Nn] region of each node in [0, n_regions), or -1 */
} oracle_problem;

/* Outputs for days [d_begin, d_end); indices are relative to d_begin. */
typedef struct oracle_output {
    int32_t *prevalence;   /* [D*R] nodes with an infected individual */
    int64_t *transitions;  /* [D*R] SSA transitions applied on the day */
    int64_t *totals;       /* [D*R*Nc] compartment sums over nodes */
    int32_t n_record;
    const int32_t *record_days; /* absolute day indices, ascending */
    int32_t *snap_u;       /* [n_record*R*Nn*Nc] */
    double *snap_v;        /* [n_record*R*Nn] */
    int64_t *regional;     /* [D*R*n_regions*Nc] compartment sums over the nodes of each region (or NULL) */
    int32_t *max_trans;    /* [D*R] largest number of SSA transitions of one node on the day (or NULL) */
    /* error report: smallest (event index, replicate) that was infeasible */
    int64_t err_event;
    int32_t err_rep;
    int32_t err_day;
} oracle_output;

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al., SC'11): ten rounds of the Philox S-P network  */
/* with the published multipliers and Weyl key increments.                   */
/* ------------------------------------------------------------------------ */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += W0; k1 += W1; }
        uint64_t p0 = (uint64_t)M0 * (uint64_t)x0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)x2;
        uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)p1;
        uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)p0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* rand in (0,1): the 53-bit odd lattice point (2*floor(x/2^12)+1) / 2^53,
 * where x = hi*2^32 + lo. Exact; never 0, never 1 (eq:sampling). */
double oracle_u53(uint32_t lo, uint32_t hi)
{
    uint64_t x = ((uint64_t)hi << 32) | (uint64_t)lo;
    uint64_t odd = 2u * (x >> 12) + 1u;
    return (double)odd * 0x1p-53;
}

/* High 64 bits of the 128-bit product a*b. */
uint64_t oracle_mulhi64(uint64_t a, uint64_t b)
{
    return (uint64_t)(((unsigned __int128)a * (unsigned __int128)b) >> 64);
}

/* -log(u) for u in (0,1), from log m = 2 atanh((m-1)/(m+1)).
 * u = m * 2^e with m folded into (sqrt(2)/2, sqrt(2)]; the atanh series is
 * summed to the s^23 term (coefficients 1/(2k+1)); ln 2 is split into a
 * 32-significant-bit head (so e*LN2_HI is exact) and a tail. Only + - * / are
 * used, in this fixed order, so the result is a fixed function of u. */
double oracle_neglog(double u)
{
    const double RT2 = 0x1.6a09e667f3bcdp+0;     /* nearest double to sqrt(2) */
    const double LN2_HI = 0x1.62e42ff000000p-1;   /* ln 2 to 32 bits */
    const double LN2_LO = -0x1.718432a1b0e26p-35; /* ln 2 - LN2_HI */
    uint64_t bits;
    memcpy(&bits, &u, sizeof bits);
    int32_t e = (int32_t)((bits >> 52) & 0x7ffu) - 1023;
    uint64_t mbits = (bits & 0x000fffffffffffffull) | 0x3ff0000000000000ull;
    double m;
    memcpy(&m, &mbits, sizeof m);
    if (m > RT2) { m = m * 0.5; e = e + 1; }
    double f = m - 1.0;
    double s = f / (2.0 + f);
    double z = s * s;
    double p = 1.0 / 23.0;
    p = 1.0 / 21.0 + z * p;
    p = 1.0 / 19.0 + z * p;
    p = 1.0 / 17.0 + z * p;
    p = 1.0 / 15.0 + z * p;
    p = 1.0 / 13.0 + z * p;
    p = 1.0 / 11.0 + z * p;
    p = 1.0 / 9.0 + z * p;
    p = 1.0 / 7.0 + z * p;
    p = 1.0 / 5.0 + z * p;
    p = 1.0 / 3.0 + z * p;
    double Rz = z * p;
    double t = s + s * Rz;
    double lm = t + t;
    double de = (double)e;
    double logu = de * LN2_HI + (lm + de * LN2_LO);
    return -logu;
}

/* Season index of beta(t) (Sec. 4.1): t mod 365 in [0,91], (91,182],
 * (182,273], (273,364]. */
int oracle_quarter(int64_t t)
{
    int64_t doy = t % 365;
    if (doy < 0) doy += 365;
    if (doy <= 91) return 0;
    if (doy <= 182) return 1;
    if (doy <= 273) return 2;
    return 3;
}

/* Rates omega_k and their sum lambda (Sec. 3.3; eq:rate_s_to_i,
 * eq:recovery_rates): omega_k = c_k * (phi if rate k uses phi) * X[a_k],
 * lambda summed left to right in transition order. */
static double rates(const oracle_problem *p, int r, const int32_t *x, double phi, double *w)
{
    double lam = 0.0;
    for (int k = 0; k < p->Nt; ++k) {
        double v = p->coef[(size_t)r * p->Nt + k];
        if (p->uses_phi[k]) v = v * phi;
        v = v * (double)x[p->reactant[k]];
        /* a bimolecular rate (mass action, e.g. the SIR example of Sec. 2.1)
         * is also proportional to its second reactant's count */
        if (p->reactant2 && p->reactant2[k] >= 0) v = v * (double)x[p->reactant2[k]];
        w[k] = v;
        lam = lam + w[k];
    }
    return lam;
}

/* One node, one window: Gillespie's direct method (Algorithm 1, the inner
 * while-loop; eq:sampling for the waiting time, eq:sampling2 for the choice
 * of transition). Returns the number of transitions applied. */
static int64_t ssa_node(const oracle_problem *p, int r, int32_t node, int32_t d,
                        int32_t *x, double phi)
{
    double w[OR_MAXT];
    double lam = rates(p, r, x, phi, w);
    double s = 0.0;
    uint32_t k = 0;
    int64_t ntrans = 0;
    const uint32_t key[2] = { p->seed, p->replicate_id[r] };
    while (lam > 0.0) {
        uint32_t ctr[4] = { k, (uint32_t)node, (uint32_t)d, 0u };
        uint32_t o[4];
        oracle_philox4x32_10(ctr, key, o);
        k = k + 1;
        double tau = oracle_neglog(oracle_u53(o[0], o[1])) / lam;
        if (!(s + tau < 1.0)) break;          /* next event falls past the window */
        s = s + tau;
        double target = oracle_u53(o[2], o[3]) * lam;
        int j = -1, last_pos = -1;
        double cum = 0.0;
        for (int kk = 0; kk < p->Nt; ++kk) {
            cum = cum + w[kk];
            if (w[kk] > 0.0) {
                last_pos = kk;
                if (cum >= target) { j = kk; break; }
            }
        }
        if (j < 0) j = last_pos;
        for (int c = 0; c < p->Nc; ++c) x[c] += p->S[(size_t)c * p->Nt + j];
        ntrans = ntrans + 1;
        lam = rates(p, r, x, phi, w);          /* full recompute (dependency graph = all) */
    }
    return ntrans;
}

/* Sample n individuals without replacement from the compartments selected by
 * mask at a node whose state is x (Sec. 3.2: the event moves n individuals;
 * which ones is drawn uniformly). m receives the sampled composition.
 * Returns 0, or -1 if fewer than n individuals are present. */
static int sample_individuals(const oracle_problem *p, int r, int64_t g, int32_t d,
                              const int32_t *x, uint32_t mask, int32_t n, int32_t *m)
{
    int64_t tot = 0;
    int32_t rem[OR_MAXC];
    for (int c = 0; c < p->Nc; ++c) {
        m[c] = 0;
        rem[c] = x[c];
        if (mask & (1u << c)) tot += x[c];
    }
    if ((int64_t)n > tot) return -1;
    const uint32_t key[2] = { p->seed, p->replicate_id[r] };
    uint32_t o[4] = { 0, 0, 0, 0 };
    for (int32_t q = 0; q < n; ++q) {
        if ((q & 1) == 0) {
            uint32_t ctr[4] = { (uint32_t)(q / 2), (uint32_t)g, (uint32_t)d, 1u };
            oracle_philox4x32_10(ctr, key, o);
        }
        uint64_t x64 = (q & 1) == 0 ? (((uint64_t)o[1] << 32) | o[0])
                                    : (((uint64_t)o[3] << 32) | o[2]);
        uint64_t pick = oracle_mulhi64(x64, (uint64_t)tot);  /* uniform in [0, tot) */
        int chosen = -1;
        for (int c = 0; c < p->Nc; ++c) {
            if (!(mask & (1u << c))) continue;
            if (pick < (uint64_t)rem[c]) { chosen = c; break; }
            pick -= (uint64_t)rem[c];
        }
        rem[chosen] -= 1;
        m[chosen] += 1;
        tot -= 1;
    }
    return 0;
}

static uint32_t select_mask(const oracle_problem *p, int32_t s)
{
    uint32_t mask = 0;
    for (int c = 0; c < p->Nc; ++c)
        if (p->E[(size_t)c * p->n_select + s]) mask |= 1u << c;
    return mask;
}

/* The deterministic step for one event (Sec. 3.2: X <- X + R n, with R the
 * event's transition column; E1 events touch one node, E2 events two). */
static int apply_event(const oracle_problem *p, int r, int64_t g, int32_t d, int32_t *u)
{
    const int32_t Nc = p->Nc;
    int32_t kind = p->ev_kind[g], node = p->ev_node[g], n = p->ev_n[g];
    int32_t sel = p->ev_select[g], sh = p->ev_shift[g];
    uint32_t mask = select_mask(p, sel);
    int32_t *xs = u + (size_t)node * Nc;
    if (kind == EV_ENTER) {
        int c = 0;
        while (!(mask & (1u << c))) ++c;       /* the single selected compartment */
        xs[c] += n;
        return 0;
    }
    int32_t m[OR_MAXC];
    if (sample_individuals(p, r, g, d, xs, mask, n, m) != 0) return -1;
    for (int c = 0; c < Nc; ++c) xs[c] -= m[c];
    if (kind == EV_EXIT) return 0;
    int32_t *xt = (kind == EV_INTERNAL) ? xs : u + (size_t)p->ev_dest[g] * Nc;
    for (int c = 0; c < Nc; ++c) {
        if (m[c] == 0) continue;
        int32_t to = c + (sh >= 0 ? p->Nsh[(size_t)c * p->n_shift + sh] : 0);
        xt[to] += m[c];
    }
    return 0;
}

/* phi_{d+1} = phi_d + dt * (alpha * I/N - beta(t) * phi_d), dt = 1, written
 * as (1 - beta) * phi + alpha * (I/N) (eq:siminfpressure, eq:numstep5). */
static double phi_update(const oracle_problem *p, int r, int32_t d, const int32_t *x, double phi)
{
    int64_t I = 0, N = 0;
    for (int c = 0; c < p->Nc; ++c) {
        if (p->phi_I_mask & (1u << c)) I += x[c];
        if (p->phi_N_mask & (1u << c)) N += x[c];
    }
    int q = oracle_quarter((int64_t)p->day0 + d);
    double a = 1.0 - p->beta[(size_t)r * 4 + q];
    double b = a * phi;
    double shed = N > 0 ? p->alpha[r] * ((double)I / (double)N) : 0.0;
    return b + shed;
}

/* Run days [d_begin, d_end) for every replicate, starting from state
 * (u[R*Nn*Nc] node-major per replicate, v[R*Nn]) which is updated in place.
 * threads > 1 runs the two node loops of each day (SSA and phi) fork-join
 * with OpenMP, as the paper's fork-join variant does; events stay serial. */
int oracle_run(const oracle_problem *p, int32_t *u, double *v, int32_t d_begin, int32_t d_end,
               int32_t threads, oracle_output *out)
{
    if (p->Nc < 1 || p->Nc > OR_MAXC || p->Nt < 1 || p->Nt > OR_MAXT || p->R < 1 || p->Nn < 0)
        return OR_EINVAL;
    if (d_end < d_begin) return OR_EINVAL;
    const int32_t Nn = p->Nn, Nc = p->Nc, R = p->R;
    out->err_event = -1; out->err_rep = -1; out->err_day = -1;
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#else
    (void)threads;
#endif
    int64_t *ntr = (int64_t *)malloc(sizeof(int64_t) * (size_t)(Nn > 0 ? Nn : 1));
    if (!ntr) return OR_ENOMEM;
    /* first event of each day: events are sorted by day */
    int64_t ev_lo = 0;
    while (ev_lo < p->n_events && p->ev_day[ev_lo] < d_begin) ++ev_lo;
    int rc = OR_OK;
    for (int32_t r = 0; r < R; ++r) {
        int32_t *ur = u + (size_t)r * Nn * Nc;
        double *vr = v + (size_t)r * Nn;
        int64_t e = ev_lo;
        int failed = 0;
        int rec = 0;
        for (int32_t d = d_begin; d < d_end && !failed; ++d) {
            const int32_t dd = d - d_begin;
            /* 1. stochastic step, every node independently */
            #pragma omp parallel for schedule(dynamic, 64) if (threads > 1)
            for (int32_t i = 0; i < Nn; ++i)
                ntr[i] = ssa_node(p, r, i, d, ur + (size_t)i * Nc, vr[i]);
            int64_t trans = 0, most = 0;
            for (int32_t i = 0; i < Nn; ++i) {
                trans += ntr[i];
                if (ntr[i] > most) most = ntr[i];
            }
            /* the longest chain of the day: the straggler of the stochastic step */
            if (out->max_trans) out->max_trans[(size_t)dd * R + r] = (int32_t)most;
            /* eq:numstep5 as written feeds phi with the state before the
             * events (the variant reading; the default follows Algorithm 1) */
            if (p->phi_pre_events) {
                #pragma omp parallel for schedule(static) if (threads > 1)
                for (int32_t i = 0; i < Nn; ++i)
                    vr[i] = phi_update(p, r, d, ur + (size_t)i * Nc, vr[i]);
            }
            /* 2. deterministic step: this day's events in list order */
            while (e < p->n_events && p->ev_day[e] == d) {
                if (apply_event(p, r, e, d, ur) != 0) {
                    if (rc == OR_OK || e < out->err_event ||
                        (e == out->err_event && r < out->err_rep)) {
                        out->err_event = e; out->err_rep = r; out->err_day = d;
                    }
                    rc = OR_EINFEASIBLE;
                    failed = 1;
                    break;
                }
                ++e;
            }
            if (failed) break;
            /* 3. continuous-state update (Algorithm 1: after the events) */
            if (!p->phi_pre_events) {
                #pragma omp parallel for schedule(static) if (threads > 1)
                for (int32_t i = 0; i < Nn; ++i)
                    vr[i] = phi_update(p, r, d, ur + (size_t)i * Nc, vr[i]);
            }
            /* 4. record */
            if (out->transitions) out->transitions[(size_t)dd * R + r] = trans;
            if (out->prevalence) {
                int32_t prev = 0;
                for (int32_t i = 0; i < Nn; ++i) {
                    int64_t I = 0;
                    for (int c = 0; c < Nc; ++c)
                        if (p->phi_I_mask & (1u << c)) I += ur[(size_t)i * Nc + c];
                    prev += I > 0;
                }
                out->prevalence[(size_t)dd * R + r] = prev;
            }
            if (out->totals) {
                for (int c = 0; c < Nc; ++c) {
                    int64_t t = 0;
                    for (int32_t i = 0; i < Nn; ++i) t += ur[(size_t)i * Nc + c];
                    out->totals[((size_t)dd * R + r) * Nc + c] = t;
                }
            }
            /* regional aggregates: X summed over the nodes of each region
             * (the inner sum of eq:goal, one sample trajectory) */
            if (out->regional && p->n_regions > 0) {
                int64_t *g = out->regional + ((size_t)dd * R + r) * p->n_regions * Nc;
                for (int64_t q = 0; q < (int64_t)p->n_regions * Nc; ++q) g[q] = 0;
                for (int32_t i = 0; i < Nn; ++i) {
                    const int32_t j = p->region[i];
                    if (j < 0) continue;
                    for (int c = 0; c < Nc; ++c) g[(size_t)j * Nc + c] += ur[(size_t)i * Nc + c];
                }
            }
            while (rec < out->n_record && out->record_days[rec] < d) ++rec;
            if (rec < out->n_record && out->record_days[rec] == d) {
                if (out->snap_u)
                    memcpy(out->snap_u + ((size_t)rec * R + r) * Nn * Nc, ur,
                           sizeof(int32_t) * (size_t)Nn * Nc);
                if (out->snap_v)
                    memcpy(out->snap_v + ((size_t)rec * R + r) * Nn, vr,
                           sizeof(double) * (size_t)Nn);
            }
        }
    }
    free(ntr);
    return rc;
}
