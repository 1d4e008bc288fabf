/*
 * oracle.c - plain, single-threaded CPU oracle for the Independent algorithm
 * (Langenstein 2021, "Communication-free and Parallel Simulation of Neutral
 * Biodiversity Models", arXiv 2108.05815).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call
 * this file; only the tests, the smoke check and the benchmark's CPU-baseline
 * leg use it.  It shares no code with the HIP library: every primitive below
 * (Philox, logarithm, Vose alias build, torus, dispersal, next-event search,
 * culling) is written here a second time, from the paper and the published
 * definitions it cites, so that a mistake on one side cannot hide on the other.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -fPIC -shared
 * (no FMA contraction: every fused multiply-add below is an explicit fma()).
 *
 * Section references are to the paper:
 *   [ind]   "The Independent Algorithm" chapter, sections "Environmental RNG
 *           Priming", "Aligning the RNGs of Colliding Individuals",
 *           "Exponential inter-event Times" (memoryless sums of exponentials)
 *           and "Summary of the Independent Algorithm";
 *   [cbrng] related-work section "Counter-based Pseudo-Random Number Generators"
 *           (Salmon et al. 2011, Philox);
 *   [dist]  appendix "Sampling Probability Distributions" (U(0,1) from 64 bits,
 *           inverse transform for Exp(lambda));
 *   [dedup] section "Deduplicating Redundant Individuals" and the Water-Level
 *           algorithm (time-aligned rounds);
 *   [comp]  section "The Statically Checked Component System" (habitat,
 *           dispersal sampler, coalescence sampler = uniform deme index);
 *   [impl]  background section "Spatially Implicit" and its appendix (a local
 *           community of J with per-event migration probability m into a
 *           non-spatial metacommunity of J_m with speciation nu_m; no
 *           speciation in the local community; the metacommunity simulated
 *           alongside, i.e. dynamic and finite);
 *   [hppp]  section "Homogeneous Poisson Point Process" of the Independent
 *           Algorithm chapter (the log-free alternative to the exponential
 *           sums: a Poisson count per interval, the events uniform in it) and
 *           appendix "Iterative Sampling: Geometric and Poisson" (the count by
 *           a linear search over the Poisson cdf, one uniform per count);
 *   [prot]  appendix "Protracted Speciation" (a speciation completes only
 *           after tau generations, so the draws at events younger than tau
 *           are ignored);
 *   [evs]   sections "Sorting Events using the Water-Level Algorithm" and
 *           "Reporting Coalescence Events Independently" (every lineage's
 *           events in one stream sorted by event time, then prior event
 *           time; copies of one event adjacent; the first copy is the
 *           parent's, and a later distinct prior time marks a coalescence).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_EXPORT __attribute__((visibility("default")))

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 [cbrng]: 10 rounds of two 32x32->64 multiplies with the      */
/* published multipliers and Weyl key increments (Salmon et al., SC'11).      */
/* ------------------------------------------------------------------------- */
OR_EXPORT void or_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
    uint32_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c[0];
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c[2];
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c[1] ^ k0;
        uint32_t n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
    memcpy(out, c, sizeof c);
}

/* Counter layout of the primeable hash RNG ("prime on seed, location, time",
 * [ind] Environmental RNG Priming): key = seed, counter = (location, two time
 * words, domain<<30 | call).  Domain 0 keys the inter-event search on the
 * interval index k, domain 1 keys the event draws on the bits of the event
 * time, domain 2 keys the species identity of a speciation event. */
enum { DOM_INTERVAL = 0u, DOM_EVENT = 1u, DOM_SPECIES = 2u };

static void hash_block(uint64_t seed, uint32_t loc, uint64_t tword, uint32_t domain, uint32_t call,
                       uint64_t *a, uint64_t *b) {
    uint32_t ctr[4] = {loc, (uint32_t)tword, (uint32_t)(tword >> 32), (domain << 30) | call};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t o[4];
    or_philox4x32_10(ctr, key, o);
    *a = ((uint64_t)o[1] << 32) | o[0];
    *b = ((uint64_t)o[3] << 32) | o[2];
}

static uint64_t f64_bits(double x) {
    uint64_t u;
    memcpy(&u, &x, sizeof u);
    return u;
}

/* [dist] U(0,1) from the top 53 bits: [0,1) ... */
static double u53(uint64_t r) { return (double)(r >> 11) * 0x1.0p-53; }
/* ... and the same grid shifted by one step, (0,1], so that log never sees 0. */
static double u53_open0(uint64_t r) { return (double)((r >> 11) + 1u) * 0x1.0p-53; }

/* floor(r * n / 2^64): a uniform index in [0, n) from one 64-bit draw. */
static uint32_t mulhi64_u32(uint64_t r, uint32_t n) {
    return (uint32_t)(((unsigned __int128)r * (unsigned __int128)n) >> 64);
}

/* ------------------------------------------------------------------------- */
/* Natural logarithm with a fixed, fully specified operation sequence, so    */
/* that the exponential waiting times are reproducible bit for bit on any    */
/* IEEE-754 binary64 machine.  Mathematics: x = m * 2^e with m in            */
/* [sqrt(1/2), sqrt(2)); log(m) = 2 atanh(s), s = (m-1)/(m+1), expanded as   */
/* 2s (1 + z/3 + z^2/5 + ... + z^10/21), z = s^2 (|s| <= 0.1716, so the      */
/* truncated tail is below 1e-18 relative); log(x) = e ln2 + log(m) with ln2 */
/* split into a 32-bit head and a tail.                                       */
/* ------------------------------------------------------------------------- */
OR_EXPORT double or_log(double x) {
    int e;
    double m = frexp(x, &e); /* x = m 2^e, m in [1/2, 1) */
    if (m < 0x1.6a09e667f3bcdp-1) {
        m = m * 2.0;
        e = e - 1;
    }
    double f = m - 1.0;
    double s = f / (2.0 + f);
    double z = s * s;
    double p = 1.0 / 21.0;
    p = fma(p, z, 1.0 / 19.0);
    p = fma(p, z, 1.0 / 17.0);
    p = fma(p, z, 1.0 / 15.0);
    p = fma(p, z, 1.0 / 13.0);
    p = fma(p, z, 1.0 / 11.0);
    p = fma(p, z, 1.0 / 9.0);
    p = fma(p, z, 1.0 / 7.0);
    p = fma(p, z, 1.0 / 5.0);
    p = fma(p, z, 1.0 / 3.0);
    p = p * z;
    double two_s = s + s;
    double log_m = fma(two_s, p, two_s);
    double de = (double)e;
    return fma(de, 0x1.62e42fee00000p-1, fma(de, 0x1.a39ef35793c76p-33, log_m));
}

/* ------------------------------------------------------------------------- */
/* Vose alias table.  The paper names the alias method for O(1) sampling of  */
/* a discrete distribution (Gillespie background, Slepoy et al.); the build  */
/* order is Vose (1991):                                                      */
/*   p_i = (w_i * n) / W with W summed in index order;                        */
/*   stacks "small" (p < 1) and "large" (p >= 1) filled by an ascending scan; */
/*   repeatedly pop s from small and l from large (last pushed first):       */
/*   prob[s] = p_s, alias[s] = l, p_l = (p_l + p_s) - 1, push l by its value;*/
/*   leftovers in either stack get prob 1 and alias = self.                   */
/* ------------------------------------------------------------------------- */
OR_EXPORT int or_alias_build(const double *w, uint32_t n, double *prob, uint32_t *alias) {
    if (n == 0) return -1;
    double total = 0.0;
    for (uint32_t i = 0; i < n; ++i) {
        if (!(w[i] >= 0.0) || isinf(w[i])) return -1;
        total = total + w[i];
    }
    if (!(total > 0.0) || isinf(total)) return -1;
    double *p = (double *)malloc(sizeof(double) * n);
    uint32_t *small = (uint32_t *)malloc(sizeof(uint32_t) * n);
    uint32_t *large = (uint32_t *)malloc(sizeof(uint32_t) * n);
    if (!p || !small || !large) {
        free(p); free(small); free(large);
        return -2;
    }
    uint32_t ns = 0, nl = 0;
    for (uint32_t i = 0; i < n; ++i) {
        p[i] = (w[i] * (double)n) / total;
        if (p[i] < 1.0) small[ns++] = i;
        else large[nl++] = i;
    }
    while (ns > 0 && nl > 0) {
        uint32_t s = small[--ns];
        uint32_t l = large[--nl];
        prob[s] = p[s];
        alias[s] = l;
        p[l] = (p[l] + p[s]) - 1.0;
        if (p[l] < 1.0) small[ns++] = l;
        else large[nl++] = l;
    }
    while (nl > 0) {
        uint32_t l = large[--nl];
        prob[l] = 1.0;
        alias[l] = l;
    }
    while (ns > 0) {
        uint32_t s = small[--ns];
        prob[s] = 1.0;
        alias[s] = s;
    }
    free(p); free(small); free(large);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Scenario: a W x H torus of demes with capacities cap[c] (c = y W + x), a  */
/* (2R+1)^2 dispersal kernel of weights (row = dy + R, column = dx + R), the */
/* speciation probability nu, turnover rate lambda and repriming interval dt.*/
/* Dispersal mode 0: one table over the positive-weight kernel cells, shared */
/* by every deme (all capacities must be positive).  Mode 1: one table per   */
/* habitable deme over weight * capacity of each target, zero-mass targets   */
/* dropped ("restricted to habitable cells"; parents drawn in proportion to  */
/* individuals).  Tables list kernel cells in row-major kernel order.        */
/* ------------------------------------------------------------------------- */
typedef struct {
    uint32_t n;      /* entries */
    double *prob;
    uint32_t *alias;
    uint32_t *kidx;  /* kernel cell index of each entry: dx = kidx % (2R+1) - R */
} or_table;

typedef struct {
    uint32_t W, H, R, mode; /* mode 0 shared table, 1 per-deme tables, 2 spatially implicit [impl] */
    double mig;             /* mode 2: migration probability of a local event */
    uint32_t *cap;
    uint64_t *prefix; /* prefix[c] = sum of cap before cell c; prefix[W H] = N */
    uint32_t cmax;
    double *weights;  /* (2R+1)^2 */
    double nu, lambda, inv_lambda, dt, inv_dt;
    uint32_t sampler; /* 0: exponential sums; 1: Poisson count + uniform points [hppp] */
    double mu, p0;    /* sampler 1: lambda * dt and exp(-lambda * dt) */
    double tau;       /* protracted speciation: generations; 0 is point speciation [prot] */
    or_table shared;  /* mode 0 */
    or_table **cells; /* mode 1, built on first visit */
} or_scenario;

static void table_free(or_table *t) {
    free(t->prob); free(t->alias); free(t->kidx);
    t->prob = NULL; t->alias = NULL; t->kidx = NULL; t->n = 0;
}

static int table_build(const or_scenario *s, int64_t cell, or_table *out) {
    uint32_t side = 2 * s->R + 1, nk = side * side;
    double *w = (double *)malloc(sizeof(double) * nk);
    uint32_t *kidx = (uint32_t *)malloc(sizeof(uint32_t) * nk);
    if (!w || !kidx) { free(w); free(kidx); return -2; }
    uint32_t n = 0;
    for (uint32_t k = 0; k < nk; ++k) {
        double wk = s->weights[k];
        if (cell >= 0) {
            int64_t x = cell % s->W, y = cell / s->W;
            int64_t dx = (int64_t)(k % side) - s->R, dy = (int64_t)(k / side) - s->R;
            int64_t tx = ((x + dx) % (int64_t)s->W + s->W) % s->W;
            int64_t ty = ((y + dy) % (int64_t)s->H + s->H) % s->H;
            wk = wk * (double)s->cap[ty * s->W + tx];
        }
        if (wk > 0.0) {
            w[n] = wk;
            kidx[n] = k;
            ++n;
        }
    }
    if (n == 0) { free(w); free(kidx); return -1; }
    out->n = n;
    out->prob = (double *)malloc(sizeof(double) * n);
    out->alias = (uint32_t *)malloc(sizeof(uint32_t) * n);
    out->kidx = (uint32_t *)realloc(kidx, sizeof(uint32_t) * n);
    int rc = (out->prob && out->alias && out->kidx) ? or_alias_build(w, n, out->prob, out->alias) : -2;
    free(w);
    if (rc != 0) table_free(out);
    return rc;
}

OR_EXPORT void or_scenario_destroy(or_scenario *s) {
    if (!s) return;
    if (s->cells) {
        for (uint64_t c = 0; c < (uint64_t)s->W * s->H; ++c) {
            if (s->cells[c]) { table_free(s->cells[c]); free(s->cells[c]); }
        }
        free(s->cells);
    }
    table_free(&s->shared);
    free(s->cap); free(s->prefix); free(s->weights);
    free(s);
}

static int is_pow2(double x) {
    int e;
    double m = frexp(x, &e);
    return x > 0.0 && !isinf(x) && m == 0.5;
}

/* Returns 0 and *out on success; -1 on invalid arguments, -2 on allocation failure. */
OR_EXPORT int or_scenario_create(uint32_t W, uint32_t H, const uint32_t *cap, uint32_t R, const double *weights,
                                 uint32_t mode, double nu, double lambda, double dt, or_scenario **out) {
    *out = NULL;
    if (W == 0 || H == 0 || mode > 1) return -1;
    if (2ull * R + 1 > W || 2ull * R + 1 > H) return -1;
    if (!(nu > 0.0 && nu <= 1.0)) return -1;
    if (!(lambda > 0.0) || isinf(lambda) || !is_pow2(dt)) return -1;
    if (lambda * dt > 1048576.0) return -1;
    or_scenario *s = (or_scenario *)calloc(1, sizeof(or_scenario));
    if (!s) return -2;
    s->W = W; s->H = H; s->R = R; s->mode = mode;
    s->nu = nu; s->lambda = lambda; s->inv_lambda = 1.0 / lambda; s->dt = dt; s->inv_dt = 1.0 / dt;
    uint64_t cells = (uint64_t)W * H;
    uint32_t side = 2 * R + 1;
    s->cap = (uint32_t *)malloc(sizeof(uint32_t) * cells);
    s->prefix = (uint64_t *)malloc(sizeof(uint64_t) * (cells + 1));
    s->weights = (double *)malloc(sizeof(double) * side * side);
    if (!s->cap || !s->prefix || !s->weights) { or_scenario_destroy(s); return -2; }
    memcpy(s->cap, cap, sizeof(uint32_t) * cells);
    memcpy(s->weights, weights, sizeof(double) * side * side);
    for (uint32_t k = 0; k < side * side; ++k) {
        if (!(weights[k] >= 0.0) || isinf(weights[k])) { or_scenario_destroy(s); return -1; }
    }
    uint64_t acc = 0;
    uint32_t cmax = 0;
    for (uint64_t c = 0; c < cells; ++c) {
        s->prefix[c] = acc;
        acc += cap[c];
        if (cap[c] > cmax) cmax = cap[c];
        if (mode == 0 && cap[c] == 0) { or_scenario_destroy(s); return -1; }
    }
    s->prefix[cells] = acc;
    s->cmax = cmax;
    if (acc == 0 || cells * (uint64_t)cmax >= (1ull << 32)) { or_scenario_destroy(s); return -1; }
    if (mode == 0) {
        int rc = table_build(s, -1, &s->shared);
        if (rc != 0) { or_scenario_destroy(s); return rc; }
    } else {
        s->cells = (or_table **)calloc(cells, sizeof(or_table *));
        if (!s->cells) { or_scenario_destroy(s); return -2; }
        /* every habitable deme must have habitable mass in its kernel */
        for (uint64_t c = 0; c < cells; ++c) {
            if (cap[c] == 0) continue;
            int any = 0;
            int64_t x = c % W, y = c / W;
            for (uint32_t k = 0; k < side * side && !any; ++k) {
                if (!(weights[k] > 0.0)) continue;
                int64_t dx = (int64_t)(k % side) - R, dy = (int64_t)(k / side) - R;
                int64_t tx = ((x + dx) % (int64_t)W + W) % W, ty = ((y + dy) % (int64_t)H + H) % H;
                if (cap[ty * W + tx] > 0) any = 1;
            }
            if (!any) { or_scenario_destroy(s); return -1; }
        }
    }
    *out = s;
    return 0;
}

/* [impl] The spatially implicit scenario: two communities, the local one of J
 * individuals (cell 0, sample ids 0 .. J-1) and the metacommunity of J_m
 * (cell 1, ids J .. J+J_m-1).  0 < m <= 1 (with m = 0 a local lineage could
 * never speciate) and 0 < nu_m <= 1. */
OR_EXPORT int or_scenario_create_implicit(uint32_t J, uint32_t J_meta, double m, double nu_meta, double lambda,
                                          double dt, or_scenario **out) {
    *out = NULL;
    if (J == 0 || J_meta == 0 || !(m > 0.0 && m <= 1.0)) return -1;
    const uint32_t cap[2] = {J, J_meta};
    const double w = 1.0;
    int rc = or_scenario_create(2, 1, cap, 0, &w, 0, nu_meta, lambda, dt, out);
    if (rc != 0) return rc;
    (*out)->mode = 2;
    (*out)->mig = m;
    return 0;
}

OR_EXPORT uint64_t or_scenario_individuals(const or_scenario *s) { return s->prefix[(uint64_t)s->W * s->H]; }

static const or_table *table_for(or_scenario *s, uint32_t cell) {
    if (s->mode == 0) return &s->shared;
    if (!s->cells[cell]) {
        or_table *t = (or_table *)calloc(1, sizeof(or_table));
        if (!t || table_build(s, cell, t) != 0) abort();
        s->cells[cell] = t;
    }
    return s->cells[cell];
}

/* Exposed for the alias-exactness pin: copy out the table a deme samples from. */
OR_EXPORT uint32_t or_scenario_table(or_scenario *s, uint32_t cell, double *prob, uint32_t *alias, uint32_t *kidx,
                                     uint32_t cap_entries) {
    const or_table *t = table_for(s, cell);
    if (t->n <= cap_entries) {
        memcpy(prob, t->prob, sizeof(double) * t->n);
        memcpy(alias, t->alias, sizeof(uint32_t) * t->n);
        memcpy(kidx, t->kidx, sizeof(uint32_t) * t->n);
    }
    return t->n;
}

/* Dense sample id n -> indexed location (cell, deme index) -> loc = cell*Cmax + i. */
static uint32_t sample_location(const or_scenario *s, uint64_t n) {
    uint64_t lo = 0, hi = (uint64_t)s->W * s->H; /* find last c with prefix[c] <= n */
    while (hi - lo > 1) {
        uint64_t mid = lo + (hi - lo) / 2;
        if (s->prefix[mid] <= n) lo = mid;
        else hi = mid;
    }
    /* lo is the last cell with prefix[lo] <= n; since prefix[lo + 1] > n, cap[lo] > 0 */
    return (uint32_t)(lo * s->cmax + (n - s->prefix[lo]));
}

/* ------------------------------------------------------------------------- */
/* [ind] Aligning the RNGs + memoryless sums of exponentials.  Time grows    */
/* into the past from 0; interval k is [k dt, (k+1) dt).  From t_last in     */
/* interval k: prime on (loc, k), start at k dt and add Exp(lambda) draws    */
/* X_j = -log(U_j) / lambda (inverse transform, [dist]); a sum that reaches  */
/* (k+1) dt leaves the interval, so restart at (k+1) dt primed on k+1; the   */
/* first sum strictly beyond t_last is the next event time.                  */
/* ------------------------------------------------------------------------- */
static uint64_t interval_draw(uint64_t seed, uint32_t loc, uint64_t k, uint32_t j) {
    uint64_t a, b;
    hash_block(seed, loc, k, DOM_INTERVAL, j >> 1, &a, &b);
    return (j & 1u) ? b : a;
}

/* [hppp] The events of interval k at loc are a Poisson(mu = lambda dt)    */
/* number of points, uniform in [k dt, (k+1) dt): draw 0 of the interval's  */
/* stream gives the count by inverting the Poisson cdf with a linear search  */
/* (p_0 = exp(-mu), p_n = p_{n-1} mu / n, stop at the first n whose         */
/* cumulative sum reaches u; also stop if p_n underflows to 0), draws        */
/* 1 .. N place the points at k dt + U(r) dt.  The next event after t_last  */
/* is the smallest point beyond it; an interval without one moves the        */
/* search to interval k+1.  Needs mu <= 700 so that exp(-mu) is normal.      */
/* The count itself: inversion of the Poisson cdf by sequential search         */
/* (Devroye 1986, Non-Uniform Random Variate Generation, ch. X.3): the       */
/* smallest n with u <= F(n) = sum_{j<=n} p_j, each term from the one before  */
/* by one binary64 division and one product, the sum left to right.          */
static uint32_t poisson_count(const or_scenario *s, double u) {
    uint32_t n;
    double term = s->p0, cdf = s->p0;
    for (n = 0; u > cdf && term > 0.0;) {
        ++n;
        term *= s->mu / (double)n;
        cdf += term;
    }
    return n;
}

static double next_event_time_poisson(const or_scenario *s, uint64_t seed, uint32_t loc, double t_last) {
    uint64_t k = (uint64_t)floor(t_last * s->inv_dt);
    for (;;) {
        const double start = (double)k * s->dt;
        const uint32_t n = poisson_count(s, u53(interval_draw(seed, loc, k, 0)));
        double best = INFINITY;
        for (uint32_t i = 1; i <= n; ++i) {
            const double t = start + u53(interval_draw(seed, loc, k, i)) * s->dt;
            if (t > t_last && t < best) best = t;
        }
        if (best < INFINITY) return best;
        k = k + 1;
    }
}

/* Switches the scenario's event-time sampler (0 or 1, [hppp]); -1 if the   */
/* sampler is unknown or lambda * dt > 700 for sampler 1.                    */
OR_EXPORT int or_scenario_set_sampler(or_scenario *s, uint32_t sampler) {
    if (sampler > 1) return -1;
    const double mu = s->lambda * s->dt; /* exact: dt is a power of two */
    if (sampler == 1 && !(mu <= 700.0)) return -1;
    s->sampler = sampler;
    s->mu = mu;
    s->p0 = exp(-mu);
    return 0;
}

/* [prot] Protracted speciation: a speciation takes tau generations to    */
/* complete, so a speciation draw at an event less than tau generations     */
/* before the present is ignored and that event is an ordinary dispersal.  */
/* A generation is one mean lifetime, 1/lambda time units, so an event at   */
/* time t is lambda * t generations old.  -1 unless tau is finite, >= 0.    */
OR_EXPORT int or_scenario_set_protracted(or_scenario *s, double tau) {
    if (!(tau >= 0.0) || isinf(tau)) return -1;
    s->tau = tau;
    return 0;
}

/* Whether a speciation draw at time t counts ([prot]). */
static int speciation_counts(const or_scenario *s, double t) {
    return !(s->lambda * t < s->tau);
}

OR_EXPORT double or_next_event_time(const or_scenario *s, uint64_t seed, uint32_t loc, double t_last) {
    if (s->sampler == 1) return next_event_time_poisson(s, seed, loc, t_last);
    uint64_t k = (uint64_t)floor(t_last * s->inv_dt);
    for (;;) {
        double e = (double)k * s->dt;
        double end = (double)(k + 1) * s->dt;
        for (uint32_t j = 0;; ++j) {
            double x = (-or_log(u53_open0(interval_draw(seed, loc, k, j)))) * s->inv_lambda;
            e = e + x;
            if (e >= end) break;
            if (e > t_last) return e;
        }
        k = k + 1;
    }
}

/* [ind] Summary: at the event (loc, t) prime on (loc, t); speciate iff      */
/* U(r0) < nu (and the event is at least tau generations old, [prot]); else */
/* disperse: alias column from r1, alias coin from r2, the torus offset,    */
/* then a uniform deme index from r3 ([comp] coalescence       */
/* sampler).  Returns 1 on speciation (species id in *species), else 0 and   */
/* the new location in *loc.                                                  */
static int commit_event(or_scenario *s, uint64_t seed, uint32_t *loc, double t, uint64_t *species,
                        int32_t *dx_out, int32_t *dy_out) {
    uint64_t r0, r1, r2, r3;
    uint64_t tb = f64_bits(t);
    hash_block(seed, *loc, tb, DOM_EVENT, 0, &r0, &r1);
    if (s->mode == 2) {
        /* [impl] cell 0 is the local community, cell 1 the metacommunity: only the latter
         * speciates (r0); a local event migrates with probability m (r1); the deme index
         * is uniform over the target community (r3). */
        const uint32_t cell = *loc / s->cmax;
        if (cell == 1 && speciation_counts(s, t) && u53(r0) < s->nu) {
            uint64_t a, b;
            hash_block(seed, *loc, tb, DOM_SPECIES, 0, &a, &b);
            *species = a;
            return 1;
        }
        hash_block(seed, *loc, tb, DOM_EVENT, 1, &r2, &r3);
        const uint32_t target = (cell == 0 && u53(r1) < s->mig) ? 1u : cell;
        *loc = target * s->cmax + mulhi64_u32(r3, s->cap[target]);
        if (dx_out) *dx_out = 0;
        if (dy_out) *dy_out = 0;
        return 0;
    }
    if (speciation_counts(s, t) && u53(r0) < s->nu) {
        uint64_t a, b;
        hash_block(seed, *loc, tb, DOM_SPECIES, 0, &a, &b);
        *species = a;
        return 1;
    }
    hash_block(seed, *loc, tb, DOM_EVENT, 1, &r2, &r3);
    uint32_t cell = *loc / s->cmax;
    const or_table *tab = table_for(s, cell);
    uint32_t col = mulhi64_u32(r1, tab->n);
    uint32_t entry = (u53(r2) < tab->prob[col]) ? col : tab->alias[col];
    uint32_t side = 2 * s->R + 1;
    int64_t dx = (int64_t)(tab->kidx[entry] % side) - (int64_t)s->R;
    int64_t dy = (int64_t)(tab->kidx[entry] / side) - (int64_t)s->R;
    int64_t x = cell % s->W, y = cell / s->W;
    int64_t tx = x + dx, ty = y + dy;
    if (tx < 0) tx += s->W;
    if (tx >= (int64_t)s->W) tx -= s->W;
    if (ty < 0) ty += s->H;
    if (ty >= (int64_t)s->H) ty -= s->H;
    uint32_t target = (uint32_t)(ty * s->W + tx);
    uint32_t i = mulhi64_u32(r3, s->cap[target]);
    *loc = target * s->cmax + i;
    if (dx_out) *dx_out = (int32_t)dx;
    if (dy_out) *dy_out = (int32_t)dy;
    return 0;
}

/* ------------------------------------------------------------------------- */
/* The plain definition: each sample traced on its own until it speciates    */
/* ([ind] Summary loop); no deduplication at all.                             */
/* ------------------------------------------------------------------------- */
OR_EXPORT int or_simulate_naive(or_scenario *s, uint64_t seed, const uint64_t *samples, uint64_t n,
                                uint64_t *species, double *t_spec, uint64_t *events) {
    uint64_t N = or_scenario_individuals(s);
    for (uint64_t q = 0; q < n; ++q)
        if (samples[q] >= N) return -1;
    for (uint64_t q = 0; q < n; ++q) {
        uint32_t loc = sample_location(s, samples[q]);
        double t = or_next_event_time(s, seed, loc, 0.0);
        uint64_t ev = 0, sp = 0;
        for (;;) {
            ++ev;
            if (commit_event(s, seed, &loc, t, &sp, NULL, NULL)) break;
            t = or_next_event_time(s, seed, loc, t);
        }
        species[q] = sp;
        if (t_spec) t_spec[q] = t;
        if (events) events[q] = ev;
    }
    return 0;
}

/* Event trace of one sample for the statistical pins: event times, the      */
/* location each event happens at, and the realised (dx, dy) of dispersals.  */
/* Returns the number of events written (the last one is the speciation if   */
/* it fits and *done is set).                                                 */
OR_EXPORT uint64_t or_trace(or_scenario *s, uint64_t seed, uint64_t sample, uint64_t max_events, double *times,
                            uint32_t *locs, int32_t *dxs, int32_t *dys, int *done) {
    uint32_t loc = sample_location(s, sample);
    double t = or_next_event_time(s, seed, loc, 0.0);
    uint64_t n = 0, sp = 0;
    *done = 0;
    while (n < max_events) {
        times[n] = t;
        locs[n] = loc;
        int32_t dx = 0, dy = 0;
        int stop = commit_event(s, seed, &loc, t, &sp, &dx, &dy);
        dxs[n] = dx;
        dys[n] = dy;
        ++n;
        if (stop) { *done = 1; break; }
        t = or_next_event_time(s, seed, loc, t);
    }
    return n;
}

/* ------------------------------------------------------------------------- */
/* The culled form ([dedup], water level): all live lineages advance to a    */
/* common horizon W_r = r * dW; a lineage whose next event lies beyond W_r   */
/* waits.  The future of a lineage is a function of (location, next event    */
/* time) alone, so lineages sharing that pair are merged: sort by            */
/* (loc, bits(t_next), id), keep the first of each run, point the others at  */
/* it.  Species per sample follow the merge pointers to the representative.  */
/* Output is identical to or_simulate_naive for every dW.                     */
/* ------------------------------------------------------------------------- */
typedef struct {
    uint32_t loc;
    uint64_t tb;
    uint64_t id;
} live_rec;

static int live_cmp(const void *pa, const void *pb) {
    const live_rec *a = (const live_rec *)pa, *b = (const live_rec *)pb;
    if (a->loc != b->loc) return a->loc < b->loc ? -1 : 1;
    if (a->tb != b->tb) return a->tb < b->tb ? -1 : 1;
    if (a->id != b->id) return a->id < b->id ? -1 : 1;
    return 0;
}

OR_EXPORT int or_simulate_culled(or_scenario *s, uint64_t seed, const uint64_t *samples, uint64_t n, double dW,
                                 uint64_t *species, uint64_t *events_out, uint64_t *rounds_out) {
    uint64_t N = or_scenario_individuals(s);
    if (!(dW > 0.0)) return -1;
    for (uint64_t q = 0; q < n; ++q)
        if (samples[q] >= N) return -1;
    uint64_t *parent = (uint64_t *)malloc(sizeof(uint64_t) * (n ? n : 1));
    uint64_t *sp = (uint64_t *)calloc(n ? n : 1, sizeof(uint64_t));
    uint32_t *loc = (uint32_t *)malloc(sizeof(uint32_t) * (n ? n : 1));
    double *tn = (double *)malloc(sizeof(double) * (n ? n : 1));
    live_rec *live = (live_rec *)malloc(sizeof(live_rec) * (n ? n : 1));
    if (!parent || !sp || !loc || !tn || !live) {
        free(parent); free(sp); free(loc); free(tn); free(live);
        return -2;
    }
    uint64_t nlive = 0, events = 0, rounds = 0;
    for (uint64_t q = 0; q < n; ++q) {
        parent[q] = q;
        loc[q] = sample_location(s, samples[q]);
        tn[q] = or_next_event_time(s, seed, loc[q], 0.0);
        live[nlive].id = q;
        ++nlive;
    }
    for (uint64_t r = 1; nlive > 0; ++r) {
        double horizon = (double)r * dW;
        uint64_t keep = 0;
        for (uint64_t a = 0; a < nlive; ++a) {
            uint64_t id = live[a].id;
            int gone = 0;
            while (tn[id] <= horizon) {
                ++events;
                if (commit_event(s, seed, &loc[id], tn[id], &sp[id], NULL, NULL)) { gone = 1; break; }
                tn[id] = or_next_event_time(s, seed, loc[id], tn[id]);
            }
            if (!gone) {
                live[keep].id = id;
                live[keep].loc = loc[id];
                live[keep].tb = f64_bits(tn[id]);
                ++keep;
            }
        }
        qsort(live, keep, sizeof(live_rec), live_cmp);
        uint64_t m = 0;
        for (uint64_t a = 0; a < keep; ++a) {
            if (m > 0 && live[a].loc == live[m - 1].loc && live[a].tb == live[m - 1].tb) {
                parent[live[a].id] = live[m - 1].id;
            } else {
                live[m++] = live[a];
            }
        }
        nlive = m;
        rounds = r;
    }
    for (uint64_t q = 0; q < n; ++q) {
        uint64_t x = q;
        while (parent[x] != x) x = parent[x];
        species[q] = sp[x];
    }
    if (events_out) *events_out = events;
    if (rounds_out) *rounds_out = rounds;
    free(parent); free(sp); free(loc); free(tn); free(live);
    return 0;
}

/* Species richness = number of distinct species identities among the samples
 * (background section on the coalescence simulation: one new species per
 * observed speciation event).  Plain definition: sort a copy, count runs. */
static int u64_cmp(const void *pa, const void *pb) {
    uint64_t a = *(const uint64_t *)pa, b = *(const uint64_t *)pb;
    return a < b ? -1 : (a > b ? 1 : 0);
}

OR_EXPORT uint64_t or_richness(const uint64_t *species, uint64_t n) {
    if (n == 0) return 0;
    uint64_t *c = (uint64_t *)malloc(sizeof(uint64_t) * n);
    if (!c) abort();
    memcpy(c, species, sizeof(uint64_t) * n);
    qsort(c, n, sizeof(uint64_t), u64_cmp);
    uint64_t k = 1;
    for (uint64_t i = 1; i < n; ++i)
        if (c[i] != c[i - 1]) ++k;
    free(c);
    return k;
}

/* Species identity of a speciation event at (loc, t): first word pair of the
 * species-domain block.  Exposed so tests can rebuild an id from a trace. */
OR_EXPORT uint64_t or_species_id(uint64_t seed, uint32_t loc, double t) {
    uint64_t a, b;
    hash_block(seed, loc, f64_bits(t), DOM_SPECIES, 0, &a, &b);
    return a;
}

OR_EXPORT uint32_t or_sample_location(const or_scenario *s, uint64_t sample) { return sample_location(s, sample); }
OR_EXPORT uint32_t or_scenario_cmax(const or_scenario *s) { return s->cmax; }

/* ------------------------------------------------------------------------- */
/* [evs] The event stream, from its definition: every sample's lineage is    */
/* traced alone to its speciation and every event it goes through is listed  */
/* as (event time t, prior event time, origin location, outcome: the new     */
/* location or OR_EVENT_SPECIATION); the prior event time of a sample's      */
/* first event is 0, the present.  Sorted by event time, then origin, then   */
/* prior event time, the copies of one event made by lineages that share it  */
/* are adjacent.  The reduced stream keeps each event once, with the         */
/* smallest prior event time of its copies (the parent's); every further     */
/* distinct prior event time among the copies is a coalescence: a lineage   */
/* that arrived at the origin at that time found it occupied, by the lineage  */
/* that arrived first.  Coalescences are listed as (time, parent's arrival,  */
/* location) sorted by time, then location, then parent's arrival.           */
/* Returns the counts; at most *_cap records are written to each output.     */
/* -1 for an invalid sample id.                                               */
/* ------------------------------------------------------------------------- */
#define OR_EVENT_SPECIATION 0xFFFFFFFFu

typedef struct {
    double t, prior;
    uint32_t from, to;
} or_ev;

typedef struct {
    double t, parent;
    uint32_t loc;
} or_co;

static int f64_cmp(double a, double b) { return a < b ? -1 : (a > b ? 1 : 0); }
static int u32_cmp(uint32_t a, uint32_t b) { return a < b ? -1 : (a > b ? 1 : 0); }

static int ev_cmp(const void *pa, const void *pb) {
    const or_ev *a = (const or_ev *)pa, *b = (const or_ev *)pb;
    int c = f64_cmp(a->t, b->t);
    if (!c) c = u32_cmp(a->from, b->from);
    if (!c) c = f64_cmp(a->prior, b->prior);
    if (!c) c = u32_cmp(a->to, b->to);
    return c;
}

static int co_cmp(const void *pa, const void *pb) {
    const or_co *a = (const or_co *)pa, *b = (const or_co *)pb;
    int c = f64_cmp(a->t, b->t);
    if (!c) c = u32_cmp(a->loc, b->loc);
    if (!c) c = f64_cmp(a->parent, b->parent);
    return c;
}

OR_EXPORT int or_event_stream(or_scenario *s, uint64_t seed, const uint64_t *samples, uint64_t n, uint64_t ev_cap,
                              double *ev_t, double *ev_prior, uint32_t *ev_from, uint32_t *ev_to, uint64_t co_cap,
                              double *co_t, double *co_parent, uint32_t *co_loc, uint64_t *n_events,
                              uint64_t *n_coalescences) {
    uint64_t N = or_scenario_individuals(s);
    for (uint64_t q = 0; q < n; ++q)
        if (samples[q] >= N) return -1;
    uint64_t len = 0, cap = 1024;
    or_ev *all = (or_ev *)malloc(sizeof(or_ev) * cap);
    if (!all) abort();
    for (uint64_t q = 0; q < n; ++q) {
        uint32_t loc = sample_location(s, samples[q]);
        double prior = 0.0, t = or_next_event_time(s, seed, loc, 0.0);
        for (;;) {
            if (len == cap) {
                cap *= 2;
                all = (or_ev *)realloc(all, sizeof(or_ev) * cap);
                if (!all) abort();
            }
            uint64_t sp = 0;
            const uint32_t from = loc;
            const int stop = commit_event(s, seed, &loc, t, &sp, NULL, NULL);
            all[len].t = t;
            all[len].prior = prior;
            all[len].from = from;
            all[len].to = stop ? OR_EVENT_SPECIATION : loc;
            ++len;
            if (stop) break;
            prior = t;
            t = or_next_event_time(s, seed, loc, t);
        }
    }
    qsort(all, len, sizeof(or_ev), ev_cmp);
    uint64_t co_len = n + 1;
    or_co *co = (or_co *)malloc(sizeof(or_co) * co_len);
    if (!co) abort();
    uint64_t ne = 0, nc = 0, first = 0;
    for (uint64_t i = 0; i < len; ++i) {
        const int same_event = i > 0 && all[i].t == all[i - 1].t && all[i].from == all[i - 1].from;
        if (!same_event) {
            first = i;
            if (ne < ev_cap) {
                ev_t[ne] = all[i].t;
                ev_prior[ne] = all[i].prior;
                ev_from[ne] = all[i].from;
                ev_to[ne] = all[i].to;
            }
            ++ne;
        } else if (all[i].prior != all[i - 1].prior) {
            if (nc == co_len) {
                co_len *= 2;
                co = (or_co *)realloc(co, sizeof(or_co) * co_len);
                if (!co) abort();
            }
            co[nc].t = all[i].prior;
            co[nc].parent = all[first].prior;
            co[nc].loc = all[i].from;
            ++nc;
        }
    }
    qsort(co, nc, sizeof(or_co), co_cmp);
    for (uint64_t k = 0; k < nc && k < co_cap; ++k) {
        co_t[k] = co[k].t;
        co_parent[k] = co[k].parent;
        co_loc[k] = co[k].loc;
    }
    free(co);
    free(all);
    *n_events = ne;
    *n_coalescences = nc;
    return 0;
}

/* Outcome of the event at (loc, t) ([ind] Summary): the new location, or      */
/* OR_EVENT_SPECIATION.                                                       */
OR_EXPORT uint32_t or_event_outcome(or_scenario *s, uint64_t seed, uint32_t loc, double t) {
    uint64_t sp = 0;
    return commit_event(s, seed, &loc, t, &sp, NULL, NULL) ? OR_EVENT_SPECIATION : loc;
}

/* ------------------------------------------------------------------------- */
/* Array forms of the primitives, for comparing many inputs at once (test    */
/* infrastructure; each item is the single-item function above).            */
/* ------------------------------------------------------------------------- */
OR_EXPORT void or_philox_array(const uint32_t *ctr, const uint32_t key[2], uint64_t n, uint32_t *out) {
    for (uint64_t i = 0; i < n; ++i) or_philox4x32_10(ctr + 4 * i, key, out + 4 * i);
}

OR_EXPORT void or_log_u53o_array(const uint64_t *r, uint64_t n, double *out) {
    for (uint64_t i = 0; i < n; ++i) out[i] = or_log(u53_open0(r[i]));
}

OR_EXPORT void or_next_event_time_array(const or_scenario *s, uint64_t seed, const uint32_t *loc, const double *t,
                                        uint64_t n, double *out) {
    for (uint64_t i = 0; i < n; ++i) out[i] = or_next_event_time(s, seed, loc[i], t[i]);
}

OR_EXPORT void or_event_outcome_array(or_scenario *s, uint64_t seed, const uint32_t *loc, const double *t, uint64_t n,
                                      uint32_t *out) {
    for (uint64_t i = 0; i < n; ++i) out[i] = or_event_outcome(s, seed, loc[i], t[i]);
}
