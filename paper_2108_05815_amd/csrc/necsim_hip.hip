// necsim_hip.hip - gfx950 kernels and C ABI of libnecsim_hip: the Independent
// algorithm for neutral Moran biodiversity models (Langenstein 2021,
// arXiv 2108.05815).  The public contract is include/necsim_hip.h.
//
// Paper sections this file implements (all in the chapter "The Declaration of
// Independence" unless noted):
//   "Environmental RNG Priming"         - counter-based hash keyed on (seed, location, time)
//   "Aligning the RNGs of Colliding Individuals" and "Exponential inter-event
//   Times" (memoryless sums)            - next_event_time(), next_event_time_group(), group_step()
//   "Homogeneous Poisson Point Process" and appendix "Iterative Sampling"
//                                       - the Poisson-count sampler (poisson_interval())
//   "Summary of the Independent Algorithm" - commit_event(), disperse(), species_of(), the lane loops
//   implementation chapter, "Deduplicating Redundant Individuals" and the
//   Water-Level algorithm               - horizon rounds + (job, location, next time) hash cull
//   appendix "Sampling Probability Distributions" - 53-bit uniforms, inverse-transform Exp
//   related work "Counter-based Pseudo-Random Number Generators" - Philox4x32-10
//
// Layout: lineage state is structure-of-arrays in HBM (loc u32 and next-event
// time f64 double-buffered by round parity, parent u32, species u64, job u32,
// events u32, speciation event), touched once per lineage per round;
// everything inside a round lives in registers.  A round kernel runs a fixed
// grid over the round's queue: waves reserve chunks of it with one atomic and
// hand items to idle lanes; each lineage runs one lane (long queues) or 8
// lanes (short queues, and the solo queue of nearly finished jobs in runs of
// several jobs) until its next event lies beyond its job's horizon; a lineage
// whose (job, location, next time) another lineage already holds is merged at
// pickup; survivors are staged per wave in LDS and appended to the next queue.
// A one-thread epilogue publishes survivors and job completions to
// host-mapped memory.  Round kernels are replayed from captured HIP graphs
// while the host polls that status word.  Between rounds the workspace is a
// complete checkpoint (suspend and resume).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "necsim_hip.h"
#include "stream_sort.h"

#define NH_API extern "C" __attribute__((visibility("default")))

namespace {

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------
thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

#define HIP_TRY(expr)                                                                         \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail(NH_EDEVICE, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_),    \
                        __FILE__, __LINE__);                                                  \
    } while (0)

constexpr uint32_t kModeImplicit = 2u; // scenario mode set by nh_scenario_create_implicit
constexpr uint32_t kErrBadSample = 1u;
constexpr uint32_t kJobSentinelSpecies = 1u; // JobState.flags: a species id equal to the set's empty marker
constexpr uint32_t kJobBadSample = 2u;       // JobState.flags: a sample id was not below N
constexpr uint32_t kErrRunaway = 2u;
constexpr uint32_t kErrHashFull = 4u;
constexpr uint32_t kMaxHorizons = 1024;
constexpr double kLongRoundS = 40e-6;  // mean round time from which the host enqueues the tail round by round
constexpr uint32_t kLdsTableMax = 4096; // shared-table entries staged in LDS (64 KiB)

// ---------------------------------------------------------------------------
// Device data
// ---------------------------------------------------------------------------
// One simulate request, as the kernels see it.  Scenario constants first.
struct JobDev {
    uint64_t seed;
    uint64_t nu_thresh;      // speciation iff (r0 >> 11) < ceil(nu * 2^53)
    double inv_lambda;       // 1 / lambda
    double dt, inv_dt;       // repriming interval (power of two) and its inverse
    const uint4 *table;      // alias entries {thresh lo, thresh hi, packed offsets, 0}
    const uint32_t *row_ptr; // per-deme mode: first entry of each cell (cells + 1)
    const uint32_t *cap;     // capacity per cell
    const uint64_t *prefix;  // capacity prefix (cells + 1)
    const uint64_t *samples; // dense sample ids
    unsigned long long *species_out;
    unsigned long long *richness_out;
    unsigned long long *rich_set; // open-addressing set of species ids, rich_mask + 1 slots
    uint64_t n_individuals;
    uint32_t W, H, cmax, R;
    uint32_t mode, n_shared, cap_const, rich_mask;
    uint32_t lin_base, n, start_round;
    uint32_t caps_in_table; // per-deme entries hold both targets' capacities (every capacity < 2^16)
    // reporters (nullable): speciation event per sample, (species, samples) pairs
    uint32_t *spec_loc_out;
    double *spec_time_out;
    unsigned long long *abund_ids_out;
    uint32_t *abund_counts_out;
    uint32_t *rich_counts;   // samples per slot of rich_set (abundance reporter)
    uint64_t rich_off;       // offset of rich_set in the run's species-set area
    uint32_t sampler, sampler_pad; // NH_SAMPLER_EXP / NH_SAMPLER_POISSON
    double mu, p0;                 // Poisson sampler: lambda * dt, exp(-lambda * dt)
    uint64_t mig_thresh;           // spatially implicit: a local event migrates iff (r1 >> 11) < mig_thresh
    double tau_t;                  // protracted speciation: no speciation at events with t < tau_t
};

// Per-job counters, written by the kernels.
struct JobState {
    uint32_t remaining;   // lineages not yet retired (speciated, merged or rejected)
    uint32_t flags;       // kJobSentinelSpecies | kJobBadSample
    uint32_t done_round;
    uint32_t start_round; // round before the job's first round
    unsigned long long rich_count;
    unsigned long long events;
    unsigned long long speciated;
    unsigned long long merged;
    uint32_t solo_round;  // first round of the job's solo schedule (0: not solo)
    uint32_t solo_pad;
    double h_base;        // the job's horizon in round solo_round - 1
    uint32_t abund_n;     // abundance pairs written
    uint32_t sentinel_count; // samples whose species id equals the set's empty marker
};

// One counter of the persistent run's two-level grid barrier, on a cache line
// of its own: arrivals at the current barrier, barriers completed, and the
// next round's control words (round, main queue, solo queue, stop) published
// with the release so a waiter reads them from the line it polled.
constexpr uint32_t kBarGroup = 32;     // workgroups per first-level counter
constexpr uint32_t kMaxBarGroups = 64; // persistent grids up to 2048 workgroups
struct alignas(128) BarSlot {
    uint32_t arrived;
    uint32_t gen;
    uint32_t pub[4];
};

// Op counts of a run (Philox blocks evaluated in all domains, exponential
// waiting-time draws), spread over lines so that workgroups finishing together
// do not queue on one address.
constexpr uint32_t kOpSlots = 32;
struct alignas(128) OpSlot {
    unsigned long long philox, draws;
};

// Run control block (device memory, inside the workspace).
struct Ctl {
    uint32_t round;      // round the next round kernel runs
    uint32_t count[3];   // queue length of round r is count[r % 3]
    uint32_t cursor[3];  // work-queue cursor of round r is cursor[r % 3]
    uint32_t solo[3];    // solo-queue length of round r (multi-job runs), stored from the top of act
    uint32_t solo_cursor[3];
    uint32_t blocks_done;
    uint32_t error;
    uint32_t n_jobs;
    uint32_t ring_head;  // completions pushed (job slots whose lineages are all retired)
    uint32_t ring_pub;   // completions already copied to the host-mapped ring
    OpSlot ops[kOpSlots];            // op counts, summed over the slots: workgroup b adds to slot b % kOpSlots
    // Persistent runs (k_run): grid barrier and stop state, reset before every launch.
    uint32_t stop;                   // kStop*: why the run ended (0: running)
    uint32_t first_round;            // round the launch started with
    unsigned long long t_start;      // device wall clock when the launch started
    BarSlot top;                     // second barrier level: one arrival per group of workgroups
    BarSlot grp[kMaxBarGroups];      // first level: kBarGroup workgroups each
};

// Why a persistent run ended.
constexpr uint32_t kStopDone = 1u;      // every lineage retired
constexpr uint32_t kStopSuspended = 2u; // the round limit of the call was reached
constexpr uint32_t kStopError = 3u;     // a kernel error flag, the run's time limit or a stalled barrier
constexpr uint32_t kStopEndgame = 4u;   // few lineages are left: k_endgame walks each to its end
constexpr uint32_t kErrTimeout = 16u;   // the run exceeded its time limit
constexpr uint32_t kErrStall = 32u;     // a barrier wait exceeded its limit (workgroups not all resident)

// Lineage state.  loc/t are double-buffered by round parity: round r reads
// [r & 1] and writes survivors to [(r + 1) & 1], so the state a cull insert
// compares against never changes during the kernel that compares it.
struct Lin {
    uint32_t *loc[2];
    double *t[2];
    uint32_t *parent;
    unsigned long long *species;
    uint32_t *job;
    uint32_t *events;
    uint32_t *spec_loc;   // location and time of the lineage's speciation event
    double *spec_t;
    uint32_t *act[2];
    unsigned long long *hash;
    uint32_t hmask;
};

// Scenario constants a lane needs per event, loaded once per lineage.
struct JobView {
    uint32_t key0, key1;
    uint64_t nu_thresh;
    double inv_lambda, dt, inv_dt;
    const uint4 *table;
    const uint32_t *row_ptr;
    const uint32_t *cap;
    uint32_t W, H, cmax, R, mode, n_shared, cap_const, caps_in_table, sampler;
    double mu, p0;
    uint64_t mig_thresh;
    uint32_t cap_local, cap_meta; // spatially implicit: the two communities' sizes
    double tau_t;                 // protracted speciation threshold time
    uint32_t lds_base;            // first entry of the table's LDS copy (kLds forms)
};

// Op counters of one lane (summed per wave at the end of a kernel).
struct Counters {
    uint32_t philox = 0, draws = 0;
};

__device__ __forceinline__ JobView load_view(const JobDev *__restrict__ J) {
    JobView v;
    v.key0 = (uint32_t)J->seed;
    v.key1 = (uint32_t)(J->seed >> 32);
    v.nu_thresh = J->nu_thresh;
    v.inv_lambda = J->inv_lambda;
    v.dt = J->dt;
    v.inv_dt = J->inv_dt;
    v.table = J->table;
    v.row_ptr = J->row_ptr;
    v.cap = J->cap;
    v.W = J->W;
    v.H = J->H;
    v.cmax = J->cmax;
    v.R = J->R;
    v.mode = J->mode;
    v.n_shared = J->n_shared;
    v.cap_const = J->cap_const;
    v.caps_in_table = J->caps_in_table;
    v.sampler = J->sampler;
    v.mu = J->mu;
    v.p0 = J->p0;
    v.mig_thresh = J->mig_thresh;
    v.tau_t = J->tau_t;
    v.lds_base = 0;
    if (J->mode == kModeImplicit) {
        v.cap_local = J->cap[0];
        v.cap_meta = J->cap[1];
    }
    return v;
}

// Philox4x32-10 (Salmon et al. 2011): 10 rounds, two 32x32->64 products per
// round; the Weyl key bump after the last round is never used.  Each
// three-way xor is one gfx950 bitop3 instruction (truth table 0x96).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ void philox10(uint32_t &c0, uint32_t &c1, uint32_t &c2, uint32_t &c3, uint32_t k0,
                                         uint32_t k1) {
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        const uint32_t n0 = xor3((uint32_t)(p1 >> 32), c1, k0);
        const uint32_t n2 = xor3((uint32_t)(p0 >> 32), c3, k1);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// The search block of the group step, Philox4x32-10 of the counter
// (loc, kk, 0, c3) under (k0, k1), as one draw: words 1:0, or words 3:2 when
// second.  The location is known last; n0 = kk ^ k0 (the first round's word 0,
// its other product being of 0) and m = 0xD2511F53 * n0 (the second round's
// first product) do not depend on it and come from the caller, computed before
// the event's dispersal.  The last round forms only the product the draw needs.
__device__ __forceinline__ uint64_t philox10_late_loc(uint32_t loc, uint32_t n0, uint64_t m, uint32_t c3,
                                                      uint32_t k0, uint32_t k1, bool second) {
    const uint64_t pa = (uint64_t)0xD2511F53u * loc;
    uint32_t c0 = n0, c1 = 0u, c2 = xor3((uint32_t)(pa >> 32), c3, k1);
    c3 = (uint32_t)pa;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
    {
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0b = xor3((uint32_t)(p1 >> 32), c1, k0);
        const uint32_t n2b = xor3((uint32_t)(m >> 32), c3, k1);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)m;
        c0 = n0b;
        c2 = n2b;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
#pragma unroll
    for (int i = 2; i < 9; ++i) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        const uint32_t n0b = xor3((uint32_t)(p1 >> 32), c1, k0);
        const uint32_t n2b = xor3((uint32_t)(p0 >> 32), c3, k1);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0b;
        c2 = n2b;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    const uint32_t a = second ? c0 : c2, mul = second ? 0xD2511F53u : 0xCD9E8D57u;
    const uint32_t xo = second ? c3 : c1, kx = second ? k1 : k0;
    const uint64_t p = (uint64_t)mul * a;
    return ((uint64_t)(uint32_t)p << 32) | xor3((uint32_t)(p >> 32), xo, kx);
}

// Dynamic LDS: the shared dispersal table of a single-job round kernel.
extern __shared__ uint4 nh_lds_table[];

// floor(r * n / 2^64) for n < 2^32, from two 32x32->64 products.
__device__ __forceinline__ uint32_t mulhi_index(uint64_t r, uint32_t n) {
    const uint64_t lo = (uint64_t)(uint32_t)r * n;
    const uint64_t hi = (uint64_t)(uint32_t)(r >> 32) * n + (lo >> 32);
    return (uint32_t)(hi >> 32);
}

// log(u) for u = ((r >> 11) + 1) * 2^-53 in (0, 1].  The decomposition
// u = m * 2^e with m in [sqrt(1/2), sqrt(2)) is done on the integer q, then
// log(m) = 2 atanh(s), s = (m - 1) / (m + 1), with the series
// 2s (1 + z/3 + ... + z^10/21), z = s^2, and log(u) = e ln2 + log(m) with ln2
// split into a 32-bit head and a tail.  Every floating-point operation is
// spelled out (no contraction), so the result is the same bits on any
// IEEE-754 binary64 machine that evaluates the same sequence.
__device__ __forceinline__ double log_u53o(uint64_t r) {
    const uint64_t q = (r >> 11) + 1ull;          // 1 .. 2^53
    const int nb = 64 - __clzll((long long)q);     // bit length, 1 .. 54
    const uint64_t frac = ((q << (64 - nb)) << 1) >> 12; // 52 bits after the leading one
    int e = nb - 53;
    uint64_t mbits;
    if (frac < 0x6a09e667f3bcdull) {               // m = q / 2^nb < sqrt(1/2): use 2m
        mbits = (1023ull << 52) | frac;
        e -= 1;
    } else {
        mbits = (1022ull << 52) | frac;
    }
    const double m = __longlong_as_double((long long)mbits);
    const double f = m - 1.0;
    const double s = f / (2.0 + f);
    const double z = s * s;
    double p = 1.0 / 21.0;
    p = __builtin_fma(p, z, 1.0 / 19.0);
    p = __builtin_fma(p, z, 1.0 / 17.0);
    p = __builtin_fma(p, z, 1.0 / 15.0);
    p = __builtin_fma(p, z, 1.0 / 13.0);
    p = __builtin_fma(p, z, 1.0 / 11.0);
    p = __builtin_fma(p, z, 1.0 / 9.0);
    p = __builtin_fma(p, z, 1.0 / 7.0);
    p = __builtin_fma(p, z, 1.0 / 5.0);
    p = __builtin_fma(p, z, 1.0 / 3.0);
    p = p * z;
    const double two_s = s + s;
    const double log_m = __builtin_fma(two_s, p, two_s);
    const double de = (double)e;
    return __builtin_fma(de, 0x1.62e42fee00000p-1, __builtin_fma(de, 0x1.a39ef35793c76p-33, log_m));
}

// Next event time after t_last at location loc: interval k = [k dt, (k+1) dt)
// is primed on (loc, k); Exp(lambda) draws are summed from k dt; a sum that
// reaches (k+1) dt moves the search to interval k+1 (restarting at its start);
// the first sum strictly beyond t_last is the answer.  Returns a negative
// value (and flags the run) only if the search runs away, which needs a
// broken scenario.
__device__ __forceinline__ double next_event_time_wide(const JobView &v, uint32_t loc, double t_last, uint32_t *err,
                                                       Counters &cnt) {
    uint64_t k = (uint64_t)floor(t_last * v.inv_dt);
    double e = (double)k * v.dt;
    double end = (double)(k + 1) * v.dt;
    uint32_t j = 0;
    uint64_t second = 0;
    for (uint32_t guard = 0; guard < (1u << 24); ++guard) {
        uint64_t r;
        if ((j & 1u) == 0u) {
            uint32_t c0 = loc, c1 = (uint32_t)k, c2 = (uint32_t)(k >> 32), c3 = j >> 1; // domain 0
            philox10(c0, c1, c2, c3, v.key0, v.key1);
            ++cnt.philox;
            r = ((uint64_t)c1 << 32) | c0;
            second = ((uint64_t)c3 << 32) | c2;
        } else {
            r = second;
        }
        const double x = (-log_u53o(r)) * v.inv_lambda;
        ++cnt.draws;
        e = e + x;
        if (e >= end) {
            k += 1;
            e = (double)k * v.dt;
            end = (double)(k + 1) * v.dt;
            j = 0;
            continue;
        }
        if (e > t_last) return e;
        ++j;
    }
    atomicOr(err, kErrRunaway);
    return -1.0;
}

// The Poisson sampler (section "Homogeneous Poisson Point Process"): the
// events of interval k at loc are a Poisson(mu = lambda dt) count, from draw 0
// of the interval's stream by a linear search over the Poisson cdf (p_0 =
// exp(-mu), p_n = p_{n-1} mu / n, the first n whose cumulative sum reaches u;
// also stop if p_n underflows), placed at k dt + U dt by draws 1 .. n.  The
// next event after t_last is the smallest of them beyond it; an interval
// without one moves the search to interval k+1.
__device__ __forceinline__ double u53(uint64_t r) { return (double)(r >> 11) * 0x1.0p-53; }

// Inversion of the Poisson cdf by sequential search (Devroye 1986, Non-Uniform
// Random Variate Generation, ch. X.3): the smallest n with u <= F(n).
__device__ __forceinline__ uint32_t poisson_count(const JobView &v, double u) {
    uint32_t n;
    double term = v.p0, cdf = v.p0;
    for (n = 0; u > cdf && term > 0.0;) {
        ++n;
        term *= v.mu / (double)n; // one division, one product, as the definition orders them
        cdf += term;
    }
    return n;
}

// Smallest event of interval k beyond t_last, or +inf; draws and blocks
// receive what the interval consumes in the definition (draw 0 and points
// 1 .. n, two draws per Philox call).  The first two calls are evaluated side
// by side, so counts up to 3 need no further call in sequence.
__device__ __forceinline__ double poisson_interval(const JobView &v, uint32_t loc, uint64_t k, double t_last,
                                                   uint32_t &draws, uint32_t &blocks) {
    const double start = (double)k * v.dt;
    uint32_t a0 = loc, a1 = (uint32_t)k, a2 = (uint32_t)(k >> 32), a3 = 0; // domain 0, call 0
    uint32_t b0 = loc, b1 = (uint32_t)k, b2 = (uint32_t)(k >> 32), b3 = 1; // call 1
    philox10(a0, a1, a2, a3, v.key0, v.key1);
    philox10(b0, b1, b2, b3, v.key0, v.key1);
    const uint32_t n = poisson_count(v, u53(((uint64_t)a1 << 32) | a0));
    const double t1 = start + u53(((uint64_t)a3 << 32) | a2) * v.dt;
    const double t2 = start + u53(((uint64_t)b1 << 32) | b0) * v.dt;
    const double t3 = start + u53(((uint64_t)b3 << 32) | b2) * v.dt;
    double best = __builtin_inf();
    best = (n >= 1u && t1 > t_last) ? t1 : best;
    best = (n >= 2u && t2 > t_last && t2 < best) ? t2 : best;
    best = (n >= 3u && t3 > t_last && t3 < best) ? t3 : best;
    uint64_t second = 0;
    for (uint32_t i = 4; i <= n; ++i) { // rare: more than three events in the interval
        uint64_t r = second;
        if ((i & 1u) == 0u) { // draw i opens call i / 2
            uint32_t d0 = loc, d1 = (uint32_t)k, d2 = (uint32_t)(k >> 32), d3 = i >> 1;
            philox10(d0, d1, d2, d3, v.key0, v.key1);
            r = ((uint64_t)d1 << 32) | d0;
            second = ((uint64_t)d3 << 32) | d2;
        }
        const double t = start + u53(r) * v.dt;
        if (t > t_last && t < best) best = t;
    }
    draws = 1u + n;
    blocks = (n >> 1) + 1u;
    return best;
}

__device__ __forceinline__ double next_event_time_poisson(const JobView &v, uint32_t loc, double t_last,
                                                          uint32_t *err, Counters &cnt) {
    uint64_t k = (uint64_t)floor(t_last * v.inv_dt);
    for (uint32_t guard = 0; guard < (1u << 24); ++guard, ++k) {
        uint32_t draws, blocks;
        const double e = poisson_interval(v, loc, k, t_last, draws, blocks);
        cnt.draws += draws;
        cnt.philox += blocks;
        if (e < __builtin_inf()) return e;
    }
    atomicOr(err, kErrRunaway);
    return -1.0;
}

// The same search for interval indices below 2^31 (every time below 2^31 dt):
// the index is a u32, so its conversions are single instructions, and the
// interval end is start + dt, which equals (k + 1) dt exactly because dt is a
// power of two.  Bit-identical to next_event_time_wide.
__device__ __forceinline__ double next_event_time(const JobView &v, uint32_t loc, double t_last, uint32_t *err,
                                                  Counters &cnt) {
    if (v.sampler == NH_SAMPLER_POISSON) return next_event_time_poisson(v, loc, t_last, err, cnt);
    const double kf = floor(t_last * v.inv_dt);
    if (!(kf < 2147483648.0)) return next_event_time_wide(v, loc, t_last, err, cnt);
    uint32_t k = (uint32_t)kf;
    double e = (double)k * v.dt;
    double end = e + v.dt;
    uint32_t j = 0;
    uint64_t second = 0;
    for (uint32_t guard = 0; guard < (1u << 24); ++guard) {
        uint64_t r;
        if ((j & 1u) == 0u) {
            uint32_t c0 = loc, c1 = k, c2 = 0, c3 = j >> 1; // domain 0
            philox10(c0, c1, c2, c3, v.key0, v.key1);
            ++cnt.philox;
            r = ((uint64_t)c1 << 32) | c0;
            second = ((uint64_t)c3 << 32) | c2;
        } else {
            r = second;
        }
        const double x = (-log_u53o(r)) * v.inv_lambda;
        ++cnt.draws;
        e = e + x;
        if (e >= end) {
            k += 1;
            e = end;
            end = e + v.dt;
            j = 0;
            continue;
        }
        if (e > t_last) return e;
        ++j;
    }
    atomicOr(err, kErrRunaway);
    return -1.0;
}

// Lineage position in registers: torus coordinates, deme index and the packed
// location loc = (y W + x) * cmax + i that keys the hash.
struct Pos {
    uint32_t x, y, i, loc;
};

__device__ __forceinline__ Pos pos_from_loc(const JobView &v, uint32_t loc) {
    Pos p;
    const uint32_t cell = loc / v.cmax;
    p.i = loc - cell * v.cmax;
    p.y = cell / v.W;
    p.x = cell - p.y * v.W;
    p.loc = loc;
    return p;
}

// Speciation threshold of the event at (p, t): nu, except in the local community
// of a spatially implicit scenario, which never speciates, and at events younger
// than the protracted-speciation time (appendix "Protracted Speciation": a
// speciation completes only tau generations after it happens, so going back
// from the present the draws of the first tau generations are ignored and the
// event disperses).  tau_t is the smallest time with lambda * tau_t >= tau in
// binary64, so t < tau_t exactly when lambda * t < tau.
template <bool kLds>
__device__ __forceinline__ uint64_t speciation_threshold(const JobView &v, const Pos &p, double t) {
    const bool young = t < v.tau_t;
    if (kLds) return young ? 0ull : v.nu_thresh; // an LDS-staged table means the shared mode
    return (young | (v.mode == kModeImplicit && p.x == 0u)) ? 0ull : v.nu_thresh;
}

// Species id of a lineage that speciates at (loc, t): the species domain of
// the hash, keyed like the event draws.
__device__ __forceinline__ uint64_t species_of(const JobView &v, uint32_t loc, double t) {
    const uint64_t tb = (uint64_t)__double_as_longlong(t);
    uint32_t s0 = loc, s1 = (uint32_t)tb, s2 = (uint32_t)(tb >> 32), s3 = (2u << 30);
    philox10(s0, s1, s2, s3, v.key0, v.key1);
    return ((uint64_t)s1 << 32) | s0;
}

// The alias-table row of the lineage's cell: its first and one-past-last
// entries.  The row pointers depend on the cell alone, so a caller issues this
// before the event's hash and the loads overlap it: they are unconditional
// (every scenario has row pointers; a shared table is the single row {0, n},
// also read by the spatially implicit scenario, whose dispersal ignores it),
// and a scheduling barrier keeps them ahead of the hash, whose first use of
// them comes after it.
// kUni: the wave works on one lineage (every active lane holds the same
// values), so the table is read through the scalar data cache: the first
// active lane's address, read as constant memory (tables never change while
// kernels run).
typedef const __attribute__((address_space(4))) uint32_t *ConstU32;

__device__ __forceinline__ ConstU32 uniform_ptr(const void *p) {
    const uint64_t b = (uint64_t)p;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)b);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
    return (ConstU32)(((uint64_t)hi << 32) | lo);
}

template <bool kLds, bool kUni = false>
__device__ __forceinline__ uint2 table_row(const JobView &v, const Pos &p) {
    if (kLds) return make_uint2(v.lds_base, v.lds_base + v.n_shared);
    const uint32_t cell = v.mode == NH_DISPERSAL_PER_DEME ? p.y * v.W + p.x : 0u;
    if (kUni) {
        const ConstU32 rp = uniform_ptr(v.row_ptr);
        const uint32_t c = (uint32_t)__builtin_amdgcn_readfirstlane(cell);
        const uint2 row = make_uint2(rp[c], rp[c + 1]);
        __builtin_amdgcn_sched_barrier(0);
        return row;
    }
    const uint2 row = make_uint2(v.row_ptr[cell], v.row_ptr[cell + 1]);
    __builtin_amdgcn_sched_barrier(0);
    return row;
}

// Dispersal from the event draws: the alias column from r1, the alias coin
// from r2, the torus offset of the chosen entry, and the deme index from r3;
// row is table_row of the lineage's cell (first and one-past-last entry).  A
// table staged in LDS is always the shared one.
template <bool kLds, bool kUni = false>
__device__ __forceinline__ void disperse(const JobView &v, Pos &p, uint64_t r1, uint64_t r2, uint64_t r3,
                                         uint2 row) {
    if (!kLds && v.mode == kModeImplicit) {
        // Spatially implicit (background section "Spatially Implicit"): cell 0 is the local
        // community, cell 1 the metacommunity; a local event migrates with probability m (r1),
        // and the deme index is uniform over the target community (r3).
        const uint32_t target = (p.x == 0u && (r1 >> 11) < v.mig_thresh) ? 1u : p.x;
        p.x = target;
        p.i = mulhi_index(r3, target ? v.cap_meta : v.cap_local);
        p.loc = target * v.cmax + p.i;
        return;
    }
    const uint32_t first = row.x, n = row.y - row.x;
    const uint32_t col = mulhi_index(r1, n);
    uint4 ent;
    if (kUni) {
        const ConstU32 tp = uniform_ptr(v.table);
        const uint32_t e = 4u * (uint32_t)__builtin_amdgcn_readfirstlane(first + col);
        ent = make_uint4(tp[e], tp[e + 1], tp[e + 2], tp[e + 3]);
    } else {
        ent = kLds ? nh_lds_table[first + col] : v.table[first + col];
    }
    const uint64_t thresh = ((uint64_t)ent.y << 32) | ent.x;
    const bool primary = (r2 >> 11) < thresh;
    const uint32_t off = primary ? (ent.z & 0xFFFFu) : (ent.z >> 16);
    // Torus wrap without compares: a = x + dx + W lies in [W - R, 2W + R) because 2R + 1 <= W,
    // and of a, a - W, a - 2W (unsigned, so the ones below zero are huge) the smallest is a mod W.
    const uint32_t ax = p.x + (off & 0xFFu) + (v.W - v.R), ay = p.y + (off >> 8) + (v.H - v.R);
    const uint32_t tx = min(ax, min(ax - v.W, ax - 2u * v.W));
    const uint32_t ty = min(ay, min(ay - v.H, ay - 2u * v.H));
    const uint32_t target = ty * v.W + tx;
    const uint32_t capt = v.cap_const       ? v.cap_const
                          : v.caps_in_table ? (primary ? (ent.w & 0xFFFFu) : (ent.w >> 16))
                                            : v.cap[target];
    p.x = tx;
    p.y = ty;
    p.i = mulhi_index(r3, capt);
    p.loc = target * v.cmax + p.i;
}

// The event at (loc, t): draws r0, r1 (call 0) and r2, r3 (call 1) from the
// event domain keyed on the bits of t.  Speciation iff U(r0) < nu (the caller
// then takes the species id from species_of); otherwise the lineage disperses.
// Returns true on speciation.
template <bool kLds = false>
__device__ __forceinline__ bool commit_event(const JobView &v, Pos &p, double t, Counters &cnt) {
    const uint2 row = table_row<kLds>(v, p);
    const uint64_t tb = (uint64_t)__double_as_longlong(t);
    const uint32_t tlo = (uint32_t)tb, thi = (uint32_t)(tb >> 32);
    // Both blocks side by side (two independent chains in one lane), block 1
    // even when the lineage speciates.
    uint32_t a0 = p.loc, a1 = tlo, a2 = thi, a3 = (1u << 30);
    uint32_t b0 = p.loc, b1 = tlo, b2 = thi, b3 = (1u << 30) | 1u;
    philox10(a0, a1, a2, a3, v.key0, v.key1);
    philox10(b0, b1, b2, b3, v.key0, v.key1);
    const uint64_t r0 = ((uint64_t)a1 << 32) | a0;
    const uint64_t r1 = ((uint64_t)a3 << 32) | a2;
    const uint64_t r2 = ((uint64_t)b1 << 32) | b0;
    const uint64_t r3 = ((uint64_t)b3 << 32) | b2;
    cnt.philox += 2;
    if (__builtin_expect((r0 >> 11) < speciation_threshold<kLds>(v, p, t), 0)) return true;
    disperse<kLds>(v, p, r1, r2, r3, row);
    return false;
}

__device__ __forceinline__ uint64_t mix_key(uint32_t loc, uint64_t tb, uint32_t job) {
    uint64_t h = tb ^ ((uint64_t)loc * 0x9E3779B97F4A7C15ull) ^ ((uint64_t)job << 40);
    h ^= h >> 31;
    h *= 0xBF58476D1CE4E5B9ull;
    h ^= h >> 29;
    h *= 0x94D049BB133111EBull;
    h ^= h >> 32;
    return h;
}

// Cull insert at the start of round r, for a lineage taken from the round's
// queue with state (job, loc, t_next) = state_in[g].  Returns g if it becomes
// the representative of that state, else the representative's id.  Slots hold
// (r << 32 | lineage); a slot of an older round is empty.  Every state compared
// here was written by an earlier kernel and is read-only in this one, so the
// only synchronisation needed is the slot's own atomic.
__device__ __forceinline__ uint32_t cull_insert(const Lin &lin, const uint32_t *__restrict__ loc_in,
                                                const double *__restrict__ t_in, uint32_t r, uint32_t g,
                                                uint32_t loc, uint64_t tb, uint32_t job, uint32_t *err) {
    uint32_t idx = (uint32_t)mix_key(loc, tb, job) & lin.hmask;
    const unsigned long long mine = ((unsigned long long)r << 32) | g;
    for (uint32_t probe = 0; probe <= lin.hmask; ++probe) {
        unsigned long long cur = __hip_atomic_load(&lin.hash[idx], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        while ((uint32_t)(cur >> 32) != r) {
            if (__hip_atomic_compare_exchange_strong(&lin.hash[idx], &cur, mine, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT))
                return g;
        }
        const uint32_t owner = (uint32_t)cur;
        if (loc_in[owner] == loc && (uint64_t)__double_as_longlong(t_in[owner]) == tb && lin.job[owner] == job)
            return owner;
        idx = (idx + 1u) & lin.hmask;
    }
    atomicOr(err, kErrHashFull);
    return g;
}

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Horizon of a job's lr-th round: the host table, extended linearly by the
// table's last step beyond its end.
__device__ __forceinline__ double horizon_of(const double *__restrict__ htab, uint32_t lr) {
    if (lr < kMaxHorizons) return htab[lr];
    const double step = htab[kMaxHorizons - 1] - htab[kMaxHorizons - 2];
    return htab[kMaxHorizons - 1] + (double)(lr - (kMaxHorizons - 1)) * step;
}

// Wave sum of a u64 over all 64 lanes.
__device__ __forceinline__ unsigned long long wave_sum(unsigned long long x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

// Op counters: per-wave sums go to LDS, one global atomic per workgroup.
// Every thread of the block must call it.
__device__ __forceinline__ void flush_counters_block(Ctl *ctl, unsigned long long philox, unsigned long long draws) {
    __shared__ unsigned long long acc[2];
    if (threadIdx.x == 0) {
        acc[0] = 0;
        acc[1] = 0;
    }
    __syncthreads();
    const unsigned long long ph = wave_sum(philox), dr = wave_sum(draws);
    if (lane_id() == 0 && (ph | dr)) {
        atomicAdd(&acc[0], ph);
        atomicAdd(&acc[1], dr);
    }
    __syncthreads();
    if (threadIdx.x == 0 && (acc[0] | acc[1])) {
        OpSlot &o = ctl->ops[blockIdx.x % kOpSlots];
        atomicAdd(&o.philox, acc[0]);
        atomicAdd(&o.draws, acc[1]);
    }
}

__device__ __forceinline__ void flush_counters_block(Ctl *ctl, const Counters &c) {
    flush_counters_block(ctl, (unsigned long long)c.philox, (unsigned long long)c.draws);
}

__device__ __forceinline__ uint32_t wave_reserve(uint64_t mask, uint32_t *counter) {
    // One atomic per wave for the lanes set in mask; each lane gets base + rank.
    const uint32_t lane = lane_id();
    const int leader = __ffsll((unsigned long long)mask) - 1;
    uint32_t base = 0;
    if ((int)lane == leader) base = atomicAdd(counter, (uint32_t)__popcll(mask));
    base = __shfl(base, leader, 64);
    return base + (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
}

__device__ __forceinline__ uint64_t shfl_u64(uint64_t x, int src) {
    const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)x, src, 64);
    const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(x >> 32), src, 64);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ double shfl_f64(double x, int src) {
    return __longlong_as_double((long long)shfl_u64((uint64_t)__double_as_longlong(x), src));
}

// ---------------------------------------------------------------------------
// Cooperative forms for lineages that are few: a group of 8 lanes works on
// one lineage and evaluates the independent Philox blocks of one event side
// by side.  Results are bit-identical to the one-lane functions above.
// ---------------------------------------------------------------------------
constexpr uint32_t kGroup = 8;

// Broadcast lane J of each quad (4 lanes) to the whole quad: two DPP moves.
template <int J>
__device__ __forceinline__ double quad_bcast(double x) {
    constexpr int ctrl = J | (J << 2) | (J << 4) | (J << 6); // quad_perm [J,J,J,J]
    const uint64_t b = (uint64_t)__double_as_longlong(x);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)b, ctrl, 0xF, 0xF, true);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(b >> 32), ctrl, 0xF, 0xF, true);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Exchange a 32-bit value between the two quads of each 8-lane half row
// (lane i <-> lane 7 - i): one DPP move.
__device__ __forceinline__ uint32_t half_mirror(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x141 /* row_half_mirror */, 0xF, 0xF, true);
}

__device__ __forceinline__ double half_mirror_f64(double x) {
    const uint64_t b = (uint64_t)__double_as_longlong(x);
    const uint32_t lo = half_mirror((uint32_t)b), hi = half_mirror((uint32_t)(b >> 32));
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Next event time by a group of 8 lanes, bit-identical to next_event_time().
// First pass: lanes 0-3 take draws 0-3 of the interval k holding t_last (two
// Philox blocks, one per lane pair, and four logarithms in one pass); lanes
// 4-7 take the first draw of intervals k+1 .. k+4, which start beyond t_last,
// so that draw alone decides them (an event iff it lands before the
// interval's end).  Each quad shares its four draws by DPP and resolves its
// own part in order -- quad 0 the walk through interval k, quad 1 the lowest
// of its four intervals with an event -- and the two quads then swap outcomes
// with one more DPP move; interval k, when it decides, comes first.  Interval
// k keeps walking on its own in the rare case that four draws neither pass
// t_last nor leave it.  Later passes give one interval to each lane.
// Counters record what the one-lane search needs.
__device__ __forceinline__ double next_event_time_group(const JobView &v, uint32_t loc, double t_last, uint32_t gl,
                                                        uint32_t grp_base, uint32_t *err, Counters &cnt) {
    if (v.sampler == NH_SAMPLER_POISSON) { // every lane runs the one-lane search; lane 0 counts
        Counters dummy;
        return next_event_time_poisson(v, loc, t_last, err, gl == 0u ? cnt : dummy);
    }
    const double kf = floor(t_last * v.inv_dt);
    if (__builtin_expect(!(kf < 2147483648.0), 0)) { // every lane runs the one-lane search; lane 0 counts
        Counters dummy;
        return next_event_time_wide(v, loc, t_last, err, gl == 0u ? cnt : dummy);
    }
    uint32_t k = (uint32_t)kf;
    {
        const bool q0 = gl < 4u;
        const uint32_t kk = q0 ? k : k + (gl - 3u);
        uint32_t c0 = loc, c1 = kk, c2 = 0, c3 = q0 ? (gl >> 1) : 0u;
        philox10(c0, c1, c2, c3, v.key0, v.key1);
        const uint64_t first = ((uint64_t)c1 << 32) | c0, second = ((uint64_t)c3 << 32) | c2;
        const double x = (-log_u53o((q0 && (gl & 1u)) ? second : first)) * v.inv_lambda;
        const double x0 = quad_bcast<0>(x), x1 = quad_bcast<1>(x), x2 = quad_bcast<2>(x), x3 = quad_bcast<3>(x);
        // Interval starts and ends are exact: dt is a power of two and every index is below 2^31.
        const double s0 = (double)k * v.dt, s1 = s0 + v.dt, s2 = s1 + v.dt, s3 = s2 + v.dt, s4 = s3 + v.dt,
                     s5 = s4 + v.dt;
        // Quad 0, interval k in the one-lane order (leave on e >= end, accept on e > t_last): the partial
        // sums never decrease, so the first sum that either leaves or passes t_last decides.  Bitwise
        // operators keep the selection free of branches.
        const double e0 = s0 + x0, e1 = e0 + x1, e2 = e1 + x2, e3 = e2 + x3;
        const bool d0 = (e0 >= s1) | (e0 > t_last), d1 = (e1 >= s1) | (e1 > t_last);
        const bool d2 = (e2 >= s1) | (e2 > t_last), d3 = (e3 >= s1) | (e3 > t_last);
        double e = d0 ? e0 : (d1 ? e1 : (d2 ? e2 : e3));
        uint32_t draws_k = d0 ? 1u : (d1 ? 2u : (d2 ? 3u : 4u));
        uint32_t philox_k = (draws_k + 1u) >> 1;
        bool hit_k = d3 & (e < s1);
        if (__builtin_expect(q0 && !d3, 0)) { // four draws neither left interval k nor passed t_last
            uint64_t sec = 0;
            for (uint32_t j = 4; j < (1u << 24); ++j) {
                uint64_t r;
                if ((j & 1u) == 0u) {
                    uint32_t d0w = loc, d1w = k, d2w = 0, d3w = j >> 1;
                    philox10(d0w, d1w, d2w, d3w, v.key0, v.key1);
                    ++philox_k;
                    r = ((uint64_t)d1w << 32) | d0w;
                    sec = ((uint64_t)d3w << 32) | d2w;
                } else {
                    r = sec;
                }
                ++draws_k;
                e = e + (-log_u53o(r)) * v.inv_lambda;
                if (e >= s1) {
                    hit_k = false;
                    break;
                }
                if (e > t_last) {
                    hit_k = true;
                    break;
                }
            }
        }
        // Quad 1: the lowest of intervals k+1 .. k+4 whose first draw lands before its end.
        const double f0 = s1 + x0, f1 = s2 + x1, f2 = s3 + x2, f3 = s4 + x3;
        const bool g0 = f0 < s2, g1 = f1 < s3, g2 = f2 < s4, g3 = f3 < s5;
        const double q1_e = g0 ? f0 : (g1 ? f1 : (g2 ? f2 : f3));
        const uint32_t q1_tag = (uint32_t)(g0 | g1 | g2 | g3) | ((g0 ? 0u : (g1 ? 1u : (g2 ? 2u : 3u))) << 1);
        // Swap outcomes between the quads; a = interval k's, b = the later intervals'.
        const double my_e = q0 ? e : q1_e;
        const uint32_t my_tag = q0 ? (uint32_t)hit_k : q1_tag;
        const double o_e = half_mirror_f64(my_e);
        const uint32_t o_tag = half_mirror(my_tag);
        const uint32_t a_tag = q0 ? my_tag : o_tag, b_tag = q0 ? o_tag : my_tag;
        const double a_e = q0 ? my_e : o_e, b_e = q0 ? o_e : my_e;
        const bool a_hit = (a_tag & 1u) != 0u, b_hit = (b_tag & 1u) != 0u;
        if (gl == 0u) {
            const uint32_t later = a_hit ? 0u : (b_hit ? (b_tag >> 1) + 1u : 4u);
            cnt.philox += philox_k + later;
            cnt.draws += draws_k + later;
        }
        if (__builtin_expect(a_hit | b_hit, 1)) return a_hit ? a_e : b_e;
        k += 5u;
    }
    for (uint32_t batch = 0; batch < (1u << 20); ++batch) {
        const uint32_t kk = k + batch * kGroup + gl;
        const double start = (double)kk * v.dt;
        const double end = start + v.dt;
        uint32_t c0 = loc, c1 = kk, c2 = 0, c3 = 0;
        philox10(c0, c1, c2, c3, v.key0, v.key1);
        const double e = start + (-log_u53o(((uint64_t)c1 << 32) | c0)) * v.inv_lambda;
        const bool hit = e < end;
        const uint32_t hits = (uint32_t)((__ballot(hit) >> grp_base) & 0xFFu);
        if (gl == 0u) {
            const uint32_t used = hits ? (uint32_t)__ffs(hits) : kGroup;
            cnt.philox += used;
            cnt.draws += used;
        }
        if (hits) return shfl_f64(e, (int)(grp_base + __ffs(hits) - 1));
    }
    atomicOr(err, kErrRunaway);
    return -1.0;
}

// Swap a 32-bit value with the neighbouring lane (lane ^ 1): one DPP move.
__device__ __forceinline__ uint32_t swap_neighbour(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0xB1 /* quad_perm [1,0,3,2] */, 0xF, 0xF, true);
}

// The value of the even (odd) lane of each lane pair, in both lanes: one DPP move.
__device__ __forceinline__ uint32_t from_even(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0xA0 /* quad_perm [0,0,2,2] */, 0xF, 0xF, true);
}
__device__ __forceinline__ uint32_t from_odd(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0xF5 /* quad_perm [1,1,3,3] */, 0xF, 0xF, true);
}

// One event of a group plus the first pass of the following event-time
// search, as straight-line code with a single outcome: kStepOk (the lineage
// dispersed and t is its next event time), kStepSpeciated (t is left at the
// event; p holds the discarded dispersal, so the caller keeps the event's
// location) or kStepSlow (the lineage dispersed, t is unchanged, and the
// search must be finished by next_event_time_group: interval k needs more
// than four draws, no interval of k .. k+4 holds an event, or t is beyond the
// 32-bit interval range).  Dispersal and the search are evaluated even when
// the lineage speciates, whose outcome then discards them; every table read
// stays in bounds either way.  The search is the first pass of
// next_event_time_group, with the walk flag of quad 0 carried in bit 3 of
// its tag; counters match what the one-lane path records.
constexpr uint32_t kStepOk = 0, kStepSpeciated = 1, kStepSlow = 2;

// Sum over the 8 lanes of a group, in every lane: three DPP moves.
__device__ __forceinline__ uint32_t group_sum8(uint32_t x) {
    x += swap_neighbour(x);
    x += (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x4E /* quad_perm [2,3,0,1] */, 0xF, 0xF, true);
    return x + half_mirror(x);
}

// row is table_row of p on entry and of the moved p on return: the next
// event's row pointers are requested as soon as the dispersal is known, so
// their loads overlap the search and the next event's hash.
template <bool kLds, bool kUni = false>
__device__ __forceinline__ uint32_t group_step(const JobView &v, Pos &p, double &t, uint2 &row, uint32_t gl,
                                               uint32_t grp_base, Counters &cnt) {
    const uint64_t tb = (uint64_t)__double_as_longlong(t);
    // the search's interval and the part of its block that does not depend on the new location
    const double kf = floor(t * v.inv_dt);
    const bool wide = !(kf < 2147483648.0);
    const uint32_t k = wide ? 0u : (uint32_t)kf;
    const bool q0 = gl < 4u;
    const uint32_t kk = q0 ? k : k + (gl - 3u);
    const uint32_t s_n0 = kk ^ v.key0;
    const uint64_t s_m = (uint64_t)0xD2511F53u * s_n0;
    const uint32_t call = gl & 1u;
    uint32_t a0 = p.loc, a1 = (uint32_t)tb, a2 = (uint32_t)(tb >> 32), a3 = (1u << 30) | call;
    philox10(a0, a1, a2, a3, v.key0, v.key1);
    // even lanes evaluated block 0 (call 0), odd lanes block 1: broadcasts give every lane both
    const uint64_t r0 = ((uint64_t)from_even(a1) << 32) | from_even(a0);
    const uint64_t r1 = ((uint64_t)from_even(a3) << 32) | from_even(a2);
    const uint64_t r2 = ((uint64_t)from_odd(a1) << 32) | from_odd(a0);
    const uint64_t r3 = ((uint64_t)from_odd(a3) << 32) | from_odd(a2);
    const bool spec = (r0 >> 11) < speciation_threshold<kLds>(v, p, t);
    Pos q = p;
    disperse<kLds, kUni>(v, q, r1, r2, r3, row);
    row = table_row<kLds, kUni>(v, q);

    if (v.sampler == NH_SAMPLER_POISSON) {
        // Lane gl takes interval k + gl whole (every event of a later interval lies beyond t); the
        // lowest interval with an event decides.  No event in k .. k+7 (or a wide index) is slow.
        uint32_t draws_i, blocks_i;
        const double best = poisson_interval(v, q.loc, (uint64_t)k + gl, t, draws_i, blocks_i);
        const uint32_t hits = (uint32_t)((__ballot(best < __builtin_inf()) >> grp_base) & 0xFFu);
        const bool slow = wide | (hits == 0u);
        const uint32_t first = hits ? (uint32_t)(__ffs(hits) - 1) : 0u;
        const double e = shfl_f64(best, (int)(grp_base + first));
        const uint32_t sd = group_sum8(gl <= first ? draws_i : 0u), sb = group_sum8(gl <= first ? blocks_i : 0u);
        const bool counted = (gl == 0u) & !spec & !slow;
        cnt.philox += (gl == 0u ? 2u : 0u) + (counted ? sb : 0u);
        cnt.draws += counted ? sd : 0u;
        p = q;
        t = (spec | slow) ? t : e;
        return spec ? kStepSpeciated : (slow ? kStepSlow : kStepOk);
    }
    const uint64_t draw = philox10_late_loc(q.loc, s_n0, s_m, q0 ? (gl >> 1) : 0u, v.key0, v.key1, q0 && (gl & 1u));
    const double x = (-log_u53o(draw)) * v.inv_lambda;
    const double x0 = quad_bcast<0>(x), x1 = quad_bcast<1>(x), x2 = quad_bcast<2>(x), x3 = quad_bcast<3>(x);
    const double s0 = kf * v.dt, s1 = s0 + v.dt, s2 = s1 + v.dt, s3 = s2 + v.dt, s4 = s3 + v.dt,
                 s5 = s4 + v.dt;
    const double e0 = s0 + x0, e1 = e0 + x1, e2 = e1 + x2, e3 = e2 + x3;
    const bool d0 = (e0 >= s1) | (e0 > t), d1 = (e1 >= s1) | (e1 > t);
    const bool d2 = (e2 >= s1) | (e2 > t), d3 = (e3 >= s1) | (e3 > t);
    const double e = d0 ? e0 : (d1 ? e1 : (d2 ? e2 : e3));
    const uint32_t draws_k = d0 ? 1u : (d1 ? 2u : (d2 ? 3u : 4u));
    const bool hit_k = d3 & (e < s1);
    const double f0 = s1 + x0, f1 = s2 + x1, f2 = s3 + x2, f3 = s4 + x3;
    const bool g0 = f0 < s2, g1 = f1 < s3, g2 = f2 < s4, g3 = f3 < s5;
    const double q1_e = g0 ? f0 : (g1 ? f1 : (g2 ? f2 : f3));
    const uint32_t q1_tag = (uint32_t)(g0 | g1 | g2 | g3) | ((g0 ? 0u : (g1 ? 1u : (g2 ? 2u : 3u))) << 1);
    const double my_e = q0 ? e : q1_e;
    const uint32_t my_tag = q0 ? ((uint32_t)hit_k | ((uint32_t)!d3 << 3)) : q1_tag;
    const double o_e = half_mirror_f64(my_e);
    const uint32_t o_tag = half_mirror(my_tag);
    const uint32_t a_tag = q0 ? my_tag : o_tag, b_tag = q0 ? o_tag : my_tag;
    const double a_e = q0 ? my_e : o_e, b_e = q0 ? o_e : my_e;
    const bool a_hit = (a_tag & 1u) != 0u, b_hit = (b_tag & 1u) != 0u;
    const bool slow = wide | ((a_tag >> 3) & 1u) | !(a_hit | b_hit);

    const uint32_t later = a_hit ? 0u : (b_hit ? ((b_tag >> 1) & 3u) + 1u : 4u);
    const bool counted = (gl == 0u) & !spec & !slow;
    cnt.philox += (gl == 0u ? 2u : 0u) + (counted ? ((draws_k + 1u) >> 1) + later : 0u);
    cnt.draws += counted ? draws_k + later : 0u;

    p = q;
    t = (spec | slow) ? t : (a_hit ? a_e : b_e);
    return spec ? kStepSpeciated : (slow ? kStepSlow : kStepOk);
}

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------
__global__ void k_fill_u64(unsigned long long *p, uint64_t n, unsigned long long value) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

__global__ void k_setup(Ctl *ctl, JobState *js, const JobDev *jobs, uint32_t n_jobs, uint32_t first_round) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t == 0) {
        ctl->round = first_round;
        for (int k = 0; k < 3; ++k) {
            ctl->count[k] = 0;
            ctl->cursor[k] = 0;
            ctl->solo[k] = 0;
            ctl->solo_cursor[k] = 0;
        }
        ctl->blocks_done = 0;
        ctl->error = 0;
        ctl->n_jobs = n_jobs;
        for (uint32_t k = 0; k < kOpSlots; ++k) ctl->ops[k] = OpSlot{};
        ctl->ring_head = 0;
        ctl->ring_pub = 0;
        ctl->stop = 0;
        ctl->first_round = first_round;
        ctl->t_start = 0;
    }
    for (uint32_t j = t; j < n_jobs; j += gridDim.x * blockDim.x) {
        js[j].remaining = jobs[j].n;
        js[j].flags = 0;
        js[j].done_round = 0;
        js[j].start_round = jobs[j].start_round;
        js[j].rich_count = 0;
        js[j].events = 0;
        js[j].speciated = 0;
        js[j].merged = 0;
        js[j].solo_round = 0;
        js[j].h_base = 0.0;
        js[j].abund_n = 0;
        js[j].sentinel_count = 0;
    }
}

// Set-up of a single-job run from kernel arguments alone (enqueue-only calls
// copy nothing from the host): the job descriptor, the horizon table (the
// same recurrence, in the same binary64 operations, as the host table of
// nh_batch_run), the control block and the job's counters.
__global__ void k_setup_single(Ctl *ctl, JobState *js, JobDev *jobs, JobDev job, double *htab, double h0,
                               double growth, double step_max) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    jobs[0] = job;
    htab[0] = 0.0;
    htab[1] = h0;
    for (uint32_t i = 2; i < kMaxHorizons; ++i) htab[i] = htab[i - 1] + fmin(step_max, htab[i - 1] * (growth - 1.0));
    ctl->round = 1;
    for (int k = 0; k < 3; ++k) {
        ctl->count[k] = 0;
        ctl->cursor[k] = 0;
        ctl->solo[k] = 0;
        ctl->solo_cursor[k] = 0;
    }
    ctl->blocks_done = 0;
    ctl->error = 0;
    ctl->n_jobs = 1;
    for (uint32_t k = 0; k < kOpSlots; ++k) ctl->ops[k] = OpSlot{};
    ctl->ring_head = 0;
    ctl->ring_pub = 0;
    ctl->stop = 0;
    ctl->first_round = 1;
    ctl->t_start = 0;
    js[0] = JobState{};
    js[0].remaining = job.n;
}

// Binary search: the job whose lineage range holds g (jobs sorted by lin_base).
__device__ __forceinline__ uint32_t job_of(const JobDev *jobs, uint32_t n_jobs, uint32_t g) {
    uint32_t lo = 0, hi = n_jobs;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (jobs[mid].lin_base <= g) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Relaxed agent-scope accesses to control words that other workgroups write.
__device__ __forceinline__ uint32_t ld_agent(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(uint32_t *p, uint32_t x) {
    __hip_atomic_store(p, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Tail lane (servers): a job whose last lineage is all that is left of it
// needs no more rounds, since a lone lineage has nothing to merge with.  The
// round kernel hands such a lineage to this queue and a separate kernel
// (k_tail, on compute units of its own) walks it to its speciation without
// waiting for anyone's rounds.  Entry i sits in slot i % kTailCap: seq holds
// i + 1 once it is filled and i + 1 | kTailCopied once a tail wave has read
// it, which frees the slot for entry i + kTailCap.
constexpr uint32_t kTailCap = 1024;
constexpr uint32_t kTailCopied = 0x80000000u;
struct TailQ {
    uint32_t push;   // entries filled (reserved by a CAS that checks the slot is free)
    uint32_t take;   // entries claimed by tail waves (only ready entries are claimed)
    uint32_t ring_n; // completions published to the host
    uint32_t done;   // entries whose walk has ended
    uint32_t busy;   // waves walking now
    uint32_t pad[3];
    uint32_t seq[kTailCap];
    uint32_t g[kTailCap], loc[kTailCap];
    double t[kTailCap];
};

struct RoundArgs {
    Ctl *ctl;
    const JobDev *jobs;
    JobState *js;
    uint32_t *ring;    // completion ring (device), ring_cap slots
    Lin lin;
    const double *htab;
    uint32_t coop_max; // queues shorter than this run groups of 8 lanes per lineage
    uint32_t ring_cap;
    uint32_t n_cap;    // slots of each act array (main queue from the bottom, solo queue from the top)
    uint32_t solo_max; // multi-job runs: jobs with at most this many live lineages turn solo (0: never)
    double solo_step;  // horizon advance per round of a solo job
    TailQ *tail;       // servers with a tail lane, else null
    uint32_t tail_walkers; // waves of the tail lane: hand-offs never wait for one
};

// A lineage goes to the tail lane only if its job's speciation probability
// leaves it a long expected walk (1 / nu events, at least this many): short
// tails finish in the rounds as well as anywhere.
constexpr uint64_t kTailMinWalk = 16384;

// Hands solo lineage g of job jb (its state (loc, t) after its round) to the
// tail lane if it is the job's last one and a slot is free.  The live count
// only falls, so reading 1 while g is live means g is the last.  One lane.
__device__ __forceinline__ bool tail_handoff(const RoundArgs &A, uint32_t jb, uint32_t g, uint32_t loc, double t) {
    TailQ *T = A.tail;
    if (__hip_atomic_load(&A.js[jb].remaining, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 1u) return false;
    if (A.jobs[jb].nu_thresh > (1ull << 53) / kTailMinWalk) return false;
    uint32_t push = ld_agent(&T->push);
    while (true) {
        if (push - ld_agent(&T->done) >= A.tail_walkers) return false; // every walker busy
        const uint32_t sq = ld_agent(&T->seq[push % kTailCap]);
        if (sq != (push < kTailCap ? 0u : ((push - kTailCap + 1u) | kTailCopied))) return false; // slot busy
        const uint32_t seen = atomicCAS(&T->push, push, push + 1u);
        if (seen == push) break;
        push = seen;
    }
    const uint32_t i = push % kTailCap;
    T->g[i] = g;
    T->loc[i] = loc;
    T->t[i] = t;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    st_agent(&T->seq[i], push + 1u);
    return true;
}

// Horizon of job jb in round r: its schedule by age, or, once the job has
// turned solo, a fixed advance per round from the horizon it had then.  A
// job's solo round is set while round solo_round - 1 runs and only read for
// later rounds, so every lineage of the job sees the same horizon.
__device__ __forceinline__ double job_horizon(const RoundArgs &A, uint32_t r, uint32_t jb) {
    const uint32_t sr = A.js[jb].solo_round;
    if (sr != 0u && r >= sr) return A.js[jb].h_base + (double)(r - sr + 1u) * A.solo_step;
    return horizon_of(A.htab, r - A.jobs[jb].start_round);
}

// Where a survivor of round r goes (multi-job runs): a job whose live count
// has fallen to solo_max or below turns solo from round r + 1 (the first lane
// to see it records the round and its current horizon) and its survivors go
// to the solo queue.  Reads of the live count may be stale; that only moves
// the switch by a round.
__device__ __forceinline__ bool route_solo(const RoundArgs &A, uint32_t r, uint32_t jb, double horizon) {
    if (A.solo_max == 0u) return false;
    JobState &J = A.js[jb];
    if (__hip_atomic_load(&J.solo_round, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) return true;
    if (__hip_atomic_load(&J.remaining, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) > A.solo_max) return false;
    if (atomicCAS(&J.solo_round, 0u, r + 1u) == 0u) J.h_base = horizon;
    return true;
}

__device__ __forceinline__ void push_solo(const RoundArgs &A, uint32_t *solo_count, uint32_t *act_out, uint32_t g) {
    const uint32_t i = atomicAdd(solo_count, 1u);
    act_out[A.n_cap - 1u - i] = g;
}

// Retires lineages (speciated, merged, or rejected at init) from their jobs'
// live counts, one atomic per wave when the retiring lanes share a job.  The
// lane that brings a job to zero records the round and pushes the job onto
// the completion ring.  All active lanes call it.
__device__ __forceinline__ void job_retired(Ctl *ctl, JobState *js, uint32_t *ring, uint32_t ring_cap, uint32_t r,
                                            uint32_t jb, uint32_t count) {
    const uint32_t old = atomicSub(&js[jb].remaining, count);
    if (old == count) {
        js[jb].done_round = r;
        const uint32_t at = atomicAdd(&ctl->ring_head, 1u);
        ring[at % ring_cap] = jb;
    }
}

__device__ __forceinline__ void wave_retire(Ctl *ctl, JobState *js, uint32_t *ring, uint32_t ring_cap, uint32_t r,
                                            bool retiring, uint32_t jb) {
    const uint64_t m = __ballot(retiring);
    if (!m) return;
    const int first = __ffsll((unsigned long long)m) - 1;
    const uint32_t jb0 = __shfl(jb, first, 64);
    if (__ballot(retiring && jb != jb0) == 0) {
        if (lane_id() == (uint32_t)first) job_retired(ctl, js, ring, ring_cap, r, jb0, (uint32_t)__popcll(m));
    } else if (retiring) {
        job_retired(ctl, js, ring, ring_cap, r, jb, 1u);
    }
}

// Location of dense individual id (< N): the cell whose capacity prefix holds
// it, and the id's offset in that cell as the deme index.
__device__ __forceinline__ uint32_t sample_loc(const JobDev *__restrict__ J, const JobView &v, uint64_t id) {
    const uint32_t cells = v.W * v.H;
    uint32_t lo = 0, hi = cells; // last cell with prefix <= id
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (J->prefix[mid] <= id) lo = mid;
        else hi = mid;
    }
    return lo * v.cmax + (uint32_t)(id - J->prefix[lo]);
}

// Lineage init: dense sample id -> (cell, deme index) -> loc; first event time
// from t = 0; append to the current round's queue.  Lineages [g_begin, g_end)
// belong to job `fixed_job`, or (fixed_job < 0) to the job found by binary
// search over jobs sorted by lineage base.  An id >= N flags the job (and the
// run) and the lineage is retired at once instead of queued.
__global__ void k_init(Ctl *ctl, const JobDev *__restrict__ jobs, uint32_t n_jobs, int fixed_job, JobState *js,
                       uint32_t *ring, uint32_t ring_cap, Lin lin, uint32_t g_begin, uint32_t g_end) {
    const uint32_t g = g_begin + blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t r = ctl->round;
    bool push = false, bad = false;
    uint32_t jb = 0;
    Counters cnt;
    if (g < g_end) {
        jb = fixed_job >= 0 ? (uint32_t)fixed_job : job_of(jobs, n_jobs, g);
        const JobDev *J = &jobs[jb];
        const JobView v = load_view(J);
        const uint64_t id = J->samples[g - J->lin_base];
        uint32_t loc = 0;
        double t = 0.0;
        if (id >= J->n_individuals) {
            atomicOr(&ctl->error, kErrBadSample);
            atomicOr(&js[jb].flags, kJobBadSample);
            bad = true;
        } else {
            loc = sample_loc(J, v, id);
            t = next_event_time(v, loc, 0.0, &ctl->error, cnt);
            push = t >= 0.0;
            bad = !push;
        }
        lin.loc[r & 1][g] = loc;
        lin.t[r & 1][g] = t;
        lin.parent[g] = g;
        lin.species[g] = 0;
        lin.spec_loc[g] = 0;
        lin.spec_t[g] = 0.0;
        lin.job[g] = jb;
        lin.events[g] = 0;
    }
    const uint64_t mask = __ballot(push);
    if (mask) {
        const uint32_t slot = wave_reserve(mask, &ctl->count[r % 3]);
        if (push) lin.act[r & 1][slot] = g;
    }
    wave_retire(ctl, js, ring, ring_cap, r, bad, jb);
    flush_counters_block(ctl, cnt);
}

// Admission of one job into a running engine: its counters, its species set
// and its first round (the job's horizons count from the round it joins).
__global__ void k_job_setup(Ctl *ctl, JobDev *jobs, JobState *js, uint32_t slot) {
    JobDev *J = &jobs[slot];
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    if (tid == 0) {
        J->start_round = ctl->round - 1;
        js[slot].start_round = ctl->round - 1;
        js[slot].remaining = J->n;
        js[slot].flags = 0;
        js[slot].done_round = 0;
        js[slot].rich_count = 0;
        js[slot].events = 0;
        js[slot].speciated = 0;
        js[slot].merged = 0;
        js[slot].solo_round = 0;
        js[slot].h_base = 0.0;
        js[slot].abund_n = 0;
        js[slot].sentinel_count = 0;
    }
    for (uint64_t i = tid; i <= (uint64_t)J->rich_mask; i += (uint64_t)gridDim.x * blockDim.x) {
        J->rich_set[i] = ~0ull;
        J->rich_counts[i] = 0u;
    }
}

// Round kernels.  Round r takes the queue of round r, drops lineages whose
// (job, loc, t_next) another lineage already holds (cull), advances the rest
// event by event until the next event lies beyond the job's horizon, retires
// speciated lineages and queues the others for round r + 1.  Two lane
// layouts: one lane per lineage (many lineages), or a group of 8 lanes per
// lineage when the queue is short enough that the chip would otherwise idle.
// Per-wave access to the round's queues with few atomics.  Input: the wave
// reserves chunks of the queue with one atomic and hands items to its idle
// lanes from the chunk.  Output: survivors are staged in a per-wave LDS
// buffer and appended to the next queue one buffer-full at a time.
constexpr uint32_t kWavesPerBlock = 4; // block size 256 at most
constexpr uint32_t kOutBuf = 256;      // staged survivor ids per wave

struct WaveQueues {
    uint32_t chunk_pos = 0, chunk_end = 0; // wave-uniform: unread part of the reserved chunk
    bool open = true;                      // wave-uniform: the round's queue may still hold items
    uint32_t staged = 0;                   // wave-uniform: ids in this wave's output buffer
};

// Hands out at most one queue position per lane in `want`; returns the
// position (or ~0u) for each wanting lane.  All active lanes call it.  A
// reservation takes max(#wanting, chunk) items: chunk is the caller's fair
// share, so a short queue is spread over many waves instead of one.
__device__ __forceinline__ uint32_t wave_take(WaveQueues &q, uint64_t want, uint32_t *cursor, uint32_t n_in,
                                              uint32_t chunk) {
    const uint32_t lane = lane_id();
    chunk = max(chunk, (uint32_t)__popcll(want));
    if (q.chunk_pos >= q.chunk_end && q.open) {
        const int leader = __ffsll((unsigned long long)__ballot(1)) - 1;
        uint32_t base = 0;
        if ((int)lane == leader) base = atomicAdd(cursor, chunk);
        base = __shfl(base, leader, 64);
        if (base >= n_in) {
            q.open = false;
            q.chunk_pos = q.chunk_end = 0;
        } else {
            q.chunk_pos = base;
            q.chunk_end = min(base + chunk, n_in);
            if (q.chunk_end == n_in) q.open = false;
        }
    }
    const uint32_t avail = q.chunk_end - q.chunk_pos;
    const uint32_t rank = (uint32_t)__popcll(want & ((1ull << lane) - 1ull));
    const uint32_t pos = ((want >> lane) & 1ull) && rank < avail ? q.chunk_pos + rank : 0xFFFFFFFFu;
    q.chunk_pos += min((uint32_t)__popcll(want), avail);
    return pos;
}

__device__ __forceinline__ void wave_flush(WaveQueues &q, uint32_t *buf, uint32_t *count_out, uint32_t *act_out) {
    if (q.staged == 0) return;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const uint32_t lane = lane_id();
    const int leader = __ffsll((unsigned long long)__ballot(1)) - 1;
    uint32_t base = 0;
    if ((int)lane == leader) base = atomicAdd(count_out, q.staged);
    base = __shfl(base, leader, 64);
    for (uint32_t i = lane; i < q.staged; i += 64) act_out[base + i] = buf[i];
    __builtin_amdgcn_wave_barrier();
    q.staged = 0;
}

// Stages the ids of lanes with `push` set; flushes when the buffer is nearly full.
__device__ __forceinline__ void wave_push(WaveQueues &q, bool push, uint32_t id, uint32_t *buf, uint32_t *count_out,
                                          uint32_t *act_out) {
    const uint64_t pm = __ballot(push);
    if (!pm) return;
    const uint32_t lane = lane_id();
    if (push) buf[q.staged + (uint32_t)__popcll(pm & ((1ull << lane) - 1ull))] = id;
    q.staged += (uint32_t)__popcll(pm);
    if (q.staged > kOutBuf - 64) wave_flush(q, buf, count_out, act_out);
}

template <bool kSingleJob, bool kLds>
__device__ __forceinline__ void round_one_lane(const RoundArgs &A, uint32_t r, uint32_t n_in, Counters &cnt,
                                               uint32_t *obuf, uint32_t chunk, bool solo) {
    Ctl *ctl = A.ctl;
    const Lin &lin = A.lin;
    const uint32_t *__restrict__ act_in = lin.act[r & 1];
    uint32_t *__restrict__ act_out = lin.act[(r + 1) & 1];
    const uint32_t *__restrict__ loc_in = lin.loc[r & 1];
    const double *__restrict__ t_in = lin.t[r & 1];
    uint32_t *__restrict__ loc_out = lin.loc[(r + 1) & 1];
    double *__restrict__ t_out = lin.t[(r + 1) & 1];
    uint32_t *err = &ctl->error;
    const uint32_t qin = r % 3, qout = (r + 1) % 3;
    // the round's input queue: the main queue from the bottom of act_in, or the solo queue from its top
    uint32_t *cursor = solo ? &ctl->solo_cursor[qin] : &ctl->cursor[qin];
    const uint32_t pos_base = solo ? A.n_cap - 1u : 0u;
    const uint32_t pos_sign = solo ? 0xFFFFFFFFu : 1u; // item i sits at pos_base + pos_sign * i

    JobView v;
    double w_single = 0.0;
    if (kSingleJob) {
        v = load_view(&A.jobs[0]);
        w_single = horizon_of(A.htab, r - A.jobs[0].start_round);
    }
    WaveQueues q;
    uint32_t iter = 0; // wave-uniform
    bool has = false;
    uint32_t g = 0, jb = 0, ev = 0;
    Pos p = {0, 0, 0, 0};
    double t = 0.0, horizon = w_single;

    while (true) {
        // A wave whose lanes are all busy does not reserve, so it would not learn that other waves
        // have reserved the rest of the queue: every 8th iteration it reads the shared cursor (one
        // relaxed load, consumed after the event step, so its latency hides behind it).
        const bool peek = q.open && q.chunk_pos >= q.chunk_end && (++iter & 7u) == 0u;
        uint32_t reserved = 0;
        if (peek) reserved = __hip_atomic_load(cursor, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint64_t need = __ballot(!has);
        bool retire = false;
        if (need && (q.open || q.chunk_pos < q.chunk_end)) {
            const uint32_t pos = wave_take(q, need, cursor, n_in, chunk);
            if (pos != 0xFFFFFFFFu) {
                g = act_in[pos_base + pos_sign * pos];
                if (!kSingleJob) jb = lin.job[g];
                const uint32_t loc = loc_in[g];
                t = t_in[g];
                const uint32_t owner =
                    cull_insert(lin, loc_in, t_in, r, g, loc, (uint64_t)__double_as_longlong(t), jb, err);
                if (owner != g) {
                    lin.parent[g] = owner;
                    retire = true;
                } else {
                    if (!kSingleJob) {
                        v = load_view(&A.jobs[jb]);
                        horizon = job_horizon(A, r, jb);
                    }
                    p = pos_from_loc(v, loc);
                    ev = 0;
                    has = true;
                }
            }
        }
        if (__ballot(has) == 0) {
            wave_retire(ctl, A.js, A.ring, A.ring_cap, r, retire, jb);
            if (!q.open && q.chunk_pos >= q.chunk_end) break;
            continue;
        }

        bool finish_live = false, finish_dead = false, speciated = false;
        // Once the wave has drained its share of the queue there is nothing to pick up, so a lane
        // stays in the event loop until its lineage leaves the round (no per-event bookkeeping).
        const bool drained = !q.open && q.chunk_pos >= q.chunk_end;
        if (has) {
            if (t > horizon) {
                finish_live = true;
            } else {
                do {
                    ++ev;
                    if (commit_event<kLds>(v, p, t, cnt)) {
                        finish_dead = true;
                        speciated = true;
                    } else {
                        t = next_event_time(v, p.loc, t, err, cnt);
                        if (t < 0.0) finish_dead = true; // runaway search (flagged)
                        else if (t > horizon) finish_live = true;
                    }
                } while (drained && !(finish_dead | finish_live));
            }
        }
        if (peek && __builtin_amdgcn_readfirstlane(reserved) >= n_in) q.open = false; // the cursor only grows
        if (finish_dead) {
            lin.species[g] = speciated ? species_of(v, p.loc, t) : 0ull;
            lin.spec_loc[g] = p.loc;
            lin.spec_t[g] = t;
            lin.events[g] += ev;
            has = false;
        }
        if (finish_live) {
            loc_out[g] = p.loc;
            t_out[g] = t;
            lin.events[g] += ev;
            has = false;
        }
        wave_retire(ctl, A.js, A.ring, A.ring_cap, r, retire || finish_dead, jb);
        const bool to_solo = !kSingleJob && finish_live && route_solo(A, r, jb, horizon);
        if (to_solo) push_solo(A, &ctl->solo[qout], act_out, g);
        wave_push(q, finish_live && !to_solo, g, obuf, &ctl->count[qout], act_out);
    }
    wave_flush(q, obuf, &ctl->count[qout], act_out);
}

template <bool kSingleJob, bool kLds>
__device__ __forceinline__ void round_group(const RoundArgs &A, uint32_t r, uint32_t n_in, Counters &cnt,
                                            uint32_t *obuf, uint32_t chunk, bool solo) {
    Ctl *ctl = A.ctl;
    const Lin &lin = A.lin;
    const uint32_t *__restrict__ act_in = lin.act[r & 1];
    uint32_t *__restrict__ act_out = lin.act[(r + 1) & 1];
    const uint32_t *__restrict__ loc_in = lin.loc[r & 1];
    const double *__restrict__ t_in = lin.t[r & 1];
    uint32_t *__restrict__ loc_out = lin.loc[(r + 1) & 1];
    double *__restrict__ t_out = lin.t[(r + 1) & 1];
    uint32_t *err = &ctl->error;
    const uint32_t qin = r % 3, qout = (r + 1) % 3;
    // the round's input queue: the main queue from the bottom of act_in, or the solo queue from its top
    uint32_t *cursor = solo ? &ctl->solo_cursor[qin] : &ctl->cursor[qin];
    const uint32_t pos_base = solo ? A.n_cap - 1u : 0u;
    const uint32_t pos_sign = solo ? 0xFFFFFFFFu : 1u; // item i sits at pos_base + pos_sign * i
    const uint32_t lane = lane_id(), gl = lane & (kGroup - 1), grp_base = lane & ~(kGroup - 1);
    const bool leader = gl == 0;

    JobView v;
    double w_single = 0.0;
    if (kSingleJob) {
        v = load_view(&A.jobs[0]);
        w_single = horizon_of(A.htab, r - A.jobs[0].start_round);
    }
    WaveQueues q;
    uint32_t iter = 0; // wave-uniform
    bool has = false;
    uint32_t g = 0, jb = 0, ev = 0;
    Pos p = {0, 0, 0, 0};
    double t = 0.0, horizon = w_single;

    while (true) {
        // as in the one-lane layout: a wave whose groups are all busy learns from the shared cursor
        // (every 8th iteration) that the queue is fully reserved
        const bool peek = q.open && q.chunk_pos >= q.chunk_end && (++iter & 7u) == 0u;
        uint32_t reserved = 0;
        if (peek) reserved = __hip_atomic_load(cursor, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint64_t need = __ballot(leader && !has);
        bool retire = false;     // set on the leader lane of a group whose candidate was merged
        uint32_t retire_jb = 0;
        if (need && (q.open || q.chunk_pos < q.chunk_end)) {
            const uint32_t pos = wave_take(q, need, cursor, n_in, chunk);
            uint32_t take = 0xFFFFFFFFu; // lineage id the group leader took, or none
            if (pos != 0xFFFFFFFFu) {
                const uint32_t cand = act_in[pos_base + pos_sign * pos];
                const uint32_t cjb = kSingleJob ? 0u : lin.job[cand];
                const uint32_t owner = cull_insert(lin, loc_in, t_in, r, cand, loc_in[cand],
                                                   (uint64_t)__double_as_longlong(t_in[cand]), cjb, err);
                if (owner != cand) {
                    lin.parent[cand] = owner;
                    retire = true;
                    retire_jb = cjb;
                } else {
                    take = cand;
                }
            }
            take = (uint32_t)__shfl((int)take, (int)grp_base, 64);
            if (!has && take != 0xFFFFFFFFu) {
                g = take;
                if (!kSingleJob) {
                    jb = lin.job[g];
                    v = load_view(&A.jobs[jb]);
                    horizon = job_horizon(A, r, jb);
                }
                p = pos_from_loc(v, loc_in[g]);
                t = t_in[g];
                ev = 0;
                has = true;
            }
        }
        if (__ballot(has) == 0) {
            wave_retire(ctl, A.js, A.ring, A.ring_cap, r, retire, retire_jb);
            if (!q.open && q.chunk_pos >= q.chunk_end) break;
            continue;
        }

        bool finish_live = false, finish_dead = false, speciated = false;
        uint32_t at = p.loc; // location of the last event (a speciation keeps it)
        // As in the one-lane layout: a drained wave keeps each group in its event loop.  The 8 lanes
        // of a group always agree, so they leave the loop together.
        const bool drained = !q.open && q.chunk_pos >= q.chunk_end;
        if (has) {
            if (t > horizon) {
                finish_live = true;
            } else {
                // The rare slow search is finished inside the iteration: a group that left the loop
                // for it would wait there until every other group of the wave had left the loop too.
                uint32_t st;
                uint2 row = table_row<kLds>(v, p);
                do {
                    ++ev;
                    at = p.loc;
                    st = group_step<kLds>(v, p, t, row, gl, grp_base, cnt);
                    if (__builtin_expect(st == kStepSlow, 0)) {
                        t = next_event_time_group(v, p.loc, t, gl, grp_base, err, cnt);
                        st = t < 0.0 ? kStepSlow : kStepOk; // kStepSlow now marks a runaway search
                    }
                } while (drained && st == kStepOk && !(t > horizon));
                if (st == kStepSpeciated) {
                    finish_dead = true;
                    speciated = true;
                } else if (st == kStepSlow) {
                    finish_dead = true;
                } else if (t > horizon) {
                    finish_live = true;
                }
            }
        }
        if (peek && __builtin_amdgcn_readfirstlane(reserved) >= n_in) q.open = false; // the cursor only grows
        if (finish_dead) {
            if (leader) {
                const uint32_t sloc = speciated ? at : p.loc;
                lin.species[g] = speciated ? species_of(v, sloc, t) : 0ull;
                lin.spec_loc[g] = sloc;
                lin.spec_t[g] = t;
                lin.events[g] += ev;
            }
            has = false;
        }
        if (finish_live) {
            if (leader) {
                loc_out[g] = p.loc;
                t_out[g] = t;
                lin.events[g] += ev;
            }
            has = false;
        }
        // a group leader retires either the candidate it merged at pickup or its speciated lineage
        const bool dead_leader = finish_dead && leader;
        wave_retire(ctl, A.js, A.ring, A.ring_cap, r, retire || dead_leader, retire ? retire_jb : jb);
        const bool to_tail = !kSingleJob && solo && finish_live && leader && A.tail && tail_handoff(A, jb, g, p.loc, t);
        const bool to_solo = !kSingleJob && finish_live && leader && !to_tail && route_solo(A, r, jb, horizon);
        if (to_solo) push_solo(A, &ctl->solo[qout], act_out, g);
        wave_push(q, finish_live && leader && !to_solo && !to_tail, g, obuf, &ctl->count[qout], act_out);
    }
    wave_flush(q, obuf, &ctl->count[qout], act_out);
}

// Which part of a round a workgroup takes.  Multi-job runs: the first
// workgroups take the solo queue, 8 lanes per lineage at raised wave priority
// (the long serial tails of nearly finished jobs), at most a quarter of the
// grid; the others take the main queue, as many as its length needs.  The
// plan is workgroup-uniform.
constexpr uint32_t kPlanIdle = 0, kPlanSolo = 1, kPlanLanes = 2, kPlanGroups = 3;
struct RoundPlan {
    uint32_t mode;  // kPlan*
    uint32_t chunk; // queue items per reservation
};

template <bool kSingleJob>
__device__ __forceinline__ RoundPlan plan_round(const RoundArgs &A, uint32_t n_main, uint32_t n_solo) {
    RoundPlan pl{kPlanIdle, 0u};
    const uint32_t waves_per_block = blockDim.x / 64;
    uint32_t solo_blocks = 0;
    if constexpr (!kSingleJob) {
        if (n_solo) {
            const uint64_t need = ((uint64_t)n_solo * kGroup + blockDim.x - 1) / blockDim.x;
            solo_blocks = (uint32_t)min<uint64_t>(need, gridDim.x / 4); // the host keeps the grid >= 4
        }
        if (blockIdx.x < solo_blocks) {
            const uint64_t waves = (uint64_t)solo_blocks * waves_per_block;
            pl.mode = kPlanSolo;
            pl.chunk = (uint32_t)min<uint64_t>(32u, n_solo / (4 * waves));
            return pl;
        }
    }
    if (n_main == 0) return pl;
    const uint32_t b = blockIdx.x - solo_blocks, grid = gridDim.x - solo_blocks;
    const bool group = n_main < A.coop_max;
    const uint64_t lanes_needed = (uint64_t)n_main * (group ? kGroup : 1u);
    const uint64_t blocks_needed = (lanes_needed + blockDim.x - 1) / blockDim.x;
    if (b >= blocks_needed) return pl; // whole workgroup sits the round out
    // fair share of the queue per participating wave (a quarter of it per reservation), capped
    const uint64_t waves = min((uint64_t)grid, blocks_needed) * waves_per_block;
    pl.mode = group ? kPlanGroups : kPlanLanes;
    pl.chunk = (uint32_t)min<uint64_t>(group ? 32u : 256u, n_main / (4 * waves));
    return pl;
}

// Stages the shared dispersal table (single job, shared mode, small table) in LDS.
__device__ __forceinline__ void stage_table(const RoundArgs &A) {
    const uint32_t n_tab = A.jobs[0].n_shared;
    const uint4 *__restrict__ src = A.jobs[0].table;
    for (uint32_t i = threadIdx.x; i < n_tab; i += blockDim.x) nh_lds_table[i] = src[i];
    __syncthreads();
}

// This workgroup's share of round r (plan pl), lane layout by the plan.
template <bool kSingleJob, bool kLds>
__device__ __forceinline__ void round_share(const RoundArgs &A, uint32_t r, const RoundPlan &pl, uint32_t n_main,
                                            uint32_t n_solo, Counters &cnt, uint32_t *obuf) {
    if constexpr (!kSingleJob) {
        if (pl.mode == kPlanSolo) {
            __builtin_amdgcn_s_setprio(2);
            round_group<false, false>(A, r, n_solo, cnt, obuf, pl.chunk, true);
            __builtin_amdgcn_s_setprio(0);
            return;
        }
    }
    if (pl.mode == kPlanGroups) round_group<kSingleJob, kLds>(A, r, n_main, cnt, obuf, pl.chunk, false);
    else round_one_lane<kSingleJob, kLds>(A, r, n_main, cnt, obuf, pl.chunk, false);
}

template <bool kSingleJob, bool kLds>
__global__ __launch_bounds__(256) void k_round(RoundArgs A) {
    const uint32_t r = A.ctl->round;
    const uint32_t n_main = A.ctl->count[r % 3];
    const uint32_t n_solo = kSingleJob ? 0u : A.ctl->solo[r % 3];
    const RoundPlan pl = plan_round<kSingleJob>(A, n_main, n_solo);
    if (pl.mode == kPlanIdle) return;
    __shared__ uint32_t out_stage[kWavesPerBlock][kOutBuf];
    uint32_t *obuf = out_stage[threadIdx.x / 64];
    Counters cnt;
    if (kLds && pl.mode != kPlanSolo) stage_table(A);
    round_share<kSingleJob, kLds>(A, r, pl, n_main, n_solo, cnt, obuf);
    flush_counters_block(A.ctl, cnt);
}

// ---------------------------------------------------------------------------
// Persistent run: one launch carries a run through all of its rounds.  The
// workgroups (all resident: the grid is sized from the occupancy and launched
// cooperatively) run a round, meet at a grid barrier whose last arrival runs
// the round epilogue (advance the round, reset the next queues, decide whether
// the run goes on), and start the next round.  Nothing returns to the host
// between rounds, so the call that enqueues it can return at once.
// ---------------------------------------------------------------------------
struct RunArgs {
    uint32_t max_rounds;          // rounds of this launch before it suspends (0: no limit)
    uint32_t endgame;             // stop for k_endgame once at most this many lineages remain (0: never)
    unsigned long long spin_ticks; // wall-clock ticks one barrier wait may take
    unsigned long long run_ticks;  // wall-clock ticks the whole launch may take
};

struct RoundCtl {
    uint32_t r, n_main, n_solo, stop;
};

// The round control words as the host-side set-up left them (launch start).
__device__ __forceinline__ RoundCtl read_round_ctl(Ctl *ctl, bool single) {
    RoundCtl c;
    c.r = ld_agent(&ctl->round);
    c.n_main = ld_agent(&ctl->count[c.r % 3]);
    c.n_solo = single ? 0u : ld_agent(&ctl->solo[c.r % 3]);
    c.stop = ld_agent(&ctl->stop);
    return c;
}

// Device wall clock at the start of the launch (set by the first workgroup to start).
__device__ __forceinline__ unsigned long long run_start(Ctl *ctl) {
    return __hip_atomic_load(&ctl->t_start, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Round epilogue of a persistent run (one thread, after every workgroup has
// finished round r): the same bookkeeping as k_advance, then the stop
// decision; returns the next round's control words.
__device__ __forceinline__ RoundCtl run_epilogue(Ctl *ctl, const RunArgs &R) {
    const uint32_t r = ld_agent(&ctl->round);
    // independent loads (the queue words of every slot), selected afterwards
    uint32_t cnt[3], solo[3];
    for (int k = 0; k < 3; ++k) {
        cnt[k] = ld_agent(&ctl->count[k]);
        solo[k] = ld_agent(&ctl->solo[k]);
    }
    const uint32_t err = ld_agent(&ctl->error), first = ld_agent(&ctl->first_round);
    const uint32_t q = (r + 1) % 3;
    const uint32_t n_out = cnt[q] + solo[q];
    st_agent(&ctl->count[(r + 2) % 3], 0u);
    st_agent(&ctl->solo[(r + 2) % 3], 0u);
    st_agent(&ctl->solo_cursor[q], 0u);
    st_agent(&ctl->cursor[q], 0u);
    st_agent(&ctl->round, r + 1);
    uint32_t stop = 0;
    if (n_out == 0) {
        stop = kStopDone;
    } else if ((err & ~kErrBadSample) != 0u) {
        stop = kStopError; // a bad sample id only fails its own job
    } else if (n_out <= R.endgame) {
        stop = kStopEndgame;
    } else if (R.max_rounds != 0u && r + 1u - first >= R.max_rounds) {
        stop = kStopSuspended;
    } else if (wall_clock64() - run_start(ctl) > R.run_ticks) {
        atomicOr(&ctl->error, kErrTimeout);
        stop = kStopError;
    }
    // a workgroup that gave up waiting has stopped the run already (if it has and the run goes on,
    // the workgroups learn it in their next wait)
    if (stop) {
        const uint32_t old = atomicCAS(&ctl->stop, 0u, stop);
        if (old != 0u) stop = old;
    }
    return RoundCtl{r + 1, cnt[q], solo[q], stop};
}

// Waits (one thread) until *gen moves past `seen`, the run stops, or a limit
// passes: past the run's own time limit the run has timed out; otherwise a
// wait longer than R.spin_ticks means workgroups that never arrive.  Returns
// false if it gave up (and has stopped the run).
__device__ __forceinline__ bool wait_gen(Ctl *ctl, const RunArgs &R, const uint32_t *gen, uint32_t seen) {
    const unsigned long long t0 = wall_clock64();
    for (uint32_t poll = 1;; ++poll) {
        // relaxed polls (an acquire per poll would invalidate the L2 each time)
        if (ld_agent(gen) != seen) return true;
        if ((poll & 31u) == 0u) {
            if (ld_agent(&ctl->stop) != 0u) return false;
            const unsigned long long now = wall_clock64();
            const bool late = now - run_start(ctl) > R.run_ticks;
            if (late || now - t0 > R.spin_ticks) {
                atomicOr(&ctl->error, late ? kErrTimeout : kErrStall);
                atomicCAS(&ctl->stop, 0u, kStopError);
                return false;
            }
        }
        // poll quickly at first (short rounds), then back off: long rounds would otherwise have every
        // idle workgroup reading the barrier lines while the busy ones work
        if (poll < 256u) __builtin_amdgcn_s_sleep(2);
        else __builtin_amdgcn_s_sleep(32);
    }
}

// Grid barrier between rounds, two levels: a workgroup arrives at its group's
// counter (kBarGroup workgroups); the last of a group arrives at the top
// counter; the last group runs the epilogue and publishes the next round's
// control words with the release of the top counter; each group's last
// arrival, which waited there, copies them to its group's line and releases
// the group.  `gen` is the number of barriers passed.  A workgroup that did
// work in the round releases it first (agent scope); the caller acquires
// before it touches lineage state again.  On return sc holds the next round's
// control words (stop set if any wait gave up).
__device__ __forceinline__ void grid_sync(Ctl *ctl, const RunArgs &R, uint32_t gen, bool worked, RoundCtl &sc) {
    __syncthreads();
    if (threadIdx.x == 0) {
        if (worked) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const uint32_t g = blockIdx.x / kBarGroup;
        const uint32_t n_groups = (gridDim.x + kBarGroup - 1) / kBarGroup;
        const uint32_t members = min(kBarGroup, gridDim.x - g * kBarGroup);
        BarSlot &G = ctl->grp[g];
        RoundCtl c{0u, 0u, 0u, kStopError};
        if (atomicAdd(&G.arrived, 1u) == members - 1u) {
            st_agent(&G.arrived, 0u);
            if (atomicAdd(&ctl->top.arrived, 1u) == n_groups - 1u) {
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                st_agent(&ctl->top.arrived, 0u);
                c = run_epilogue(ctl, R);
                st_agent(&ctl->top.pub[0], c.r);
                st_agent(&ctl->top.pub[1], c.n_main);
                st_agent(&ctl->top.pub[2], c.n_solo);
                st_agent(&ctl->top.pub[3], c.stop);
                __hip_atomic_store(&ctl->top.gen, gen + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            } else if (wait_gen(ctl, R, &ctl->top.gen, gen)) {
                c = RoundCtl{ld_agent(&ctl->top.pub[0]), ld_agent(&ctl->top.pub[1]), ld_agent(&ctl->top.pub[2]),
                             ld_agent(&ctl->top.pub[3])};
            }
            // release the group, also after giving up (its members then read the stop)
            st_agent(&G.pub[0], c.r);
            st_agent(&G.pub[1], c.n_main);
            st_agent(&G.pub[2], c.n_solo);
            st_agent(&G.pub[3], c.stop);
            __hip_atomic_store(&G.gen, gen + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else if (wait_gen(ctl, R, &G.gen, gen)) {
            c = RoundCtl{ld_agent(&G.pub[0]), ld_agent(&G.pub[1]), ld_agent(&G.pub[2]), ld_agent(&G.pub[3])};
        }
        sc = c;
    }
    __syncthreads();
}

template <bool kSingleJob, bool kLds>
__global__ __launch_bounds__(256) void k_run(RoundArgs A, RunArgs R) {
    __shared__ uint32_t out_stage[kWavesPerBlock][kOutBuf];
    __shared__ RoundCtl sc;
    uint32_t *obuf = out_stage[threadIdx.x / 64];
    if (threadIdx.x == 0) {
        // the first workgroup to start sets the launch's start time (k_run_reset cleared it)
        atomicCAS(&A.ctl->t_start, 0ull, wall_clock64());
        sc = read_round_ctl(A.ctl, kSingleJob);
    }
    __syncthreads();
    if (kLds) stage_table(A);
    unsigned long long philox = 0, draws = 0; // this lane's op counts over all rounds
    for (uint32_t gen = 0;; ++gen) {
        const RoundCtl c = sc; // workgroup-uniform
        if (c.stop != 0u) break;
        const RoundPlan pl = plan_round<kSingleJob>(A, c.n_main, c.n_solo);
        const bool work = pl.mode != kPlanIdle;
        if (work) {
            // acquire the previous rounds' lineage state (other workgroups' releases)
            if (threadIdx.x == 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            __syncthreads();
            Counters cnt;
            round_share<kSingleJob, kLds>(A, c.r, pl, c.n_main, c.n_solo, cnt, obuf);
            philox += cnt.philox;
            draws += cnt.draws;
        }
        grid_sync(A.ctl, R, gen, work, sc);
    }
    flush_counters_block(A.ctl, philox, draws);
}

// Clears a persistent run's barrier and stop state before a launch (a resume
// included: the run goes on from the round its control block holds).
__global__ void k_run_reset(Ctl *ctl) {
    const uint32_t t = threadIdx.x;
    if (t < kMaxBarGroups) ctl->grp[t] = BarSlot{};
    if (t == 0) {
        ctl->top = BarSlot{};
        ctl->stop = 0;
        ctl->first_round = ctl->round;
        ctl->t_start = 0;
    }
}

// Tail lane kernel: each wave claims ready entries of the tail queue one at a
// time and walks the lineage with lanes 0-7 (the shared table copied to the
// wave's part of the LDS when it fits, else read through the scalar cache) to
// its speciation or a runaway search, writes the lineage's result and retires
// it; the lane that retires a job's last lineage publishes the job on the host
// ring, entry k as ((k + 1) << 32) | job slot.  A launch lasts one time slice:
// it claims nothing after the slice's end, and a walk still running then is
// queued again where it stands (its events so far counted) and the host-mapped
// more-flag set, so that the host starts the next slice.  A wave also leaves
// when it has had nothing to claim for idle_ticks while no wave walked, or when
// it sees the host's stop word (a walk checks it every 512 events): waves stay
// for new hand-offs while any walk lasts, the kernel ends once the lane is
// idle, and the host starts it again when hand-offs come.  Launched with
// enough dynamic LDS that no round workgroup fits beside it on its compute
// unit, so the walks do not share SIMDs with the main queue's waves.
struct TailArgs {
    Ctl *ctl;
    const JobDev *jobs;
    JobState *js;
    Lin lin;
    TailQ *q;
    unsigned long long *ring_host; // host-mapped, ring_cap entries
    uint32_t ring_cap;
    const uint32_t *stop_host;     // host-mapped
    unsigned long long idle_ticks;
    unsigned long long slice_ticks; // a launch's time slice (its walks are cut and queued again at its end)
    uint32_t *more_host;            // host-mapped: set when a walk was queued again (the host starts the next slice)
    uint32_t lds_entries;           // table entries each wave may copy to its part of the LDS
};

// A lone lineage's walk to its end (lanes 0-7 of a wave; the group's lanes
// agree throughout): from (p, t) event after event, with no horizon, until it
// speciates (kStepSpeciated; at = the event's location, t its time) or the
// search runs away (kStepSlow, flagged in err).  Every 512 events the walk
// reads *stop (when given) and the wall clock (when a deadline is given) and
// returns kStepOk if either says so (a passed deadline also flags kErrTimeout
// when late_is_error).  ev counts the events.
template <bool kLds, bool kUni>
__device__ __forceinline__ uint32_t walk_to_end(const JobView &v, Pos &p, double &t, uint32_t &at, uint32_t &ev,
                                                uint32_t gl, uint32_t grp_base, uint32_t *err, const uint32_t *stop,
                                                unsigned long long deadline, bool late_is_error) {
    uint2 row = table_row<kLds, kUni>(v, p);
    Counters cnt;
    uint32_t st = kStepOk;
    do {
        ++ev;
        at = p.loc;
        st = group_step<kLds, kUni>(v, p, t, row, gl, grp_base, cnt);
        if (__builtin_expect(st == kStepSlow, 0)) {
            t = next_event_time_group(v, p.loc, t, gl, grp_base, err, cnt);
            st = t < 0.0 ? kStepSlow : kStepOk; // kStepSlow now marks a runaway search
        }
        if ((ev & 511u) == 0u) {
            if (stop && __hip_atomic_load(stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) != 0u) return kStepOk;
            if (deadline && wall_clock64() > deadline) {
                if (late_is_error) atomicOr(err, kErrTimeout);
                return kStepOk;
            }
        }
    } while (st == kStepOk);
    return st;
}

// Writes the end of lineage g's walk (a speciation or a runaway search) into the
// lineage arrays.  One lane.
__device__ __forceinline__ void write_walk_end(const Lin &lin, const JobView &v, uint32_t g, uint32_t st, uint32_t at,
                                               const Pos &p, double t, uint32_t ev) {
    const bool speciated = st == kStepSpeciated;
    const uint32_t sloc = speciated ? at : p.loc;
    lin.species[g] = speciated ? species_of(v, sloc, t) : 0ull;
    lin.spec_loc[g] = sloc;
    lin.spec_t[g] = t;
    lin.events[g] += ev;
}

// Copies the shared dispersal table of v into this wave's part of the LDS
// (entries per wave, wave w of the workgroup from w * entries) when it fits;
// returns whether it did (then v reads it there).
__device__ __forceinline__ bool stage_wave_table(JobView &v, uint32_t entries) {
    if (!(v.mode == NH_DISPERSAL_SHARED && v.n_shared <= entries)) return false;
    v.lds_base = (threadIdx.x / 64) * entries;
    for (uint32_t e = lane_id(); e < v.n_shared; e += 64) nh_lds_table[v.lds_base + e] = v.table[e];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    return true;
}

// Queues lineage g at (loc, t) again (a walk cut at the end of its slice) in a
// free slot; false if none is free.  One lane.
__device__ __forceinline__ bool tail_requeue(TailQ *T, uint32_t g, uint32_t loc, double t) {
    uint32_t push = ld_agent(&T->push);
    while (true) {
        const uint32_t sq = ld_agent(&T->seq[push % kTailCap]);
        if (sq != (push < kTailCap ? 0u : ((push - kTailCap + 1u) | kTailCopied))) return false;
        const uint32_t seen = atomicCAS(&T->push, push, push + 1u);
        if (seen == push) break;
        push = seen;
    }
    const uint32_t i = push % kTailCap;
    T->g[i] = g;
    T->loc[i] = loc;
    T->t[i] = t;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    st_agent(&T->seq[i], push + 1u);
    return true;
}

// One walk of the tail lane: lineage g of job jb from (loc0, t0) until its end
// (its result written, the lineage retired, the job's completion on the host
// ring) or the end of the launch's slice (it is queued again where it stands,
// its events so far counted; if no slot is free it walks on).
template <bool kLds, bool kUni>
__device__ __forceinline__ void tail_walk(const TailArgs &A, const JobView &v, uint32_t g, uint32_t jb, uint32_t loc0,
                                          double t0, uint32_t gl, uint32_t grp_base, unsigned long long slice_end) {
    TailQ *T = A.q;
    Pos p = pos_from_loc(v, loc0);
    double t = t0;
    uint32_t at = p.loc, ev = 0, st = kStepOk;
    for (unsigned long long end = slice_end;; end = wall_clock64() + A.slice_ticks / 8) {
        st = walk_to_end<kLds, kUni>(v, p, t, at, ev, gl, grp_base, &A.ctl->error, A.stop_host, end, false);
        if (st != kStepOk) break;
        if (__hip_atomic_load(A.stop_host, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) != 0u) return; // going away
        bool queued = false;
        if (gl == 0u) queued = tail_requeue(T, g, p.loc, t);
        if (__shfl((int)queued, (int)grp_base, 64)) {
            if (gl == 0u) {
                A.lin.events[g] += ev;
                atomicAdd(&T->done, 1u);
                __hip_atomic_store(A.more_host, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            }
            return;
        }
    }
    if (gl != 0u) return;
    write_walk_end(A.lin, v, g, st, at, p, t, ev);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if (atomicSub(&A.js[jb].remaining, 1u) == 1u) {
        A.js[jb].done_round = ld_agent(&A.ctl->round);
        const uint32_t k = atomicAdd(&T->ring_n, 1u);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_store(&A.ring_host[k % A.ring_cap], ((unsigned long long)(k + 1u) << 32) | jb, __ATOMIC_RELEASE,
                           __HIP_MEMORY_SCOPE_SYSTEM);
    }
    atomicAdd(&T->done, 1u);
}

// Endgame of a persistent multi-job run (the launch stopped with
// kStopEndgame): the few lineages queued for the next round are walked to
// their ends independently, one wave each (lanes 0-7), with the shared table
// staged in the wave's part of the LDS when it fits, else read through the
// scalar cache.  Lineages that would still have merged walk the same events
// twice and reach the same species (an individual's species is a function of
// its own path alone), so only the event counts see the difference.  Wave w
// takes queue item w: the main queue first, then the solo queue from the top.
// A walk that passes the run's deadline flags kErrTimeout and stops.
__global__ __launch_bounds__(256) void k_endgame(RoundArgs A, unsigned long long run_ticks, uint32_t lds_entries) {
    Ctl *ctl = A.ctl;
    if (ld_agent(&ctl->stop) != kStopEndgame) return;
    const uint32_t r = ld_agent(&ctl->round);
    const uint32_t n_main = ld_agent(&ctl->count[r % 3]), n_solo = ld_agent(&ctl->solo[r % 3]);
    const uint32_t w = (blockIdx.x * blockDim.x + threadIdx.x) / 64, lane = lane_id();
    if (w >= n_main + n_solo) return;
    const uint32_t *act = A.lin.act[r & 1];
    const uint32_t g = w < n_main ? act[w] : act[A.n_cap - 1u - (w - n_main)];
    const uint32_t jb = A.lin.job[g];
    JobView v = load_view(&A.jobs[jb]);
    const bool stage = stage_wave_table(v, lds_entries);
    if (lane >= kGroup) return;
    Pos p = pos_from_loc(v, A.lin.loc[r & 1][g]);
    double t = A.lin.t[r & 1][g];
    uint32_t at = p.loc, ev = 0;
    const unsigned long long deadline = run_start(ctl) + run_ticks;
    const uint32_t st = stage ? walk_to_end<true, false>(v, p, t, at, ev, lane, 0u, &ctl->error, nullptr, deadline, true)
                              : walk_to_end<false, true>(v, p, t, at, ev, lane, 0u, &ctl->error, nullptr, deadline, true);
    if (st == kStepOk || lane != 0u) return; // past the deadline (flagged)
    write_walk_end(A.lin, v, g, st, at, p, t, ev);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    job_retired(ctl, A.js, A.ring, A.ring_cap, r, jb, 1u);
}

// After k_endgame: the run is over (unless a walk timed out).
__global__ void k_endgame_done(Ctl *ctl) {
    if (ctl->stop == kStopEndgame && (ctl->error & kErrTimeout) == 0u) ctl->stop = kStopDone;
}

__global__ __launch_bounds__(256) void k_tail(TailArgs A) {
    const uint32_t lane = lane_id(), gl = lane & (kGroup - 1), grp_base = lane & ~(kGroup - 1);
    TailQ *T = A.q;
    unsigned long long idle_from = wall_clock64();
    const unsigned long long slice_end = idle_from + A.slice_ticks;
    for (uint32_t poll = 0;; ++poll) {
        if (wall_clock64() >= slice_end) break; // claims nothing past its slice
        uint32_t take = 0, got = 0, stop = 0;
        if (lane == 0) {
            // the stop word lives in host memory: read it seldom (every 32nd poll, about 0.1 ms)
            if ((poll & 31u) == 0u) stop = __hip_atomic_load(A.stop_host, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            take = ld_agent(&T->take);
            if (!stop && ld_agent(&T->seq[take % kTailCap]) == take + 1u)
                got = atomicCAS(&T->take, take, take + 1u) == take ? 1u : 0u;
        }
        stop = (uint32_t)__builtin_amdgcn_readfirstlane(stop);
        got = (uint32_t)__builtin_amdgcn_readfirstlane(got);
        take = (uint32_t)__builtin_amdgcn_readfirstlane(take);
        if (stop) break;
        if (!got) {
            if (wall_clock64() - idle_from > A.idle_ticks && ld_agent(&T->busy) == 0u) break;
            __builtin_amdgcn_s_sleep(127); // about 3 us between polls
            continue;
        }
        if (lane == 0) atomicAdd(&T->busy, 1u);
        const uint32_t i = take % kTailCap;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        const uint32_t g = T->g[i], loc0 = T->loc[i];
        const double t0 = T->t[i];
        // the entry's loads complete before the slot is given back to the producers
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        if (lane == 0) st_agent(&T->seq[i], (take + 1u) | kTailCopied);
        {
            const uint32_t jb = A.lin.job[g];
            JobView v = load_view(&A.jobs[jb]);
            // a shared table that fits the wave's part of the LDS is copied there (the wave's 64 lanes),
            // else read through the scalar cache
            const bool stage = stage_wave_table(v, A.lds_entries);
            if (lane < kGroup) {
                if (stage) tail_walk<true, false>(A, v, g, jb, loc0, t0, gl, grp_base, slice_end);
                else tail_walk<false, true>(A, v, g, jb, loc0, t0, gl, grp_base, slice_end);
            }
        }
        __builtin_amdgcn_wave_barrier();
        if (lane == 0) atomicSub(&T->busy, 1u);
        idle_from = wall_clock64();
    }
}

// Single-thread epilogue of a round: publish the survivor count to the
// host-mapped status word and new job completions to the host-mapped ring,
// advance the round, reset the next queues.
// Once a round has left no survivors the run is over (stop = kStopDone): the
// rounds enqueued past it leave the round number and the status word alone,
// so the host reads the true last round however late it polls.
// tail/tail_host (servers with a tail lane): the count of tail hand-offs is
// copied to the host-mapped word, where the host sees that the lane has work.
__global__ void k_advance(Ctl *ctl, unsigned long long *status_host, const uint32_t *ring, uint32_t ring_cap,
                          uint32_t *ring_host, const TailQ *tail = nullptr, uint32_t *tail_host = nullptr) {
    if (ctl->stop == kStopDone) return;
    const uint32_t r = ctl->round;
    const uint32_t n_out = ctl->count[(r + 1) % 3] + ctl->solo[(r + 1) % 3];
    if (n_out == 0 && ring_host == nullptr) ctl->stop = kStopDone;
    ctl->count[(r + 2) % 3] = 0;
    ctl->solo[(r + 2) % 3] = 0;
    ctl->solo_cursor[(r + 1) % 3] = 0;
    ctl->cursor[(r + 1) % 3] = 0;
    ctl->round = r + 1;
    if (tail_host)
        __hip_atomic_store(tail_host, __hip_atomic_load(&tail->push, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    if (ring_host) {
        const uint32_t head = ctl->ring_head;
        for (uint32_t i = ctl->ring_pub; i != head; ++i)
            __hip_atomic_store(&ring_host[1 + i % ring_cap], ring[i % ring_cap], __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_SYSTEM);
        ctl->ring_pub = head;
        __hip_atomic_store(&ring_host[0], head, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    // a bad sample id only fails its own job (reported at completion); other flags stop the run
    const unsigned long long word = ((unsigned long long)(r + 1) << 32) | n_out |
                                    ((unsigned long long)((ctl->error & ~kErrBadSample) != 0) << 31);
    __hip_atomic_store(status_host, word, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Output: follow merge pointers to the representative, write species per
// sample; representatives insert their species into the job's set.  Counters
// are summed per wave when the whole wave belongs to one job.
// gate (nullable): the control block of a persistent run; nothing is done unless it finished.
__global__ void k_resolve(const JobDev *__restrict__ jobs, JobState *js, Lin lin, uint32_t g_begin, uint32_t g_end,
                          const Ctl *gate) {
    if (gate && gate->stop != kStopDone) return;
    const uint32_t g = g_begin + blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = g < g_end;
    uint32_t jb = 0;
    unsigned long long events = 0;
    bool is_root = false;
    if (valid) {
        jb = lin.job[g];
        const JobDev *J = &jobs[jb];
        uint32_t x = g;
        while (lin.parent[x] != x) x = lin.parent[x];
        const unsigned long long sp = lin.species[x];
        const uint32_t q = g - J->lin_base;
        J->species_out[q] = sp;
        if (J->spec_time_out) {
            J->spec_loc_out[q] = lin.spec_loc[x];
            J->spec_time_out[q] = lin.spec_t[x];
        }
        events = lin.events[g];
        is_root = x == g;
        // Representatives insert their species into the job's set; with the abundance reporter
        // every sample inserts-or-finds its species and counts itself at its slot.
        const bool count = J->abund_counts_out != nullptr;
        if (is_root || count) {
            if (sp == ~0ull) {
                if (is_root) atomicOr(&js[jb].flags, kJobSentinelSpecies);
                if (count) atomicAdd(&js[jb].sentinel_count, 1u);
            } else {
                uint32_t idx = (uint32_t)sp & J->rich_mask;
                for (uint32_t probe = 0; probe <= J->rich_mask; ++probe) {
                    unsigned long long cur = ~0ull;
                    if (__hip_atomic_compare_exchange_strong(&J->rich_set[idx], &cur, sp, __ATOMIC_RELAXED,
                                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                        atomicAdd(&js[jb].rich_count, 1ull);
                        break;
                    }
                    if (cur == sp) break;
                    idx = (idx + 1u) & J->rich_mask;
                }
                if (count) atomicAdd(&J->rich_counts[idx], 1u);
            }
        }
    }
    const uint64_t vmask = __ballot(valid);
    const int first = __ffsll((unsigned long long)vmask) - 1;
    const uint32_t jb0 = __shfl(jb, first < 0 ? 0 : first, 64);
    const bool uniform = __ballot(valid && jb != jb0) == 0;
    if (uniform) {
        const unsigned long long ev_sum = wave_sum(valid ? events : 0ull);
        const unsigned long long roots = (unsigned long long)__popcll(__ballot(valid && is_root));
        const unsigned long long n_valid = (unsigned long long)__popcll(vmask);
        if (vmask && lane_id() == (uint32_t)first) {
            atomicAdd(&js[jb0].events, ev_sum);
            atomicAdd(&js[jb0].speciated, roots);
            atomicAdd(&js[jb0].merged, n_valid - roots);
        }
    } else if (valid) {
        atomicAdd(&js[jb].events, events);
        atomicAdd(is_root ? &js[jb].speciated : &js[jb].merged, 1ull);
    }
}

// Per-event latency of one lineage on an otherwise idle device: a single group
// of 8 lanes (one wave, 56 lanes idle, as in the last rounds of a run) walks
// `steps` events of the round kernel's group step from sample 0's location,
// the shared table staged in LDS when the round kernel would stage it.  A
// speciation does not stop the walk (the step has moved the lineage anyway);
// a runaway search ends it.
template <bool kLds>
__global__ void k_event_latency(const JobDev *__restrict__ J, uint32_t steps, uint32_t *err,
                                unsigned long long *sink) {
    const JobView v = load_view(J);
    if (kLds) {
        for (uint32_t i = threadIdx.x; i < v.n_shared; i += blockDim.x) nh_lds_table[i] = v.table[i];
        __syncthreads();
    }
    const uint32_t lane = lane_id(), gl = lane & (kGroup - 1), grp_base = lane & ~(kGroup - 1);
    Counters cnt;
    Pos p = pos_from_loc(v, sample_loc(J, v, 0));
    double t = next_event_time(v, p.loc, 0.0, err, cnt);
    uint2 row = table_row<kLds>(v, p);
    for (uint32_t k = 0; k < steps && !(t < 0.0); ++k) {
        const uint32_t st = group_step<kLds>(v, p, t, row, gl, grp_base, cnt);
        if (st == kStepSlow) t = next_event_time_group(v, p.loc, t, gl, grp_base, err, cnt);
    }
    if (lane == 0) sink[0] = (unsigned long long)p.loc ^ (unsigned long long)__double_as_longlong(t);
}

// The path's primitives on given inputs, for device-level unit tests: 8 lanes
// per item (the group forms need a whole group; lane 0 runs the one-lane
// forms and writes).  An item whose location is not a slot of the scenario, or
// whose time is not a finite non-negative number below 2^40, gets NaN and
// 0xFFFFFFFF outputs and reads no table.
template <bool kLds>
__global__ void k_primitives(const JobDev *__restrict__ J, uint64_t n, nh_primitive_io io, uint32_t *err) {
    const JobView v = load_view(J);
    if (kLds) {
        for (uint32_t i = threadIdx.x; i < v.n_shared; i += blockDim.x) nh_lds_table[i] = v.table[i];
        __syncthreads();
    }
    const uint32_t lane = lane_id(), gl = lane & (kGroup - 1), grp_base = lane & ~(kGroup - 1);
    const uint64_t groups = (uint64_t)gridDim.x * (blockDim.x / kGroup);
    // the 8 lanes of a group hold the same item, so they take every branch together
    for (uint64_t i = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kGroup; i < n; i += groups) {
        if (io.d_ctr && io.d_philox_out && gl == 0u) {
            uint32_t c0 = io.d_ctr[4 * i], c1 = io.d_ctr[4 * i + 1], c2 = io.d_ctr[4 * i + 2], c3 = io.d_ctr[4 * i + 3];
            philox10(c0, c1, c2, c3, v.key0, v.key1);
            io.d_philox_out[4 * i] = c0;
            io.d_philox_out[4 * i + 1] = c1;
            io.d_philox_out[4 * i + 2] = c2;
            io.d_philox_out[4 * i + 3] = c3;
        }
        if (io.d_r && io.d_log_out && gl == 0u) io.d_log_out[i] = log_u53o(io.d_r[i]);
        if (!io.d_loc || !io.d_t) continue;
        const uint32_t loc = io.d_loc[i];
        const double t = io.d_t[i];
        const uint32_t cell = loc / v.cmax;
        const bool ok = cell < v.W * v.H && loc - cell * v.cmax < J->cap[cell] && t >= 0.0 && t < 0x1p40;
        if (!ok) {
            if (gl == 0u) {
                if (io.d_next_out) io.d_next_out[i] = __builtin_nan("");
                if (io.d_next_group_out) io.d_next_group_out[i] = __builtin_nan("");
                if (io.d_outcome_out) io.d_outcome_out[i] = 0xFFFFFFFFu;
                if (io.d_step_loc_out) io.d_step_loc_out[i] = 0xFFFFFFFFu;
                if (io.d_step_t_out) io.d_step_t_out[i] = __builtin_nan("");
            }
            continue;
        }
        Counters cnt;
        if (io.d_next_out && gl == 0u) io.d_next_out[i] = next_event_time(v, loc, t, err, cnt);
        if (io.d_next_group_out) {
            const double e = next_event_time_group(v, loc, t, gl, grp_base, err, cnt);
            if (gl == 0u) io.d_next_group_out[i] = e;
        }
        if (io.d_outcome_out && gl == 0u) {
            Pos p = pos_from_loc(v, loc);
            io.d_outcome_out[i] = commit_event<kLds>(v, p, t, cnt) ? NH_EVENT_SPECIATION : p.loc;
        }
        if (io.d_step_loc_out && io.d_step_t_out) {
            // one group step (event, then the search from the new location, finished by the full
            // group search when the first pass cannot decide)
            Pos p = pos_from_loc(v, loc);
            double tt = t;
            uint2 row = table_row<kLds>(v, p);
            const uint32_t st = group_step<kLds>(v, p, tt, row, gl, grp_base, cnt);
            if (st == kStepSlow) tt = next_event_time_group(v, p.loc, tt, gl, grp_base, err, cnt);
            if (gl == 0u) {
                io.d_step_loc_out[i] = st == kStepSpeciated ? NH_EVENT_SPECIATION : p.loc;
                io.d_step_t_out[i] = st == kStepSpeciated ? t : tt;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Event stream (sections "Sorting Events using the Water-Level Algorithm" and
// "Reporting Coalescence Events Independently").  After a completed run each
// lineage knows how many events it committed (redundant copies of an event it
// shared with another lineage included) and whether it stopped by merging.
// Replaying those events from the sample's start gives one record (t, prior
// event time, origin, outcome) per committed event; a merged lineage adds one
// record for the state it was merged at (its next event, committed by the
// lineage it merged into).  Every lineage that reaches an event leaves a copy
// of it with its own prior event time, so after a stable sort by (job, t,
// origin, prior) the first copy of each event carries the parent's prior time
// and every further distinct prior time is the arrival of a lineage that found
// the origin occupied: a coalescence.  That is the same reduced stream as
// tracing every sample alone to its speciation, without the redundant work.
// ---------------------------------------------------------------------------
constexpr uint32_t kRecMerged = 0xFFFFFFFEu; // outcome of a merge-state record
constexpr uint32_t kErrStream = 8u;          // a replay did not retrace its lineage

struct StreamRecs {   // one entry per record (structure of arrays)
    uint64_t *t;      // bits of the event time (non-negative doubles order as their bits)
    uint64_t *prior;  // bits of the prior event time
    uint32_t *from;   // origin location
    uint32_t *to;     // new location, NH_EVENT_SPECIATION or kRecMerged
    uint32_t *job;
};

struct StreamDev {    // per-job outputs
    nh_event *ev;
    uint64_t ev_cap;
    nh_coalescence *co;
    uint64_t co_cap;
};

__device__ __forceinline__ bool stream_bad(const JobDev *__restrict__ J, uint32_t g) {
    return J->samples[g - J->lin_base] >= J->n_individuals;
}

// Records per lineage: its committed events, plus one if it was merged.
__global__ void k_stream_count(const JobDev *__restrict__ jobs, Lin lin, uint32_t n_total, uint64_t *n_rec) {
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n_total) return;
    const JobDev *J = &jobs[lin.job[g]];
    n_rec[g] = stream_bad(J, g) ? 0ull : (uint64_t)lin.events[g] + (lin.parent[g] != g ? 1ull : 0ull);
}

// Replays lineage g's committed events into records off[g] ..: 8 lanes per
// lineage with the round kernel's group step (the same bits as its one-lane
// form), so the longest lineage, which sets the replay time, moves at the
// tail rate.  The group leader writes the records.
__global__ void k_stream_replay(const JobDev *__restrict__ jobs, Lin lin, uint32_t n_total,
                                const uint64_t *__restrict__ off, StreamRecs R, uint32_t *err) {
    const uint32_t lane = lane_id(), gl = lane & (kGroup - 1), grp_base = lane & ~(kGroup - 1);
    const uint32_t groups = gridDim.x * (blockDim.x / kGroup);
    // the 8 lanes of a group hold the same g and the same state throughout, so they leave
    // every loop together
    for (uint32_t g = (blockIdx.x * blockDim.x + threadIdx.x) / kGroup; g < n_total; g += groups) {
        const uint32_t jb = lin.job[g];
        const JobDev *J = &jobs[jb];
        if (stream_bad(J, g)) continue;
        const JobView v = load_view(J);
        Counters cnt;
        Pos p = pos_from_loc(v, sample_loc(J, v, J->samples[g - J->lin_base]));
        double t = next_event_time(v, p.loc, 0.0, err, cnt), prior = 0.0;
        uint64_t o = off[g];
        const uint32_t n_ev = lin.events[g];
        const bool merged = lin.parent[g] != g;
        bool ended = false, bad = false;
        uint2 row = table_row<false>(v, p);
        for (uint32_t k = 0; k < n_ev; ++k) {
            if (t < 0.0) { // runaway search (flagged by the search)
                bad = true;
                break;
            }
            const uint32_t from = p.loc;
            const double te = t;
            const uint32_t st = group_step<false>(v, p, t, row, gl, grp_base, cnt);
            const bool spec = st == kStepSpeciated;
            if (gl == 0u) {
                R.t[o] = (uint64_t)__double_as_longlong(te);
                R.prior[o] = (uint64_t)__double_as_longlong(prior);
                R.from[o] = from;
                R.to[o] = spec ? NH_EVENT_SPECIATION : p.loc;
                R.job[o] = jb;
            }
            ++o;
            if (spec) {
                // only a representative's last event speciates
                bad = k + 1 != n_ev || merged;
                ended = true;
                break;
            }
            if (st == kStepSlow) t = next_event_time_group(v, p.loc, te, gl, grp_base, err, cnt);
            prior = te;
        }
        if (!bad && !ended) {
            // a representative must have ended by speciating
            bad = !merged || t < 0.0;
            if (!bad && gl == 0u) {
                R.t[o] = (uint64_t)__double_as_longlong(t);
                R.prior[o] = (uint64_t)__double_as_longlong(prior);
                R.from[o] = p.loc;
                R.to[o] = kRecMerged;
                R.job[o] = jb;
            }
        }
        if (bad && gl == 0u) atomicOr(err, kErrStream);
    }
}

__global__ void k_iota(uint32_t *v, uint32_t n) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) v[i] = i;
}

template <typename T>
__global__ void k_gather(const T *__restrict__ src, const uint32_t *__restrict__ perm, T *__restrict__ dst,
                         uint32_t n) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) dst[i] = src[perm[i]];
}

__device__ __forceinline__ bool same_event(const StreamRecs &R, uint32_t a, uint32_t b) {
    return R.job[a] == R.job[b] && R.t[a] == R.t[b] && R.from[a] == R.from[b];
}

// Over the sorted records: the first copy of an event, and the copies whose prior
// time differs from the previous copy's (coalescences); counts per job.
// The per-job counts are added once per wave when the wave's records belong to
// one job (the usual case: records are sorted by job), so a single-job stream
// does not funnel every record through one atomic counter.
__global__ void k_stream_flags(StreamRecs R, const uint32_t *__restrict__ perm, uint32_t n, uint32_t *flag_ev,
                               uint32_t *flag_co, unsigned long long *ev_count, unsigned long long *co_count) {
    // every lane of a wave runs the same number of iterations, so the ballots see the whole wave
    for (uint32_t base = blockIdx.x * blockDim.x; base < n; base += gridDim.x * blockDim.x) {
        const uint32_t i = base + threadIdx.x;
        const bool valid = i < n;
        bool first = false, coal = false;
        uint32_t jb = 0;
        if (valid) {
            const uint32_t e = perm[i];
            first = i == 0 || !same_event(R, perm[i - 1], e);
            coal = !first && R.prior[perm[i - 1]] != R.prior[e];
            flag_ev[i] = first;
            flag_co[i] = coal;
            jb = R.job[e];
        }
        const uint64_t vmask = __ballot(valid);
        if (vmask == 0) continue;
        const int lead = __ffsll((unsigned long long)vmask) - 1;
        const uint32_t jb0 = __shfl(jb, lead, 64);
        if (__ballot(valid && jb != jb0) == 0) {
            const unsigned long long ne = (unsigned long long)__popcll(__ballot(first));
            const unsigned long long nc = (unsigned long long)__popcll(__ballot(coal));
            if (lane_id() == (uint32_t)lead) {
                if (ne) atomicAdd(&ev_count[jb0], ne);
                if (nc) atomicAdd(&co_count[jb0], nc);
            }
        } else {
            if (first) atomicAdd(&ev_count[jb], 1ull);
            if (coal) atomicAdd(&co_count[jb], 1ull);
        }
    }
}

// Writes each event (its first copy, the outcome of a copy that committed it)
// at its rank within the job, and gathers the coalescences, each with the
// prior time of its event's first copy (the parent's arrival).
__global__ void k_stream_emit(StreamRecs R, const uint32_t *__restrict__ perm, uint32_t n,
                              const uint32_t *__restrict__ flag_ev, const uint32_t *__restrict__ rank_ev,
                              const uint32_t *__restrict__ flag_co, const uint32_t *__restrict__ rank_co,
                              const uint64_t *__restrict__ ev_base, const StreamDev *__restrict__ outs,
                              StreamRecs C, uint32_t *err) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const uint32_t e = perm[i];
        if (flag_ev[i]) {
            const uint32_t jb = R.job[e];
            const uint64_t local = rank_ev[i] - ev_base[jb];
            if (local < outs[jb].ev_cap) {
                uint32_t k = i;
                while (k < n && same_event(R, perm[k], e) && R.to[perm[k]] == kRecMerged) ++k;
                const bool found = k < n && same_event(R, perm[k], e);
                if (!found) atomicOr(err, kErrStream);
                nh_event out;
                out.t = __longlong_as_double((long long)R.t[e]);
                out.t_prior = __longlong_as_double((long long)R.prior[e]);
                out.origin = R.from[e];
                out.outcome = found ? R.to[perm[k]] : NH_EVENT_SPECIATION;
                outs[jb].ev[local] = out;
            }
        }
        if (flag_co[i]) {
            uint32_t k = i;
            while (k > 0 && same_event(R, perm[k - 1], e)) --k;
            const uint32_t c = rank_co[i];
            C.t[c] = R.prior[e];
            C.prior[c] = R.prior[perm[k]];
            C.from[c] = R.from[e];
            C.job[c] = R.job[e];
        }
    }
}

// Writes the sorted coalescences at their rank within the job.
__global__ void k_stream_coal_write(StreamRecs C, const uint32_t *__restrict__ perm, uint32_t n,
                                    const uint64_t *__restrict__ co_base, const StreamDev *__restrict__ outs) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const uint32_t e = perm[i];
        const uint32_t jb = C.job[e];
        const uint64_t local = i - co_base[jb];
        if (local < outs[jb].co_cap) {
            nh_coalescence out;
            out.t = __longlong_as_double((long long)C.t[e]);
            out.t_parent = __longlong_as_double((long long)C.prior[e]);
            out.loc = C.from[e];
            out.reserved = 0;
            outs[jb].co[local] = out;
        }
    }
}

// Abundance reporter: every occupied slot of the species sets of jobs
// [j_lo, j_hi) (contiguous in the species-set area, n_slots in all) appends its
// (species, samples) pair to its job's output.
__global__ void k_abundance(const JobDev *__restrict__ jobs, JobState *js, uint32_t j_lo, uint32_t j_hi,
                            uint64_t n_slots, const Ctl *gate) {
    if (gate && gate->stop != kStopDone) return;
    const uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_slots) return;
    const uint64_t base = jobs[j_lo].rich_off;
    uint32_t lo = j_lo, hi = j_hi; // the last job whose set starts at or before slot s
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (jobs[mid].rich_off - base <= s) lo = mid;
        else hi = mid;
    }
    const JobDev *J = &jobs[lo];
    if (!J->abund_counts_out) return;
    const uint64_t local = s - (J->rich_off - base);
    if (local > J->rich_mask) return;
    const unsigned long long id = J->rich_set[local];
    if (id == ~0ull) return;
    const uint32_t at = atomicAdd(&js[lo].abund_n, 1u);
    J->abund_ids_out[at] = id;
    J->abund_counts_out[at] = J->rich_counts[local];
}

// gate as for k_resolve.  mark_failure (enqueue-only calls, which return no
// status): a job of a run that did not finish, or with a sample id >= N, gets
// the richness ~0 instead.
__global__ void k_finalize(const JobDev *__restrict__ jobs, JobState *js, uint32_t j_begin, uint32_t j_end,
                           const Ctl *gate, uint32_t mark_failure) {
    const uint32_t j = j_begin + blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= j_end) return;
    if ((gate && gate->stop != kStopDone) || (mark_failure && (js[j].flags & kJobBadSample))) {
        if (mark_failure && jobs[j].richness_out) *jobs[j].richness_out = ~0ull;
        return;
    }
    const bool sentinel = (js[j].flags & kJobSentinelSpecies) != 0u;
    const unsigned long long rich = js[j].rich_count + (sentinel ? 1ull : 0ull);
    js[j].rich_count = rich;
    if (jobs[j].richness_out) *jobs[j].richness_out = rich;
    if (sentinel && jobs[j].abund_counts_out) {
        const uint32_t at = js[j].abund_n++;
        jobs[j].abund_ids_out[at] = ~0ull;
        jobs[j].abund_counts_out[at] = js[j].sentinel_count;
    }
}

// ---------------------------------------------------------------------------
// Measurement helpers (not part of the method): the throughput the chip
// sustains for the event path's own instruction mix with every lane busy, and
// for random 16-byte gathers from a large table.
// ---------------------------------------------------------------------------
constexpr uint32_t kMixPhilox = 3, kMixDraws = 2; // per iteration: about the event path's 1.6 blocks per draw

__global__ __launch_bounds__(256) void k_peak_mix(uint32_t iters, uint64_t seed, unsigned long long *sink) {
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    uint32_t s0 = g, s1 = 0;
    double acc = 0.0;
    for (uint32_t i = 0; i < iters; ++i) {
        uint32_t w[kMixPhilox][4];
#pragma unroll
        for (uint32_t b = 0; b < kMixPhilox; ++b) {
            w[b][0] = s0;
            w[b][1] = i;
            w[b][2] = s1;
            w[b][3] = b;
            philox10(w[b][0], w[b][1], w[b][2], w[b][3], k0, k1);
        }
#pragma unroll
        for (uint32_t d = 0; d < kMixDraws; ++d) acc += log_u53o(((uint64_t)w[d][1] << 32) | w[d][0]);
        s1 ^= w[kMixPhilox - 1][2];
    }
    if (acc == 1.0) sink[g] = s1; // never true (a sum of logs of (0,1] draws); keeps the work live
}

__global__ __launch_bounds__(256) void k_peak_gather(const uint4 *__restrict__ table, uint64_t n_entries,
                                                     uint32_t iters, unsigned long long *sink) {
    const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t h = g * 0x9E3779B97F4A7C15ull + 1ull;
    uint32_t acc = 0;
    for (uint32_t i = 0; i < iters; ++i) {
        h ^= h >> 31;
        h *= 0xBF58476D1CE4E5B9ull;
        h ^= h >> 29;
        const uint4 e = table[mulhi_index(h, (uint32_t)min<uint64_t>(n_entries, 0xFFFFFFFFull))];
        acc += e.x ^ e.y ^ e.z ^ e.w;
    }
    if (acc == 0x12345678u) sink[g] = acc; // keeps the loads live
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
inline uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

inline uint64_t pow2_at_least(uint64_t x, uint64_t floor_value) {
    uint64_t p = floor_value;
    while (p < x) p <<= 1;
    return p;
}

// ceil(p * 2^53) for p in [0, 1]: the integer threshold with
// (r >> 11) < ceil(p 2^53)  <=>  (r >> 11) * 2^-53 < p.
inline uint64_t u53_threshold(double p) { return (uint64_t)std::ceil(std::ldexp(p, 53)); }

// Smallest binary64 t >= 0 with lambda * t >= tau after rounding.  The rounded
// product is non-decreasing in t, so lambda * t < tau holds exactly for t below
// it: the protracted-speciation test needs one compare per event and no product.
double protracted_threshold(double tau, double lambda) {
    if (!(tau > 0.0)) return 0.0;
    double t = tau / lambda;
    while (lambda * t < tau) t = std::nextafter(t, INFINITY);
    while (t > 0.0) {
        const double below = std::nextafter(t, 0.0);
        if (lambda * below < tau) break;
        t = below;
    }
    return t;
}

bool is_power_of_two(double x) {
    int e;
    const double m = std::frexp(x, &e);
    return x > 0.0 && std::isfinite(x) && m == 0.5;
}

// Vose alias construction in a fixed order (the same steps as any conforming
// implementation must take for bit-identical tables): p_i = (w_i n) / W with W
// summed in index order; ascending scan into "small" (p < 1) and "large"
// stacks; pop one of each (last pushed first), prob[s] = p_s, alias[s] = l,
// p_l = (p_l + p_s) - 1, push l by its new value; leftovers keep prob 1.
void vose(const double *w, uint32_t n, double *prob, uint32_t *alias, std::vector<double> &p,
          std::vector<uint32_t> &small, std::vector<uint32_t> &large) {
    double total = 0.0;
    for (uint32_t i = 0; i < n; ++i) total = total + w[i];
    p.resize(n);
    small.resize(n);
    large.resize(n);
    uint32_t ns = 0, nl = 0;
    for (uint32_t i = 0; i < n; ++i) {
        p[i] = (w[i] * (double)n) / total;
        if (p[i] < 1.0) small[ns++] = i;
        else large[nl++] = i;
    }
    while (ns > 0 && nl > 0) {
        const uint32_t s = small[--ns];
        const uint32_t l = large[--nl];
        prob[s] = p[s];
        alias[s] = l;
        p[l] = (p[l] + p[s]) - 1.0;
        if (p[l] < 1.0) small[ns++] = l;
        else large[nl++] = l;
    }
    while (nl > 0) {
        const uint32_t l = large[--nl];
        prob[l] = 1.0;
        alias[l] = l;
    }
    while (ns > 0) {
        const uint32_t s = small[--ns];
        prob[s] = 1.0;
        alias[s] = s;
    }
}

// Alias table of one deme (cell < 0: the shared table) packed for the device:
// x,y = threshold of the column, z = offsets of the column (low 16 bits) and of
// its alias (high 16 bits), each as (dx + R) | (dy + R) << 8.
struct TableBuilder {
    uint32_t W, H, R, side;
    const uint32_t *cap;
    const double *weights;
    std::vector<double> w, prob, p;
    std::vector<uint32_t> kidx, alias, small, large;

    uint32_t count(int64_t cell) const {
        uint32_t n = 0;
        for (uint32_t k = 0; k < side * side; ++k)
            if (mass(cell, k) > 0.0) ++n;
        return n;
    }
    uint32_t target_cap(int64_t cell, uint32_t k) const {
        const int64_t x = cell % W, y = cell / W;
        const int64_t dx = (int64_t)(k % side) - R, dy = (int64_t)(k / side) - R;
        const int64_t tx = ((x + dx) % (int64_t)W + W) % W;
        const int64_t ty = ((y + dy) % (int64_t)H + H) % H;
        return cap[ty * W + tx];
    }
    double mass(int64_t cell, uint32_t k) const {
        double wk = weights[k];
        if (cell >= 0) {
            const int64_t x = cell % W, y = cell / W;
            const int64_t dx = (int64_t)(k % side) - R, dy = (int64_t)(k / side) - R;
            const int64_t tx = ((x + dx) % (int64_t)W + W) % W;
            const int64_t ty = ((y + dy) % (int64_t)H + H) % H;
            wk = wk * (double)cap[ty * W + tx];
        }
        return wk;
    }
    uint32_t build(int64_t cell, uint4 *out) {
        w.clear();
        kidx.clear();
        for (uint32_t k = 0; k < side * side; ++k) {
            const double m = mass(cell, k);
            if (m > 0.0) {
                w.push_back(m);
                kidx.push_back(k);
            }
        }
        const uint32_t n = (uint32_t)w.size();
        prob.resize(n);
        alias.resize(n);
        vose(w.data(), n, prob.data(), alias.data(), p, small, large);
        auto pack = [&](uint32_t k) { return (k % side) | ((k / side) << 8); };
        // Per-deme tables also carry both candidate targets' capacities (16 bits each, 0 when one
        // does not fit), so dispersal needs no further dependent load for the deme index.
        auto cap16 = [&](uint32_t k) { const uint32_t c = target_cap(cell, k); return c <= 0xFFFFu ? c : 0u; };
        for (uint32_t c = 0; c < n; ++c) {
            const uint64_t th = u53_threshold(prob[c]);
            const uint32_t caps = cell >= 0 ? (cap16(kidx[c]) | (cap16(kidx[alias[c]]) << 16)) : 0u;
            out[c] = make_uint4((uint32_t)th, (uint32_t)(th >> 32), pack(kidx[c]) | (pack(kidx[alias[c]]) << 16), caps);
        }
        return n;
    }
};

} // namespace

struct nh_scenario {
    int device = 0;
    uint32_t sampler = NH_SAMPLER_EXP;
    double mu = 1.0, p0 = 0.0; // Poisson sampler: lambda * delta_t and exp(-lambda * delta_t)
    uint64_t mig_thresh = 0;   // spatially implicit scenario: ceil(m 2^53)
    double tau = 0, tau_t = 0; // protracted speciation: generations, and the threshold time
    uint32_t W = 0, H = 0, R = 0, mode = 0, cmax = 0, cap_const = 0, n_shared = 0;
    uint64_t cells = 0, N = 0, n_entries = 0;
    double nu = 0, lambda = 1, dt = 1;
    uint64_t nu_thresh = 0;
    uint4 *d_table = nullptr;
    uint32_t *d_row_ptr = nullptr;
    uint32_t *d_cap = nullptr;
    uint64_t *d_prefix = nullptr;
    uint64_t table_bytes = 0;
};

namespace {

// Library-internal non-blocking stream per device: scenario tables are
// allocated, uploaded and freed stream-ordered on it, so creating or
// destroying a scenario never synchronises work on other streams.
hipStream_t table_stream(int device) {
    static std::mutex mu;
    static hipStream_t streams[64] = {};
    std::lock_guard<std::mutex> lock(mu);
    if (device < 0 || device >= 64) return nullptr;
    if (!streams[device]) {
        int prev = 0;
        (void)hipGetDevice(&prev);
        (void)hipSetDevice(device);
        if (hipStreamCreateWithFlags(&streams[device], hipStreamNonBlocking) != hipSuccess) streams[device] = nullptr;
        (void)hipSetDevice(prev);
    }
    return streams[device];
}

void scenario_free(nh_scenario *s) {
    if (!s) return;
    if (s->device < 0 || !(s->d_table || s->d_row_ptr || s->d_cap || s->d_prefix)) {
        delete s;
        return;
    }
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(s->device);
    hipStream_t ts = table_stream(s->device);
    if (s->d_table) (void)hipFreeAsync(s->d_table, ts);
    if (s->d_row_ptr) (void)hipFreeAsync(s->d_row_ptr, ts);
    if (s->d_cap) (void)hipFreeAsync(s->d_cap, ts);
    if (s->d_prefix) (void)hipFreeAsync(s->d_prefix, ts);
    (void)hipSetDevice(prev);
    delete s;
}

struct Workspace {
    uint64_t off_ctl, off_jobs, off_js, off_ring, off_htab, off_loc0, off_loc1, off_t0, off_t1, off_parent, off_species,
        off_job, off_events, off_sloc, off_st, off_act0, off_act1, off_hash, off_rich, off_rcount, total;
    uint64_t hcap;
};

Workspace layout(uint64_t n_total, uint32_t n_jobs) {
    Workspace w{};
    const uint64_t N = std::max<uint64_t>(n_total, 1);
    uint64_t o = 0;
    auto take = [&](uint64_t bytes) {
        const uint64_t at = o;
        o = align_up(o + bytes, 256);
        return at;
    };
    w.off_ctl = take(sizeof(Ctl));
    w.off_jobs = take(sizeof(JobDev) * std::max<uint32_t>(n_jobs, 1));
    w.off_js = take(sizeof(JobState) * std::max<uint32_t>(n_jobs, 1));
    w.off_ring = take(sizeof(uint32_t) * std::max<uint32_t>(n_jobs, 1));
    w.off_htab = take(sizeof(double) * kMaxHorizons);
    w.off_loc0 = take(4 * N);
    w.off_loc1 = take(4 * N);
    w.off_t0 = take(8 * N);
    w.off_t1 = take(8 * N);
    w.off_parent = take(4 * N);
    w.off_species = take(8 * N);
    w.off_job = take(4 * N);
    w.off_events = take(4 * N);
    w.off_sloc = take(4 * N);
    w.off_st = take(8 * N);
    w.off_act0 = take(4 * N);
    w.off_act1 = take(4 * N);
    w.hcap = pow2_at_least(2 * N, 1024);
    w.off_hash = take(8 * w.hcap);
    w.off_rich = take(8 * (4 * N + 64ull * std::max<uint32_t>(n_jobs, 1)));
    w.off_rcount = take(4 * (4 * N + 64ull * std::max<uint32_t>(n_jobs, 1)));
    w.total = o;
    return w;
}

// The lineage arrays of a batch workspace.
Lin lin_view(char *ws, const Workspace &L) {
    Lin lin;
    lin.loc[0] = (uint32_t *)(ws + L.off_loc0);
    lin.loc[1] = (uint32_t *)(ws + L.off_loc1);
    lin.t[0] = (double *)(ws + L.off_t0);
    lin.t[1] = (double *)(ws + L.off_t1);
    lin.parent = (uint32_t *)(ws + L.off_parent);
    lin.species = (unsigned long long *)(ws + L.off_species);
    lin.job = (uint32_t *)(ws + L.off_job);
    lin.events = (uint32_t *)(ws + L.off_events);
    lin.spec_loc = (uint32_t *)(ws + L.off_sloc);
    lin.spec_t = (double *)(ws + L.off_st);
    lin.act[0] = (uint32_t *)(ws + L.off_act0);
    lin.act[1] = (uint32_t *)(ws + L.off_act1);
    lin.hash = (unsigned long long *)(ws + L.off_hash);
    lin.hmask = (uint32_t)(L.hcap - 1);
    return lin;
}

struct PinnedStatus {
    unsigned long long *host = nullptr;
    unsigned long long *dev = nullptr;
};

int pinned_status(PinnedStatus &out) {
    thread_local PinnedStatus ps;
    if (!ps.host) {
        void *h = nullptr;
        HIP_TRY(hipHostMalloc(&h, 256, hipHostMallocMapped | hipHostMallocPortable | hipHostMallocCoherent));
        void *d = nullptr;
        HIP_TRY(hipHostGetDevicePointer(&d, h, 0));
        ps.host = (unsigned long long *)h;
        ps.dev = (unsigned long long *)d;
    }
    out = ps;
    return NH_OK;
}

void fill_config(const nh_config *in, nh_config &c) {
    c = nh_config{};
    if (in) c = *in;
    if (!(c.horizon0 > 0)) c.horizon0 = 0.5;
    if (!(c.horizon_growth > 1.0)) c.horizon_growth = 1.25;
    if (!(c.horizon_step_max > 0)) c.horizon_step_max = 4096.0;
    if (c.block_size == 0) c.block_size = 256;
    if (c.blocks_per_cu == 0) c.blocks_per_cu = 4;
    if (c.rounds_per_graph == 0) c.rounds_per_graph = 8;
    if (c.table_placement > 1) c.table_placement = 0;
    if (!(c.timeout_s > 0)) c.timeout_s = 600.0;
    if (!(c.solo_step > 0)) c.solo_step = 512.0;
}

std::vector<double> horizon_table(const nh_config &c) {
    std::vector<double> h(kMaxHorizons, 0.0);
    h[0] = 0.0;
    h[1] = c.horizon0;
    for (uint32_t i = 2; i < kMaxHorizons; ++i)
        h[i] = h[i - 1] + std::min(c.horizon_step_max, h[i - 1] * (c.horizon_growth - 1.0));
    return h;
}

} // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
NH_API const char *nh_last_error(void) { return g_last_error.c_str(); }

NH_API const char *nh_version(void) { return "libnecsim_hip 0.1 (gfx950)"; }

NH_API uint64_t nh_struct_bytes(const char *name) {
    if (!name) return 0;
    const std::pair<const char *, uint64_t> sizes[] = {
        {"nh_habitat", sizeof(nh_habitat)},           {"nh_dispersal", sizeof(nh_dispersal)},
        {"nh_params", sizeof(nh_params)},             {"nh_config", sizeof(nh_config)},
        {"nh_stats", sizeof(nh_stats)},               {"nh_job", sizeof(nh_job)},
        {"nh_event", sizeof(nh_event)},               {"nh_coalescence", sizeof(nh_coalescence)},
        {"nh_stream_out", sizeof(nh_stream_out)},     {"nh_server_config", sizeof(nh_server_config)},
        {"nh_completion", sizeof(nh_completion)},     {"nh_primitive_io", sizeof(nh_primitive_io)}};
    for (const auto &e : sizes)
        if (std::strcmp(e.first, name) == 0) return e.second;
    return 0;
}

NH_API int nh_measure_mix_peak(double *lane_ops_per_s, void *stream_ptr) {
    if (!lane_ops_per_s) return fail(NH_EINVAL, "NULL output");
    hipStream_t stream = (hipStream_t)stream_ptr;
    int dev = 0, n_cu = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
    const uint32_t blocks = (uint32_t)std::max(1, n_cu) * 8, threads = 256, iters = 2048;
    unsigned long long *sink = nullptr;
    HIP_TRY(hipMallocAsync((void **)&sink, sizeof(unsigned long long) * blocks * threads, stream));
    hipEvent_t a, b;
    HIP_TRY(hipEventCreate(&a));
    HIP_TRY(hipEventCreate(&b));
    k_peak_mix<<<blocks, threads, 0, stream>>>(64, 1, sink); // warm-up
    HIP_TRY(hipEventRecord(a, stream));
    k_peak_mix<<<blocks, threads, 0, stream>>>(iters, 2, sink);
    HIP_TRY(hipEventRecord(b, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, a, b));
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    (void)hipFreeAsync(sink, stream);
    const double ops_per_iter = 100.0 * kMixPhilox + 43.0 * kMixDraws;
    *lane_ops_per_s = (double)blocks * threads * iters * ops_per_iter / (ms * 1e-3);
    return NH_OK;
}

NH_API int nh_measure_gather(const void *d_table, uint64_t table_bytes, double *bytes_per_s, void *stream_ptr) {
    if (!d_table || !bytes_per_s || table_bytes < 16 * 1024) return fail(NH_EINVAL, "bad gather table");
    hipStream_t stream = (hipStream_t)stream_ptr;
    int dev = 0, n_cu = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
    const uint32_t blocks = (uint32_t)std::max(1, n_cu) * 8, threads = 256, iters = 256;
    unsigned long long *sink = nullptr;
    HIP_TRY(hipMallocAsync((void **)&sink, sizeof(unsigned long long) * blocks * threads, stream));
    hipEvent_t a, b;
    HIP_TRY(hipEventCreate(&a));
    HIP_TRY(hipEventCreate(&b));
    const uint64_t n = table_bytes / 16;
    k_peak_gather<<<blocks, threads, 0, stream>>>((const uint4 *)d_table, n, 16, sink); // warm-up
    HIP_TRY(hipEventRecord(a, stream));
    k_peak_gather<<<blocks, threads, 0, stream>>>((const uint4 *)d_table, n, iters, sink);
    HIP_TRY(hipEventRecord(b, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, a, b));
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    (void)hipFreeAsync(sink, stream);
    *bytes_per_s = (double)blocks * threads * iters * 16.0 / (ms * 1e-3);
    return NH_OK;
}


NH_API int nh_scenario_create(const nh_habitat *habitat, const nh_dispersal *dispersal, double nu,
                              const nh_params *params, nh_scenario **out) {
    if (!out) return fail(NH_EINVAL, "out is NULL");
    *out = nullptr;
    if (!habitat || !dispersal || !habitat->h_capacity || !dispersal->h_weights)
        return fail(NH_EINVAL, "NULL habitat or dispersal");
    const uint32_t W = habitat->width, H = habitat->height, R = dispersal->radius;
    if (W == 0 || H == 0) return fail(NH_EINVAL, "empty habitat");
    if (dispersal->mode > 1) return fail(NH_EINVAL, "unknown dispersal mode %u", dispersal->mode);
    if (R > 127 || 2ull * R + 1 > W || 2ull * R + 1 > H)
        return fail(NH_EINVAL, "kernel side 2R+1 = %llu exceeds the habitat or 255", 2ull * R + 1);
    if (!(nu > 0.0 && nu <= 1.0)) return fail(NH_EINVAL, "nu must lie in (0, 1]");
    const double lambda = params ? params->lambda : 1.0;
    const double dt = params ? params->delta_t : 1.0;
    if (!(lambda > 0.0) || !std::isfinite(lambda)) return fail(NH_EINVAL, "lambda must be positive and finite");
    if (!is_power_of_two(dt)) return fail(NH_EINVAL, "delta_t must be a positive power of two");
    if (lambda * dt > 1048576.0) return fail(NH_EINVAL, "lambda * delta_t must not exceed 2^20");
    const uint32_t sampler = params ? params->sampler : NH_SAMPLER_EXP;
    if (sampler > NH_SAMPLER_POISSON) return fail(NH_EINVAL, "unknown event-time sampler %u", sampler);
    if (sampler == NH_SAMPLER_POISSON && !(lambda * dt <= 700.0))
        return fail(NH_EINVAL, "the Poisson sampler needs lambda * delta_t <= 700");
    const double tau = params ? params->tau : 0.0;
    if (!(tau >= 0.0) || !(tau / lambda < 0x1p60))
        return fail(NH_EINVAL, "tau must be non-negative with tau / lambda below 2^60");
    const uint32_t side = 2 * R + 1;
    for (uint32_t k = 0; k < side * side; ++k) {
        const double w = dispersal->h_weights[k];
        if (!(w >= 0.0) || !std::isfinite(w)) return fail(NH_EINVAL, "weight %u is negative or not finite", k);
    }
    const uint64_t cells = (uint64_t)W * H;
    const uint32_t *cap = habitat->h_capacity;
    std::vector<uint64_t> prefix(cells + 1);
    uint64_t acc = 0;
    uint32_t cmax = 0;
    bool constant = true;
    for (uint64_t c = 0; c < cells; ++c) {
        prefix[c] = acc;
        acc += cap[c];
        cmax = std::max(cmax, cap[c]);
        if (cap[c] != cap[0]) constant = false;
        if (dispersal->mode == NH_DISPERSAL_SHARED && cap[c] == 0)
            return fail(NH_EINVAL, "the shared dispersal mode needs every deme habitable (cell %llu)",
                        (unsigned long long)c);
    }
    prefix[cells] = acc;
    if (acc == 0) return fail(NH_EINVAL, "no habitable deme");
    if (cells * (uint64_t)cmax >= (1ull << 32)) return fail(NH_EINVAL, "width*height*max capacity must be < 2^32");

    nh_scenario *s = new nh_scenario();
    if (hipGetDevice(&s->device) != hipSuccess) s->device = -1;
    hipStream_t ts = nullptr; // the device is touched only after every validation has passed
    s->W = W;
    s->H = H;
    s->R = R;
    s->mode = dispersal->mode;
    s->cmax = cmax;
    s->cap_const = constant ? cap[0] : 0;
    s->cells = cells;
    s->N = acc;
    s->nu = nu;
    s->lambda = lambda;
    s->dt = dt;
    s->sampler = sampler;
    s->mu = lambda * dt; // exact: delta_t is a power of two
    s->p0 = std::exp(-s->mu);
    s->nu_thresh = u53_threshold(nu);
    s->tau = tau;
    s->tau_t = protracted_threshold(tau, lambda);

    TableBuilder tb;
    tb.W = W;
    tb.H = H;
    tb.R = R;
    tb.side = side;
    tb.cap = cap;
    tb.weights = dispersal->h_weights;

    auto bail = [&](int code) {
        scenario_free(s);
        return code;
    };

    auto device_stream = [&]() -> bool {
        if (!ts) ts = table_stream(s->device);
        return ts != nullptr;
    };
    if (s->mode == NH_DISPERSAL_SHARED) {
        const uint32_t n = tb.count(-1);
        if (n == 0) return bail(fail(NH_EINVAL, "all dispersal weights are zero"));
        if (!device_stream()) return bail(fail(NH_EDEVICE, "no HIP device for the scenario tables"));
        std::vector<uint4> host(n);
        tb.build(-1, host.data());
        s->n_shared = n;
        s->n_entries = n;
        // the shared table is one row {0, n} of row pointers, so every scenario has them
        const uint32_t row[2] = {0u, n};
        if (hipMallocAsync((void **)&s->d_table, sizeof(uint4) * n, ts) != hipSuccess ||
            hipMallocAsync((void **)&s->d_row_ptr, sizeof row, ts) != hipSuccess)
            return bail(fail(NH_ENOMEM, "device table allocation failed"));
        if (hipMemcpyAsync(s->d_table, host.data(), sizeof(uint4) * n, hipMemcpyHostToDevice, ts) != hipSuccess ||
            hipMemcpyAsync(s->d_row_ptr, row, sizeof row, hipMemcpyHostToDevice, ts) != hipSuccess ||
            hipStreamSynchronize(ts) != hipSuccess)
            return bail(fail(NH_EDEVICE, "table upload failed"));
    } else {
        // Per-deme tables in CSR order, built by host threads in chunks and
        // uploaded through a staging buffer.
        std::vector<uint32_t> counts(cells, 0);
        const unsigned nthreads = std::max(1u, std::min(32u, std::thread::hardware_concurrency()));
        {
            std::vector<std::thread> pool;
            std::atomic<bool> bad{false};
            for (unsigned tid = 0; tid < nthreads; ++tid) {
                pool.emplace_back([&, tid] {
                    for (uint64_t c = tid; c < cells; c += nthreads) {
                        if (cap[c] == 0) continue;
                        counts[c] = tb.count((int64_t)c);
                        if (counts[c] == 0) bad = true;
                    }
                });
            }
            for (auto &th : pool) th.join();
            if (bad) return bail(fail(NH_EINVAL, "a habitable deme has no habitable mass in its dispersal kernel"));
        }
        std::vector<uint32_t> row(cells + 1);
        uint64_t total = 0;
        for (uint64_t c = 0; c < cells; ++c) {
            row[c] = (uint32_t)total;
            total += counts[c];
            if (total >= (1ull << 32)) return bail(fail(NH_EINVAL, "more than 2^32 per-deme table entries"));
        }
        row[cells] = (uint32_t)total;
        s->n_entries = total;
        if (!device_stream()) return bail(fail(NH_EDEVICE, "no HIP device for the scenario tables"));
        if (hipMallocAsync((void **)&s->d_table, sizeof(uint4) * std::max<uint64_t>(total, 1), ts) != hipSuccess)
            return bail(fail(NH_ENOMEM, "device table allocation (%llu entries) failed", (unsigned long long)total));
        if (hipMallocAsync((void **)&s->d_row_ptr, sizeof(uint32_t) * (cells + 1), ts) != hipSuccess)
            return bail(fail(NH_ENOMEM, "row pointer allocation failed"));
        if (hipMemcpyAsync(s->d_row_ptr, row.data(), sizeof(uint32_t) * (cells + 1), hipMemcpyHostToDevice, ts) !=
            hipSuccess)
            return bail(fail(NH_EDEVICE, "row pointer upload failed"));
        const uint64_t chunk_entries = 1ull << 24; // 256 MB staging
        std::vector<uint4> stage((size_t)std::min<uint64_t>(chunk_entries + side * side, total + 1));
        uint64_t c0 = 0;
        while (c0 < cells) {
            uint64_t c1 = c0;
            while (c1 < cells && (uint64_t)row[c1 + 1] - row[c0] <= chunk_entries) ++c1;
            if (c1 == c0) c1 = c0 + 1;
            const uint64_t base = row[c0];
            std::vector<std::thread> pool;
            for (unsigned tid = 0; tid < nthreads; ++tid) {
                pool.emplace_back([&, tid] {
                    TableBuilder local = tb;
                    for (uint64_t c = c0 + tid; c < c1; c += nthreads)
                        if (counts[c]) local.build((int64_t)c, stage.data() + (row[c] - base));
                });
            }
            for (auto &th : pool) th.join();
            const uint64_t n = (uint64_t)row[c1] - base;
            if (n && (hipMemcpyAsync(s->d_table + base, stage.data(), sizeof(uint4) * n, hipMemcpyHostToDevice, ts) !=
                          hipSuccess ||
                      hipStreamSynchronize(ts) != hipSuccess))
                return bail(fail(NH_EDEVICE, "table upload failed"));
            c0 = c1;
        }
    }
    if (hipMallocAsync((void **)&s->d_cap, sizeof(uint32_t) * cells, ts) != hipSuccess ||
        hipMallocAsync((void **)&s->d_prefix, sizeof(uint64_t) * (cells + 1), ts) != hipSuccess)
        return bail(fail(NH_ENOMEM, "capacity allocation failed"));
    if (hipMemcpyAsync(s->d_cap, cap, sizeof(uint32_t) * cells, hipMemcpyHostToDevice, ts) != hipSuccess ||
        hipMemcpyAsync(s->d_prefix, prefix.data(), sizeof(uint64_t) * (cells + 1), hipMemcpyHostToDevice, ts) !=
            hipSuccess ||
        hipStreamSynchronize(ts) != hipSuccess)
        return bail(fail(NH_EDEVICE, "capacity upload failed"));
    s->table_bytes = sizeof(uint4) * s->n_entries + (s->mode == NH_DISPERSAL_PER_DEME ? 4 * (cells + 1) : 8) +
                     4 * cells + 8 * (cells + 1);
    *out = s;
    return NH_OK;
}

NH_API int nh_scenario_create_implicit(uint32_t J, uint32_t J_meta, double m, double nu_meta,
                                       const nh_params *params, nh_scenario **out) {
    if (!out) return fail(NH_EINVAL, "out is NULL");
    *out = nullptr;
    if (J == 0 || J_meta == 0) return fail(NH_EINVAL, "both communities need individuals");
    if (!(m > 0.0 && m <= 1.0)) return fail(NH_EINVAL, "the migration probability must lie in (0, 1]");
    const uint32_t cap[2] = {J, J_meta};
    const double w = 1.0;
    const nh_habitat hab{2, 1, cap};
    const nh_dispersal disp{0, &w, NH_DISPERSAL_SHARED};
    if (int rc = nh_scenario_create(&hab, &disp, nu_meta, params, out)) return rc;
    (*out)->mode = kModeImplicit;
    (*out)->cap_const = 0;
    (*out)->mig_thresh = u53_threshold(m);
    return NH_OK;
}

NH_API void nh_scenario_destroy(nh_scenario *s) { scenario_free(s); }

NH_API uint64_t nh_scenario_individuals(const nh_scenario *s) { return s ? s->N : 0; }

NH_API uint64_t nh_scenario_table_bytes(const nh_scenario *s) { return s ? s->table_bytes : 0; }

NH_API uint64_t nh_workspace_bytes(uint64_t n_total, uint32_t n_jobs) { return layout(n_total, n_jobs).total; }

NH_API uint64_t nh_scenario_footprint_bytes(const nh_scenario *s, uint64_t n_samples) {
    return (s ? s->table_bytes : 0) + layout(n_samples, 1).total;
}

namespace {

// One device run over many jobs, from the start or (resume) from the state a
// suspended run left in the workspace.
// Descriptor of job `job` in a batch run: its species set and counters start
// at slot rich_off of the run's set area and its lineages at index base; both
// advance past the job.
void job_descriptor_run(JobDev &d, const nh_job &job, unsigned long long *rich, uint32_t *rich_counts,
                        uint64_t &rich_off, uint64_t &base) {
    const nh_scenario *s = job.scenario;
    std::memset(&d, 0, sizeof d);
    d.seed = job.seed;
    d.nu_thresh = s->nu_thresh;
    d.inv_lambda = 1.0 / s->lambda;
    d.dt = s->dt;
    d.inv_dt = 1.0 / s->dt;
    d.table = s->d_table;
    d.row_ptr = s->d_row_ptr;
    d.cap = s->d_cap;
    d.prefix = s->d_prefix;
    d.samples = job.d_sample_ids;
    d.species_out = (unsigned long long *)job.d_species_out;
    d.richness_out = (unsigned long long *)job.d_richness_out;
    const uint64_t slots = pow2_at_least(2 * job.n, 64);
    d.rich_set = rich + rich_off;
    d.rich_counts = rich_counts + rich_off;
    d.rich_off = rich_off;
    d.rich_mask = (uint32_t)(slots - 1);
    rich_off += slots;
    d.spec_loc_out = job.d_spec_loc_out;
    d.spec_time_out = job.d_spec_time_out;
    d.abund_ids_out = (unsigned long long *)job.d_abundance_ids_out;
    d.abund_counts_out = job.d_abundance_counts_out;
    d.n_individuals = s->N;
    d.W = s->W;
    d.H = s->H;
    d.cmax = s->cmax;
    d.R = s->R;
    d.mode = s->mode;
    d.n_shared = s->n_shared;
    d.cap_const = s->cap_const;
    d.caps_in_table = (s->mode == NH_DISPERSAL_PER_DEME && s->cmax <= 0xFFFFu) ? 1u : 0u;
    d.sampler = s->sampler;
    d.mu = s->mu;
    d.p0 = s->p0;
    d.mig_thresh = s->mig_thresh;
    d.tau_t = s->tau_t;
    d.lin_base = (uint32_t)base;
    d.n = (uint32_t)job.n;
    d.start_round = 0;
    base += job.n;
}

// Per-device resources of persistent runs.  Every persistent run on a device
// is launched on one library-owned stream, so two grids sized to the whole
// device are never in flight at once (each would wait at its barriers for
// workgroups the other keeps out); events join that stream to the caller's
// stream before and after the launch, so the call stays enqueue-only.
struct PersistentLane {
    std::mutex mu;
    bool ready = false;
    hipStream_t stream = nullptr;
    hipEvent_t in = nullptr, out = nullptr;
    int n_cu = 0, coop = 0, clock_khz = 0;
};

int persistent_lane(PersistentLane *&out) {
    static PersistentLane lanes[64];
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(NH_EDEVICE, "device %d is beyond the library's 64", dev);
    PersistentLane &L = lanes[dev];
    std::lock_guard<std::mutex> lock(L.mu);
    if (!L.ready) {
        HIP_TRY(hipDeviceGetAttribute(&L.n_cu, hipDeviceAttributeMultiprocessorCount, dev));
        HIP_TRY(hipDeviceGetAttribute(&L.coop, hipDeviceAttributeCooperativeLaunch, dev));
        HIP_TRY(hipDeviceGetAttribute(&L.clock_khz, hipDeviceAttributeWallClockRate, dev));
        if (L.clock_khz <= 0) return fail(NH_EDEVICE, "the device reports no wall-clock rate");
        HIP_TRY(hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking));
        HIP_TRY(hipEventCreateWithFlags(&L.in, hipEventDisableTiming));
        HIP_TRY(hipEventCreateWithFlags(&L.out, hipEventDisableTiming));
        L.ready = true;
    }
    out = &L;
    return NH_OK;
}

// Round-kernel variants: 0 multi-job, 1 single job, 2 single job with the shared table in LDS.
const void *run_kernel(uint32_t variant) {
    if (variant == 2) return reinterpret_cast<const void *>(&k_run<true, true>);
    if (variant == 1) return reinterpret_cast<const void *>(&k_run<true, false>);
    return reinterpret_cast<const void *>(&k_run<false, false>);
}

// Grid of a persistent run: as many workgroups per compute unit as stay
// resident together (the occupancy of k_run at this block size and LDS), at
// most cfg.blocks_per_cu.
int persistent_grid(const PersistentLane &L, uint32_t variant, const nh_config &cfg, size_t lds, uint32_t &grid) {
    int per_cu = 0;
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, run_kernel(variant), (int)cfg.block_size, lds));
    per_cu = std::min<int>(per_cu, (int)cfg.blocks_per_cu);
    while (per_cu > 1 && (uint64_t)per_cu * L.n_cu > (uint64_t)kBarGroup * kMaxBarGroups) --per_cu;
    if (per_cu < 1) return fail(NH_EINVAL, "no workgroup of %u threads fits a compute unit", cfg.block_size);
    if ((uint64_t)per_cu * L.n_cu > (uint64_t)kBarGroup * kMaxBarGroups)
        return fail(NH_EDEVICE, "%d compute units exceed the grid barrier's %u workgroups", L.n_cu,
                    kBarGroup * kMaxBarGroups);
    grid = (uint32_t)(per_cu * L.n_cu);
    return NH_OK;
}

// Enqueues a persistent run of the workspace's current state on `stream`:
// reset the barrier state, then k_run on the device's persistent stream.
// t0/t1 (nullable) bracket the run kernel alone.
int enqueue_persistent(PersistentLane &L, uint32_t variant, const RoundArgs &ra, const nh_config &cfg, size_t lds,
                       uint32_t grid, hipStream_t stream, hipEvent_t t0, hipEvent_t t1, uint32_t endgame = 0) {
    RunArgs R{};
    R.max_rounds = cfg.max_rounds;
    R.endgame = endgame;
    const double khz = (double)L.clock_khz;
    const double wait_s = cfg.barrier_wait_ms ? cfg.barrier_wait_ms * 1e-3 : std::min(cfg.timeout_s, 60.0);
    R.spin_ticks = (unsigned long long)std::max(1.0, wait_s * khz * 1e3);
    R.run_ticks = (unsigned long long)std::max(1.0, cfg.timeout_s * khz * 1e3);
    RoundArgs a = ra;
    void *args[] = {&a, &R};
    std::lock_guard<std::mutex> lock(L.mu);
    HIP_TRY(hipEventRecord(L.in, stream));
    HIP_TRY(hipStreamWaitEvent(L.stream, L.in, 0));
    k_run_reset<<<1, kMaxBarGroups, 0, L.stream>>>(ra.ctl);
    if (t0) HIP_TRY(hipEventRecord(t0, L.stream));
    if (L.coop)
        HIP_TRY(hipLaunchCooperativeKernel(run_kernel(variant), dim3(grid), dim3(cfg.block_size), args,
                                           (unsigned int)lds, L.stream));
    else
        HIP_TRY(hipLaunchKernel(run_kernel(variant), dim3(grid), dim3(cfg.block_size), args, lds, L.stream));
    if (t1) HIP_TRY(hipEventRecord(t1, L.stream));
    HIP_TRY(hipEventRecord(L.out, L.stream));
    HIP_TRY(hipStreamWaitEvent(stream, L.out, 0));
    return NH_OK;
}

// Dynamic LDS of a one-wave-per-lineage walk kernel (k_tail, k_endgame): all
// the LDS a workgroup may take (so it holds a compute unit alone), opted in
// once per kernel past the default 64 KiB limit.
size_t walk_kernel_lds(const void *kernel) {
    int dev = 0, lds_cu = 0, lds_block = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds_block, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return 0;
    size_t bytes = (size_t)std::max(0, std::min(lds_cu, lds_block));
    if (bytes > 65536 && hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess)
        bytes = 65536;
    return bytes;
}

// Workspace of nh_simulate_noalloc: a file-scope device array, one copy per
// device that the library runs on, held until the process ends.  Host code
// never passes the array's name to a kernel (on the host it is only a
// stand-in for the symbol): it looks the device address up once per device
// and passes that.
constexpr uint64_t kScratchBytes = 64ull << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Device address of `scratch` on the current device (looked up at the first
// call on that device, with the device current).
int scratch_address(void *&out) {
    static std::mutex mu;
    static void *addr[64] = {};
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(NH_EDEVICE, "device %d is beyond the library's 64", dev);
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(NH_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        addr[dev] = p;
    }
    out = addr[dev];
    return NH_OK;
}

// Round-kernel arguments of a run in workspace ws laid out as L.
RoundArgs round_args(char *ws, const Workspace &L, uint32_t n_jobs, uint64_t n_total, uint32_t grid,
                     const nh_config &cfg) {
    RoundArgs ra;
    std::memset(&ra, 0, sizeof ra);
    ra.ctl = (Ctl *)(ws + L.off_ctl);
    ra.jobs = (JobDev *)(ws + L.off_jobs);
    ra.js = (JobState *)(ws + L.off_js);
    ra.ring = (uint32_t *)(ws + L.off_ring);
    ra.ring_cap = std::max<uint32_t>(n_jobs, 1);
    ra.lin = lin_view(ws, L);
    ra.htab = (const double *)(ws + L.off_htab);
    ra.coop_max = cfg.coop_max ? cfg.coop_max : (uint32_t)(((uint64_t)grid * cfg.block_size) / (2 * kGroup)) + 1;
    ra.n_cap = (uint32_t)n_total;
    ra.solo_max = (n_jobs == 1 || grid < 4) ? 0u : cfg.solo_max; // solo blocks never take more than a quarter
    ra.solo_step = cfg.solo_step;
    return ra;
}

// Enqueues a whole single-job run on `stream` in the workspace at ws (at least
// nh_workspace_bytes(n, 1) bytes): set-up from kernel arguments, lineage init,
// one persistent round launch and the output kernels, which write the species
// and the richness only if the run finished and every sample id was valid
// (else the richness reads ~0).  Nothing waits for the device and nothing is
// copied from the host.
int enqueue_single(const nh_scenario *scn, uint64_t seed, const uint64_t *d_samples, uint64_t n,
                   uint64_t *d_species, uint64_t *d_richness, char *ws, const nh_config &cfg, hipStream_t stream) {
    const Workspace L = layout(n, 1);
    PersistentLane *lane = nullptr;
    if (int rc = persistent_lane(lane)) return rc;
    const bool lds_table =
        cfg.table_placement == 0 && scn->mode == NH_DISPERSAL_SHARED && scn->n_shared <= kLdsTableMax;
    const size_t lds_bytes = lds_table ? sizeof(uint4) * scn->n_shared : 0;
    const uint32_t variant = lds_table ? 2u : 1u;
    uint32_t grid = 0;
    if (int rc = persistent_grid(*lane, variant, cfg, lds_bytes, grid)) return rc;
    const RoundArgs ra = round_args(ws, L, 1, n, grid, cfg);
    unsigned long long *rich = (unsigned long long *)(ws + L.off_rich);
    uint32_t *rich_counts = (uint32_t *)(ws + L.off_rcount);
    const nh_job job{scn, seed, d_samples, n, d_species, d_richness, nullptr, nullptr, nullptr, nullptr};
    JobDev jd;
    uint64_t rich_off = 0, base = 0;
    job_descriptor_run(jd, job, rich, rich_counts, rich_off, base);
    JobDev *d_jobs = (JobDev *)ra.jobs;
    k_setup_single<<<1, 64, 0, stream>>>(ra.ctl, ra.js, d_jobs, jd, (double *)ra.htab, cfg.horizon0,
                                         cfg.horizon_growth, cfg.horizon_step_max);
    k_fill_u64<<<1024, 256, 0, stream>>>(ra.lin.hash, L.hcap, 0ull);
    k_fill_u64<<<1024, 256, 0, stream>>>(rich, rich_off, ~0ull);
    k_fill_u64<<<1024, 256, 0, stream>>>((unsigned long long *)rich_counts, rich_off / 2, 0ull);
    if (n) {
        const uint32_t blocks = (uint32_t)((n + 255) / 256);
        k_init<<<blocks, 256, 0, stream>>>(ra.ctl, d_jobs, 1, 0, ra.js, ra.ring, ra.ring_cap, ra.lin, 0,
                                           (uint32_t)n);
        HIP_TRY(hipGetLastError());
        if (int rc = enqueue_persistent(*lane, variant, ra, cfg, lds_bytes, grid, stream, nullptr, nullptr))
            return rc;
        k_resolve<<<blocks, 256, 0, stream>>>(d_jobs, ra.js, ra.lin, 0, (uint32_t)n, ra.ctl);
    }
    k_finalize<<<1, 64, 0, stream>>>(d_jobs, ra.js, 0, 1, n ? ra.ctl : nullptr, 1u);
    HIP_TRY(hipGetLastError());
    return NH_OK;
}

// Checks of an enqueue-only single-job call that need no device access.
int check_single(const nh_scenario *scn, const uint64_t *d_samples, uint64_t n, const uint64_t *d_species,
                 const nh_config &cfg) {
    if (!scn) return fail(NH_EINVAL, "scenario is NULL");
    if (n > 0 && (!d_samples || !d_species)) return fail(NH_EINVAL, "NULL sample or output buffer");
    if (n >= (1ull << 31)) return fail(NH_EINVAL, "more than 2^31 - 1 samples in one run");
    if (cfg.block_size % 64 != 0 || cfg.block_size > 256)
        return fail(NH_EINVAL, "block_size must be a multiple of 64 up to 256");
    if (cfg.launch != NH_LAUNCH_PERSISTENT) return fail(NH_EINVAL, "enqueue-only runs are persistent launches");
    if (cfg.max_rounds != 0) return fail(NH_EINVAL, "enqueue-only runs cannot suspend (max_rounds must be 0)");
    return NH_OK;
}

int batch_run_impl(const nh_job *jobs, uint32_t n_jobs, void *d_workspace, uint64_t workspace_bytes,
                   const nh_config *cfg_in, nh_stats *stats, void *stream_ptr, bool resume) {
    using clock = std::chrono::steady_clock;
    hipStream_t stream = (hipStream_t)stream_ptr;
    if (n_jobs == 0) return NH_OK;
    if (!jobs) return fail(NH_EINVAL, "jobs is NULL");
    nh_config cfg;
    fill_config(cfg_in, cfg);
    if (cfg.block_size % 64 != 0 || cfg.block_size > 256 || cfg.rounds_per_graph > 256)
        return fail(NH_EINVAL, "block_size must be a multiple of 64 up to 256, rounds_per_graph <= 256");
    uint64_t n_total = 0;
    for (uint32_t j = 0; j < n_jobs; ++j) {
        const nh_job &jb = jobs[j];
        if (!jb.scenario) return fail(NH_EINVAL, "job %u has no scenario", j);
        if (jb.n > 0 && (!jb.d_sample_ids || !jb.d_species_out))
            return fail(NH_EINVAL, "job %u has NULL sample or output buffers", j);
        if (!jb.d_spec_loc_out != !jb.d_spec_time_out || !jb.d_abundance_ids_out != !jb.d_abundance_counts_out)
            return fail(NH_EINVAL, "job %u: reporter outputs come in pairs (both or neither)", j);
        n_total += jb.n;
    }
    if (n_total >= (1ull << 31)) return fail(NH_EINVAL, "more than 2^31 - 1 samples in one batch");
    const Workspace L = layout(n_total, n_jobs);
    if (!d_workspace || workspace_bytes < L.total)
        return fail(NH_ENOMEM, "workspace of %llu bytes is smaller than the %llu needed",
                    (unsigned long long)workspace_bytes, (unsigned long long)L.total);
    if (((uintptr_t)d_workspace & 255) != 0) return fail(NH_EINVAL, "workspace must be 256-byte aligned");

    char *ws = (char *)d_workspace;
    Ctl *ctl = (Ctl *)(ws + L.off_ctl);
    JobDev *d_jobs = (JobDev *)(ws + L.off_jobs);
    JobState *d_js = (JobState *)(ws + L.off_js);
    double *d_htab = (double *)(ws + L.off_htab);
    uint32_t *d_ring = (uint32_t *)(ws + L.off_ring);
    const uint32_t ring_cap = std::max<uint32_t>(n_jobs, 1);
    const Lin lin = lin_view(ws, L);
    unsigned long long *rich = (unsigned long long *)(ws + L.off_rich);
    uint32_t *rich_counts = (uint32_t *)(ws + L.off_rcount);

    // Job descriptors.
    std::vector<JobDev> hj(n_jobs);
    uint64_t base = 0, rich_off = 0;
    bool any_abundance = false;
    for (uint32_t j = 0; j < n_jobs; ++j) {
        job_descriptor_run(hj[j], jobs[j], rich, rich_counts, rich_off, base);
        if (hj[j].abund_counts_out) any_abundance = true;
    }
    const std::vector<double> htab = horizon_table(cfg);

    PinnedStatus st;
    if (int rc = pinned_status(st)) return rc;

    hipEvent_t ev0, ev1;
    HIP_TRY(hipEventCreate(&ev0));
    HIP_TRY(hipEventCreate(&ev1));
    struct EvGuard {
        hipEvent_t a, b;
        ~EvGuard() {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
        }
    } evg{ev0, ev1};

    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    int n_cu = 0;
    HIP_TRY(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));

    // The first round this call runs: 1 for a new run; for a resume, the round
    // the suspended run would have run next (its control block says which).
    uint32_t base_round = 1;
    if (resume) {
        Ctl c0;
        HIP_TRY(hipMemcpyAsync(&c0, ctl, sizeof(Ctl), hipMemcpyDeviceToHost, stream));
        HIP_TRY(hipStreamSynchronize(stream));
        if (c0.n_jobs != n_jobs || c0.round == 0)
            return fail(NH_EINVAL, "the workspace does not hold a suspended run of these %u jobs", n_jobs);
        base_round = c0.round;
    }
    HIP_TRY(hipEventRecord(ev0, stream));
    HIP_TRY(hipMemcpyAsync(d_jobs, hj.data(), sizeof(JobDev) * n_jobs, hipMemcpyHostToDevice, stream));
    HIP_TRY(hipMemcpyAsync(d_htab, htab.data(), sizeof(double) * kMaxHorizons, hipMemcpyHostToDevice, stream));
    if (!resume) {
        k_setup<<<std::max<uint32_t>(1, (n_jobs + 255) / 256), 256, 0, stream>>>(ctl, d_js, d_jobs, n_jobs,
                                                                                 base_round);
        k_fill_u64<<<1024, 256, 0, stream>>>(lin.hash, L.hcap, 0ull);
        if (rich_off) k_fill_u64<<<1024, 256, 0, stream>>>(rich, rich_off, ~0ull);
        if (rich_off) k_fill_u64<<<1024, 256, 0, stream>>>((unsigned long long *)rich_counts, rich_off / 2, 0ull);
        if (n_total) {
            const uint32_t blocks = (uint32_t)((n_total + 255) / 256);
            k_init<<<blocks, 256, 0, stream>>>(ctl, d_jobs, n_jobs, -1, d_js, d_ring, ring_cap, lin, 0,
                                               (uint32_t)n_total);
        }
    }
    HIP_TRY(hipGetLastError());
    // The status word: round 0 and "not finished" until the first round kernel reports.
    __atomic_store_n(st.host, (unsigned long long)1, __ATOMIC_SEQ_CST);

    // Round kernels: one persistent launch, or replayed from a captured graph of
    // cfg.rounds_per_graph launches.
    const bool single = n_jobs == 1;
    const nh_scenario *s0 = jobs[0].scenario;
    const bool lds_table =
        single && cfg.table_placement == 0 && s0->mode == NH_DISPERSAL_SHARED && s0->n_shared <= kLdsTableMax;
    const size_t lds_bytes = lds_table ? sizeof(uint4) * s0->n_shared : 0;
    const uint32_t variant = lds_table ? 2u : (single ? 1u : 0u);
    const bool persistent = cfg.launch == NH_LAUNCH_PERSISTENT;
    PersistentLane *lane = nullptr;
    uint32_t grid = (uint32_t)std::max(1, n_cu) * cfg.blocks_per_cu;
    if (persistent) {
        if (int rc = persistent_lane(lane)) return rc;
        if (int rc = persistent_grid(*lane, variant, cfg, lds_bytes, grid)) return rc;
    }
    RoundArgs ra;
    std::memset(&ra, 0, sizeof ra);
    ra.ctl = ctl;
    ra.jobs = d_jobs;
    ra.lin = lin;
    ra.htab = d_htab;
    ra.js = d_js;
    ra.ring = d_ring;
    ra.ring_cap = ring_cap;
    ra.coop_max = cfg.coop_max ? cfg.coop_max : (uint32_t)(((uint64_t)grid * cfg.block_size) / (2 * kGroup)) + 1;
    ra.n_cap = (uint32_t)n_total;
    ra.solo_max = (single || grid < 4) ? 0u : cfg.solo_max; // solo blocks never take more than a quarter
    ra.solo_step = cfg.solo_step;
    auto launch_round = [&](hipStream_t s) {
        if (lds_table)
            k_round<true, true><<<grid, cfg.block_size, lds_bytes, s>>>(ra);
        else if (single)
            k_round<true, false><<<grid, cfg.block_size, 0, s>>>(ra);
        else
            k_round<false, false><<<grid, cfg.block_size, 0, s>>>(ra);
        k_advance<<<1, 1, 0, s>>>(ctl, st.dev, d_ring, ring_cap, nullptr);
    };
    // Instantiated graphs are cached per thread: a graph bakes in the kernel
    // arguments, which depend only on the workspace, the lane layout and the
    // status word, so repeated runs on one workspace reuse it.
    struct GraphEntry {
        RoundArgs ra;
        uint32_t grid, block, rounds, variant;
        size_t lds;
        unsigned long long *status;
        hipGraph_t graph;
        hipGraphExec_t exec;
    };
    thread_local std::vector<GraphEntry> graph_cache;
    hipGraphExec_t exec = nullptr;
    bool use_graph = !persistent && cfg.rounds_per_graph > 1;
    if (use_graph && n_total) {
        for (auto &ge : graph_cache) {
            if (ge.grid == grid && ge.block == cfg.block_size && ge.rounds == cfg.rounds_per_graph &&
                ge.variant == variant && ge.lds == lds_bytes && ge.status == st.dev &&
                std::memcmp(&ge.ra, &ra, sizeof ra) == 0) {
                exec = ge.exec;
                break;
            }
        }
        if (!exec) {
            hipGraph_t graph = nullptr;
            hipStream_t cap_stream;
            HIP_TRY(hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking));
            hipError_t e = hipStreamBeginCapture(cap_stream, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                for (uint32_t k = 0; k < cfg.rounds_per_graph; ++k) launch_round(cap_stream);
                e = hipStreamEndCapture(cap_stream, &graph);
            }
            if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            (void)hipStreamDestroy(cap_stream);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                if (graph) (void)hipGraphDestroy(graph);
                exec = nullptr;
                use_graph = false;
            } else {
                if (graph_cache.size() >= 8) {
                    (void)hipGraphExecDestroy(graph_cache.front().exec);
                    (void)hipGraphDestroy(graph_cache.front().graph);
                    graph_cache.erase(graph_cache.begin());
                }
                graph_cache.push_back(GraphEntry{ra, grid, cfg.block_size, cfg.rounds_per_graph, variant, lds_bytes,
                                                 st.dev, graph, exec});
            }
        }
    }
    const uint32_t per_launch = use_graph ? cfg.rounds_per_graph : 1;
    uint64_t rounds_enqueued = 0;
    // Optional HIP-event bracketing of every round launch (graph or kernel).
    thread_local std::vector<hipEvent_t> ev_pool;
    uint32_t ev_used = 0;
    // whole: a graph of cfg.rounds_per_graph rounds (when graphs are in use), else one round
    auto enqueue = [&](bool whole) -> int {
        const bool as_graph = use_graph && whole;
        if (cfg.event_timing) {
            while (ev_pool.size() < 2ull * (ev_used + 1)) {
                hipEvent_t e;
                HIP_TRY(hipEventCreate(&e));
                ev_pool.push_back(e);
            }
            HIP_TRY(hipEventRecord(ev_pool[2 * ev_used], stream));
        }
        if (as_graph) HIP_TRY(hipGraphLaunch(exec, stream));
        else launch_round(stream);
        HIP_TRY(hipGetLastError());
        if (cfg.event_timing) {
            HIP_TRY(hipEventRecord(ev_pool[2 * ev_used + 1], stream));
            ++ev_used;
        }
        rounds_enqueued += as_graph ? per_launch : 1u;
        return NH_OK;
    };
    const auto t_start = clock::now();
    uint32_t final_round = base_round - 1;
    bool suspended = false;
    if (persistent && n_total) {
        // One launch runs every round; the output kernels run only if it finished (the control
        // block says so), so nothing here waits for the device.
        hipEvent_t t0 = nullptr, t1 = nullptr;
        if (cfg.event_timing) {
            while (ev_pool.size() < 2) {
                hipEvent_t e;
                HIP_TRY(hipEventCreate(&e));
                ev_pool.push_back(e);
            }
            t0 = ev_pool[0];
            t1 = ev_pool[1];
            ev_used = 1;
        }
        // a batch of several jobs ends with the endgame (the few last lineages walked to their ends)
        const uint32_t endgame = single ? 0u : std::min<uint32_t>(cfg.endgame, 4096u);
        if (int rc = enqueue_persistent(*lane, variant, ra, cfg, lds_bytes, grid, stream, t0, t1, endgame)) return rc;
        if (endgame) {
            static const size_t end_lds = walk_kernel_lds((const void *)k_endgame);
            const double khz = (double)lane->clock_khz;
            const unsigned long long run_ticks = (unsigned long long)std::max(1.0, cfg.timeout_s * khz * 1e3);
            k_endgame<<<(endgame + 3) / 4, 256, end_lds, stream>>>(ra, run_ticks,
                                                                    (uint32_t)(end_lds / (4 * sizeof(uint4))));
            k_endgame_done<<<1, 1, 0, stream>>>(ctl);
        }
        const uint32_t blocks = (uint32_t)((n_total + 255) / 256);
        k_resolve<<<blocks, 256, 0, stream>>>(d_jobs, d_js, lin, 0, (uint32_t)n_total, ctl);
        if (any_abundance)
            k_abundance<<<(uint32_t)((rich_off + 255) / 256), 256, 0, stream>>>(d_jobs, d_js, 0, n_jobs, rich_off,
                                                                                ctl);
        k_finalize<<<(n_jobs + 255) / 256, 256, 0, stream>>>(d_jobs, d_js, 0, n_jobs, ctl, 0u);
    } else if (n_total) {
        // Keep two launches in flight; stop when a round reports an empty queue, or, past
        // cfg.max_rounds, once every enqueued round has run.  Whatever is enqueued past the
        // last round still runs (two near-empty launches per round, about 9 us), which is
        // felt in a short single-job run.  There the host keeps one graph and two rounds
        // ahead of the device (not two graphs), and once the queue is shorter than the
        // 8-lanes-per-lineage threshold and rounds have been long enough for launch overhead
        // not to matter, it enqueues single rounds, two ahead, instead of whole graphs.  A
        // multi-job batch runs hundreds of rounds and keeps two whole graphs ahead.
        if (int rc = enqueue(true)) return rc;
        if (int rc = enqueue(true)) return rc;
        uint64_t spins = 0;
        for (;;) {
            const unsigned long long word = __atomic_load_n(st.host, __ATOMIC_ACQUIRE);
            const uint32_t next_round = (uint32_t)(word >> 32);
            const uint32_t live = (uint32_t)(word & 0x7FFFFFFFu);
            const bool errflag = (word >> 31) & 1u;
            const uint64_t completed = next_round > base_round ? next_round - base_round : 0;
            if (completed > 0 && (live == 0 || errflag)) {
                final_round = next_round - 1;
                break;
            }
            const bool capped = cfg.max_rounds != 0 && rounds_enqueued >= cfg.max_rounds;
            if (capped && completed >= rounds_enqueued) {
                final_round = next_round - 1;
                suspended = true;
                break;
            }
            bool whole = true;
            if (use_graph && single && completed > 0 && live < ra.coop_max) {
                const double el = std::chrono::duration<double>(clock::now() - t_start).count();
                whole = el < kLongRoundS * (double)completed;
            }
            const uint64_t ahead = !whole ? 2ull : single ? per_launch + 2ull : 2ull * per_launch;
            if (!capped && rounds_enqueued < completed + ahead) {
                if (int rc = enqueue(whole)) return rc;
                continue;
            }
            if ((++spins & 255) == 0) {
                const double el = std::chrono::duration<double>(clock::now() - t_start).count();
                if (el > cfg.timeout_s) {
                    (void)hipStreamSynchronize(stream);
                    return fail(NH_ETIMEOUT, "run exceeded %.1f s (round %u, %u lineages live)", cfg.timeout_s,
                                next_round, live);
                }
                std::this_thread::yield();
            }
        }
        if (!suspended) {
            const uint32_t blocks = (uint32_t)((n_total + 255) / 256);
            k_resolve<<<blocks, 256, 0, stream>>>(d_jobs, d_js, lin, 0, (uint32_t)n_total, nullptr);
            if (any_abundance)
                k_abundance<<<(uint32_t)((rich_off + 255) / 256), 256, 0, stream>>>(d_jobs, d_js, 0, n_jobs,
                                                                                    rich_off, nullptr);
        }
    }
    if (!suspended && !(persistent && n_total))
        k_finalize<<<(n_jobs + 255) / 256, 256, 0, stream>>>(d_jobs, d_js, 0, n_jobs, nullptr, 0u);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipEventRecord(ev1, stream));
    std::vector<JobState> hs(n_jobs);
    Ctl hctl;
    HIP_TRY(hipMemcpyAsync(hs.data(), d_js, sizeof(JobState) * n_jobs, hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipMemcpyAsync(&hctl, ctl, sizeof(Ctl), hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    if (persistent && n_total) {
        if (hctl.error & kErrTimeout)
            return fail(NH_ETIMEOUT, "run exceeded %.1f s (round %u)", cfg.timeout_s, hctl.round);
        if (hctl.error & kErrStall)
            return fail(NH_EDEVICE, "a grid barrier wait exceeded its limit (round %u)", hctl.round);
        if (hctl.stop != kStopDone && hctl.stop != kStopSuspended && hctl.error == 0)
            return fail(NH_EDEVICE, "the persistent run ended in state %u", hctl.stop);
        suspended = hctl.stop == kStopSuspended;
        final_round = hctl.round - 1;
        rounds_enqueued = 1; // one round-kernel launch
    }
    if (hctl.error & kErrBadSample) return fail(NH_EINVAL, "a sample id is not below the number of individuals");
    if (hctl.error) return fail(NH_EDEVICE, "kernel reported error flags 0x%x", hctl.error);
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, ev0, ev1));
    double round_ms = 0.0;
    for (uint32_t k = 0; k < ev_used; ++k) {
        float x = 0.f;
        HIP_TRY(hipEventElapsedTime(&x, ev_pool[2 * k], ev_pool[2 * k + 1]));
        round_ms += x;
    }
    unsigned long long philox_calls = 0, exp_draws = 0;
    for (uint32_t k = 0; k < kOpSlots; ++k) {
        philox_calls += hctl.ops[k].philox;
        exp_draws += hctl.ops[k].draws;
    }
    if (stats) {
        for (uint32_t j = 0; j < n_jobs; ++j) {
            stats[j].events = hs[j].events;
            stats[j].lineages = jobs[j].n;
            stats[j].speciated = hs[j].speciated;
            stats[j].merged = hs[j].merged;
            // the job's own rounds: to the round it finished in (or the run's last round, if it has not)
            stats[j].rounds = (hs[j].remaining == 0 && hs[j].done_round > hs[j].start_round)
                                  ? hs[j].done_round - hs[j].start_round
                                  : final_round;
            stats[j].richness = hs[j].rich_count;
            stats[j].device_ms = ms;
            stats[j].philox_calls = philox_calls;
            stats[j].exp_draws = exp_draws;
            stats[j].round_kernels = rounds_enqueued;
            stats[j].round_kernel_ms = round_ms;
        }
    }
    return suspended ? NH_SUSPENDED : NH_OK;
}

// Library-owned memory pool per device for the event stream's scratch.  It
// keeps what it has reserved (release threshold: never), so repeated calls
// reuse the memory of the largest one instead of mapping it again each time;
// null if the pool cannot be made (the scratch then comes from the device's
// default pool).
hipMemPool_t scratch_pool(int device) {
    static std::mutex mu;
    static hipMemPool_t pools[64] = {};
    static bool tried[64] = {};
    std::lock_guard<std::mutex> lock(mu);
    if (device < 0 || device >= 64) return nullptr;
    if (!tried[device]) {
        tried[device] = true;
        hipMemPoolProps props{};
        props.allocType = hipMemAllocationTypePinned;
        props.location.type = hipMemLocationTypeDevice;
        props.location.id = device;
        hipMemPool_t pool = nullptr;
        if (hipMemPoolCreate(&pool, &props) == hipSuccess) {
            uint64_t keep = ~0ull;
            if (hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep) == hipSuccess) pools[device] = pool;
            else (void)hipMemPoolDestroy(pool);
        }
    }
    return pools[device];
}

// Stream-ordered scratch allocations of one call, released (stream-ordered)
// when the call returns.
struct AsyncScratch {
    hipStream_t stream;
    hipMemPool_t pool;
    std::vector<void *> held;
    ~AsyncScratch() {
        for (void *q : held) (void)hipFreeAsync(q, stream);
    }
    template <typename T>
    int take(T *&out, uint64_t count) {
        void *q = nullptr;
        const uint64_t bytes = std::max<uint64_t>(count, 1) * sizeof(T);
        if (pool) HIP_TRY(hipMallocFromPoolAsync(&q, bytes, pool, stream));
        else HIP_TRY(hipMallocAsync(&q, bytes, stream));
        held.push_back(q);
        out = (T *)q;
        return 0;
    }
};

// Scratch bytes the sorts and scans over n items need.
int sort_scratch_bytes(uint32_t n, size_t &bytes) {
    size_t a = 0, b = 0, c = 0;
    HIP_TRY(nh_sort::sort_pairs_u64(nullptr, a, nullptr, nullptr, nullptr, nullptr, n, 64, nullptr));
    HIP_TRY(nh_sort::sort_pairs_u32(nullptr, b, nullptr, nullptr, nullptr, nullptr, n, 32, nullptr));
    HIP_TRY(nh_sort::exclusive_sum_u32(nullptr, c, nullptr, nullptr, n, nullptr));
    bytes = std::max(a, std::max(b, c));
    return 0;
}

// Stable LSD passes: perm (initially the identity) ends sorted by (job, key2,
// key1, key0) over the records' fields; returns the array holding the result.
int stream_sort(const StreamRecs &R, uint32_t n, uint32_t n_jobs, const uint64_t *key0_64, const uint32_t *key1_32,
                const uint64_t *key2_64, uint32_t *perm_a, uint32_t *perm_b, uint64_t *k64_a, uint64_t *k64_b,
                uint32_t *k32_a, uint32_t *k32_b, void *tmp, size_t tmp_bytes, hipStream_t stream,
                uint32_t *&sorted) {
    const uint32_t blocks = (uint32_t)std::min<uint64_t>((n + 255) / 256, 65535);
    size_t b = tmp_bytes;
    k_iota<<<blocks, 256, 0, stream>>>(perm_a, n);
    HIP_TRY(nh_sort::sort_pairs_u64(tmp, b, key0_64, k64_b, perm_a, perm_b, n, 64, stream));
    k_gather<uint32_t><<<blocks, 256, 0, stream>>>(key1_32, perm_b, k32_a, n);
    b = tmp_bytes;
    HIP_TRY(nh_sort::sort_pairs_u32(tmp, b, k32_a, k32_b, perm_b, perm_a, n, 32, stream));
    k_gather<uint64_t><<<blocks, 256, 0, stream>>>(key2_64, perm_a, k64_a, n);
    b = tmp_bytes;
    HIP_TRY(nh_sort::sort_pairs_u64(tmp, b, k64_a, k64_b, perm_a, perm_b, n, 64, stream));
    sorted = perm_b;
    if (n_jobs > 1) {
        int bits = 0;
        while (bits < 32 && ((n_jobs - 1) >> bits) != 0) ++bits;
        k_gather<uint32_t><<<blocks, 256, 0, stream>>>(R.job, perm_b, k32_a, n);
        b = tmp_bytes;
        HIP_TRY(nh_sort::sort_pairs_u32(tmp, b, k32_a, k32_b, perm_b, perm_a, n, bits, stream));
        sorted = perm_a;
    }
    HIP_TRY(hipGetLastError());
    return 0;
}

int event_stream_impl(const nh_job *jobs, uint32_t n_jobs, void *d_workspace, uint64_t workspace_bytes,
                      nh_stream_out *outs, void *stream_ptr) {
    hipStream_t stream = (hipStream_t)stream_ptr;
    if (n_jobs == 0 || !jobs || !outs) return fail(NH_EINVAL, "no jobs or no outputs");
    uint64_t n_total = 0;
    for (uint32_t j = 0; j < n_jobs; ++j) {
        if (!jobs[j].scenario) return fail(NH_EINVAL, "job %u has no scenario", j);
        if (outs[j].events_cap && !outs[j].d_events) return fail(NH_EINVAL, "job %u: events_cap > 0 with NULL d_events", j);
        if (jobs[j].n && !outs[j].d_coalescences) return fail(NH_EINVAL, "job %u has NULL d_coalescences", j);
        n_total += jobs[j].n;
    }
    if (n_total >= (1ull << 31)) return fail(NH_EINVAL, "more than 2^31 - 1 samples in one batch");
    const Workspace L = layout(n_total, n_jobs);
    if (!d_workspace || workspace_bytes < L.total)
        return fail(NH_ENOMEM, "workspace of %llu bytes is smaller than the %llu of this batch",
                    (unsigned long long)workspace_bytes, (unsigned long long)L.total);
    if (((uintptr_t)d_workspace & 255) != 0) return fail(NH_EINVAL, "workspace must be 256-byte aligned");
    char *ws = (char *)d_workspace;
    const Ctl *ctl = (const Ctl *)(ws + L.off_ctl);
    const JobDev *d_jobs = (const JobDev *)(ws + L.off_jobs);
    const JobState *d_js = (const JobState *)(ws + L.off_js);

    // The workspace must hold a finished, error-free run of exactly these jobs.
    Ctl hc;
    std::vector<JobDev> hd(n_jobs);
    std::vector<JobState> hs(n_jobs);
    HIP_TRY(hipMemcpyAsync(&hc, ctl, sizeof hc, hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipMemcpyAsync(hd.data(), d_jobs, sizeof(JobDev) * n_jobs, hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipMemcpyAsync(hs.data(), d_js, sizeof(JobState) * n_jobs, hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    if (hc.n_jobs != n_jobs) return fail(NH_EINVAL, "the workspace does not hold a run of these %u jobs", n_jobs);
    if (hc.error) return fail(NH_EINVAL, "the run in the workspace failed (error flags %#x)", hc.error);
    for (uint32_t j = 0; j < n_jobs; ++j) {
        if (hd[j].seed != jobs[j].seed || hd[j].samples != jobs[j].d_sample_ids || hd[j].n != jobs[j].n ||
            hd[j].table != jobs[j].scenario->d_table || hd[j].tau_t != jobs[j].scenario->tau_t)
            return fail(NH_EINVAL, "job %u differs from the run in the workspace", j);
        if (hs[j].remaining != 0)
            return fail(NH_EINVAL, "the run in the workspace has not finished (job %u; suspended?)", j);
        outs[j].n_events = 0;
        outs[j].n_coalescences = 0;
    }
    if (n_total == 0) return NH_OK;
    const Lin lin = lin_view(ws, L);
    const uint32_t nt = (uint32_t)n_total;
    const uint32_t lin_blocks = (nt + 255) / 256;
    int device = 0;
    HIP_TRY(hipGetDevice(&device));
    AsyncScratch S{stream, scratch_pool(device), {}};

    // Records per lineage and their offsets.
    uint64_t *n_rec = nullptr, *off = nullptr;
    uint32_t *err = nullptr;
    if (int rc = S.take(n_rec, nt)) return rc;
    if (int rc = S.take(off, nt)) return rc;
    if (int rc = S.take(err, 1)) return rc;
    HIP_TRY(hipMemsetAsync(err, 0, sizeof(uint32_t), stream));
    k_stream_count<<<lin_blocks, 256, 0, stream>>>(d_jobs, lin, nt, n_rec);
    size_t scan_bytes = 0;
    HIP_TRY(nh_sort::exclusive_sum_u64(nullptr, scan_bytes, n_rec, off, nt, stream));
    char *scan_tmp = nullptr;
    if (int rc = S.take(scan_tmp, scan_bytes)) return rc;
    HIP_TRY(nh_sort::exclusive_sum_u64(scan_tmp, scan_bytes, n_rec, off, nt, stream));
    uint64_t last[2];
    HIP_TRY(hipMemcpyAsync(&last[0], off + (nt - 1), sizeof(uint64_t), hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipMemcpyAsync(&last[1], n_rec + (nt - 1), sizeof(uint64_t), hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    const uint64_t n_records = last[0] + last[1];
    if (n_records >= (1ull << 31)) return fail(NH_EINVAL, "%llu event records exceed 2^31 - 1",
                                              (unsigned long long)n_records);
    if (n_records == 0) return NH_OK;
    const uint32_t nr = (uint32_t)n_records;
    const uint32_t rec_blocks = (uint32_t)std::min<uint64_t>((nr + 255) / 256, 65535);

    // Replay, then sort by (job, t, origin, prior).
    StreamRecs R;
    if (int rc = S.take(R.t, nr)) return rc;
    if (int rc = S.take(R.prior, nr)) return rc;
    if (int rc = S.take(R.from, nr)) return rc;
    if (int rc = S.take(R.to, nr)) return rc;
    if (int rc = S.take(R.job, nr)) return rc;
    // a replay that fails leaves records unwritten: their job index must still be valid
    HIP_TRY(hipMemsetAsync(R.job, 0, sizeof(uint32_t) * nr, stream));
    const uint32_t group_blocks = (uint32_t)std::min<uint64_t>(((uint64_t)nt * kGroup + 255) / 256, 1u << 20);
    k_stream_replay<<<group_blocks, 256, 0, stream>>>(d_jobs, lin, nt, off, R, err);
    uint32_t *perm_a, *perm_b, *k32_a, *k32_b, *flag_ev, *flag_co, *rank_ev, *rank_co;
    uint64_t *k64_a, *k64_b;
    for (uint32_t **q : {&perm_a, &perm_b, &k32_a, &k32_b, &flag_ev, &flag_co, &rank_ev, &rank_co})
        if (int rc = S.take(*q, nr)) return rc;
    if (int rc = S.take(k64_a, nr)) return rc;
    if (int rc = S.take(k64_b, nr)) return rc;
    size_t tmp_bytes = 0;
    if (int rc = sort_scratch_bytes(nr, tmp_bytes)) return rc;
    char *tmp = nullptr;
    if (int rc = S.take(tmp, tmp_bytes)) return rc;
    uint32_t *sorted = nullptr;
    if (int rc = stream_sort(R, nr, n_jobs, R.prior, R.from, R.t, perm_a, perm_b, k64_a, k64_b, k32_a, k32_b, tmp,
                             tmp_bytes, stream, sorted))
        return rc;

    // Reduce: events and coalescences per job.
    unsigned long long *counts = nullptr; // [0, n_jobs) events, [n_jobs, 2 n_jobs) coalescences
    if (int rc = S.take(counts, 2ull * n_jobs)) return rc;
    k_fill_u64<<<std::max<uint32_t>(1, (2 * n_jobs + 255) / 256), 256, 0, stream>>>(counts, 2ull * n_jobs, 0ull);
    k_stream_flags<<<rec_blocks, 256, 0, stream>>>(R, sorted, nr, flag_ev, flag_co, counts, counts + n_jobs);
    size_t b = tmp_bytes;
    HIP_TRY(nh_sort::exclusive_sum_u32(tmp, b, flag_ev, rank_ev, nr, stream));
    b = tmp_bytes;
    HIP_TRY(nh_sort::exclusive_sum_u32(tmp, b, flag_co, rank_co, nr, stream));
    std::vector<unsigned long long> hcnt(2ull * n_jobs);
    HIP_TRY(hipMemcpyAsync(hcnt.data(), counts, sizeof(unsigned long long) * 2 * n_jobs, hipMemcpyDeviceToHost,
                           stream));
    HIP_TRY(hipStreamSynchronize(stream));
    std::vector<uint64_t> base(2ull * n_jobs);
    uint64_t n_coal = 0, ev_acc = 0;
    for (uint32_t j = 0; j < n_jobs; ++j) {
        base[j] = ev_acc;
        base[n_jobs + j] = n_coal;
        ev_acc += hcnt[j];
        n_coal += hcnt[n_jobs + j];
        if (hcnt[n_jobs + j] > jobs[j].n) return fail(NH_EDEVICE, "job %u: more coalescences than samples", j);
    }
    std::vector<StreamDev> hout(n_jobs);
    for (uint32_t j = 0; j < n_jobs; ++j)
        hout[j] = StreamDev{outs[j].d_events, outs[j].d_events ? outs[j].events_cap : 0, outs[j].d_coalescences,
                            jobs[j].n};
    uint64_t *d_base = nullptr;
    StreamDev *d_out = nullptr;
    if (int rc = S.take(d_base, 2ull * n_jobs)) return rc;
    if (int rc = S.take(d_out, n_jobs)) return rc;
    HIP_TRY(hipMemcpyAsync(d_base, base.data(), sizeof(uint64_t) * 2 * n_jobs, hipMemcpyHostToDevice, stream));
    HIP_TRY(hipMemcpyAsync(d_out, hout.data(), sizeof(StreamDev) * n_jobs, hipMemcpyHostToDevice, stream));
    StreamRecs C{};
    const uint32_t nc = (uint32_t)n_coal;
    if (int rc = S.take(C.t, nc)) return rc;
    if (int rc = S.take(C.prior, nc)) return rc;
    if (int rc = S.take(C.from, nc)) return rc;
    if (int rc = S.take(C.job, nc)) return rc;
    k_stream_emit<<<rec_blocks, 256, 0, stream>>>(R, sorted, nr, flag_ev, rank_ev, flag_co, rank_co, d_base, d_out,
                                                  C, err);
    if (nc) {
        // coalescences by (job, t, loc, parent's arrival)
        size_t need = 0;
        if (int rc = sort_scratch_bytes(nc, need)) return rc;
        if (need > tmp_bytes) {
            if (int rc = S.take(tmp, need)) return rc;
            tmp_bytes = need;
        }
        uint32_t *csorted = nullptr;
        if (int rc = stream_sort(C, nc, n_jobs, C.prior, C.from, C.t, perm_a, perm_b, k64_a, k64_b, k32_a, k32_b,
                                 tmp, tmp_bytes, stream, csorted))
            return rc;
        k_stream_coal_write<<<(uint32_t)std::min<uint64_t>((nc + 255) / 256, 65535), 256, 0, stream>>>(
            C, csorted, nc, d_base + n_jobs, d_out);
    }
    HIP_TRY(hipGetLastError());
    uint32_t herr = 0;
    HIP_TRY(hipMemcpyAsync(&herr, err, sizeof herr, hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    if (herr) return fail(NH_EDEVICE, "event stream: a replay did not retrace its lineage (flags %#x)", herr);
    for (uint32_t j = 0; j < n_jobs; ++j) {
        outs[j].n_events = hcnt[j];
        outs[j].n_coalescences = hcnt[n_jobs + j];
    }
    return NH_OK;
}

} // namespace

NH_API int nh_batch_run(const nh_job *jobs, uint32_t n_jobs, void *d_workspace, uint64_t workspace_bytes,
                        const nh_config *cfg, nh_stats *stats, void *stream) {
    return batch_run_impl(jobs, n_jobs, d_workspace, workspace_bytes, cfg, stats, stream, false);
}

NH_API int nh_batch_resume(const nh_job *jobs, uint32_t n_jobs, void *d_workspace, uint64_t workspace_bytes,
                           const nh_config *cfg, nh_stats *stats, void *stream) {
    if (n_jobs == 0) return fail(NH_EINVAL, "no jobs to resume");
    return batch_run_impl(jobs, n_jobs, d_workspace, workspace_bytes, cfg, stats, stream, true);
}

NH_API int nh_event_stream(const nh_job *jobs, uint32_t n_jobs, void *d_workspace, uint64_t workspace_bytes,
                           nh_stream_out *outs, void *stream) {
    return event_stream_impl(jobs, n_jobs, d_workspace, workspace_bytes, outs, stream);
}

NH_API int nh_simulate_device(const nh_scenario *scenario, uint64_t seed, const uint64_t *d_sample_ids, uint64_t n,
                              uint64_t *d_species_out, uint64_t *d_richness_out, const nh_config *cfg,
                              nh_stats *stats, void *stream_ptr) {
    if (!scenario) return fail(NH_EINVAL, "scenario is NULL");
    hipStream_t stream = (hipStream_t)stream_ptr;
    nh_job job{scenario, seed, d_sample_ids, n, d_species_out, d_richness_out};
    const uint64_t bytes = nh_workspace_bytes(n, 1);
    void *ws = nullptr;
    HIP_TRY(hipMallocAsync(&ws, bytes, stream));
    const int rc = nh_batch_run(&job, 1, ws, bytes, cfg, stats, stream_ptr);
    (void)hipFreeAsync(ws, stream);
    return rc;
}

NH_API int nh_simulate_async(const nh_scenario *scenario, uint64_t seed, const uint64_t *d_sample_ids, uint64_t n,
                             uint64_t *d_species_out, uint64_t *d_richness_out, const nh_config *cfg_in,
                             void *stream_ptr) {
    nh_config cfg;
    fill_config(cfg_in, cfg);
    if (int rc = check_single(scenario, d_sample_ids, n, d_species_out, cfg)) return rc;
    hipStream_t stream = (hipStream_t)stream_ptr;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    const uint64_t bytes = nh_workspace_bytes(n, 1);
    void *ws = nullptr;
    if (hipMemPool_t pool = scratch_pool(dev)) HIP_TRY(hipMallocFromPoolAsync(&ws, bytes, pool, stream));
    else HIP_TRY(hipMallocAsync(&ws, bytes, stream));
    const int rc = enqueue_single(scenario, seed, d_sample_ids, n, d_species_out, d_richness_out, (char *)ws, cfg,
                                  stream);
    (void)hipFreeAsync(ws, stream);
    return rc;
}

NH_API int nh_simulate_noalloc(const nh_scenario *scenario, uint64_t seed, const uint64_t *d_sample_ids,
                               uint64_t n, uint64_t *d_species_out, uint64_t *d_richness_out, const nh_config *cfg_in,
                               void *stream_ptr) {
    nh_config cfg;
    fill_config(cfg_in, cfg);
    if (int rc = check_single(scenario, d_sample_ids, n, d_species_out, cfg)) return rc;
    if (nh_workspace_bytes(n, 1) > kScratchBytes) {
        uint64_t lo = 0, hi = n; // the largest run the scratch holds
        while (hi - lo > 1) {
            const uint64_t mid = lo + (hi - lo) / 2;
            if (nh_workspace_bytes(mid, 1) <= kScratchBytes) lo = mid;
            else hi = mid;
        }
        return fail(NH_EINVAL, "nh_simulate_noalloc: %llu samples need %llu workspace bytes; its scratch holds %llu "
                    "bytes, at most %llu samples", (unsigned long long)n,
                    (unsigned long long)nh_workspace_bytes(n, 1), (unsigned long long)kScratchBytes,
                    (unsigned long long)lo);
    }
    void *ws = nullptr;
    if (int rc = scratch_address(ws)) return rc;
    return enqueue_single(scenario, seed, d_sample_ids, n, d_species_out, d_richness_out, (char *)ws, cfg,
                          (hipStream_t)stream_ptr);
}

NH_API int nh_simulate(const nh_scenario *scenario, uint64_t seed, const uint64_t *h_sample_ids, uint64_t n,
                       uint64_t *h_species_out, uint64_t *h_richness_out, nh_stats *stats) {
    if (!scenario) return fail(NH_EINVAL, "scenario is NULL");
    if (n > 0 && (!h_sample_ids || !h_species_out)) return fail(NH_EINVAL, "NULL sample or output buffer");
    for (uint64_t q = 0; q < n; ++q)
        if (h_sample_ids[q] >= scenario->N) return fail(NH_EINVAL, "sample id %llu out of range", (unsigned long long)h_sample_ids[q]);
    uint64_t *d_s = nullptr, *d_o = nullptr, *d_r = nullptr;
    const uint64_t m = std::max<uint64_t>(n, 1);
    HIP_TRY(hipMalloc(&d_s, 8 * m));
    struct Free {
        void *p;
        ~Free() {
            if (p) (void)hipFree(p);
        }
    } f1{d_s};
    HIP_TRY(hipMalloc(&d_o, 8 * m));
    Free f2{d_o};
    HIP_TRY(hipMalloc(&d_r, 8));
    Free f3{d_r};
    if (n) HIP_TRY(hipMemcpy(d_s, h_sample_ids, 8 * n, hipMemcpyHostToDevice));
    const uint64_t bytes = nh_workspace_bytes(n, 1);
    void *ws = nullptr;
    HIP_TRY(hipMalloc(&ws, bytes));
    Free f4{ws};
    nh_job job{scenario, seed, d_s, n, d_o, d_r};
    const int rc = nh_batch_run(&job, 1, ws, bytes, nullptr, stats, nullptr);
    if (rc != NH_OK) return rc;
    if (n) HIP_TRY(hipMemcpy(h_species_out, d_o, 8 * n, hipMemcpyDeviceToHost));
    uint64_t rich = 0;
    HIP_TRY(hipMemcpy(&rich, d_r, 8, hipMemcpyDeviceToHost));
    if (h_richness_out) *h_richness_out = rich;
    return NH_OK;
}

// ---------------------------------------------------------------------------
// Continuous batching: nh_server
// ---------------------------------------------------------------------------
namespace {

// First-fit allocator of [start, start + len) ranges with coalescing frees.
struct RangeAlloc {
    std::vector<std::pair<uint64_t, uint64_t>> free; // sorted by start: (start, len)
    void reset(uint64_t total) {
        free.clear();
        if (total) free.emplace_back(0, total);
    }
    bool alloc(uint64_t n, uint64_t &at) {
        for (size_t k = 0; k < free.size(); ++k) {
            if (free[k].second >= n) {
                at = free[k].first;
                free[k].first += n;
                free[k].second -= n;
                if (free[k].second == 0) free.erase(free.begin() + (long)k);
                return true;
            }
        }
        return false;
    }
    void release(uint64_t at, uint64_t n) {
        if (n == 0) return;
        size_t k = 0;
        while (k < free.size() && free[k].first < at) ++k;
        free.insert(free.begin() + (long)k, {at, n});
        if (k + 1 < free.size() && free[k].first + free[k].second == free[k + 1].first) {
            free[k].second += free[k + 1].second;
            free.erase(free.begin() + (long)k + 1);
        }
        if (k > 0 && free[k - 1].first + free[k - 1].second == free[k].first) {
            free[k - 1].second += free[k].second;
            free.erase(free.begin() + (long)k);
        }
    }
};

enum SlotState { kSlotFree = 0, kSlotActive = 1, kSlotResolving = 2 };

struct ServerSlot {
    int state = kSlotFree;
    uint64_t tag = 0;
    nh_job job{};
    uint64_t lin_base = 0, n = 0, rich_base = 0, rich_slots = 0;
    hipEvent_t ev = nullptr;
};

} // namespace

struct nh_server {
    int device = 0;
    hipStream_t stream = nullptr;        // rounds, admissions and outputs
    bool own_stream = false;
    hipStream_t user_stream = nullptr;   // the caller's stream when the server runs its own
    hipEvent_t submit_ev = nullptr;
    nh_config cfg{};
    uint64_t cap_lin = 0;
    uint32_t max_jobs = 0, lookahead = 0;
    void *ws = nullptr;
    Workspace L{};
    Ctl *ctl = nullptr;
    JobDev *d_jobs = nullptr;
    JobState *d_js = nullptr;
    uint32_t *d_ring = nullptr;
    double *d_htab = nullptr;
    Lin lin{};
    unsigned long long *rich = nullptr;
    uint32_t *rich_counts = nullptr;
    uint64_t rich_total = 0;
    // host-mapped / pinned
    unsigned long long *status_h = nullptr, *status_d = nullptr;
    uint32_t *ring_h = nullptr, *ring_hd = nullptr;
    JobState *js_h = nullptr;
    JobDev *jobdev_h = nullptr;
    RangeAlloc lin_alloc, rich_alloc;
    std::vector<ServerSlot> slots;
    std::vector<uint32_t> free_slots;
    std::vector<std::pair<nh_job, uint64_t>> pending;
    std::vector<nh_completion> done;
    uint32_t ring_read = 0;
    uint32_t active = 0, resolving = 0;
    uint64_t rounds_enqueued = 0;
    uint64_t admitted_at = 0; // rounds enqueued when the last job was admitted (its k_init follows them)
    uint32_t grid = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // tail lane
    uint32_t tail_blocks = 0;
    size_t tail_lds = 0;
    hipStream_t tail_stream = nullptr;
    hipEvent_t tail_ev = nullptr;
    TailQ *d_tail = nullptr;
    unsigned long long *tail_ring_h = nullptr, *tail_ring_d = nullptr;
    uint32_t *tail_word_h = nullptr, *tail_word_d = nullptr; // [0]: hand-offs (copied each round), [1]: stop,
                                                             // [2]: cut walks queued again
    uint32_t tail_read = 0, tail_seen = 0;
    bool tail_launched = false;
    unsigned long long tail_idle_ticks = 0;
};

namespace {

void server_free(nh_server *s) {
    if (!s) return;
    if (s->tail_stream) {
        // the tail kernel leaves on the stop word (a walk within 512 events)
        if (s->tail_word_h) __atomic_store_n(&s->tail_word_h[1], 1u, __ATOMIC_SEQ_CST);
        (void)hipStreamSynchronize(s->tail_stream);
        (void)hipStreamDestroy(s->tail_stream);
    }
    if (s->tail_ev) (void)hipEventDestroy(s->tail_ev);
    if (s->d_tail) (void)hipFree(s->d_tail);
    if (s->tail_ring_h) (void)hipHostFree(s->tail_ring_h);
    if (s->tail_word_h) (void)hipHostFree(s->tail_word_h);
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    for (auto &sl : s->slots)
        if (sl.ev) (void)hipEventDestroy(sl.ev);
    if (s->exec) (void)hipGraphExecDestroy(s->exec);
    if (s->graph) (void)hipGraphDestroy(s->graph);
    if (s->ws) (void)hipFree(s->ws);
    if (s->status_h) (void)hipHostFree(s->status_h);
    if (s->ring_h) (void)hipHostFree(s->ring_h);
    if (s->js_h) (void)hipHostFree(s->js_h);
    if (s->jobdev_h) (void)hipHostFree(s->jobdev_h);
    if (s->submit_ev) (void)hipEventDestroy(s->submit_ev);
    if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
}

void job_descriptor(JobDev &d, const nh_job &job, unsigned long long *rich_set, uint32_t *rich_counts,
                    uint64_t rich_off, uint64_t rich_slots, uint64_t lin_base) {
    const nh_scenario *sc = job.scenario;
    std::memset(&d, 0, sizeof d);
    d.seed = job.seed;
    d.nu_thresh = sc->nu_thresh;
    d.inv_lambda = 1.0 / sc->lambda;
    d.dt = sc->dt;
    d.inv_dt = 1.0 / sc->dt;
    d.table = sc->d_table;
    d.row_ptr = sc->d_row_ptr;
    d.cap = sc->d_cap;
    d.prefix = sc->d_prefix;
    d.samples = job.d_sample_ids;
    d.species_out = (unsigned long long *)job.d_species_out;
    d.richness_out = (unsigned long long *)job.d_richness_out;
    d.rich_set = rich_set;
    d.rich_counts = rich_counts;
    d.rich_off = rich_off;
    d.rich_mask = (uint32_t)(rich_slots - 1);
    d.spec_loc_out = job.d_spec_loc_out;
    d.spec_time_out = job.d_spec_time_out;
    d.abund_ids_out = (unsigned long long *)job.d_abundance_ids_out;
    d.abund_counts_out = job.d_abundance_counts_out;
    d.n_individuals = sc->N;
    d.W = sc->W;
    d.H = sc->H;
    d.cmax = sc->cmax;
    d.R = sc->R;
    d.mode = sc->mode;
    d.n_shared = sc->n_shared;
    d.cap_const = sc->cap_const;
    d.caps_in_table = (sc->mode == NH_DISPERSAL_PER_DEME && sc->cmax <= 0xFFFFu) ? 1u : 0u;
    d.sampler = sc->sampler;
    d.mu = sc->mu;
    d.p0 = sc->p0;
    d.mig_thresh = sc->mig_thresh;
    d.tau_t = sc->tau_t;
    d.lin_base = (uint32_t)lin_base;
    d.n = (uint32_t)job.n;
    d.start_round = 0;
}

// The tail lane's queue, host ring and words, its stream, and the LDS a tail
// workgroup takes so that no round workgroup (which needs a few KiB) fits on
// its compute unit.  tail_blocks == 0 (or no solo jobs): no lane.
int server_tail_setup(nh_server *s, uint32_t tail_blocks) {
    if (tail_blocks == 0 || !s->tail_stream || s->grid < 4) return NH_OK;
    s->tail_blocks = std::min<uint32_t>(tail_blocks, 64);
    int lds_cu = 0, lds_block = 0, khz = 0;
    if (hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, s->device) !=
            hipSuccess ||
        hipDeviceGetAttribute(&lds_block, hipDeviceAttributeMaxSharedMemoryPerBlock, s->device) != hipSuccess ||
        hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, s->device) != hipSuccess || khz <= 0)
        return fail(NH_EDEVICE, "device query failed");
    s->tail_lds = (size_t)std::max(0, std::min(lds_cu, lds_block));
    if (s->tail_lds > 65536 &&
        hipFuncSetAttribute((const void *)k_tail, hipFuncAttributeMaxDynamicSharedMemorySize, (int)s->tail_lds) !=
            hipSuccess)
        s->tail_lds = 65536;
    s->tail_idle_ticks = (unsigned long long)khz / 5; // 200 us
    if (hipMalloc(&s->d_tail, sizeof(TailQ)) != hipSuccess) return fail(NH_ENOMEM, "tail queue allocation failed");
    if (hipMemsetAsync(s->d_tail, 0, sizeof(TailQ), s->stream) != hipSuccess)
        return fail(NH_EDEVICE, "tail queue clear failed");
    void *h = nullptr;
    if (hipHostMalloc(&h, sizeof(unsigned long long) * s->max_jobs, hipHostMallocMapped | hipHostMallocCoherent) !=
        hipSuccess)
        return fail(NH_ENOMEM, "pinned tail ring allocation failed");
    s->tail_ring_h = (unsigned long long *)h;
    std::memset(s->tail_ring_h, 0, sizeof(unsigned long long) * s->max_jobs);
    if (hipHostGetDevicePointer((void **)&s->tail_ring_d, h, 0) != hipSuccess)
        return fail(NH_EDEVICE, "tail ring mapping failed");
    if (hipHostMalloc(&h, 64, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess)
        return fail(NH_ENOMEM, "pinned tail word allocation failed");
    s->tail_word_h = (uint32_t *)h;
    std::memset(s->tail_word_h, 0, 64);
    if (hipHostGetDevicePointer((void **)&s->tail_word_d, h, 0) != hipSuccess)
        return fail(NH_EDEVICE, "tail word mapping failed");
    if (hipEventCreateWithFlags(&s->tail_ev, hipEventDisableTiming) != hipSuccess)
        return fail(NH_EDEVICE, "tail event creation failed");
    return NH_OK;
}

// Starts the tail kernel once its last launch has left, if hand-offs have come
// since that launch started or it queued cut walks again.  A launch sees every
// entry filled before it started; it leaves at the end of its time slice (so
// it never holds a hardware queue it may share with the rounds for long) or
// after idle_ticks with nothing ready.
int server_tail_kick(nh_server *s) {
    if (!s->tail_stream) return NH_OK;
    if (s->tail_launched) {
        const hipError_t q = hipEventQuery(s->tail_ev);
        if (q == hipErrorNotReady) return NH_OK;
        if (q != hipSuccess) return fail(NH_EDEVICE, "tail lane failed: %s", hipGetErrorString(q));
    }
    const uint32_t pushed = __atomic_load_n(&s->tail_word_h[0], __ATOMIC_ACQUIRE);
    const uint32_t more = __atomic_load_n(&s->tail_word_h[2], __ATOMIC_ACQUIRE);
    if (pushed == s->tail_seen && !more) return NH_OK;
    __atomic_store_n(&s->tail_word_h[2], 0u, __ATOMIC_RELEASE);
    s->tail_seen = pushed;
    TailArgs ta;
    ta.ctl = s->ctl;
    ta.jobs = s->d_jobs;
    ta.js = s->d_js;
    ta.lin = s->lin;
    ta.q = s->d_tail;
    ta.ring_host = s->tail_ring_d;
    ta.ring_cap = s->max_jobs;
    ta.stop_host = s->tail_word_d + 1;
    ta.idle_ticks = s->tail_idle_ticks;
    ta.slice_ticks = s->tail_idle_ticks * 40; // 8 ms
    ta.more_host = s->tail_word_d + 2;
    ta.lds_entries = (uint32_t)(s->tail_lds / (4 * sizeof(uint4)));
    k_tail<<<s->tail_blocks, 256, s->tail_lds, s->tail_stream>>>(ta);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipEventRecord(s->tail_ev, s->tail_stream));
    s->tail_launched = true;
    return NH_OK;
}

int server_launch_round(nh_server *s) {
    if (s->exec) HIP_TRY(hipGraphLaunch(s->exec, s->stream));
    else return fail(NH_EDEVICE, "server round graph missing");
    HIP_TRY(hipGetLastError());
    s->rounds_enqueued += s->cfg.rounds_per_graph;
    return NH_OK;
}

// Output of a completed job, enqueued on the server stream.
int server_resolve(nh_server *s, uint32_t slot) {
    ServerSlot &sl = s->slots[slot];
    const uint32_t blocks = (uint32_t)((sl.n + 255) / 256);
    k_resolve<<<blocks, 256, 0, s->stream>>>(s->d_jobs, s->d_js, s->lin, (uint32_t)sl.lin_base,
                                              (uint32_t)(sl.lin_base + sl.n), nullptr);
    if (sl.job.d_abundance_counts_out)
        k_abundance<<<(uint32_t)((sl.rich_slots + 255) / 256), 256, 0, s->stream>>>(s->d_jobs, s->d_js, slot, slot + 1,
                                                                                  sl.rich_slots, nullptr);
    k_finalize<<<1, 1, 0, s->stream>>>(s->d_jobs, s->d_js, slot, slot + 1, nullptr, 0u);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(&s->js_h[slot], &s->d_js[slot], sizeof(JobState), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipEventRecord(sl.ev, s->stream));
    sl.state = kSlotResolving;
    --s->active;
    ++s->resolving;
    return NH_OK;
}

int server_admit(nh_server *s, const nh_job &job, uint64_t tag, bool &admitted) {
    admitted = false;
    if (s->free_slots.empty()) return NH_OK;
    const uint64_t rich_slots = pow2_at_least(2 * job.n, 64);
    uint64_t lin_at = 0, rich_at = 0;
    if (job.n && !s->lin_alloc.alloc(job.n, lin_at)) return NH_OK;
    if (!s->rich_alloc.alloc(rich_slots, rich_at)) {
        if (job.n) s->lin_alloc.release(lin_at, job.n);
        return NH_OK;
    }
    const uint32_t slot = s->free_slots.back();
    s->free_slots.pop_back();
    ServerSlot &sl = s->slots[slot];
    sl.state = kSlotActive;
    sl.tag = tag;
    sl.job = job;
    sl.lin_base = lin_at;
    sl.n = job.n;
    sl.rich_base = rich_at;
    sl.rich_slots = rich_slots;
    JobDev &d = s->jobdev_h[slot];
    job_descriptor(d, job, s->rich + rich_at, s->rich_counts + rich_at, rich_at, rich_slots, lin_at);
    HIP_TRY(hipMemcpyAsync(&s->d_jobs[slot], &d, sizeof(JobDev), hipMemcpyHostToDevice, s->stream));
    const uint32_t fill_blocks = (uint32_t)std::min<uint64_t>(1024, (rich_slots + 255) / 256);
    k_job_setup<<<fill_blocks, 256, 0, s->stream>>>(s->ctl, s->d_jobs, s->d_js, slot);
    if (job.n) {
        const uint32_t blocks = (uint32_t)((job.n + 255) / 256);
        k_init<<<blocks, 256, 0, s->stream>>>(s->ctl, s->d_jobs, s->max_jobs, (int)slot, s->d_js, s->d_ring,
                                               s->max_jobs, s->lin, (uint32_t)lin_at, (uint32_t)(lin_at + job.n));
    } else {
        // nothing to simulate: resolve (richness 0) right away
        k_finalize<<<1, 1, 0, s->stream>>>(s->d_jobs, s->d_js, slot, slot + 1, nullptr, 0u);
        HIP_TRY(hipMemcpyAsync(&s->js_h[slot], &s->d_js[slot], sizeof(JobState), hipMemcpyDeviceToHost, s->stream));
        HIP_TRY(hipEventRecord(sl.ev, s->stream));
        sl.state = kSlotResolving;
        ++s->resolving;
        admitted = true;
        return NH_OK;
    }
    HIP_TRY(hipGetLastError());
    ++s->active;
    s->admitted_at = s->rounds_enqueued;
    admitted = true;
    return NH_OK;
}

} // namespace

NH_API uint64_t nh_server_bytes(uint64_t lineage_capacity, uint32_t max_jobs) {
    return layout(lineage_capacity, max_jobs).total;
}

NH_API int nh_server_create(const nh_server_config *config, void *stream, nh_server **out) {
    if (!out) return fail(NH_EINVAL, "out is NULL");
    *out = nullptr;
    if (!config || config->lineage_capacity == 0 || config->max_jobs == 0)
        return fail(NH_EINVAL, "server needs a positive lineage capacity and job count");
    if (config->lineage_capacity >= (1ull << 31)) return fail(NH_EINVAL, "lineage capacity must be < 2^31");
    nh_server *s = new nh_server();
    fill_config(&config->cfg, s->cfg);
    if (s->cfg.block_size % 64 != 0 || s->cfg.block_size > 256) {
        delete s;
        return fail(NH_EINVAL, "block_size must be a multiple of 64 up to 256");
    }
    s->cap_lin = config->lineage_capacity;
    s->max_jobs = config->max_jobs;
    s->lookahead = config->lookahead;
    auto bail = [&](int code) {
        server_free(s);
        return code;
    };
    if (hipGetDevice(&s->device) != hipSuccess) return bail(fail(NH_EDEVICE, "no HIP device"));
    // A tail lane's kernel runs for as long as tails walk, and a hardware queue runs its kernels in
    // order: the rounds and the lane each get a stream of the server's own, created one after the
    // other so that the runtime puts them on different hardware queues.  The caller's stream then
    // only orders submissions (the server stream waits for the caller's work at each submit).
    const bool want_tail = config->tail_blocks > 0 && s->cfg.solo_max > 0;
    if (stream && !want_tail) {
        s->stream = (hipStream_t)stream;
    } else {
        if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess)
            return bail(fail(NH_EDEVICE, "stream creation failed"));
        s->own_stream = true;
        s->user_stream = (hipStream_t)stream;
        if (want_tail && hipStreamCreateWithFlags(&s->tail_stream, hipStreamNonBlocking) != hipSuccess)
            return bail(fail(NH_EDEVICE, "tail stream creation failed"));
        if (s->user_stream && hipEventCreateWithFlags(&s->submit_ev, hipEventDisableTiming) != hipSuccess)
            return bail(fail(NH_EDEVICE, "event creation failed"));
    }
    s->L = layout(s->cap_lin, s->max_jobs);
    if (hipMalloc(&s->ws, s->L.total) != hipSuccess)
        return bail(fail(NH_ENOMEM, "server pool of %llu bytes", (unsigned long long)s->L.total));
    char *ws = (char *)s->ws;
    s->ctl = (Ctl *)(ws + s->L.off_ctl);
    s->d_jobs = (JobDev *)(ws + s->L.off_jobs);
    s->d_js = (JobState *)(ws + s->L.off_js);
    s->d_ring = (uint32_t *)(ws + s->L.off_ring);
    s->d_htab = (double *)(ws + s->L.off_htab);
    s->lin.loc[0] = (uint32_t *)(ws + s->L.off_loc0);
    s->lin.loc[1] = (uint32_t *)(ws + s->L.off_loc1);
    s->lin.t[0] = (double *)(ws + s->L.off_t0);
    s->lin.t[1] = (double *)(ws + s->L.off_t1);
    s->lin.parent = (uint32_t *)(ws + s->L.off_parent);
    s->lin.species = (unsigned long long *)(ws + s->L.off_species);
    s->lin.job = (uint32_t *)(ws + s->L.off_job);
    s->lin.events = (uint32_t *)(ws + s->L.off_events);
    s->lin.spec_loc = (uint32_t *)(ws + s->L.off_sloc);
    s->lin.spec_t = (double *)(ws + s->L.off_st);
    s->lin.act[0] = (uint32_t *)(ws + s->L.off_act0);
    s->lin.act[1] = (uint32_t *)(ws + s->L.off_act1);
    s->lin.hash = (unsigned long long *)(ws + s->L.off_hash);
    s->lin.hmask = (uint32_t)(s->L.hcap - 1);
    s->rich = (unsigned long long *)(ws + s->L.off_rich);
    s->rich_counts = (uint32_t *)(ws + s->L.off_rcount);
    s->rich_total = 4 * s->cap_lin + 64ull * s->max_jobs;
    void *h = nullptr;
    if (hipHostMalloc(&h, 256, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess)
        return bail(fail(NH_ENOMEM, "pinned status allocation failed"));
    s->status_h = (unsigned long long *)h;
    if (hipHostGetDevicePointer((void **)&s->status_d, h, 0) != hipSuccess)
        return bail(fail(NH_EDEVICE, "status mapping failed"));
    if (hipHostMalloc(&h, sizeof(uint32_t) * (1 + s->max_jobs), hipHostMallocMapped | hipHostMallocCoherent) !=
        hipSuccess)
        return bail(fail(NH_ENOMEM, "pinned ring allocation failed"));
    s->ring_h = (uint32_t *)h;
    std::memset(s->ring_h, 0, sizeof(uint32_t) * (1 + s->max_jobs));
    if (hipHostGetDevicePointer((void **)&s->ring_hd, h, 0) != hipSuccess)
        return bail(fail(NH_EDEVICE, "ring mapping failed"));
    if (hipHostMalloc(&h, sizeof(JobState) * s->max_jobs, hipHostMallocDefault) != hipSuccess)
        return bail(fail(NH_ENOMEM, "pinned job-state allocation failed"));
    s->js_h = (JobState *)h;
    if (hipHostMalloc(&h, sizeof(JobDev) * s->max_jobs, hipHostMallocDefault) != hipSuccess)
        return bail(fail(NH_ENOMEM, "pinned job staging allocation failed"));
    s->jobdev_h = (JobDev *)h;
    s->slots.resize(s->max_jobs);
    for (uint32_t k = 0; k < s->max_jobs; ++k) {
        if (hipEventCreateWithFlags(&s->slots[k].ev, hipEventDisableTiming) != hipSuccess)
            return bail(fail(NH_EDEVICE, "event creation failed"));
        s->free_slots.push_back(s->max_jobs - 1 - k);
    }
    s->lin_alloc.reset(s->cap_lin);
    s->rich_alloc.reset(s->rich_total);
    __atomic_store_n(s->status_h, (unsigned long long)1, __ATOMIC_SEQ_CST);

    const std::vector<double> htab = horizon_table(s->cfg);
    if (hipMemcpyAsync(s->d_htab, htab.data(), sizeof(double) * kMaxHorizons, hipMemcpyHostToDevice, s->stream) !=
        hipSuccess)
        return bail(fail(NH_EDEVICE, "horizon upload failed"));
    k_setup<<<1, 256, 0, s->stream>>>(s->ctl, s->d_js, s->d_jobs, 0, 1);
    k_fill_u64<<<1024, 256, 0, s->stream>>>(s->lin.hash, s->L.hcap, 0ull);
    if (hipGetLastError() != hipSuccess) return bail(fail(NH_EDEVICE, "server setup launch failed"));

    int n_cu = 0;
    if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, s->device) != hipSuccess)
        return bail(fail(NH_EDEVICE, "device query failed"));
    s->grid = (uint32_t)std::max(1, n_cu) * s->cfg.blocks_per_cu;
    RoundArgs ra;
    std::memset(&ra, 0, sizeof ra);
    ra.ctl = s->ctl;
    ra.jobs = s->d_jobs;
    ra.js = s->d_js;
    ra.ring = s->d_ring;
    ra.ring_cap = s->max_jobs;
    ra.lin = s->lin;
    ra.htab = s->d_htab;
    ra.coop_max =
        s->cfg.coop_max ? s->cfg.coop_max : (uint32_t)(((uint64_t)s->grid * s->cfg.block_size) / (2 * kGroup)) + 1;
    ra.n_cap = (uint32_t)s->cap_lin;
    ra.solo_max = s->grid < 4 ? 0u : s->cfg.solo_max; // solo blocks never take more than a quarter
    ra.solo_step = s->cfg.solo_step;
    if (int rc = server_tail_setup(s, config->tail_blocks)) return bail(rc);
    ra.tail = s->d_tail;
    ra.tail_walkers = s->tail_blocks * 4;
    hipStream_t cap_stream;
    if (hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking) != hipSuccess)
        return bail(fail(NH_EDEVICE, "capture stream creation failed"));
    hipError_t e = hipStreamBeginCapture(cap_stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        for (uint32_t k = 0; k < s->cfg.rounds_per_graph; ++k) {
            k_round<false, false><<<s->grid, s->cfg.block_size, 0, cap_stream>>>(ra);
            k_advance<<<1, 1, 0, cap_stream>>>(s->ctl, s->status_d, s->d_ring, s->max_jobs, s->ring_hd, s->d_tail,
                                               s->d_tail ? s->tail_word_d : nullptr);
        }
        e = hipStreamEndCapture(cap_stream, &s->graph);
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&s->exec, s->graph, nullptr, nullptr, 0);
    (void)hipStreamDestroy(cap_stream);
    if (e != hipSuccess) return bail(fail(NH_EDEVICE, "round graph capture failed: %s", hipGetErrorString(e)));
    if (hipStreamSynchronize(s->stream) != hipSuccess) return bail(fail(NH_EDEVICE, "server setup failed"));
    *out = s;
    return NH_OK;
}

NH_API int nh_server_submit(nh_server *s, const nh_job *job, uint64_t tag) {
    if (!s || !job || !job->scenario) return fail(NH_EINVAL, "NULL server, job or scenario");
    if (job->n > 0 && (!job->d_sample_ids || !job->d_species_out))
        return fail(NH_EINVAL, "NULL sample or output buffer");
    if (!job->d_spec_loc_out != !job->d_spec_time_out || !job->d_abundance_ids_out != !job->d_abundance_counts_out)
        return fail(NH_EINVAL, "reporter outputs come in pairs (both or neither)");
    if (job->n > s->cap_lin)
        return fail(NH_EINVAL, "job of %llu lineages exceeds the server capacity %llu", (unsigned long long)job->n,
                    (unsigned long long)s->cap_lin);
    if (pow2_at_least(2 * job->n, 64) > s->rich_total) return fail(NH_EINVAL, "job too large for the species pool");
    if (s->user_stream) { // the job's buffers may still be written by work on the caller's stream
        HIP_TRY(hipEventRecord(s->submit_ev, s->user_stream));
        HIP_TRY(hipStreamWaitEvent(s->stream, s->submit_ev, 0));
    }
    s->pending.emplace_back(*job, tag);
    return NH_OK;
}

NH_API int nh_server_progress(nh_server *s, uint32_t *active_out, uint32_t *pending_out) {
    if (!s) return fail(NH_EINVAL, "NULL server");
    // (a) completions published by the round epilogue
    const uint32_t head = __atomic_load_n(&s->ring_h[0], __ATOMIC_ACQUIRE);
    while (s->ring_read != head) {
        const uint32_t slot = __atomic_load_n(&s->ring_h[1 + s->ring_read % s->max_jobs], __ATOMIC_ACQUIRE);
        ++s->ring_read;
        if (slot >= s->max_jobs || s->slots[slot].state != kSlotActive)
            return fail(NH_EDEVICE, "corrupt completion ring entry %u", slot);
        if (int rc = server_resolve(s, slot)) return rc;
    }
    // (a') completions published by the tail lane
    while (s->tail_ring_h) {
        const unsigned long long e = __atomic_load_n(&s->tail_ring_h[s->tail_read % s->max_jobs], __ATOMIC_ACQUIRE);
        if ((uint32_t)(e >> 32) != s->tail_read + 1u) break;
        const uint32_t slot = (uint32_t)e;
        ++s->tail_read;
        if (slot >= s->max_jobs || s->slots[slot].state != kSlotActive)
            return fail(NH_EDEVICE, "corrupt tail ring entry %u", slot);
        if (int rc = server_resolve(s, slot)) return rc;
    }
    if (int rc = server_tail_kick(s)) return rc;
    // (b) resolved jobs: report, free their slots and ranges
    if (s->resolving) {
        for (uint32_t k = 0; k < s->max_jobs; ++k) {
            ServerSlot &sl = s->slots[k];
            if (sl.state != kSlotResolving) continue;
            const hipError_t q = hipEventQuery(sl.ev);
            if (q == hipErrorNotReady) continue;
            if (q != hipSuccess) return fail(NH_EDEVICE, "job event failed: %s", hipGetErrorString(q));
            const JobState &js = s->js_h[k];
            nh_completion c{};
            c.tag = sl.tag;
            c.status = (js.flags & kJobBadSample) ? NH_EINVAL : NH_OK;
            c.rounds = js.done_round > js.start_round ? js.done_round - js.start_round : 0;
            c.richness = js.rich_count;
            c.events = js.events;
            c.lineages = sl.n;
            c.speciated = js.speciated;
            c.merged = js.merged;
            s->done.push_back(c);
            if (sl.n) s->lin_alloc.release(sl.lin_base, sl.n);
            s->rich_alloc.release(sl.rich_base, sl.rich_slots);
            sl.state = kSlotFree;
            s->free_slots.push_back(k);
            --s->resolving;
        }
    }
    // (c) admission: FIFO, with backfill over `lookahead` jobs behind a head that does not fit
    size_t k = 0;
    uint32_t skipped = 0;
    while (k < s->pending.size() && !s->free_slots.empty()) {
        bool admitted = false;
        if (int rc = server_admit(s, s->pending[k].first, s->pending[k].second, admitted)) return rc;
        if (admitted) {
            s->pending.erase(s->pending.begin() + (long)k);
        } else {
            if (++skipped > s->lookahead) break;
            ++k;
        }
    }
    // (d) rounds: keep two launches in flight while lineages are in the rounds (the last round
    // left some queued, or a job was admitted after the rounds enqueued so far); jobs whose last
    // lineage walks in the tail lane need none
    if (s->active) {
        const unsigned long long word = __atomic_load_n(s->status_h, __ATOMIC_ACQUIRE);
        if ((word >> 31) & 1u) return fail(NH_EDEVICE, "kernel reported an error");
        const uint32_t next_round = (uint32_t)(word >> 32);
        const uint64_t completed = next_round >= 1 ? next_round - 1 : 0;
        const bool queued = (word & 0x7FFFFFFFull) != 0 || completed <= s->admitted_at;
        while (queued && s->rounds_enqueued < completed + 2ull * s->cfg.rounds_per_graph)
            if (int rc = server_launch_round(s)) return rc;
    }
    if (active_out) *active_out = s->active + s->resolving;
    if (pending_out) *pending_out = (uint32_t)s->pending.size();
    return NH_OK;
}

NH_API int nh_server_poll(nh_server *s, nh_completion *out, uint32_t max, uint32_t *n_out) {
    if (!s || (!out && max)) return fail(NH_EINVAL, "NULL server or output");
    const uint32_t n = (uint32_t)std::min<size_t>(max, s->done.size());
    for (uint32_t k = 0; k < n; ++k) out[k] = s->done[k];
    s->done.erase(s->done.begin(), s->done.begin() + n);
    if (n_out) *n_out = n;
    return NH_OK;
}

NH_API int nh_server_drain(nh_server *s, double timeout_s) {
    if (!s) return fail(NH_EINVAL, "NULL server");
    const auto t0 = std::chrono::steady_clock::now();
    for (uint64_t spin = 0;; ++spin) {
        uint32_t act = 0, pend = 0;
        if (int rc = nh_server_progress(s, &act, &pend)) return rc;
        if (act == 0 && pend == 0) return NH_OK;
        if ((spin & 255) == 0) {
            if (std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count() > timeout_s)
                return fail(NH_ETIMEOUT, "drain exceeded %.1f s (%u active, %u queued)", timeout_s, act, pend);
            std::this_thread::yield();
        }
    }
}

NH_API void nh_server_destroy(nh_server *s) { server_free(s); }

NH_API int nh_measure_event_latency(const nh_scenario *scenario, uint64_t seed, uint32_t steps,
                                    double *ns_per_event, void *stream_ptr) {
    if (!scenario || !ns_per_event || steps == 0) return fail(NH_EINVAL, "NULL scenario or output, or no steps");
    hipStream_t stream = (hipStream_t)stream_ptr;
    nh_job job{};
    job.scenario = scenario;
    job.seed = seed;
    JobDev hd;
    job_descriptor(hd, job, nullptr, nullptr, 0, 64, 0);
    const bool lds = scenario->mode == NH_DISPERSAL_SHARED && scenario->n_shared <= kLdsTableMax;
    const size_t lds_bytes = lds ? sizeof(uint4) * scenario->n_shared : 0;
    int device = 0;
    HIP_TRY(hipGetDevice(&device));
    AsyncScratch S{stream, nullptr, {}};
    JobDev *d_job = nullptr;
    uint32_t *err = nullptr;
    unsigned long long *sink = nullptr;
    if (int rc = S.take(d_job, 1)) return rc;
    if (int rc = S.take(err, 1)) return rc;
    if (int rc = S.take(sink, 1)) return rc;
    HIP_TRY(hipMemcpyAsync(d_job, &hd, sizeof hd, hipMemcpyHostToDevice, stream));
    HIP_TRY(hipMemsetAsync(err, 0, sizeof(uint32_t), stream));
    hipEvent_t a, b;
    HIP_TRY(hipEventCreate(&a));
    HIP_TRY(hipEventCreate(&b));
    struct EvGuard {
        hipEvent_t a, b;
        ~EvGuard() {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
        }
    } guard{a, b};
    auto launch = [&](uint32_t n) {
        if (lds) k_event_latency<true><<<1, kGroup, lds_bytes, stream>>>(d_job, n, err, sink);
        else k_event_latency<false><<<1, kGroup, 0, stream>>>(d_job, n, err, sink);
    };
    launch(std::min<uint32_t>(steps, 256)); // warm-up
    HIP_TRY(hipEventRecord(a, stream));
    launch(steps);
    HIP_TRY(hipEventRecord(b, stream));
    HIP_TRY(hipGetLastError());
    uint32_t herr = 0;
    HIP_TRY(hipMemcpyAsync(&herr, err, sizeof herr, hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    if (herr) return fail(NH_EDEVICE, "the latency walk ran away (flags %#x)", herr);
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, a, b));
    *ns_per_event = (double)ms * 1e6 / steps;
    return NH_OK;
}

NH_API int nh_eval_primitives(const nh_scenario *scenario, uint64_t seed, uint64_t n, const nh_primitive_io *io,
                              uint32_t use_lds, void *stream_ptr) {
    if (!scenario || !io) return fail(NH_EINVAL, "NULL scenario or io");
    if ((!io->d_ctr) != (!io->d_philox_out) || (!io->d_r) != (!io->d_log_out) || (!io->d_loc) != (!io->d_t) ||
        (!io->d_step_loc_out) != (!io->d_step_t_out))
        return fail(NH_EINVAL, "primitive inputs and outputs come in pairs");
    if (!io->d_loc && (io->d_next_out || io->d_next_group_out || io->d_outcome_out || io->d_step_loc_out))
        return fail(NH_EINVAL, "event outputs need d_loc and d_t");
    if (n == 0) return NH_OK;
    hipStream_t stream = (hipStream_t)stream_ptr;
    nh_job job{};
    job.scenario = scenario;
    job.seed = seed;
    JobDev hd;
    job_descriptor(hd, job, nullptr, nullptr, 0, 64, 0);
    const bool lds = use_lds && scenario->mode == NH_DISPERSAL_SHARED && scenario->n_shared <= kLdsTableMax;
    const size_t lds_bytes = lds ? sizeof(uint4) * scenario->n_shared : 0;
    AsyncScratch S{stream, nullptr, {}};
    JobDev *d_job = nullptr;
    uint32_t *err = nullptr;
    if (int rc = S.take(d_job, 1)) return rc;
    if (int rc = S.take(err, 1)) return rc;
    HIP_TRY(hipMemcpyAsync(d_job, &hd, sizeof hd, hipMemcpyHostToDevice, stream));
    HIP_TRY(hipMemsetAsync(err, 0, sizeof(uint32_t), stream));
    const uint32_t blocks = (uint32_t)std::min<uint64_t>((n * kGroup + 255) / 256, 1u << 16);
    if (lds) k_primitives<true><<<blocks, 256, lds_bytes, stream>>>(d_job, n, *io, err);
    else k_primitives<false><<<blocks, 256, 0, stream>>>(d_job, n, *io, err);
    HIP_TRY(hipGetLastError());
    uint32_t herr = 0;
    HIP_TRY(hipMemcpyAsync(&herr, err, sizeof herr, hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    if (herr) return fail(NH_EDEVICE, "an event-time search ran away (flags %#x)", herr);
    return NH_OK;
}
