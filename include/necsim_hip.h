/*
 * necsim_hip.h - C ABI of libnecsim_hip, an MI355X (gfx950) implementation of
 * the communication-free Independent algorithm for neutral Moran biodiversity
 * models (Langenstein 2021, arXiv 2108.05815).
 *
 * The method (paper chapter "The Declaration of Independence"): every sampled
 * individual's lineage is traced backwards in time on its own.  Its random
 * numbers come from a counter-based hash keyed on (seed, indexed location,
 * time) ("Environmental RNG Priming"), and waiting times are sums of
 * exponentials restarted at fixed interval boundaries ("Aligning the RNGs of
 * Colliding Individuals", "Exponential inter-event Times"), so lineages that
 * meet draw identical numbers from then on and merge with no communication.
 * At each event a lineage speciates with probability nu, otherwise it moves to
 * a parent drawn from the dispersal kernel and a uniform deme index ("Summary
 * of the Independent Algorithm").  Species identities are hashed from the
 * speciation event; richness is the number of distinct identities among the
 * samples.  Lineages that reach the same (location, next event time) are
 * merged after time-aligned horizon rounds ("Deduplicating Redundant
 * Individuals", Water-Level algorithm).
 *
 * Conventions used by every entry point:
 *   - Return value: NH_OK (0) or a negative NH_E* code; the message of the
 *     last failure on the calling thread is available from nh_last_error().
 *   - Ownership: the caller owns every buffer it passes.  nh_scenario_create
 *     deep-copies its host inputs and owns the device tables until
 *     nh_scenario_destroy.  Outputs are written only on success.
 *   - Host vs device pointers: arguments named h_* are host memory, d_* are
 *     device memory of the current HIP device (for instance a PyTorch tensor's
 *     data_ptr()).  Streams are hipStream_t passed as void* (NULL = default).
 *   - Sample ids are dense individual indices in [0, N), N = sum of
 *     capacities, in row-major cell order then deme index.  Duplicates are
 *     allowed and give identical species.
 *   - Results are a pure function of (scenario, seed, sample id): they do not
 *     depend on the order or partition of the samples, on the batch a job
 *     runs in, or on any tuning parameter in nh_config.
 *   - Threads: a scenario is immutable after nh_scenario_create, so any
 *     number of calls may use it at once.  Calls from different host threads
 *     with different workspaces (and streams) may run concurrently: the
 *     library's own state is per thread (error message, captured graphs,
 *     timing events, status word) or guarded by a lock (per-device streams and
 *     pools).  A workspace, and a server, serves one call at a time.
 */
#ifndef NECSIM_HIP_H
#define NECSIM_HIP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NH_OK 0
#define NH_EINVAL (-1)   /* invalid argument (see each function) */
#define NH_ENOMEM (-2)   /* host or device allocation failed, or workspace too small */
#define NH_EDEVICE (-3)  /* HIP runtime error or kernel-reported failure */
#define NH_ETIMEOUT (-4) /* the run exceeded nh_config.timeout_s */
#define NH_SUSPENDED 1   /* not an error: the run stopped at nh_config.max_rounds with its state in the
                            workspace; nh_batch_resume continues it */

#define NH_DISPERSAL_SHARED 0u   /* one alias table over the kernel, shared by every deme */
#define NH_DISPERSAL_PER_DEME 1u /* one table per habitable deme over weight x target capacity */

typedef struct nh_scenario nh_scenario; /* opaque, library-owned, immutable after creation */

/* Landscape: a width x height torus of demes; capacity is a host array of
 * height*width u32 in row-major order (cell c = y*width + x). */
typedef struct {
    uint32_t width, height;
    const uint32_t *h_capacity;
} nh_habitat;

/* Dispersal kernel: (2R+1)^2 non-negative f64 weights on the host, row-major
 * with row = dy + R and column = dx + R (paper: the dispersal sampler maps a
 * habitable origin to a habitable target, possibly the origin itself).
 * mode NH_DISPERSAL_SHARED: parent cell drawn in proportion to the weight;
 *   every deme must have capacity > 0.
 * mode NH_DISPERSAL_PER_DEME: parent cell drawn in proportion to weight times
 *   the target's capacity, uninhabitable targets excluded (a dispersal map
 *   restricted to habitable cells).  Radius 0 with a 1x1 torus is the paper's
 *   non-spatial scenario. */
typedef struct {
    uint32_t radius;
    const double *h_weights;
    uint32_t mode;
} nh_dispersal;

/* Scenario constants that change the random draws (never tuned):
 * lambda > 0 is the per-individual turnover rate, delta_t the repriming
 * interval, a positive power of two with lambda*delta_t <= 2^20.
 * tau >= 0 selects protracted speciation (appendix "Protracted Speciation"):
 * a speciation completes only tau generations (tau / lambda time units) after
 * it happens, so the speciation draw of an event at time t with lambda*t < tau
 * (binary64 product) is ignored and that event disperses like any other; tau = 0
 * is point speciation.  tau / lambda must lie below 2^60 (NH_EINVAL otherwise).
 * A zero-filled struct is not valid: lambda and delta_t have no zero default. */
typedef struct {
    double lambda;
    double delta_t;
    uint32_t sampler;  /* NH_SAMPLER_EXP (0, default) or NH_SAMPLER_POISSON (1) */
    uint32_t reserved; /* set to zero */
    double tau;        /* protracted speciation, generations; 0 for point speciation */
} nh_params;

/* Event-time samplers (both give Exp(lambda) gaps; they draw different bits):
 * NH_SAMPLER_EXP: from t_last, Exp(lambda) draws -log(U)/lambda summed from the
 *   interval start (section "Exponential inter-event Times");
 * NH_SAMPLER_POISSON: per interval a Poisson(lambda*delta_t) count, by a linear
 *   search over its cdf from one uniform (appendix "Iterative Sampling"), of
 *   events at start + U*delta_t; the next event is the smallest beyond t_last
 *   (section "Homogeneous Poisson Point Process").  Needs lambda*delta_t <= 700. */
#define NH_SAMPLER_EXP 0
#define NH_SAMPLER_POISSON 1

/* Tuning knobs; none of them changes any result.  Zero fields take defaults. */
typedef struct {
    double horizon0;      /* first cull horizon (time units), default 0.5 */
    double horizon_growth;/* horizon multiplier per round (> 1), default 1.25 */
    double horizon_step_max; /* cap on one round's horizon advance, default 4096 */
    uint32_t block_size;  /* threads per workgroup of the round kernel: a multiple of 64 up to 256,
                             default 256 */
    uint32_t blocks_per_cu; /* workgroups per compute unit, default 4; a persistent run takes at most as
                               many as stay resident together (the kernel's occupancy) */
    uint32_t rounds_per_graph; /* NH_LAUNCH_GRAPHS only: round kernels per captured graph (1 = plain
                                  launches), default 8; a single-job run launches its tail (queue below
                                  coop_max, rounds of 40 us or more on average) one round at a time */
    uint32_t event_timing; /* 1: bracket the round kernels with HIP events (fills round_kernel_ms) */
    uint32_t coop_max;    /* queues shorter than this many lineages run 8 lanes per lineage; default
                             (0): a launch's lane count / 16 + 1; 1 keeps one lane per lineage always */
    uint32_t table_placement; /* 0: stage a shared dispersal table in LDS for single-job runs when it
                                 fits (4096 entries); 1: read every table from global memory */
    double timeout_s;     /* wall-clock limit of one run, default 600 */
    uint32_t solo_max;    /* runs of several jobs (batches, the server): a job whose live lineage count
                             has fallen to this many or fewer runs its lineages 8 lanes each, at raised
                             wave priority, on blocks of their own, and advances its horizon by
                             solo_step per round (its serial tail no longer waits on the horizon
                             schedule of young jobs); default 0: off */
    uint32_t launch;      /* NH_LAUNCH_PERSISTENT (0, default): one launch runs every round of the run
                             (a grid barrier between rounds); NH_LAUNCH_GRAPHS: one launch per round,
                             replayed from captured graphs while the host polls the round count */
    double solo_step;     /* horizon advance per round of such a job, default 512 */
    uint32_t max_rounds;  /* nh_batch_run / nh_batch_resume: stop after at least this many rounds of the
                             call (at the first launch boundary past it) and return NH_SUSPENDED with
                             the run's whole state in the workspace; default 0: run to the end */
    uint32_t barrier_wait_ms; /* persistent launches: the longest a workgroup waits at one grid barrier
                                 before it stops the run (NH_EDEVICE; the kernel exits either way);
                                 default 0: min(timeout_s, 60 s) */
    uint32_t endgame;     /* persistent runs of several jobs: once at most this many lineages (up to
                             4096) are left, the rounds end and each is walked to its end by a wave of
                             its own (lineages that would still merge then walk the same events twice:
                             the results are the same, the event counts larger); default 0: never */
} nh_config;

#define NH_LAUNCH_PERSISTENT 0u
#define NH_LAUNCH_GRAPHS 1u

/* Per-job counters of one run. */
typedef struct {
    uint64_t events;    /* committed events (speciations + dispersals) of every lane, duplicates included */
    uint64_t lineages;  /* samples simulated */
    uint64_t speciated; /* lineages that ended by speciating (representatives) */
    uint64_t merged;    /* lineages merged into an identical one by culling */
    uint64_t rounds;    /* horizon rounds the job took part in: to the round its last lineage retired in
                           (for a suspended run, the rounds so far) */
    uint64_t richness;
    double device_ms;   /* stream time of the whole run (same for every job of a batch) */
    /* Totals of the whole run (the same for every job of a batch): */
    uint64_t philox_calls;   /* Philox4x32-10 blocks evaluated */
    uint64_t exp_draws;      /* exponential waiting-time draws (logarithms) */
    uint64_t round_kernels;  /* round-kernel launches (1 for a persistent run) */
    double round_kernel_ms;  /* HIP-event time of all round launches (cfg.event_timing), else 0 */
} nh_stats;

/* One simulate request of a batch.  Device pointers; species_out has n slots.
 * Optional reporters (each may be NULL; zero-initialise the struct):
 * - speciation events (chapter "The Declaration of Independence", the species
 *   identity is hashed from the speciation event): d_spec_loc_out[n] (u32
 *   location (y*W + x)*C_max + i) and d_spec_time_out[n] (f64 time) receive, per
 *   sample, the event at which its lineage (or the lineage it coalesced with)
 *   speciated, so species_out[q] is the species hash of exactly that event;
 *   both or neither.
 * - species abundance (the community's species-abundance distribution, the
 *   output beside richness): d_abundance_ids_out[n] and d_abundance_counts_out[n]
 *   receive one (species id, number of samples) pair per species, in no
 *   particular order; the number of pairs written is the richness.  Both or
 *   neither. */
typedef struct {
    const nh_scenario *scenario;
    uint64_t seed;
    const uint64_t *d_sample_ids;
    uint64_t n;
    uint64_t *d_species_out;
    uint64_t *d_richness_out; /* one u64, may be NULL */
    uint32_t *d_spec_loc_out;
    double *d_spec_time_out;
    uint64_t *d_abundance_ids_out;
    uint32_t *d_abundance_counts_out;
} nh_job;

/* Builds the scenario's tables on the host (Vose alias tables, capacity prefix)
 * and uploads them to the current device.
 * Errors: NH_EINVAL if width or height is 0, 2R+1 exceeds width or height,
 * nu is not in (0, 1], a weight is negative, NaN or infinite, all weights are
 * zero, a habitable deme has no habitable mass in its kernel, the shared mode
 * meets a zero-capacity deme, width*height*max(capacity) >= 2^32, lambda is
 * not positive and finite, delta_t is not a power of two, or
 * lambda*delta_t > 2^20; NH_ENOMEM / NH_EDEVICE on allocation or copy failure.
 * params may be NULL (lambda = 1, delta_t = 1). */
int nh_scenario_create(const nh_habitat *habitat, const nh_dispersal *dispersal, double nu, const nh_params *params,
                       nh_scenario **out);

/* The spatially implicit scenario (background section "Spatially Implicit" and
 * its appendix): a local community of J individuals (cell 0; sample ids
 * 0 .. J-1) that never speciates and whose lineages migrate, with probability
 * m per event, into a non-spatial metacommunity of J_meta individuals (cell 1;
 * ids J .. J+J_meta-1) simulated alongside (finite and dynamic), which
 * speciates with probability nu_meta.  Within a community the parent's deme
 * index is uniform (event draw r3); the migration coin is draw r1 (U < m);
 * speciation is tested on r0 in the metacommunity only.  params as for
 * nh_scenario_create.  NH_EINVAL for J or J_meta = 0, m outside (0, 1] (with
 * m = 0 a local lineage would never speciate) or nu_meta outside (0, 1]. */
int nh_scenario_create_implicit(uint32_t J, uint32_t J_meta, double m, double nu_meta, const nh_params *params,
                                nh_scenario **out);

void nh_scenario_destroy(nh_scenario *scenario);

/* Number of individuals N (sum of capacities). */
uint64_t nh_scenario_individuals(const nh_scenario *scenario);

/* Device bytes held by the scenario's tables. */
uint64_t nh_scenario_table_bytes(const nh_scenario *scenario);

/* Device workspace needed by nh_batch_run for jobs with n_total samples in all
 * (sum of job sizes) and n_jobs jobs. */
uint64_t nh_workspace_bytes(uint64_t n_total, uint32_t n_jobs);

/* Scenario tables plus the workspace of one job of n samples: the HBM an
 * admission controller must reserve for it. */
uint64_t nh_scenario_footprint_bytes(const nh_scenario *scenario, uint64_t n_samples);

/* Simulates every job in one device run: all lineages of all jobs share the
 * round kernels (captured in HIP graphs), the cull hash table and the work
 * queue.  d_workspace must hold nh_workspace_bytes(sum n, n_jobs) bytes of
 * device memory, 256-byte aligned.  Work is enqueued on `stream`; the call
 * returns when the results are written (it blocks the calling thread, polling
 * a host-mapped status word; other streams are not synchronised).
 * stats (nullable) receives n_jobs entries.  cfg may be NULL.
 * Errors: NH_EINVAL for a NULL job field with n > 0, a sample id >= N (the
 * device checks every id), or a bad cfg; NH_ENOMEM if the workspace is too
 * small; NH_EDEVICE on a HIP error; NH_ETIMEOUT if cfg->timeout_s passes. */
int nh_batch_run(const nh_job *jobs, uint32_t n_jobs, void *d_workspace, uint64_t workspace_bytes,
                 const nh_config *cfg, nh_stats *stats, void *stream);

/* Continues a run that nh_batch_run (or an earlier resume) left suspended
 * (NH_SUSPENDED). Between rounds the workspace is a complete checkpoint: every
 * future draw depends only on (seed, location, time) (chapter "The Declaration of
 * Independence", priming), and the workspace holds each lineage's location and
 * next event time, the merge links, the cull table and the per-job counters; the
 * device addresses it also holds (job descriptors) are written again by the
 * resume. So the caller may copy the workspace bytes to the host, free or reuse
 * the device memory, and later copy them back into any 256-byte-aligned buffer of
 * the same size; the results are bitwise those of an uninterrupted run. Bytes
 * that are not such a copy give undefined results. jobs must be the same list
 * (same order, scenarios, seeds, sizes and sample ids; the output buffers may
 * move). cfg may differ (tuning knobs never change results); cfg->max_rounds may
 * suspend again. Returns as nh_batch_run; stats count the events of the whole run
 * so far and rounds since its start. */
int nh_batch_resume(const nh_job *jobs, uint32_t n_jobs, void *d_workspace, uint64_t workspace_bytes,
                    const nh_config *cfg, nh_stats *stats, void *stream);

/* Event stream (sections "Sorting Events using the Water-Level Algorithm" and
 * "Reporting Coalescence Events Independently").  The stream of a simulation
 * lists every event that the samples' lineages go through, each once, sorted
 * by event time t and then origin: a dispersal from `origin` to `outcome`, or a
 * speciation (outcome NH_EVENT_SPECIATION), with t_prior the time of the
 * previous event of the first lineage to reach it (0 for a sample's first
 * event).  Lineages that share an event have coalesced: a coalescence is the
 * arrival of a lineage, at time t, at a location `loc` already holding another
 * sampled lineage, which arrived there at t_parent (0: it was sampled there);
 * they are listed sorted by t, loc, t_parent.  Every lineage ends in one
 * speciation or one coalescence, so the distinct samples of a job number its
 * speciation events plus its coalescences.  Locations are loc32 =
 * (y*W + x)*C_max + i as for the speciation-event reporter. */
#define NH_EVENT_SPECIATION 0xFFFFFFFFu
typedef struct {
    double t;
    double t_prior;
    uint32_t origin;
    uint32_t outcome;
} nh_event;

typedef struct {
    double t;
    double t_parent;
    uint32_t loc;
    uint32_t reserved;
} nh_coalescence;

/* Per-job outputs: d_events (device, events_cap records; may be NULL with
 * events_cap 0 to count only) and d_coalescences (device, room for the job's n
 * records, never more are needed).  n_events and n_coalescences are set by the
 * call; when n_events exceeds events_cap only the first events_cap events were
 * written, and a second call with room for them all gives the whole stream. */
typedef struct {
    nh_event *d_events;
    uint64_t events_cap;
    nh_coalescence *d_coalescences;
    uint64_t n_events;
    uint64_t n_coalescences;
} nh_stream_out;

/* The event stream of every job of the batch run that just finished in
 * d_workspace: jobs must be the run's own jobs (same scenarios, seeds and sample
 * buffers, all still alive and the samples unchanged, since the replay reads
 * them again), the run complete (not suspended) and free of errors; the
 * workspace is only read.  The library replays each lineage's
 * committed events on the GPU, sorts the records with device radix sorts and
 * reduces them to events and coalescences; it allocates its scratch
 * stream-ordered (about 100 bytes per committed event, below 2^31 of them) from
 * a library-owned pool per device, which keeps the memory of the largest call
 * reserved until the process ends, and returns it to that pool before
 * returning.  Synchronises `stream`.  Runs of the nh_server_*
 * engine have no such workspace.  NH_EINVAL if the workspace holds no finished,
 * error-free run of these jobs or the run committed 2^31 events or more;
 * NH_EDEVICE on a HIP error (an allocation that fails included). */
int nh_event_stream(const nh_job *jobs, uint32_t n_jobs, void *d_workspace, uint64_t workspace_bytes,
                    nh_stream_out *outs, void *stream);

/* One job with device buffers; allocates its own workspace (hipMallocAsync on
 * the stream).  Same semantics as nh_batch_run with one job. */
int nh_simulate_device(const nh_scenario *scenario, uint64_t seed, const uint64_t *d_sample_ids, uint64_t n,
                       uint64_t *d_species_out, uint64_t *d_richness_out, const nh_config *cfg, nh_stats *stats,
                       void *stream);

/* One job with device buffers, enqueue-only: every step of the run (set-up from
 * kernel arguments, lineage init, one persistent launch that runs all horizon
 * rounds on the device with a grid barrier between them, output) is enqueued
 * on `stream` and the call returns without waiting for the device (paper,
 * section "The Independent Algorithm on the GPU": the host<->device crossing
 * between steps is what the GPU path paid for).  The caller synchronises
 * `stream` (or records an event) before reading d_species_out (n u64) and
 * *d_richness_out (one u64, may be NULL).  The workspace is taken
 * stream-ordered from a library-owned pool of the current device and given
 * back stream-ordered; the persistent launch itself runs on a library stream
 * per device joined to `stream` by events, so persistent runs of one device
 * never overlap.  cfg may be NULL; cfg->launch must be NH_LAUNCH_PERSISTENT and
 * cfg->max_rounds 0.
 * Errors found before enqueueing are returned (NH_EINVAL: NULL buffers with
 * n > 0, n >= 2^31, a bad cfg; NH_EDEVICE: a HIP error).  Errors found on the
 * device cannot be returned: a sample id >= N, or a run that stops early (its
 * time limit cfg->timeout_s, a kernel error flag, a barrier wait beyond
 * cfg->barrier_wait_ms), set *d_richness_out to ~0 (UINT64_MAX) and leave
 * d_species_out unspecified. */
int nh_simulate_async(const nh_scenario *scenario, uint64_t seed, const uint64_t *d_sample_ids, uint64_t n,
                      uint64_t *d_species_out, uint64_t *d_richness_out, const nh_config *cfg, void *stream);

/* nh_simulate_async for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same enqueue-only run, outputs and failure reporting, with no
 * allocation at all.  The workspace is a 64 MiB device array inside the
 * library (one per device, reserved when the library's code is loaded on that
 * device and held until the process ends), which limits a run to the samples
 * whose nh_workspace_bytes(n, 1) fits 64 MiB (about 480,000; NH_EINVAL beyond,
 * with the limit in the message).  Every call on a device shares that array
 * and overwrites what the last call left there (each call initialises what it
 * reads), so calls on one device whose work can overlap (different streams
 * with no ordering between them) race; calls on one stream are ordered.  The
 * first call on a device looks the array's address up and creates the
 * library's per-device stream and events; later calls only enqueue. */
int nh_simulate_noalloc(const nh_scenario *scenario, uint64_t seed, const uint64_t *d_sample_ids, uint64_t n,
                        uint64_t *d_species_out, uint64_t *d_richness_out, const nh_config *cfg, void *stream);

/* One job with host buffers: uploads the samples, runs, downloads species
 * (n u64) and the richness.  Blocking; uses the default stream. */
int nh_simulate(const nh_scenario *scenario, uint64_t seed, const uint64_t *h_sample_ids, uint64_t n,
                uint64_t *h_species_out, uint64_t *h_richness_out, nh_stats *stats);

/* ------------------------------------------------------------------------
 * Continuous batching (a served request stream).  A server owns a resident
 * pool of lineage slots in HBM and runs the same round kernels as
 * nh_batch_run over whichever jobs are admitted: a job submitted while others
 * are running is admitted at the next round boundary as soon as a contiguous
 * range of lineage slots (its HBM footprint) and a job slot are free, its
 * lineages join the shared queue and hash table, and it completes on its own
 * when its last lineage retires.  Results are bitwise those of nh_simulate.
 * One thread drives a server; the caller keeps each job's buffers and
 * scenario alive until its completion is polled.
 * ------------------------------------------------------------------------ */
typedef struct nh_server nh_server;

typedef struct {
    uint64_t lineage_capacity; /* resident lineage slots (the HBM budget / nh_server_bytes per lineage) */
    uint32_t max_jobs;         /* job slots in flight */
    uint32_t lookahead;        /* pending jobs past the head that may be admitted first when the head
                                  does not fit (backfill); 0 = strict FIFO */
    nh_config cfg;             /* round-kernel tuning; cfg.rounds_per_graph rounds per launch */
    uint32_t tail_blocks;      /* tail lane: workgroups (4 waves each, one compute unit each; at most 64)
                                  that walk the last lineage of a solo job (cfg.solo_max > 0) whose nu is
                                  at most 1/16384 outside the rounds, to its end; 0 = none.  The lane's
                                  kernel runs on a stream of the server's own in launches of 8 ms (a walk
                                  still going then is queued again and continues in the next launch)
                                  while such lineages exist, and leaves when idle */
} nh_server_config;

typedef struct {
    uint64_t tag;       /* the caller's tag from nh_server_submit */
    int status;         /* NH_OK, or NH_EINVAL if a sample id was not below N */
    uint32_t rounds;    /* rounds the job took part in */
    uint64_t richness;
    uint64_t events;
    uint64_t lineages;
    uint64_t speciated;
    uint64_t merged;
} nh_completion;

/* Device bytes of a server's resident pool. */
uint64_t nh_server_bytes(uint64_t lineage_capacity, uint32_t max_jobs);

/* Allocates the pool on the current device and captures the round graph.
 * stream may be NULL (the server then creates its own non-blocking stream).  With a
 * tail lane the server always runs on streams of its own (a long-running lane kernel
 * must not share a hardware queue with the rounds); a given stream then only orders
 * submissions: each nh_server_submit makes the server wait for the work enqueued on it
 * so far.  Outputs are complete once the job's completion is polled.
 * Errors: NH_EINVAL for zero capacity or jobs; NH_ENOMEM; NH_EDEVICE. */
int nh_server_create(const nh_server_config *config, void *stream, nh_server **out);

/* Queues a job (device buffers as in nh_batch_run).  Never blocks.
 * Errors: NH_EINVAL if the job can never fit (n > lineage_capacity) or has
 * NULL buffers with n > 0. */
int nh_server_submit(nh_server *server, const nh_job *job, uint64_t tag);

/* Non-blocking step: collects finished jobs, admits queued jobs that fit,
 * and keeps round launches in flight while any job is active.  Reports the
 * jobs on the device and those still queued (either pointer may be NULL). */
int nh_server_progress(nh_server *server, uint32_t *active, uint32_t *pending);

/* Moves up to max finished jobs into out (oldest first); *n_out receives the count. */
int nh_server_poll(nh_server *server, nh_completion *out, uint32_t max, uint32_t *n_out);

/* Calls nh_server_progress until nothing is queued, active or resolving.
 * NH_ETIMEOUT after timeout_s seconds. */
int nh_server_drain(nh_server *server, double timeout_s);

/* Waits for the server's stream and frees the pool. */
void nh_server_destroy(nh_server *server);

/* Per-event latency of a lone lineage (the quantity that bounds a run's last
 * rounds, when a few lineages remain and each event waits on the previous one:
 * chapter "The Declaration of Independence", each lineage's events form a
 * sequential chain).  One group of 8 lanes on an otherwise idle device walks
 * `steps` events of the scenario from sample 0's location with the same group
 * step as the round kernel (table in LDS where the round kernel would stage
 * it); *ns_per_event receives the stream time per event.  The walk ignores
 * speciation.  Synchronises `stream`.  NH_EINVAL for a NULL argument or steps
 * = 0; NH_EDEVICE on a HIP error. */
int nh_measure_event_latency(const nh_scenario *scenario, uint64_t seed, uint32_t steps, double *ns_per_event,
                             void *stream);

/* Device evaluation of the path's primitives on given inputs, for unit tests
 * of the kernels' building blocks against a host implementation (chapter "The
 * Declaration of Independence": priming, exponential waiting times, the event
 * summary).  For item i < n (device arrays; each pair may be NULL):
 *   d_ctr[4i..4i+3] -> d_philox_out[4i..4i+3]: the Philox4x32-10 block of that
 *     counter under key (seed low word, seed high word);
 *   d_r[i] -> d_log_out[i]: log(((r >> 11) + 1) 2^-53), the logarithm the
 *     event-time search applies to a draw;
 *   (d_loc[i], d_t[i]) -> d_next_out[i]: the next event time after t at loc
 *     (one-lane search); d_next_group_out[i]: the same by the 8-lane group
 *     search; d_outcome_out[i]: the outcome of an event at (loc, t), the new
 *     location or NH_EVENT_SPECIATION; (d_step_loc_out[i], d_step_t_out[i]):
 *     one group step from (loc, t), the new location and its next event time,
 *     or (NH_EVENT_SPECIATION, t).
 * Locations are loc32 of the scenario; an item whose location is no slot of
 * the scenario, or whose time is not finite, non-negative and below 2^40, gets
 * NaN or 0xFFFFFFFF outputs.  use_lds stages a small shared table in LDS as the
 * single-job round kernel does.  Synchronises `stream`.  NH_EINVAL for a NULL
 * scenario or io, unpaired arrays, or event outputs without d_loc and d_t;
 * NH_EDEVICE on a HIP error or a search that ran away. */
typedef struct {
    const uint32_t *d_ctr;
    uint32_t *d_philox_out;
    const uint64_t *d_r;
    double *d_log_out;
    const uint32_t *d_loc;
    const double *d_t;
    double *d_next_out;
    double *d_next_group_out;
    uint32_t *d_outcome_out;
    uint32_t *d_step_loc_out;
    double *d_step_t_out;
} nh_primitive_io;

int nh_eval_primitives(const nh_scenario *scenario, uint64_t seed, uint64_t n, const nh_primitive_io *io,
                       uint32_t use_lds, void *stream);

/* Message of the last failure on the calling thread ("" if none). */
const char *nh_last_error(void);

/* Library version string. */
const char *nh_version(void);

/* sizeof the public struct of that name (e.g. "nh_config"), 0 for an unknown name: for
 * bindings to check that their copies of these layouts match the library's. */
uint64_t nh_struct_bytes(const char *name);

/* Measurement helpers, not part of the method; callers are benchmarks that
 * price the hot path against what the chip sustains.
 * nh_measure_mix_peak: with 8 workgroups of 256 lanes per compute unit, every
 * lane evaluates 3 Philox4x32-10 blocks and 2 exponential-draw logarithms per
 * iteration (about the event path's mix) from registers; *lane_ops_per_s gets
 * the rate in the algorithmic units the path is counted in (100 per Philox
 * block, 43 per draw).  Allocates a small sink buffer on the stream; blocks.
 * nh_measure_gather: random 16-byte gathers from d_table (device memory of
 * table_bytes >= 16 KiB, contents irrelevant) by the same number of lanes, 256
 * per lane; *bytes_per_s gets the useful bytes (16 per gather) per second.
 * Both return NH_EINVAL on NULL arguments, NH_EDEVICE on a HIP error. */
int nh_measure_mix_peak(double *lane_ops_per_s, void *stream);
int nh_measure_gather(const void *d_table, uint64_t table_bytes, double *bytes_per_s, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* NECSIM_HIP_H */
