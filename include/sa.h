/*
 * sa.h -- C ABI of libsa.so: direct simulated annealing of quadratic and higher-order
 * unconstrained integer optimisation problems (QUIO / HUIO) on AMD Instinct MI355X (gfx950).
 *
 * Method: K. Suzuki, "Simulated Annealing for Quadratic and Higher-Order Unconstrained Integer
 * Optimization", arXiv:2511.17245.  The library runs the paper's single-variable update sweep
 * (Sec. 3.1) with the energy difference of Sec. 3.2 and the three transition rules of Sec. 3.3
 * (Metropolis, heat bath, optimal-transition Metropolis; the heat bath also with the closed-form
 * draw of Sec. 3.3.2 for linear energy differences) as HIP kernels.  A replica (read) is
 * updated by one 64-lane wavefront, or by a team of up to 16 wavefronts that update variables
 * sharing no term at the same time (the result is the sequential sweep's either way).
 *
 * Conventions shared by every entry point
 *  - All functions return an int32_t status (SA_OK or a negative SA_E* code).  On failure no
 *    output is written and sa_last_error() describes the cause.  No C++ exception crosses the ABI.
 *  - Input arrays are borrowed for the duration of the call and copied; no pointer is retained,
 *    except by the plan, batch and server objects, which copy what they need at creation.
 *  - Output arrays are allocated by the caller.
 *  - Every argument check (shapes, bounds, the int64 bound, rule support) happens on the host
 *    before any device work is queued.
 *  - The GPU work runs on the current HIP device of the calling thread.
 *  - Entry points are safe to call from several threads; calls that share one plan, batch or
 *    server object must be serialised by the caller (except the server's submit/poll/cancel).
 *
 * Results contract (what "the same result" means across launches, batches and the server):
 * read r of instance id I with seed K follows the Philox4x32-10 stream with counter
 * (variable k, sweep s, read r, I) and key (K mod 2^32, K / 2^32); the initial state uses sweep id
 * 0xFFFFFFFF.  Energies are exact int64; FP64 is used only for acceptance and heat-bath weights.
 */
#ifndef SA_H
#define SA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------------------------- */
#define SA_OK 0
#define SA_EINVAL (-1)         /* malformed argument (shape, index, bound, schedule value) */
#define SA_ERANGE (-2)         /* sum_t |J_t| prod_i max(|l_i|,|u_i|)^e >= 2^62: int64 not exact */
#define SA_EUNSUPPORTED (-3)   /* e.g. optimal-transition rule with an exponent above 4 */
#define SA_ENOMEM (-4)         /* host or device allocation failed, or a server budget is exceeded */
#define SA_EDEVICE (-5)        /* a HIP call failed (no device, launch failure, fault) */
#define SA_EBUSY (-6)          /* server: result not ready yet */
#define SA_ECANCELED (-7)      /* server: the request was cancelled */

/* ---- transition rules (Sec. 3.3) ---------------------------------------------------------- */
#define SA_METROPOLIS 0        /* uniform nonzero change, accept min[1, exp(-dE/T)]   (Sec. 3.3.1) */
#define SA_HEAT_BATH 1         /* draw the new value with probability exp(-dE/T)/sum  (Sec. 3.3.2) */
#define SA_OPT_METROPOLIS 2    /* with probability r = s/(S-1) the optimal transition: the value
                                  of smallest dE over the whole range (the unchanged value, dE = 0,
                                  included; ties to the lowest value), else the Metropolis
                                  proposal; Metropolis acceptance                      (Sec. 3.3.3) */
#define SA_HEAT_BATH_CLOSED 3  /* heat bath; a variable whose dE is linear in its new value (no
                                  exponent above one) takes the O(1) inverse-transform draw of
                                  Sec. 3.3.2, the others the enumeration of SA_HEAT_BATH */

/* ---- problem description (Sec. 2) ----------------------------------------------------------
 * E(z) = sum_t coef[t] * prod_{f = term_ptr[t]}^{term_ptr[t+1]-1} z[factor_var[f]].
 * A power z_i^m is written as index i repeated m times.  Terms with the same multiset of indices
 * are merged and zero coefficients dropped (Sec. 2: unordered index tuples).  Every term has
 * degree >= 1 (no constant terms). */
typedef struct {
    int32_t n_vars;             /* N >= 1 */
    int64_t n_terms;            /* >= 0 */
    const int64_t *term_ptr;    /* n_terms + 1 offsets, term_ptr[0] = 0, strictly increasing */
    const int32_t *factor_var;  /* term_ptr[n_terms] indices in [0, N) */
    const int64_t *coef;        /* n_terms integer coefficients J_t */
} sa_instance;

/* Integer box l_i <= z_i <= u_i (Sec. 2), with u_i - l_i <= 2^31 - 2.  l_i = u_i fixes z_i. */
typedef struct {
    const int32_t *lower;       /* N values */
    const int32_t *upper;       /* N values */
} sa_bounds;

/* Inverse temperatures beta_s = 1/T_s, one per sweep.  beta == NULL selects the automatic
 * schedule: T_init and T_final from Sec. 3.4 (a = 1/2, b = 0.001) with the geometric cooling of
 * Sec. 3.1.  Every beta must be finite and >= 0. */
typedef struct {
    int32_t n_sweeps;           /* S >= 1 */
    const double *beta;         /* S values (host memory), or NULL */
} sa_schedule;

/* ---- one-shot annealing ---------------------------------------------------------------------
 * Runs n_reads independent chains of S sweeps from random initial states and writes the final
 * states and their energies (the tracked energy, equal to E(final state)).
 *   out_states   host int32[n_reads * N], row-major (read, variable)
 *   out_energies host int64[n_reads] */
int32_t sa_anneal(const sa_instance *inst, const sa_bounds *bounds, const sa_schedule *sched,
                  int32_t rule, int32_t n_reads, uint64_t seed, int32_t *out_states,
                  int64_t *out_energies);

/* Options of the extended entry points.  Initialise with sa_opts_default(). */
typedef struct {
    uint32_t instance_id;       /* fourth Philox counter word (default 0) */
    void *hip_stream;           /* hipStream_t to queue the work on (NULL: the null stream) */
    int32_t device_buffers;     /* 1: out_states / out_energies / init_states are device pointers
                                   on the current device; the call then returns once the work is
                                   queued (no host synchronisation).  0: host pointers (default) */
    int32_t sweep_begin;        /* run sweeps [sweep_begin, sweep_end) of the S-sweep schedule */
    int32_t sweep_end;          /* <= 0 means S */
    const int32_t *init_states; /* n_reads * N start states (resume), or NULL for random ones */
    double otm_r;               /* < 0: r = s/(S-1) as in Sec. 3.3.3 (default); else a fixed r */
    int32_t waves_per_replica;  /* 0: automatic.  G > 1 lets G wavefronts of one replica update G
                                   consecutive variables that share no term at the same time (the
                                   result is identical to the sequential sweep); 1, 2, 4, 8 or 16 */
    int32_t otm_enum_max;       /* optimal transition: ranges of at most this many values (and
                                   of at most 64) take the argmin by enumeration, wider ones from
                                   the sign changes of the forward differences of the degree-<=4
                                   energy difference (exact: the same value); 0: 2048 */
    uint64_t *trace_hashes;     /* NULL: no tracing (default).  Otherwise n_reads x (sweep_end -
                                   sweep_begin) words, row-major (read, sweep), host or device memory
                                   as device_buffers says: the hash of each read's state after each
                                   sweep of the run, sum_k mix(k * 2^32 + (uint32_t)z_k) modulo 2^64
                                   with mix the 64-bit finaliser of SplitMix64.  Two runs of a chain
                                   part at the first sweep whose hashes differ.  Plain launches only
                                   (batches and the server do not trace). */
    int32_t lanes_per_update;   /* heat bath: lanes that carry one update.  0: automatic.  64: one
                                   wavefront per update (the candidate values split over its lanes,
                                   the waves of a replica over schedule windows, as waves_per_replica
                                   says).  4: one quad of lanes per update, the 16 quads of each of a
                                   workgroup's 8 waves over the dependency levels of the sweep
                                   (sparse problems, exponents <= 2, ranges of at most 128 values,
                                   waves_per_replica 0; SA_EINVAL otherwise).  Both follow the
                                   sequential sweep; they differ only in the order in which heat-bath
                                   weights are added (a quad adds them in value order). */
} sa_opts;

void sa_opts_default(sa_opts *opts);

/* sa_anneal with options.  With sweep_begin/sweep_end and init_states a run can be split into
 * pieces that reproduce the uninterrupted run exactly (the draws are counter-based). */
int32_t sa_anneal_ex(const sa_instance *inst, const sa_bounds *bounds, const sa_schedule *sched,
                     int32_t rule, int32_t n_reads, uint64_t seed, int32_t *out_states,
                     int64_t *out_energies, const sa_opts *opts);

/* ---- the same run without device allocations -------------------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): sa_anneal_ex with device outputs, whose staging (the
 * packed instance, the inverse temperatures and the sweep schedule) lives in a static device area
 * of 32 MiB per GPU, set up on the first call on each device and held until the process ends.
 * The call allocates no device memory (no hipMalloc / hipFree).  Results are those of
 * sa_anneal_ex with the same arguments.
 *   opts            required, with device_buffers = 1: out_states, out_energies, init_states and
 *                   trace_hashes are device pointers on the current device
 *   return          SA_OK once the work is queued on opts->hip_stream (the call waits only for
 *                   its own staging copy); SA_ENOMEM if the problem needs more than the 32 MiB
 *                   area (the message states the bytes needed); the other codes as sa_anneal_ex.
 * Every call on a GPU uses the same area and overwrites it: calls whose work may overlap on one
 * GPU (different streams or threads without ordering between them) race.  Calls queued on one
 * stream are ordered and safe. */
int32_t sa_anneal_noalloc(const sa_instance *inst, const sa_bounds *bounds, const sa_schedule *sched,
                          int32_t rule, int32_t n_reads, uint64_t seed, int32_t *out_states,
                          int64_t *out_energies, const sa_opts *opts);

/* ---- plans: a canonical instance packed once in device memory, run many times -------------- */
typedef struct sa_plan sa_plan;

/* Canonicalises, checks and uploads the instance for `rule` on the current device. */
int32_t sa_plan_create(const sa_instance *inst, const sa_bounds *bounds, int32_t rule,
                       sa_plan **out);
/* Same contract as sa_anneal_ex on the plan's instance and rule. */
int32_t sa_plan_run(sa_plan *plan, const sa_schedule *sched, int32_t n_reads, uint64_t seed,
                    int32_t *out_states, int64_t *out_energies, const sa_opts *opts);
void sa_plan_destroy(sa_plan *plan);

/* Facts about a plan, for reports. */
typedef struct {
    int32_t n_vars;
    int64_t n_terms;            /* canonical terms */
    int64_t n_incidences;       /* sum_k |terms containing z_k| */
    int64_t n_factor_slots;     /* other-factor indices stored for the incidences */
    int32_t max_exponent;
    int32_t max_width;          /* max_k (u_k - l_k + 1) */
    int64_t device_bytes;       /* device memory held by the plan */
    int32_t coef_bits;          /* 32 or 64: width of the stored coefficients */
    int32_t arith_bits;         /* 32 or 64: integer width of energy differences in the kernel */
    int32_t dense;              /* 1: stored as a dense coupling matrix (QUIO with >= 25% of all
                                   pairs present); 0: variable-major incidence records */
} sa_plan_info;
int32_t sa_plan_get_info(const sa_plan *plan, sa_plan_info *info);

/* Launch geometry the last sa_plan_run used (for profiling reports). */
typedef struct {
    int32_t waves_per_group;    /* replicas per workgroup */
    int32_t groups;             /* workgroups launched */
    int32_t lds_bytes;          /* dynamic LDS per workgroup */
    int32_t state_in_lds;       /* 1: replica states live in LDS, 0: in device memory */
    int32_t kernel_variant;     /* internal id of the instantiated kernel */
    int32_t waves_per_replica;  /* G: wavefronts cooperating on one replica */
    int32_t n_windows;          /* windows per sweep in the schedule (N for G = 1 without fixed vars) */
    int32_t lanes_per_update;   /* 64, or 4 for the quad kernel */
    int32_t n_levels;           /* quad kernel: dependency levels per sweep (0 otherwise) */
} sa_launch_info;
int32_t sa_plan_last_launch(const sa_plan *plan, sa_launch_info *info);

/* ---- batches: many instances annealed by one persistent launch ------------------------------
 * Every problem keeps its own rule, schedule, read count, seed and instance id, and its results
 * are identical to sa_anneal_ex of that problem alone (same Philox counters, exact arithmetic).
 * One kernel launch runs all (problem, read) replicas: each workgroup of 8 wavefronts takes the
 * next task from a device counter, longest first; a task is 8/G consecutive reads of one problem,
 * each annealed by G cooperating wavefronts (G = 1, 2, 4 or 8 per problem, larger for the
 * problems on the critical path) with its state in LDS.  Every problem's N must fit LDS
 * (N <= 40960 on MI355X); otherwise creation fails with SA_EUNSUPPORTED. */
typedef struct {
    sa_instance inst;
    sa_bounds bounds;
    sa_schedule sched;          /* beta == NULL: automatic schedule of this problem */
    int32_t rule;
    int32_t n_reads;
    uint64_t seed;
    uint32_t instance_id;
} sa_problem;

typedef struct {
    int32_t *states;            /* host int32[n_reads * N] (caller-allocated) */
    int64_t *energies;          /* host int64[n_reads] */
    int32_t status;             /* written by sa_batch_results / sa_anneal_batch */
} sa_result;

typedef struct {
    int32_t autotune;           /* 1: time candidate launch geometries once and keep the fastest
                                   (cached per batch shape within the process) */
    int32_t use_graph;          /* 1: the launch is captured once into a HIP graph and replayed */
    void *hip_stream;           /* stream of sa_batch_run (NULL: the batch creates its own) */
    int32_t waves_per_group;    /* 0 or 8 (the batch kernel's workgroup size in wavefronts) */
    int32_t groups;             /* 0: automatic / tuned; else the persistent workgroup count */
} sa_batch_opts;

typedef struct sa_batch sa_batch;

/* Validates, canonicalises and uploads every problem, then (optionally) tunes and captures the
 * launch.  Problems are copied; the caller's arrays may be freed after the call. */
int32_t sa_batch_create(const sa_problem *problems, int32_t n_problems, const sa_batch_opts *opts,
                        sa_batch **out);
/* Queues one complete annealing of every problem on the batch's stream (asynchronous). */
int32_t sa_batch_run(sa_batch *batch);
/* Waits for the queued work of the batch. */
int32_t sa_batch_wait(sa_batch *batch);
/* Waits, then copies every problem's final states and energies to results[i]. */
int32_t sa_batch_results(sa_batch *batch, sa_result *results);
typedef struct {
    int32_t n_problems;
    int64_t n_tasks;            /* replicas */
    int64_t total_updates;      /* sum over problems of n_reads * n_sweeps * N */
    int32_t waves_per_group;
    int32_t groups;
    int32_t slot_bytes;         /* dynamic LDS per workgroup */
    int32_t kernel_maxe;        /* exponent class of the batch kernel */
    int32_t kernel_bits;        /* 32 or 64: integer width of energy differences */
    int32_t state_bits;         /* 16 or 32: width of the states held in LDS */
    int32_t graph;              /* 1 if replayed from a HIP graph */
    int32_t max_team;           /* largest number of wavefronts cooperating on one replica */
    double policy;              /* team-size policy strength in use (0: one wavefront per replica) */
    double tune_ms;             /* time spent in tuning trials */
} sa_batch_info;
int32_t sa_batch_get_info(const sa_batch *batch, sa_batch_info *info);
void sa_batch_destroy(sa_batch *batch);

/* One-shot form: create, run, copy the results, destroy. */
int32_t sa_anneal_batch(const sa_problem *problems, int32_t n_problems, sa_result *results,
                        const sa_batch_opts *opts);

/* ---- serving: continuous batching ----------------------------------------------------------
 * A server owns one device (the caller's current device at creation), a stream, host threads that
 * canonicalise and upload arriving requests, and a scheduler thread.  The scheduler admits
 * prepared requests in arrival order while a slot is free and their device footprint (plan,
 * states, schedule) fits the memory budget, and advances all admitted requests together, one
 * chunk of sweeps per batched launch, with their states kept on the device in between.  A
 * request's results are identical to sa_anneal_ex of the same problem alone.  submit, poll, wait
 * and cancel may be called from any thread. */
typedef struct sa_server sa_server;

typedef struct {
    size_t mem_budget_bytes;    /* device bytes for admitted requests (0: 16 GiB) */
    int32_t max_slots;          /* requests on the device at once (0: 256) */
    int32_t chunk_sweeps;       /* sweeps per chunk launch for a request of median cost (0: 50);
                                   cheaper requests run more sweeps per chunk, dearer ones fewer
                                   (at least one), so that every chunk is about equally long */
    int32_t prep_threads;       /* host threads preparing requests (0: 4) */
} sa_server_opts;

typedef struct {
    double t_submit, t_admit, t_done;  /* seconds since the server was created (steady clock) */
    uint64_t updates;                   /* n_reads * n_sweeps * N */
    int32_t status;                     /* SA_EBUSY until done, then the request's status */
} sa_timing;

int32_t sa_server_create(const sa_server_opts *opts, sa_server **out);
/* Copies the problem and queues it.  result's buffers (host, caller-owned) must stay valid until
 * the request is done; they are written at completion.  SA_ENOMEM at once if the states alone
 * exceed the budget; a request whose full footprint exceeds it completes with SA_ENOMEM. */
int32_t sa_server_submit(sa_server *server, const sa_problem *problem, sa_result *result,
                         uint64_t *ticket);
/* Queues a run of an existing plan (shared, not copied: keep it alive until the request is done). */
int32_t sa_server_submit_plan(sa_server *server, sa_plan *plan, const sa_schedule *sched,
                              int32_t n_reads, uint64_t seed, uint32_t instance_id,
                              sa_result *result, uint64_t *ticket);
/* done = 1 once the request finished (timing->status then holds its status). */
int32_t sa_server_poll(sa_server *server, uint64_t ticket, int32_t *done, sa_timing *timing);
/* Blocks until the request is done; returns its status. */
int32_t sa_server_wait(sa_server *server, uint64_t ticket, sa_timing *timing);
/* Cancels a request: it completes with SA_ECANCELED at its next hand-over (before preparation,
 * at admission, or at the next chunk boundary); other requests are unaffected. */
int32_t sa_server_cancel(sa_server *server, uint64_t ticket);
typedef struct {
    int64_t submitted, completed, canceled, failed;
    int64_t active, queued, chunks, updates;
    size_t mem_in_use;          /* device bytes held: admitted requests and cached plans */
    double elapsed_s;
    int64_t plans_reused;       /* requests served by a plan cached from an earlier request with the
                                   same instance, bounds and rule (content hash) */
} sa_server_stats;
int32_t sa_server_get_stats(sa_server *server, sa_server_stats *stats);
/* Cancels what has not finished, joins the threads and frees everything. */
void sa_server_destroy(sa_server *server);

/* ---- utilities -------------------------------------------------------------------------------- */
/* The automatic schedule of Sec. 3.4 (host arithmetic): beta_out[0..n_sweeps-1]. */
int32_t sa_auto_schedule(const sa_instance *inst, const sa_bounds *bounds, int32_t n_sweeps,
                         double *beta_out);

/* Exact energies of n_states states (host int32[n_states * N]) computed on the GPU. */
int32_t sa_energy(const sa_instance *inst, const sa_bounds *bounds, int32_t n_states,
                  const int32_t *states, int64_t *out_energies);

/* Thread-local description of the last failure on this thread ("" if none). */
const char *sa_last_error(void);

/* Library version: major * 10000 + minor * 100 + patch. */
int32_t sa_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SA_H */
