/*
 * lik.h -- C ABI of the MI355X particle-filter likelihood library (liblik.so).
 *
 * The library evaluates, for a batch of rate vectors theta, the bootstrap
 * particle-filter estimate of log p(y | theta) for a stochastic mass-action
 * reaction network observed through noisy measurements (Mikelson & Khammash,
 * arXiv 1606.08281):
 *   - network: U species, R reactions, reaction r consumes p_ru and produces
 *     q_ru molecules of species u (Sec. "Chemical Reaction Networks");
 *   - observations: Y ~ p(. | X, theta) at T time points of M trajectories
 *     (Sec. "General Task");
 *   - likelihood: product over trajectories and time points, each factor the
 *     mean particle weight (Supplementary I, the recursion and the Algorithm
 *     "Likelihood Approximation using particle filter");
 *   - propagation: Gillespie's direct-method SSA between observation times.
 *
 * Conventions fixed by this library where the paper is silent:
 *   - propensity a_r = c_r * prod_u C(x_u, p_ru) (Gillespie's combinatorial
 *     mass-action form); theta[r] = c_r, so the parameter dimension is R;
 *   - resampling before every propagation step after the first, systematic,
 *     with integer (2^-32 fixed-point) weights;
 *   - random numbers from Philox4x32-10 keyed by the seed, with counters made
 *     of (event index, particle slot, (trajectory << 16) | interval,
 *     (theta id << 2) | purpose); results depend only on the inputs, the seed
 *     and the theta ids, never on batch composition or launch shape;
 *   - log-likelihoods are natural logs in binary64; -inf is a valid result
 *     (every particle has zero density under the noise model).
 *
 * Errors: every entry point returns LIK_OK (0) or a negative LIK_E* code and
 * then lik_last_error() (thread-local) describes the failure.  Per-theta
 * outcomes are not call errors: they are reported in status_out.
 *
 * Ownership: the caller owns every buffer it passes.  Entry points copy what
 * they keep (network tables).  Handles are immutable after creation and may
 * be shared by threads.
 */
#ifndef LIK_H
#define LIK_H

#ifndef __HIPCC_RTC__
#include <stddef.h>
#include <stdint.h>
#endif

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
#define LIK_OK 0
#define LIK_EINVAL (-1)
#define LIK_ENOMEM (-2)
#define LIK_EDEVICE (-3)
#define LIK_EUNSUPPORTED (-4)

/* per-theta status (status_out) */
#define LIK_STATUS_OK 0
#define LIK_STATUS_EVENT_CAP 1      /* a particle needed more events in one interval than the cap */
#define LIK_STATUS_COUNT_OVERFLOW 2 /* a count exceeded 2^30 at the end of an interval */
#define LIK_STATUS_BAD_THETA 3      /* a rate was negative, infinite or NaN, or (with
                                       LIK_FP32_MIXED) beyond the binary32 range */
#define LIK_STATUS_SCHEDULER 4      /* the flow schedule saw no work item finish for a
                                       minute and gave up (an internal fault; the limit,
                                       in microseconds, can be lowered through the
                                       environment variable LIK_FLOW_STALL_US for tests) */
#define LIK_STATUS_CANCELLED 5      /* server: the request was cancelled (lik_server_cancel) */
#define LIK_STATUS_TIMED_OUT 6      /* server: the request's own time limit passed first */
#define LIK_STATUS_STEP_LIMIT 7     /* deterministic model: the solver's step limit was reached */
#define LIK_STATUS_NONFINITE 8      /* deterministic model: a state or observation mean not finite */

/* observation noise models (Sec. "General Task": Y ~ p(. | X, theta)) */
#define LIK_OBS_GAUSSIAN 0  /* y = x_s + N(0, sigma^2) per observed species s */
#define LIK_OBS_LOGNORMAL 1 /* log y = log x_s + N(0, sigma^2); y > 0 required */
#define LIK_OBS_FLUORESCENCE 2 /* y = N(gain x_s, sigma^2 x_s) + B, B ~ N(bg_mean, bg_sd^2):
                                  each molecule adds an independent normal signal,
                                  background added (Supplementary "LacGfp example") */

/* arithmetic of the SSA step */
#define LIK_FP64 0       /* binary64 propensities, event times and clock */
#define LIK_FP32_MIXED 1 /* binary32 propensities / event times (two events per Philox
                            block), binary64 clock and weights */

/* propagation kernel variants (lik_eval_opts.kernel) */
#define LIK_KERNEL_AUTO 0        /* specialised when the batch amortises compiling it */
#define LIK_KERNEL_GENERIC 1     /* reaction tables read at run time */
#define LIK_KERNEL_SPECIALIZED 2 /* reaction tables compiled in (hipRTC, cached on disk) */

/* limits */
#define LIK_MAX_SPECIES 32
#define LIK_MAX_REACTIONS 64
#define LIK_MAX_OBSERVED 8
#define LIK_MAX_PARTICLES 4096
#define LIK_MAX_OBS_PER_TRAJ 65535
#define LIK_MAX_TRAJ 65535
#define LIK_MAX_EVENT_CAP 134217728ull /* 2^27 events per particle per interval */
#define LIK_DEFAULT_EVENT_CAP 100000000ull

typedef struct lik_network *lik_network_t;

/*
 * lik_create_network -- validate and copy a reaction network (Sec. "Chemical
 * Reaction Networks").
 *   n_species U in [1, LIK_MAX_SPECIES], n_reactions R in [1, LIK_MAX_REACTIONS].
 *   reactant_orders [R*U], row-major by reaction: p_ru >= 0, sum_u p_ru <= 2
 *     (mass action of order 0, 1 or 2).
 *   stoichiometry [R*U], row-major by reaction: net change nu_ru = q_ru - p_ru,
 *     with nu_ru >= -p_ru (no reaction consumes what it does not use) and
 *     |nu_ru| <= 7.
 *   out: receives the handle.  Host pointers; the arrays are copied.
 * Returns LIK_EINVAL on any violated rule, LIK_ENOMEM on allocation failure.
 */
int lik_create_network(int32_t n_species, int32_t n_reactions, const int32_t *reactant_orders,
                       const int32_t *stoichiometry, lik_network_t *out);

/*
 * Work partitioning of the propagation kernels (never changes a result).
 * A wavefront runs a pool of G * 64 particles of one filter and hands a lane
 * the next particle of its pool as soon as the lane's particle reaches the
 * observation time.  Per filter and interval, G = clamp(pool_events / e,
 * pool_min, pool_max), where e is the expected number of events per particle
 * (the total propensity of the particles' starting states times the
 * interval's length; in the first interval the total propensity at x0), and
 * pool_first when there is no estimate.  G is at most
 * H / 64 rounded up, and at most 1536 / (64 U + 32) (the pool's starting
 * counts and its order are staged in 6 KiB of LDS).  Idle lanes take new
 * particles once refill_min of them are idle; a pool's particles are taken
 * heaviest first (by the total propensity of their starting counts).
 */
typedef struct lik_tuning {
    int32_t pool_min;      /* >= 1 */
    int32_t pool_max;      /* >= pool_min, <= 64 */
    uint32_t pool_events;  /* target events per lane per work item */
    int32_t pool_first;    /* >= 1, <= 64 */
    int32_t refill_min;    /* idle lanes of a wavefront that trigger a refill, 1..64 */
    int32_t priority;      /* 1: raise the wavefront priority of the filters whose
                              particles are expected to need the most events; 0: off */
    int32_t items_per_cu;  /* pools grow only while an iteration keeps at least this
                              many work items per compute unit (>= 0; 0: always) */
    int32_t persistent;    /* 1: networks of at most 16 reactions run a persistent
                              kernel whose lanes move on to the next work item when
                              their pool runs out; 0: one wavefront per work item */
    int32_t schedule;      /* batch evaluation: 0: one launch sequence per observation
                              interval, every filter advancing together; 1: one
                              persistent launch for all intervals, each filter going on
                              to its next interval as soon as its own particles are
                              weighed (the server always advances its slots together;
                              persistent is ignored under 1; takes 0 where its kernel
                              keeps fewer than 4 wavefronts per SIMD resident (large
                              networks) and for batches of 2^26 or more filter-intervals
                              x groups of 64 particles) */
    uint32_t urgent_events; /* schedule 1: a filter whose intervals left times the expected
                               events per lane of its items reach this (one on the critical
                               path) queues its items at once; the others wait while the
                               queue is long, so urgent items are taken soon;
                               0: first come, first served */
    uint32_t backlog_per_cu; /* schedule 1: the queue counts as long from this many waiting
                                work items per compute unit (>= 1) */
} lik_tuning;

/* Sets (NULL: restores the defaults {1, 6, 1536, 1, 1, 0, 160, 0, 1, 16000, 60}) / reads a
 * network's tuning for lik_eval_batch, lik_eval_batch_device and
 * lik_eval_requests; LIK_EINVAL outside the bounds above.  Not to be called
 * while an evaluation on this network is being enqueued on another thread.
 * A server ignores the networks' tunings: it partitions every iteration by
 * lik_server_opts.tuning (NULL: the defaults). */
int lik_network_set_tuning(lik_network_t net, const lik_tuning *tuning);
int lik_network_get_tuning(lik_network_t net, lik_tuning *out);

/* Releases a handle.  The caller guarantees no evaluation using it is in flight. */
int lik_destroy_network(lik_network_t net);

/*
 * lik_network_precompile -- compile the network-specialised propagation
 * kernel for `precision` (LIK_FP64 / LIK_FP32_MIXED) into the on-disk kernel
 * cache ($LIK_KERNEL_CACHE, else $HOME/.cache/lik-kernels) so that the first
 * evaluation does not pay for it.  Needs no GPU.  Returns LIK_EDEVICE with a
 * compiler log in lik_last_error() if compilation fails.
 */
int lik_network_precompile(lik_network_t net, int32_t precision);

/*
 * Observation model (Sec. "General Task": Y ~ p(. | X, theta)): kind, observed
 * species (in order) and noise parameters.
 *   LIK_OBS_GAUSSIAN, LIK_OBS_LOGNORMAL: sigma > 0; gain, bg_mean, bg_sd unused.
 *   LIK_OBS_FLUORESCENCE: the density of y is normal with mean gain * x + bg_mean
 *     and variance sigma^2 * x + bg_sd^2 (x: the observed count), so a count of
 *     zero still has density through the background.  gain, bg_mean finite;
 *     sigma >= 0 finite; bg_sd > 0 finite.
 */
typedef struct lik_obs_model {
    int32_t kind;
    int32_t n_observed;                 /* P in [1, LIK_MAX_OBSERVED] */
    int32_t species[LIK_MAX_OBSERVED];  /* species index of observed component k */
    double sigma;
    double gain, bg_mean, bg_sd;        /* LIK_OBS_FLUORESCENCE only */
} lik_obs_model;

/*
 * Observed trajectories (Sec. "General Task": y_t^m for m < M, t < T_m).
 * Trajectory m owns observations obs_offsets[m] .. obs_offsets[m+1]-1.
 *   obs_offsets [M+1] int32, non-decreasing, obs_offsets[0] = 0, T_m >= 1;
 *   t_obs [total] binary64 observation times, strictly increasing within a
 *     trajectory and > t0[m];
 *   y [total * P] binary64 observed values, component k of observation n at
 *     y[n*P + k];
 *   t0 [M] start times; x0 [M*U] int32 known initial counts (>= 0, <= 2^30).
 *   x0_hi [M*U] int32 or NULL.  NULL: every particle starts at x0.  Otherwise
 *     the initial counts are random (Supplementary I: the filter starts from
 *     H draws of the initial distribution): particle j of trajectory m starts
 *     with species u drawn uniformly from the integers x0 .. x0_hi
 *     (x0 <= x0_hi <= 2^30), independently per species and particle, from
 *     Philox block (u / 4, j, m << 16, theta id << 2 | 2), word u % 4:
 *     x0 + floor(word * (x0_hi - x0 + 1) / 2^32).
 * Whether these are host or device pointers is fixed by the entry point.
 */
typedef struct lik_data {
    int32_t n_traj;
    const int32_t *obs_offsets;
    const double *t_obs;
    const double *y;
    const double *t0;
    const int32_t *x0;
    const int32_t *x0_hi;
} lik_data;

/* Evaluation options; a NULL pointer means all defaults. */
typedef struct lik_eval_opts {
    int32_t precision;          /* LIK_FP64 (default) or LIK_FP32_MIXED */
    int32_t kernel;             /* LIK_KERNEL_*; every variant gives identical results */
    uint64_t event_cap;         /* per particle per interval; 0 = LIK_DEFAULT_EVENT_CAP */
    const uint32_t *theta_ids;  /* [n_theta] random-stream ids (< 2^30), NULL = 0..n_theta-1;
                                   same memory space as theta */
    int32_t flags;              /* LIK_FLAG_* */
    int32_t reserved;           /* must be 0 */
} lik_eval_opts;

/* lik_eval_batch_device: capture the whole launch sequence into a HIP graph
 * the first time a given set of buffers, sizes and options is seen (per
 * network), and replay it on later calls with only the seed updated.  The
 * caller must not free or reuse any of those buffers for other shapes while
 * the network lives.  Results are identical to eager launches. */
#define LIK_FLAG_GRAPH 1

/* Optional per-filter outputs (filter f = theta index i * M + trajectory m);
 * any pointer may be NULL.  Same memory space as loglik_out. */
typedef struct lik_aux {
    uint64_t *filter_events;    /* [n_theta*M] SSA events applied */
    double *filter_loglik;      /* [n_theta*M] log-likelihood of each filter */
    int32_t *final_state;       /* [n_theta*M][U][H] counts after the last interval run */
} lik_aux;

/*
 * lik_eval_batch -- log-likelihood of every theta against all M trajectories
 * (Supplementary I: log p(y | theta) = sum_m log p(y^m | theta)), with
 * n_particles filter particles per (theta, trajectory) pair.  Synchronous.
 *   theta [n_theta * R] host, rate constants c_r per theta (row-major).
 *   data: host pointers.
 *   loglik_out [n_theta] host: the estimate, -inf if some filter had every
 *     particle at zero density, NaN when status is not LIK_STATUS_OK.
 *   status_out [n_theta] host or NULL.
 *   aux: host pointers or NULL.
 * The library allocates and frees its device memory internally.
 */
int lik_eval_batch(lik_network_t net, const lik_obs_model *obs, const lik_eval_opts *opts,
                   int32_t n_theta, const double *theta, const lik_data *data,
                   int32_t n_particles, uint64_t seed, double *loglik_out,
                   int32_t *status_out, const lik_aux *aux);

/*
 * lik_workspace_size -- bytes of device workspace lik_eval_batch_device needs.
 */
size_t lik_workspace_size(lik_network_t net, int32_t n_theta, int32_t n_traj,
                          int32_t n_particles);

/*
 * lik_eval_batch_device -- the same computation on device-resident buffers,
 * enqueued on `stream` (a hipStream_t; NULL = the default stream).  Returns
 * after enqueueing; results are valid when the stream reaches them.
 *   theta, data (all arrays), opts->theta_ids, loglik_out, status_out (may be
 *   NULL) and aux arrays are DEVICE pointers.
 *   obs_offsets_host [M+1]: a host copy of data->obs_offsets, used to plan
 *   the launches.
 *   workspace: device memory of at least lik_workspace_size(...) bytes,
 *   256-byte aligned, not used by anything else until the stream has passed
 *   this call.
 * Invalid theta values are reported per theta (LIK_STATUS_BAD_THETA);
 * observation values are not inspected on the host in this entry point.
 */
int lik_eval_batch_device(lik_network_t net, const lik_obs_model *obs,
                          const lik_eval_opts *opts, int32_t n_theta, const double *theta,
                          const lik_data *data, const int32_t *obs_offsets_host,
                          int32_t n_particles, uint64_t seed, double *loglik_out,
                          int32_t *status_out, const lik_aux *aux, void *workspace,
                          size_t workspace_bytes, void *stream);

/*
 * lik_eval_batch_device_noalloc -- lik_eval_batch_device for callers that
 * cannot allocate device memory: code under HIP graph capture (the caller's
 * own), tight serving loops, harnesses that forbid hipMalloc.  Same arguments
 * and results as lik_eval_batch_device, without the workspace: the library
 * uses a static device array of LIK_NOALLOC_SCRATCH_BYTES instead (one per
 * GPU it runs on, held until the process ends).  This entry point calls no
 * hipMalloc, hipFree or other allocating routine: it records no timing
 * events, LIK_FLAG_GRAPH is rejected (LIK_EINVAL), and it never compiles or
 * loads a specialised kernel -- it runs the one an earlier call of another
 * entry point loaded on this device, else the generic kernels
 * (LIK_KERNEL_SPECIALIZED with none loaded: LIK_EINVAL).  A batch whose
 * lik_workspace_size exceeds LIK_NOALLOC_SCRATCH_BYTES is rejected with
 * LIK_EINVAL before anything is enqueued.  Every call on a GPU uses that
 * GPU's one array, which keeps the last call's contents (every kernel
 * initialises what it reads): calls that overlap on one GPU -- on two
 * streams, or from two threads -- race and give undefined results.
 */
#define LIK_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int lik_eval_batch_device_noalloc(lik_network_t net, const lik_obs_model *obs,
                                  const lik_eval_opts *opts, int32_t n_theta, const double *theta,
                                  const lik_data *data, const int32_t *obs_offsets_host,
                                  int32_t n_particles, uint64_t seed, double *loglik_out,
                                  int32_t *status_out, const lik_aux *aux, void *stream);

/* ------------------------------------------------------------------------ */
/* Continuous-batching server                                               */
/* ------------------------------------------------------------------------ */
/*
 * A server owns one HIP stream, a device arena and a worker thread.  Requests
 * (a batch of rate vectors of one network against its trajectories, with its
 * own particle count, lengths, observation model, precision and seed) are
 * admitted while filter slots and arena memory are free, first come first
 * served.  Each worker iteration advances every resident filter by one
 * observation interval in shared launches, so requests that arrive while
 * others run join the next iteration; a request's slots and memory are
 * released when its last interval is done.  A request's result depends only
 * on its own inputs and seed: it is bit-identical to lik_eval_batch on the
 * same inputs, alone or in any mix.
 */
#define LIK_ETIMEOUT (-5)

typedef struct lik_server *lik_server_t;

typedef struct lik_server_opts {
    size_t arena_bytes;     /* device memory for resident requests; 0 = 1 GiB */
    size_t staging_bytes;   /* pinned host memory for inputs in flight; 0 = 64 MiB */
    int32_t max_filters;    /* filter slots (theta x trajectory pairs); 0 = 65536 */
    int32_t kernel;         /* LIK_KERNEL_GENERIC or LIK_KERNEL_SPECIALIZED (default, 0) */
    int32_t max_inflight;   /* iterations enqueued ahead of the GPU; 0 = 2 */
    int32_t reserved;       /* must be 0 */
    const lik_tuning *tuning; /* work partitioning for every iteration; NULL = defaults */
} lik_server_opts;

typedef struct lik_request {
    lik_network_t net;
    lik_obs_model obs;
    int32_t precision;          /* LIK_FP64 or LIK_FP32_MIXED */
    int32_t n_theta;
    const double *theta;        /* host [n_theta * R] */
    const uint32_t *theta_ids;  /* host [n_theta] random-stream ids or NULL (0..n_theta-1) */
    lik_data data;              /* host pointers */
    int32_t n_particles;
    int32_t reserved;           /* must be 0 */
    uint64_t seed;
    uint64_t event_cap;         /* 0 = default */
    int64_t timeout_us;         /* > 0: a request not finished this long after its submit is
                                   withdrawn like a cancelled one, with LIK_STATUS_TIMED_OUT;
                                   0: no limit */
} lik_request;

typedef struct lik_server_stats {
    uint64_t submitted, completed, evals;   /* requests and rate vectors */
    uint64_t iterations;                    /* engine iterations run */
    double p50_latency_us, p99_latency_us;  /* submit -> result available, completed requests */
    double busy_s;                          /* wall time with resident work */
    uint64_t cancelled;                     /* requests withdrawn (cancelled or timed out) */
} lik_server_stats;

/*
 * lik_eval_requests -- many requests evaluated together (each a lik_request:
 * its own network, observation model, rate vectors, trajectories, particle
 * count, seed and event cap; lik_request.timeout_us must be 0).  Every filter
 * of every request is admitted in one launch; with the flow schedule
 * (tuning->schedule = 1, the default) one persistent launch then runs every
 * interval of every filter, each work item with its own network's
 * propagation body (one kernel compiled for the set of networks, or the
 * generic kernel), and one launch sums each request's trajectories.  Where
 * the flow schedule does not qualify (large networks: too few resident
 * wavefronts; 2^26 or more work items) the same filters advance in shared
 * per-interval iterations.  Each request's results equal lik_eval_batch on
 * its own inputs.  Synchronous; allocates and frees its device memory.
 *   reqs [n_req] host; all of one precision; at most 16 distinct networks;
 *     at most 2^26 filters (theta x trajectory pairs) in all.
 *   tuning: work partitioning and schedule (NULL: the defaults).
 *   kernel: LIK_KERNEL_* (AUTO: specialised when the batch amortises the
 *     compile).
 *   loglik_out [sum of n_theta] host: request k's values at offset
 *     sum_{j<k} reqs[j].n_theta, as lik_eval_batch writes them; status_out
 *     likewise, or NULL.
 *   done_ms [n_req] host or NULL: device-clock time from the admission
 *     launch to the finish of the request's last filter (for completion
 *     percentiles; 0 if none of its filters ran).
 * Returns LIK_EINVAL for an invalid request (the message names it),
 * LIK_EUNSUPPORTED for more than 16 networks.
 */
int lik_eval_requests(const lik_request *reqs, int32_t n_req, const lik_tuning *tuning,
                      int32_t kernel, double *loglik_out, int32_t *status_out, double *done_ms);

/*
 * lik_precompile_requests -- compile the flow kernel lik_eval_requests uses
 * for this set of networks into the on-disk kernel cache (no GPU needed).
 * nets: the distinct networks in the order they first appear in the
 * requests; 1 to 16.  LIK_EDEVICE with the compiler log if compilation fails.
 */
int lik_precompile_requests(const lik_network_t *nets, int32_t n_nets, int32_t precision);

/*
 * lik_autotune_requests -- times lik_eval_requests on these requests for
 * the fixed set of candidate tunings (particles per wavefront, pool
 * thresholds, schedule) and writes the fastest to *chosen.  Results of
 * every candidate are identical; the timing includes the calls' copies.
 */
int lik_autotune_requests(const lik_request *reqs, int32_t n_req, int32_t kernel,
                          lik_tuning *chosen);

/* Creates a server on the current device.  LIK_ENOMEM if the arena cannot be allocated. */
int lik_server_create(const lik_server_opts *opts, lik_server_t *out);

/*
 * Validates and copies a request (the caller may free its buffers when this
 * returns) and queues it.  LIK_EINVAL for invalid requests or requests that
 * could never fit the server's arena or slots.  *ticket identifies it.
 */
int lik_server_submit(lik_server_t srv, const lik_request *req, uint64_t *ticket);

/*
 * Waits up to timeout_us (< 0: forever) for a ticket; on LIK_OK writes
 * loglik_out[n_theta] and status_out[n_theta] (may be NULL) and forgets the
 * ticket.  LIK_ETIMEOUT if it is not done yet (the ticket stays valid).
 */
int lik_server_wait(lik_server_t srv, uint64_t ticket, double *loglik_out, int32_t *status_out,
                    int64_t timeout_us);

/*
 * Withdraws a request.  Still queued: it is removed at once.  Resident: its
 * filter slots stop at the next iteration boundary and its slots and memory
 * are released once the work already enqueued for it has passed; the other
 * requests' results are unaffected.  Either way the ticket then completes:
 * lik_server_wait returns LIK_OK with LIK_STATUS_CANCELLED for every theta
 * and NaN log-likelihoods.  A request whose results are already being
 * copied back is left to finish (LIK_OK; its results stay valid).
 * LIK_EINVAL for an unknown ticket.  Thread-safe.
 */
int lik_server_cancel(lik_server_t srv, uint64_t ticket);

int lik_server_stats_get(lik_server_t srv, lik_server_stats *out);

/* Finishes every submitted request, then stops the worker and frees the server. */
int lik_server_destroy(lik_server_t srv);

/*
 * Kernel timing for measurement tools.  While enabled, every propagation
 * launch and every weighting/resampling launch is bracketed by HIP events
 * recorded on the stream it is enqueued on.  lik_timing_read waits for the
 * recorded events, returns the summed kernel durations and launch counts
 * since the previous read, and releases the events.  Process-global, not
 * thread-safe: for single-threaded benchmark drivers.
 */
typedef struct lik_timing {
    double propagate_ms;        /* summed duration of SSA propagation launches (and of
                                   lik_ode_eval's solver launches) */
    int64_t propagate_launches;
    double weigh_ms;            /* summed duration of weight/resampling launches */
    int64_t weigh_launches;
} lik_timing;

int lik_timing_enable(int enable);
int lik_timing_read(lik_timing *out);

/*
 * lik_autotune_device -- times lik_eval_batch_device on these exact buffers
 * for a fixed set of candidate tunings (synchronising `stream` after each),
 * keeps the fastest as the network's tuning and writes it to *chosen (may be
 * NULL).  The outputs are overwritten with valid results of `seed`; graph
 * mode (LIK_FLAG_GRAPH) is ignored while timing.  Arguments as for
 * lik_eval_batch_device (no aux outputs).  On error the previous tuning is
 * kept.  Same threading rule as lik_network_set_tuning.
 */
int lik_autotune_device(lik_network_t net, const lik_obs_model *obs, const lik_eval_opts *opts,
                        int32_t n_theta, const double *theta, const lik_data *data,
                        const int32_t *obs_offsets_host, int32_t n_particles, uint64_t seed,
                        double *loglik_out, int32_t *status_out, void *workspace,
                        size_t workspace_bytes, void *stream, lik_tuning *chosen);

/* ------------------------------------------------------------------------ */
/* Deterministic models                                                      */
/* ------------------------------------------------------------------------ */
/*
 * The deterministic formulation (Sec. "Chemical Reaction Networks": the state
 * follows dX/dt = f(X, t, theta)): no particle filter; the likelihood of a
 * trajectory is the noise density of its observations around the ODE solution
 * (Results, deterministic models; Supplementary "Egf-Ras-Raf-Mek-Erk model"),
 * summed over trajectories per theta.
 *
 * f is a sum of fluxes ("terms").  Term k moves one unit from species `from`
 * to species `to` (-1: none) at the rate
 *   v_k = rate_scale * theta[rate_param] * prod_f phi_f   (rate_param -1: rate_scale alone)
 * with factors phi of kind
 *   LIK_ODE_SPECIES     x_u
 *   LIK_ODE_SATURATING  x_u / (theta[param] + x_u)         (Michaelis-Menten)
 *   LIK_ODE_HILL2       x_u^2 / (theta[param] + x_u^2)     (activating, Hill 2)
 *   LIK_ODE_REPRESS2    theta[param] / (theta[param] + x_u^2) (repressing, Hill 2)
 *   LIK_ODE_INPUT       u(t), the trajectory's piecewise-constant input
 * (a Hill constant K enters as K^2 through the parameter map of the caller).
 * dx_u/dt sums -v_k over the terms leaving u and +v_k over those entering it,
 * in term order.
 *
 * Initial state of trajectory m: x_u(t0) = theta[x0_param[u]] where
 * x0_param[u] >= 0, else the trajectory's x0[u].
 *
 * Observation (one value per time point): y ~ N(g(x), sd^2), sd =
 * theta[sd_param] (or sd_const when sd_param is -1), with
 *   LIK_ODE_OBS_SPECIES  g = x_{obs_species}
 *   LIK_ODE_OBS_FRET     g = lambda (E fAA x_a / ((x_b + (1 - E) x_a) fDD) + bg),
 *                        x_a = x_{obs_species} (active), x_b = x_{obs_species2},
 *                        lambda, bg, E, fAA, fDD = theta[fret_param[0..4]]
 *                        (the FRET ratio of the Egf-Ras-Raf-Mek-Erk example).
 *
 * Solver (the paper names none): the Dormand-Prince 5(4) pair with local
 * extrapolation and first-same-as-last stages; a step is accepted when
 * max_u |e_u| / (atol + rtol max(|x_u|, |x_u new|)) <= 1, and the next step is
 * h * min(5, max(0.2, 0.9 err^(-1/5))) (err^(-1/5) from the library's log and
 * exp); steps end exactly at every observation time and input breakpoint.
 * LIK_STATUS_STEP_LIMIT if a trajectory needs more than max_steps steps or its
 * step falls below 1e-12 of its time span; LIK_STATUS_NONFINITE if the state
 * or g is not finite.  A theta with a non-finite entry, or a negative rate,
 * Hill constant, sd or initial value, is LIK_STATUS_BAD_THETA.
 */
#define LIK_ODE_MAX_SPECIES 32
#define LIK_ODE_MAX_TERMS 128
#define LIK_ODE_MAX_PARAMS 128
#define LIK_ODE_MAX_FACTORS 3

#define LIK_ODE_SPECIES 0
#define LIK_ODE_SATURATING 1
#define LIK_ODE_HILL2 2
#define LIK_ODE_REPRESS2 3
#define LIK_ODE_INPUT 4

#define LIK_ODE_OBS_SPECIES 0
#define LIK_ODE_OBS_FRET 1

typedef struct lik_ode_term {
    int32_t from, to;        /* species indices, or -1 */
    int32_t rate_param;      /* theta index, or -1 */
    int32_t n_factors;       /* 0 .. LIK_ODE_MAX_FACTORS */
    double rate_scale;       /* finite, >= 0 */
    int32_t kind[LIK_ODE_MAX_FACTORS];
    int32_t species[LIK_ODE_MAX_FACTORS];
    int32_t param[LIK_ODE_MAX_FACTORS]; /* theta index of K (saturating, Hill, repressing) */
} lik_ode_term;

typedef struct lik_ode_model {
    int32_t n_species;       /* U in [1, LIK_ODE_MAX_SPECIES] */
    int32_t n_params;        /* theta length V in [1, LIK_ODE_MAX_PARAMS] */
    int32_t n_terms;         /* in [1, LIK_ODE_MAX_TERMS] */
    const lik_ode_term *terms;
    const int32_t *x0_param; /* [U]: theta index or -1 */
    int32_t obs_kind, obs_species, obs_species2, sd_param;
    double sd_const;         /* > 0 when sd_param is -1 */
    int32_t fret_param[5];   /* lambda, bg, E, fAA, fDD (LIK_ODE_OBS_FRET) */
} lik_ode_model;

typedef struct lik_ode_t_ *lik_ode_t;

/* Validates and copies a model (host pointers).  LIK_EINVAL on a violated rule. */
int lik_ode_create(const lik_ode_model *model, lik_ode_t *out);
int lik_ode_destroy(lik_ode_t model);
/* Compiles the model-specialised kernel into the on-disk kernel cache (no GPU
 * needed); LIK_EDEVICE with the compiler log in lik_last_error() on failure. */
int lik_ode_precompile(lik_ode_t model);

/*
 * Trajectories of a deterministic batch (host pointers):
 *   obs_offsets [M+1], t_obs [total] (strictly increasing, > t0[m]), y [total];
 *   t0 [M]; x0 [M*U] binary64 initial values of the species not set by theta;
 *   in_offsets [M+1] (NULL: no input, u = 0), t_in [n_in] breakpoints, strictly
 *   increasing per trajectory, u_in [n_in]: u(t) = u_in[k] on [t_in[k],
 *   t_in[k+1]), 0 before the first breakpoint, u_in[last] after the last.
 */
typedef struct lik_ode_data {
    int32_t n_traj;
    const int32_t *obs_offsets;
    const double *t_obs, *y, *t0, *x0;
    const int32_t *in_offsets;
    const double *t_in, *u_in;
} lik_ode_data;

/*
 * lik_ode_eval -- log-likelihood of n_theta parameter vectors (theta
 * [n_theta * V], host) against the trajectories: loglik_out[i] = sum over m
 * of sum over t of log N(y_t; g(x(t_t)), sd^2) in trajectory and time order;
 * status_out[i] (may be NULL) the first non-OK trajectory status, with NaN;
 * steps_out[i * M + m] (may be NULL) the step attempts (accepted or rejected)
 * of trajectory m.  rtol, atol > 0; max_steps in [1, 2^30] per trajectory.
 * kernel: LIK_KERNEL_GENERIC (the terms read at run time),
 * LIK_KERNEL_SPECIALIZED (the model compiled with hipRTC into code with
 * constant indices, cached on disk like the networks' kernels; LIK_EDEVICE if
 * that fails) or LIK_KERNEL_AUTO (specialised, else generic); every variant
 * gives identical results.  Each (theta, trajectory) pair is integrated by
 * one GPU lane; the lanes take pairs from a shared counter, the trajectories
 * with the most stops (observations plus input breakpoints) first, which
 * changes only the speed.  Synchronous; allocates its device memory.
 */
int lik_ode_eval(lik_ode_t model, int32_t n_theta, const double *theta,
                 const lik_ode_data *data, double rtol, double atol, int32_t max_steps,
                 int32_t kernel, double *loglik_out, int32_t *status_out, int32_t *steps_out);

/*
 * lik_ode_workspace_size -- bytes of device workspace lik_ode_eval_device
 * needs for n_theta parameter vectors and n_traj trajectories (0 on a bad
 * argument).
 *
 * lik_ode_eval_device -- lik_ode_eval on device buffers, enqueued on `stream`
 * (a hipStream_t; NULL: the null stream) without waiting: theta [n_theta * V],
 * every array of `data`, loglik [n_theta], status [n_theta] (may be NULL) and
 * steps [n_theta * M] (may be NULL) are device pointers; obs_offsets_host and
 * in_offsets_host are host copies of data->obs_offsets and data->in_offsets
 * (both NULL or both given), checked like lik_ode_eval's; the values of the
 * device arrays are the caller's to keep valid (the rules of lik_ode_data),
 * and the device offsets must equal the host copies.  workspace: device
 * memory of lik_ode_workspace_size bytes, owned by the caller, not to be
 * shared by calls in flight.  The first call on a device copies the model's
 * terms there (synchronously); later calls copy nothing from the host.
 * Results are identical to lik_ode_eval's.
 */
size_t lik_ode_workspace_size(lik_ode_t model, int32_t n_theta, int32_t n_traj);
int lik_ode_eval_device(lik_ode_t model, int32_t n_theta, const double *theta,
                        const lik_ode_data *data, const int32_t *obs_offsets_host,
                        const int32_t *in_offsets_host, double rtol, double atol,
                        int32_t max_steps, int32_t kernel, double *loglik, int32_t *status,
                        int32_t *steps, void *workspace, size_t workspace_bytes, void *stream);

/* Thread-local description of the last error returned on this thread. */
const char *lik_last_error(void);

/* Library version string. */
const char *lik_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LIK_H */
