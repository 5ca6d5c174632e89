/*
 * nsmi.h - C ABI of the MI355X batched acceptance-walk nested sampler.
 *
 * The library implements the vectorised nested-sampling step of
 * arXiv:2509.04336 ("Gravitational-wave inference at GPU speed"):
 *   - delete the k lowest-likelihood live points of each event and set the
 *     threshold L* to the largest deleted log-likelihood (Sec. 2.2.3);
 *   - refill with k independent acceptance walks that make
 *     differential-evolution proposals in the unit cube and accept only when
 *     L > L*, every walk of a batch taking the same number of steps W
 *     (Sec. 3.1);
 *   - account the deletions with live counts n, n-1, ..., n-k+1 (Sec. 3.2,
 *     3.2.1) and retune W once per batch (Sec. 3.2);
 * with the frequency-domain Whittle log-likelihood ratio of an aligned-spin
 * TaylorF2 signal projected on up to three detectors (Sec. 3.3, 4.1.1).
 *
 * Conventions shared by every entry point:
 *   - Parameter vector theta[11] (physical): chirp mass [Msun], mass ratio
 *     q = m2/m1 in (0, 1], chi1, chi2, luminosity distance [Mpc], theta_JN,
 *     right ascension, declination, polarisation psi, coalescence phase,
 *     coalescence time [s] (priors of Table 1).  A sampled event of
 *     dimension 4 samples the first four and fixes the rest; dimension 11
 *     samples all, with right ascension, psi and phase periodic.
 *   - Frequencies f_k = f_lo + k*df, k = 0..n_bins-1.
 *   - Every call returns an ns_status; nothing is thrown or aborted across
 *     the ABI.  After a failure ns_last_error() gives the message.
 *   - Host pointers are read during the call only (the library copies what
 *     it keeps).  Device pointers must stay valid until the enqueued work on
 *     the context stream has finished.
 *   - All device work of a context is enqueued on cfg.stream (a hipStream_t,
 *     NULL for the default stream).  Calls on one context must not overlap.
 */
#ifndef NSMI_H
#define NSMI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ns_ctx ns_ctx; /* opaque, owned by the library */

typedef enum {
    NS_OK = 0,
    NS_EINVAL = -1,      /* bad argument (size, pointer, range) */
    NS_EHIP = -2,        /* a HIP runtime call failed */
    NS_ENOMEM = -3,      /* device or host allocation failed */
    NS_ESTATE = -4,      /* call not valid in the current state */
    NS_ENONFINITE = -5,  /* non-finite or non-positive input data */
    NS_ENOTIMPL = -6     /* feature not available in this library */
} ns_status;

typedef enum {
    NS_FP64 = 0,  /* everything in double precision */
    NS_MIXED = 1  /* FP64 phase and argument reduction, FP32 sin/cos (one
                     pair per bin, an FP32 rotation for further detectors)
                     and FP32 sums flushed into FP64 every 8 bins of a lane;
                     |dlogL| <= 1e-3 per call against FP64 */
} ns_precision;

typedef enum {
    NS_INNER_WALK = 0, /* acceptance walk (Sec. 3.1): differential-evolution
                          proposals, strict L > L* acceptance, W steps */
    NS_INNER_HRSS = 1  /* hit-and-run slice sampling (the alternative inner
                          kernel of the closing section; slice sampler of
                          Neal 2003, Sec. 4): W slice steps along
                          differential-evolution lines, each stepping out a
                          unit interval (budget 8 widths) and shrinking it
                          until a uniform draw lies in L > L* */
} ns_inner;

typedef enum {
    NS_LIKE_GW = 0,    /* Whittle log-likelihood ratio (use_ratio) */
    NS_LIKE_GAUSS = 1, /* -|u - 1/2|^2 / (2 sigma^2) in the unit cube (test
                          likelihood with a closed-form evidence) */
    NS_LIKE_GW_RB = 2  /* the Whittle likelihood with its data term
                          heterodyned around a fiducial point (relative
                          binning; the paper names heterodyning as the way to
                          cut the per-call cost, Sec. 3.3 and Sec. 5): the
                          fiducial phase factor stays exact, the ratio
                          e^{-i (Phi - Phi0)} is interpolated linearly between
                          the rb_bins + 1 nodes; <h|h> stays exact.  Always
                          evaluated in FP64. */
} ns_likelihood;

/* One event (analysis segment).  All arrays are host memory. */
typedef struct {
    int32_t n_bins;              /* >= 1 */
    int32_t n_det;               /* 1..3 */
    int32_t ndim;                /* 4 or 11 sampled parameters */
    int32_t likelihood;          /* ns_likelihood */
    double f_lo, df;             /* f_lo > 0, df > 0 */
    const double *data;          /* [n_det][n_bins][2] complex strain d(f_k) */
    const double *psd;           /* [n_det][n_bins] one-sided S(f_k) > 0 */
    const double *det_tensor;    /* [n_det][9] response tensor, row-major, or NULL
                                    when fixed_antenna is given */
    const double *det_loc;       /* [n_det][3] Earth-fixed position in metres */
    const double *fixed_antenna; /* [n_det][2] (F+, Fx) with zero time delay, or
                                    NULL to use det_tensor/det_loc */
    const double *prior_lo;      /* [11] lower prior edges (Table 1 shapes) */
    const double *prior_hi;      /* [11] upper prior edges */
    const double *fixed_theta;   /* [11] values of the parameters not sampled */
    double gmst;                 /* Greenwich mean sidereal time [rad] */
    double toy_sigma;            /* width of the Gaussian test likelihood */
    /* NS_LIKE_GW_RB only (ignored otherwise): fiducial physical parameters
     * [11] (a valid point) and rb_bins + 1 node sample indices, rb_edges[0] =
     * 0 < rb_edges[1] < ... < rb_edges[rb_bins] = n_bins (the last node lies
     * one grid step past the last sample); 1 <= rb_bins <= 4095. */
    const double *rb_theta0;
    const int32_t *rb_edges;
    int32_t rb_bins;
    int32_t rb_pad;              /* set to 0 */
} ns_event_desc;

typedef struct {
    int32_t n_live;      /* live points per event, 3..4096 */
    int32_t num_delete;  /* k deleted per batch, 1 <= k <= n_live - 2 */
    int32_t naccept;     /* target accepted steps per walk (Sec. 3.2) */
    int32_t maxmcmc;     /* cap on the walk length */
    int32_t walk0;       /* initial walk length, 1..maxmcmc */
    int32_t term_kind;   /* 0: dlogZ < term_thr; 1: Z_live/Z < term_thr */
    double delay;        /* sequential smoothing delay D; < 0 selects
                            max(n_live/10 - 1, 0) */
    double term_thr;     /* termination threshold (0.1 or 1e-3 in the paper) */
    int32_t precision;   /* ns_precision of the walk likelihood */
    int32_t flags;       /* bit 0 (NS_FLAG_TIMING): record HIP events around
                            every kernel launch of ns_step (see ns_timing) */
    uint64_t seed;       /* Philox4x64-10 key word 0 */
    void *stream;        /* hipStream_t */
} ns_config;

#define NS_FLAG_TIMING 1
#define NS_FLAG_GRAPH 2   /* replay each iteration's launches as a captured
                             hipGraph (ignored together with NS_FLAG_TIMING) */

/* Accumulated device time of the kernels launched by ns_step, from HIP
 * events recorded on the context stream (only with NS_FLAG_TIMING). */
typedef struct {
    double select_ms, walk_ms, finish_ms; /* summed event-to-event times */
    int64_t launches;                     /* ns_step calls timed */
} ns_timing_t;

/* Evidence and run statistics of one event (Sec. 3.2.1; termination rules
 * of Sec. 4.1.1 and 4.2). */
typedef struct {
    double logZ;         /* log evidence including the live points */
    double logZ_dead;    /* log evidence accumulated from dead points */
    double logZ_err;     /* sqrt(H sum(1/n_i^2) / sum(1/n_i)) over the dead
                            points' live counts n_i: Skilling's sqrt(H / n)
                            with the batched saw-tooth of live counts
                            (Sec. 3.2.1), about 1.2x sqrt(H / n_live) at
                            k = n_live / 2 */
    double H;            /* information (KL divergence posterior || prior) */
    double logX;         /* log remaining prior volume */
    double dlogZ;        /* log(Z + X max L_live) - log Z */
    double log_frac;     /* log(X mean L_live / Z) */
    double last_Lstar;   /* threshold of the last batch */
    int64_t n_dead;      /* dead points so far */
    int64_t n_calls;     /* exact likelihood evaluations in walks */
    int64_t n_accept;    /* accepted walk steps */
    int64_t n_oob;       /* proposals outside the cube (no evaluation) */
    int64_t n_steps;     /* walk steps taken (k * W summed over batches) */
    int64_t n_calls_saved; /* evaluations skipped by a surrogate screen */
    int64_t batch;       /* batches done */
    int32_t W;           /* walk length of the next batch */
    int32_t converged;   /* termination criterion met */
    int64_t last_accept; /* accepted steps in the last batch */
    int64_t last_calls;  /* evaluations in the last batch */
    int64_t n_spec_discarded; /* speculative evaluations discarded (extra work,
                                 not part of n_calls) */
    int32_t walk_capped; /* consecutive batches (the last included) whose
                            tuned walk length is maxmcmc: the chains no longer
                            reach naccept accepted steps within the cap, so
                            new points stay correlated with their starts
                            (stuck-walk guard; Sec. 3.2 tuning rule) */
    int32_t reserved;    /* zero */
} ns_evidence_t;

/* Create a context: upload n_events events (copied), build the per-bin
 * tables and weights on the device, draw the initial live sets from the
 * prior with Philox (purpose 7) and evaluate them.  Returns NS_EINVAL for
 * bad sizes, NS_ENONFINITE for non-finite data or non-positive PSD values.
 * On failure *out is NULL. */
ns_status ns_init(ns_ctx **out, const ns_config *cfg, const ns_event_desc *events,
                  int32_t n_events);

/* Release every device and host resource of the context (NULL is a no-op). */
void ns_free(ns_ctx *ctx);

/* Message of the last failure on this context (empty string if none).
 * ns_last_error(NULL) returns the message of the last failed ns_init. */
const char *ns_last_error(const ns_ctx *ctx);

/* One batched iteration on every event that has not converged (Sec. 2.2.3,
 * 3.1, 3.2): select and delete k points, walk k chains, account the
 * evidence, retune W.  k <= 0 uses cfg.num_delete; walk <= 0 uses the tuned
 * walk length of each event, walk > 0 forces that length for this batch
 * (must be <= maxmcmc).  Enqueued on the context stream; does not wait.
 * Convergence is decided on the device; the host learns it only when
 * ns_evidence reads an event back (or a checkpoint is restored).  Once every
 * event has been read back converged, ns_step returns NS_ESTATE and
 * enqueues nothing.  Before that, a step leaves converged events unchanged
 * (their kernels return at once) and only reserves dead-point rows. */
ns_status ns_step(ns_ctx *ctx, int32_t k, int32_t walk);

/* Log-likelihood ratio of n physical parameter vectors of one event:
 * theta is a device pointer to [n][11] doubles, out_logl a device pointer to
 * n doubles.  precision selects the inner-product arithmetic.  A parameter
 * vector outside the physical domain (non-finite, q not in (0, 1],
 * Mc <= 0, dL <= 0) gives -inf.  Enqueued on the context stream. */
ns_status ns_loglike_batch(ns_ctx *ctx, int32_t event, const double *theta, int64_t n,
                           double *out_logl, int32_t precision);

/* Same as ns_loglike_batch for unit-cube points u (device, [n][ndim]),
 * mapped through the event's prior transform. */
ns_status ns_loglike_batch_u(ns_ctx *ctx, int32_t event, const double *u, int64_t n,
                             double *out_logl, int32_t precision);

/* Physical parameters theta (device, [n][11], the order above) of
 * unit-cube points u (device, [n][ndim]) through the event's prior
 * transforms (Sec. 4, Tab. 1), e.g. for posterior samples from
 * ns_get_dead.  Enqueued on the context stream.  NS_EINVAL for a bad event,
 * a Gaussian-toy event, n < 0 or NULL pointers with n > 0. */
ns_status ns_theta_from_u(ns_ctx *ctx, int32_t event, const double *u, int64_t n, double *theta);

/* Evidence summary of one event; waits for the context stream. */
ns_status ns_evidence(ns_ctx *ctx, int32_t event, ns_evidence_t *out);

/* Per-chain counts of the last batch of one event (Sec. 3.2: the accepted
 * steps of the chains are what the walk-length rule reads): out receives
 * [n][4] int64 = accepted steps, exact likelihood calls, out-of-cube steps
 * and speculative evaluations discarded, for chains c = 0..n-1 with
 * n = min(k of the last batch, max_chains) written to *n_chains (0 when the
 * event was already inactive).  Chain c produced live row n_live - k + c.
 * With a surrogate screen, steps saved by it are W - calls - out-of-cube.
 * Waits for the context stream.  NS_EINVAL for a bad event or NULL
 * pointers. */
ns_status ns_get_chain_stats(ns_ctx *ctx, int32_t event, int64_t *out, int32_t max_chains,
                             int32_t *n_chains);

/* Evidence of R replicates of one event's run (App. A: the prior-volume
 * weights of the dead points are uncertain): each replicate replaces the
 * expected shrinkage of deletion i by log t_i, t_i ~ Beta(n_i, 1) with n_i
 * the live count at that deletion (log t_i = log(U_i) / n_i), and re-adds
 * the dead points and the final live set.  uniforms: device [R][n_dead]
 * values in (0, 1] (the deletion order of ns_get_dead), or NULL to draw
 * U = 1 - u01 of Philox counter (i, r, 0, 9) under key (seed, 0); out: device
 * [R], log Z of each replicate (their spread is the evidence error).
 * Enqueued on the context stream after reading the dead count (a wait).
 * NS_ESTATE before the first batch; NS_EINVAL for a bad event, R outside
 * [1, 2^20] or out NULL. */
ns_status ns_logz_replicates(ns_ctx *ctx, int32_t event, int32_t R, uint64_t seed,
                             const double *uniforms, double *out);

/* Copy the live set of one event to host memory: u [n_live][ndim],
 * logl [n_live] (either may be NULL).  Waits for the context stream. */
ns_status ns_get_live(ns_ctx *ctx, int32_t event, double *u, double *logl);

/* Replace the live set of one event from host memory (u in [0,1]^ndim,
 * logl its log-likelihoods).  The evidence accumulators are not changed. */
ns_status ns_set_live(ns_ctx *ctx, int32_t event, const double *u, const double *logl);

/* Copy up to max_rows dead points of one event to host memory in deletion
 * order: u [rows][ndim], logl, logw (log prior-volume weight) and nlive
 * (live count at deletion); any output may be NULL.  *n_rows receives the
 * number of rows copied.  Waits for the context stream. */
ns_status ns_get_dead(ns_ctx *ctx, int32_t event, int64_t max_rows, double *u, double *logl,
                      double *logw, double *nlive, int64_t *n_rows);

/* Checkpoint and resume of the sampler state of Sec. 2.2.3 and 3.2: live
 * set, dead points, evidence accumulators, walk length, counters and the
 * batch index that keys the counter-based random numbers.
 *
 * ns_checkpoint_size: *bytes receives the size of a checkpoint of the
 * current state.  ns_checkpoint: writes it into buf (caller-owned host
 * memory of at least that many bytes; NS_EINVAL if smaller); *written, if
 * not NULL, receives the size.  ns_restore: loads a checkpoint into a
 * context created with the same events and sampler configuration (live
 * points, delete count, naccept, maxmcmc, initial walk length, precision,
 * termination rule, seed, delay), the same inner kernel and the same event
 * data (a fingerprint of each event's grid, data and PSD is stored);
 * NS_EINVAL, with nothing changed, for another layout, configuration, event
 * data or size, a live u outside [0, 1], or a per-event state the sampler
 * cannot produce (walk length outside [1, maxmcmc], flags other than 0/1,
 * log X not finite and <= 0, negative counters).  A restored context continues exactly as the
 * checkpointed one would have.  The learned surrogate, harvest buffer,
 * timing and launch shape are not part of a checkpoint.  All three wait for
 * the context stream; the layout is native-endian and tied to this
 * library version. */
ns_status ns_checkpoint_size(ns_ctx *ctx, int64_t *bytes);
ns_status ns_checkpoint(ns_ctx *ctx, void *buf, int64_t bytes, int64_t *written);
ns_status ns_restore(ns_ctx *ctx, const void *buf, int64_t bytes);

/* Detector strain h_d(f_k) of one parameter vector for an event
 * description (desc->data and desc->psd are not read): theta is host [11],
 * h receives host [n_det][n_bins][2].  Evaluated on the current device with
 * the same device code as the likelihood, then copied back.  Used to build
 * injections. */
ns_status ns_signal(const ns_event_desc *desc, const double *theta, double *h);

/* ns_signal for callers that cannot allocate device memory (code under
 * graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same arguments, result bit-identical to ns_signal, with no hipMalloc,
 * hipFree or allocating library call.  The descriptor, parameter vector and
 * strain staging live in a fixed device array of about 3 MiB that each GPU
 * the library runs on holds until the process ends.  n_bins is limited to
 * 65536 (NS_EINVAL above); the copies and the kernel run on the null stream
 * and the call returns when h is written.  Calls on one GPU share that
 * array: calls that overlap in time on the same GPU (from several host
 * threads) race and must be serialised by the caller. */
ns_status ns_signal_noalloc(const ns_event_desc *desc, const double *theta, double *h);

/* Kernel times accumulated since ns_init or the last reset (reset != 0
 * clears them after reading).  Waits for the context stream.  Returns
 * NS_ESTATE when the context was created without NS_FLAG_TIMING. */
ns_status ns_timing(ns_ctx *ctx, ns_timing_t *out, int32_t reset);

/* Launch shape of the walk kernel: waves per chain (1, 2, 4, 6 or 8; 0
 * picks 4 from 256 chains per batch up, else 8).  A round evaluates as many
 * speculative proposals as there are waves (for the exact likelihood
 * two proposals per wave pair, each wave over half of the bins).  Results
 * do not depend on it, to the last bit; only the discarded work does.
 * NS_EINVAL for other values. */
ns_status ns_set_waves_per_chain(ns_ctx *ctx, int32_t waves_per_chain);

/* ---- learned surrogate (delayed acceptance) --------------------------------
 * A fully connected network s(u): 11 -> 256 -> 256 -> 256 -> 1 with SiLU,
 * BF16 matrix products with FP32 accumulation, FP32 master weights.  It is
 * fitted to y = (z(logL) - mu) / sigma on (u, logL) pairs and predicts
 * z^-1(mu + sigma s(u)).  The target map z is either v = max(logL, clip)
 * (top = +inf) or, for a finite top > clip, the log-gap z = -log(top - v)
 * (gaps floored at 1e-12) with inverse z^-1(w) = top - exp(-w): it spreads
 * the log-likelihoods just below top, where the screen has to be accurate,
 * and compresses the far tail.  The paper names batched machine-learning models
 * as a natural companion of the batched sampler (Sec. 5); the surrogate is
 * used as a screen in exact two-stage delayed acceptance, the exact
 * likelihood still deciding every accepted point. */

/* Allocate the network (training batches up to max_rows rows) and draw its
 * initial weights with Philox (purpose 5) from seed. */
ns_status ns_surrogate_init(ns_ctx *ctx, uint64_t seed, int64_t max_rows);

/* Copy the FP32 master parameters (134913 floats, layout W1[256][11], b1,
 * W2[256][256], b2, W3[256][256], b3, W4[256], b4) from or to host memory. */
ns_status ns_surrogate_set_params(ns_ctx *ctx, const float *params, int64_t n);
ns_status ns_surrogate_get_params(ns_ctx *ctx, float *params, int64_t n);

/* Target map and normalisation used by training and prediction (mu finite,
 * sigma > 0, top +inf or finite and above clip; NS_EINVAL otherwise). */
ns_status ns_surrogate_set_norm(ns_ctx *ctx, double mu, double sigma, double clip, double top);
ns_status ns_surrogate_get_norm(ns_ctx *ctx, double *mu, double *sigma, double *clip,
                                double *top);

/* Per-input standardisation x = (u - mean) / stdev applied before the
 * network (ndim values each; identity after ns_surrogate_init; set from the
 * training pairs by ns_surrogate_train). */
ns_status ns_surrogate_set_input_norm(ns_ctx *ctx, const double *mean, const double *stdev);
ns_status ns_surrogate_get_input_norm(ns_ctx *ctx, double *mean, double *stdev);

/* Predictions mu + sigma s(u) for n unit-cube points (device [n][ndim] ->
 * device [n]). */
ns_status ns_surrogate_predict(ns_ctx *ctx, const double *u, int64_t n, double *out);

/* Mean squared error on n <= max_rows pairs (device u [n][ndim], device
 * logL [n]) and its gradient with respect to the parameters (host grad,
 * 134913 floats; loss to *loss).  Waits for the context stream. */
ns_status ns_surrogate_loss_grad(ns_ctx *ctx, const double *u, const double *logl, int64_t n,
                                 float *grad, double *loss);

/* Fit the network: set the target map (clip, top), the input
 * standardisation and mu, sigma from the n device pairs, then `steps` Adam
 * steps (learning rate decaying from lr to lr/20 on a cosine schedule) on
 * batches of `batch` pairs drawn with Philox, starting from the current
 * parameters with fresh Adam moments.  *loss receives the last batch loss. */
ns_status ns_surrogate_train(ns_ctx *ctx, const double *u, const double *logl, int64_t n,
                             int32_t steps, int32_t batch, double lr, double clip, double top,
                             double *loss);

/* Screen the walks' proposals with the surrogate by exact two-stage delayed
 * acceptance (Christen & Fox 2005): with the screen density
 *   pi(x) = floor + (1 - floor) sigmoid((s(x) - L* + margin) / temperature),
 * stage 1 continues with probability min(1, pi(u')/pi(u)) without an exact
 * call (counted in n_calls_saved); stage 2 accepts iff L(u') > L* and
 * U < min(1, pi(u)/pi(u')).  The constrained prior stays the invariant
 * distribution of every walk; only the cost and the mixing change.  The floor
 * (0 <= floor < 1) bounds both ratios below by floor, so a chain whose point
 * the surrogate underrates cannot be held in place by stage 2.  Detach
 * returns to the plain walk.  NS_EINVAL for a non-finite margin, a
 * temperature <= 0 or a floor outside [0, 1). */
ns_status ns_surrogate_attach(ns_ctx *ctx, double margin, double temperature, double floor);
ns_status ns_surrogate_detach(ns_ctx *ctx);

/* Record every exact likelihood evaluation of the walks, (u, logL), into a
 * library-owned device buffer of the given capacity (0 stops recording). */
ns_status ns_harvest(ns_ctx *ctx, int64_t capacity);

/* Copy up to max_rows recorded pairs to device memory (u [rows][ndim],
 * logl [rows]); *n_rows receives the count.  Waits for the context stream. */
ns_status ns_harvest_copy(ns_ctx *ctx, double *u, double *logl, int64_t max_rows, int64_t *n_rows);

/* Inner kernel of the chains (NS_INNER_WALK, the default, or
 * NS_INNER_HRSS).  With NS_INNER_HRSS the tuned walk length counts slice
 * steps (a step that moves counts as accepted), each costing several
 * likelihood calls; the surrogate screen and ns_autotune need the walk
 * (NS_ESTATE).  NS_EINVAL for other values. */
ns_status ns_set_inner(ns_ctx *ctx, int32_t inner);

/* Pick the walk kernel's waves per chain for this context's shape by timing
 * side-effect-free trial batches (the sampler state is saved and restored on
 * the device) with walk length `trial_walk`.  If cache_path is not NULL the
 * choice is read from / appended to that text file, keyed by the shape.
 * *chosen (may be NULL) receives the choice. */
ns_status ns_autotune(ns_ctx *ctx, const char *cache_path, int32_t trial_walk, int32_t *chosen);

/* Number of events and sampled dimension of a context. */
int32_t ns_num_events(const ns_ctx *ctx);

/* Build identification string (kernel variants, target). */
const char *ns_version(void);

#ifdef __cplusplus
}
#endif

#endif /* NSMI_H */
