/*
 * saltbf.h - C ABI of the MI355X (gfx950) SALT bandflux library.
 *
 * What is computed (paper, section "Implementation"):
 *   model equation   F(p, lam) = x0 [M0(p, lam) + x1 M1(p, lam)] exp(c CL(lam)),
 *                    free parameters x0, x1, t0, c;
 *   bandflux         the integral over the band of F(lam) T(lam) lam / (h c),
 *                    taken with the trapezoidal rule along wavelength;
 *   derivatives      of the bandflux with respect to the parameters (the paper's
 *                    differentiability claim, sections "Summary" and
 *                    "Implementation"), here also with respect to z;
 *   fits             of x0, x1, t0, c to a light curve (the optimisation example
 *                    of section "Implementation").
 * Readings where the paper is silent (one definition for the whole library):
 *   s = 1/(1+z); phase p = (t - t0) s; amplitude A = x0 s; the surfaces are read
 *   at rest wavelength mu = lam s of a fixed observer-frame quadrature grid lam_k
 *   and lam/(hc) uses lam_k; M0 and M1 are interpolated by Catmull-Rom (Keys,
 *   a = -1/2) cubic convolution, linear in the first and last cell of each axis;
 *   a phase outside the grid gives zero flux; a band whose rest window leaves the
 *   wavelength grid is a range error; CL(mu) = sum_n a_n r^n with
 *   r = (mu - wave_b)/(wave_v - wave_b); the band grid has
 *   N = ceil((U - L)/spacing) equal intervals between its first and last sample
 *   with T interpolated linearly; h c = 6.62607015e-27 erg s x 2.99792458e18 A/s.
 *
 * Conventions for every call:
 *   - Device pointers belong to the caller, must stay valid until the work on
 *     the caller's stream has finished, and are never freed by the library.
 *   - Host pointers are read during the call only (the library copies).
 *   - All compute calls are asynchronous on the given HIP stream (NULL = the
 *     legacy default stream) and never synchronise it.
 *   - Errors are status codes; nothing crosses the ABI as an exception.
 *     sb_last_error() returns a thread-local message for the last failing call.
 *   - Arguments that can be checked on the host (null pointers, sizes, flags)
 *     are checked before anything is launched.  Conditions only the device can
 *     see (a band id >= the number of bands, a band window outside the surface,
 *     malformed CSR offsets) turn the affected results into NaN and set a sticky
 *     device flag that sb_device_check() reports.
 */
#ifndef SALTBF_H
#define SALTBF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SB_API_VERSION 1
#define SB_MAX_BANDS 64           /* band registry capacity per context */
#define SB_MAX_BAND_POINTS 2048   /* quadrature nodes per band */
#define SB_MAX_CL_DEGREE 8
#define SB_N_PARAMS 5             /* gradient order: z, t0, x0, x1, c */
#define SB_LATENCY_BINS 24        /* fit latency histogram bins (sb_stats_t) */

typedef int32_t sb_status;
enum {
  SB_OK = 0,
  SB_PENDING = 1,        /* fit not finished yet */
  SB_CANCELLED = 2,      /* fit cancelled before it finished */
  SB_FIT_DIVERGED = 3,   /* fit stopped: non-finite chi-square at its start */
  SB_ERR_ARG = -1,       /* invalid argument (checked on the host) */
  SB_ERR_RANGE = -2,     /* band window outside the surface, or bad band id / CSR (device flag) */
  SB_ERR_DEVICE = -3,    /* HIP runtime error */
  SB_ERR_NOMEM = -4,     /* device or host allocation failed */
  SB_ERR_BUDGET = -5,    /* fit request larger than the whole serving budget */
  SB_ERR_STATE = -6,     /* call not valid in the current state */
  SB_ERR_NOTFOUND = -7   /* unknown ticket (never issued, or its result was already taken) */
};

typedef struct sb_ctx sb_ctx;   /* opaque: device copies of model and bands, scratch, fit server */

/* SALT model surfaces and colour law (model equation).  m0/m1 are host arrays,
 * row-major [n_phase][n_wave] (phase-major, wavelength contiguous), copied at
 * sb_create.  Grid node (a, j) sits at phase phase0 + a*dphase (days) and rest
 * wavelength wave0 + j*dwave (Angstrom).  4 <= n_phase <= 256, 4 <= n_wave <= 8192.
 * cl_coef[0..cl_degree-1] are a_1..a_deg of CL (no constant term). */
typedef struct {
  int32_t n_phase, n_wave;
  double phase0, dphase, wave0, dwave;
  const float *m0, *m1;
  int32_t cl_degree;
  const double *cl_coef;
  double cl_wave_b, cl_wave_v;
} sb_model_desc;

/* Band quadrature rules on the grid of N equal intervals of width Delta <= max_spacing
 * between a band's first and last sample wavelengths.  Trapezoid (the bandflux
 * integral as the paper evaluates it, section "Implementation"): the N + 1
 * interval ends, weights Delta/2 at both ends and Delta inside.  Midpoint: the N
 * interval midpoints, weight Delta each. */
enum { SB_QUAD_TRAPEZOID = 0, SB_QUAD_MIDPOINT = 1 };

/* Library configuration; fill with sb_config_default() and override. */
typedef struct {
  double max_spacing;        /* quadrature spacing bound in Angstrom (default 5) */
  int32_t max_obs_per_fit;   /* observations per fit request (default 256, at most 1024) */
  int32_t max_slots;         /* fits resident on the device at once (default 1024) */
  int64_t hbm_budget_bytes;  /* device bytes the fit server may hold for requests (default 256 MiB) */
  int32_t iters_per_tick;    /* LM iterations per server launch (default 5) */
  int32_t fit_iters;         /* LM iterations per fit (default 50) */
  double lm_lambda0;         /* initial Marquardt damping (default 1e-3) */
  int32_t quad_rule;         /* band quadrature: SB_QUAD_TRAPEZOID (default, the paper's rule) or
                                SB_QUAD_MIDPOINT */
  int64_t lds_limit_bytes;   /* LDS a workgroup may use; 0 (default): the device's per-workgroup maximum.
                                Kernels run several waves per workgroup where that fits, else one;
                                bands whose one-wave form does not fit are refused by sb_add_band. */
  int32_t solver;            /* fit solver of the server and the batch fits: SB_SOLVER_LM (default) or
                                SB_SOLVER_LBFGSB */
  int32_t lbfgs_m;           /* L-BFGS-B correction pairs kept, 1..5 (default 5) */
} sb_config;

/* Fit solvers.  Both vary (t0, ln x0, x1, c) with z fixed and minimise
 * chi2 = sum_i (d_i - f_i)^2 / sigma_i^2 with cfg.fit_iters evaluations after the
 * one at the start.
 * SB_SOLVER_LM: Levenberg-Marquardt damped Gauss-Newton (see the fit server).
 * SB_SOLVER_LBFGSB: the bounded limited-memory quasi-Newton method of the
 *   paper's optimisation example (L-BFGS-B; Byrd, Lu, Nocedal and Zhu 1995):
 *   BFGS matrix from the last cfg.lbfgs_m correction pairs, generalized Cauchy
 *   point along the projected gradient path, subspace step cut back to the box,
 *   strong-Wolfe line search (1e-3, 0.9); bounds per fit (requests: has_bounds,
 *   lower, upper; batch fits: lower, upper arrays).  A held parameter (free_mask)
 *   is a variable whose two bounds equal its start. */
enum { SB_SOLVER_LM = 0, SB_SOLVER_LBFGSB = 1 };

void sb_config_default(sb_config *cfg);

/* Create a context on HIP device `device`: validates and uploads the surfaces
 * (as interleaved (M0, M1) float pairs, wavelength-major), prepares the band
 * registry.  cfg may be NULL for defaults.  On success *out owns device memory
 * until sb_destroy. */
sb_status sb_create(const sb_model_desc *model, const sb_config *cfg, int device, sb_ctx **out);

/* Stop the fit server (pending fits become SB_CANCELLED), free everything.
 * The caller must have finished all work it queued with this context. */
sb_status sb_destroy(sb_ctx *ctx);

/* Register a bandpass (the paper's bandpass registration): n >= 2 samples of
 * (wave [Angstrom, strictly increasing], trans >= 0), host arrays, copied.
 * Builds its quadrature grid (cfg.quad_rule, at most SB_MAX_BAND_POINTS nodes) and stores
 * lam_k and W_k = w_k lam_k T(lam_k)/(h c) in float32 on the device.
 * Synchronous.  Not allowed while compute calls of this context are in
 * flight.  *band_id receives 0, 1, 2, ... in registration order. */
sb_status sb_add_band(sb_ctx *ctx, const double *wave, const double *trans, int32_t n, int32_t *band_id);

/* Host-only helper (no context, no GPU): the quadrature grid sb_add_band builds
 * with rule (SB_QUAD_TRAPEZOID or SB_QUAD_MIDPOINT).  Writes at most cap nodes to
 * lam_out/weight_out (float32, weight = W_k above); *n_points receives the node
 * count.  SB_ERR_ARG if it exceeds cap. */
sb_status sb_band_grid(const double *wave, const double *trans, int32_t n, double max_spacing, int32_t rule,
                       int32_t cap, float *lam_out, float *weight_out, int32_t *n_points);

/* Bandpass files (the paper's bandpass loading from a file): a text file of two
 * numeric columns per line, wavelength [Angstrom] and transmission, separated by
 * spaces, tabs or a comma; '#' starts a comment; blank lines are skipped.  Host
 * only: reads at most cap rows into wave/trans, *n receives the row count.
 * SB_ERR_ARG if the file cannot be read, a line does not parse, or there are
 * more than cap rows (*n then holds the count needed). */
sb_status sb_read_band_file(const char *path, double *wave, double *trans, int32_t cap, int32_t *n);

/* sb_read_band_file followed by sb_add_band (at most 65,536 rows). */
sb_status sb_add_band_file(sb_ctx *ctx, const char *path, int32_t *band_id);

/* AB magnitude system: m_AB = -2.5 log10(f / F_AB), where F_AB is the bandflux
 * of the AB reference source, f_nu = 10^(-48.60/2.5) erg s^-1 cm^-2 Hz^-1 at
 * every frequency, through the band with the same quadrature as the model:
 * F_AB = sum_k w_k T_k f_nu / (h lam_k) (the lam/(hc) photon weight times
 * f_lam = f_nu c / lam^2).  Computed in FP64 at registration.
 * sb_band_zeropoint: the value for a registered band; sb_band_zeropoint_ab: the
 * same for band samples, host only (no context), with the given spacing and rule. */
enum { SB_MAGSYS_AB = 0 };
sb_status sb_band_zeropoint(sb_ctx *ctx, int32_t band_id, int32_t magsys, double *zp_flux);
sb_status sb_band_zeropoint_ab(const double *wave, const double *trans, int32_t n, double max_spacing,
                               int32_t rule, double *zp_flux);

/* Batch flags. */
enum {
  SB_OBS_BROADCAST = 1,  /* one observation table [n_obs] shared by all n_sn parameter samples */
  SB_OUT_CHI2 = 2,       /* sb_bandflux: write chi2 per supernova instead of fluxes;
                            sb_bandflux_vjp: cotangent = d chi2 / d f = 2 (f - data) inv_sigma2 */
  SB_PERSISTENT = 4      /* with SB_OBS_BROADCAST only (else SB_ERR_ARG): a persistent launch of a fixed
                            grid of G workgroups (16 per workgroup the device holds at once, at most
                            one per sample), workgroup g taking samples g, g + G, ..., instead of one
                            workgroup per sample; every result is bitwise the same */
};

/* A batch of supernovae in structure-of-arrays layout, all device pointers.
 * Supernova s has parameters z[s], t0[s], x0[s], x1[s], c[s] (z > -1).  A band
 * whose rest-frame window lam/(1+z) leaves the surface's wavelength grid, or
 * (only possible for z < -1/20) spans more surface columns than the context
 * sized its LDS for, cannot be evaluated: its observations give NaN and the
 * device flag that sb_device_check reports as SB_ERR_RANGE is set.
 * Without SB_OBS_BROADCAST its observations are i in [sn_offsets[s], sn_offsets[s+1])
 * (CSR, non-decreasing, sn_offsets[0] = 0, sn_offsets[n_sn] = n_obs), at time t[i]
 * (days, same origin as t0) through band band[i].  With SB_OBS_BROADCAST,
 * sn_offsets is ignored and every sample sees all n_obs observations.
 * data / inv_sigma2 ([n_obs]) are read only with SB_OUT_CHI2. */
typedef struct {
  int32_t n_sn, n_obs, flags;
  const float *z, *t0, *x0, *x1, *c;
  const float *t;
  const int32_t *band;
  const int32_t *sn_offsets;
  const float *data, *inv_sigma2;
} sb_batch;

/* Bandflux of every observation (the bandflux equation).
 * out: [n_obs] fluxes; with SB_OBS_BROADCAST [n_sn][n_obs]; with SB_OUT_CHI2
 * [n_sn] chi2_s = sum_i (f_i - data_i)^2 inv_sigma2_i.  One workgroup per
 * supernova, or, with SB_OBS_BROADCAST, per parameter sample (every sample
 * reads the one shared observation table); its waves build different bands. */
sb_status sb_bandflux(sb_ctx *ctx, const sb_batch *batch, float *out, void *hip_stream);

/* Forward pass plus adjoint: grad[s*5 + q] = sum_i gbar_i d f_i / d theta_s[q],
 * theta = (z, t0, x0, x1, c), where gbar_i = cotangent[i], or with SB_OUT_CHI2
 * gbar_i = 2 (f_i - data_i) inv_sigma2_i (cotangent must then be NULL).
 * grad is required ([n_sn*5]); flux_out ([n_obs], or [n_sn][n_obs] with
 * broadcast), jac_out ([n_obs][5], or [n_sn][n_obs][5]) and chi2_out ([n_sn],
 * SB_OUT_CHI2 only) may be NULL.  Each supernova's sums are reduced in a fixed
 * order (with at most 8 bands registered: per band over one wave's lanes, then over
 * its bands in band order by one thread; otherwise by one workgroup): results are
 * bitwise reproducible and do not depend on the rest of the batch.  With at most 8
 * bands the per-band sums live in a device workspace the context keeps per stream
 * (24 bytes per supernova and registered band), grown on demand: a call that must
 * grow it waits for the stream's earlier work, and is SB_ERR_STATE while the stream
 * is being captured into a graph (one call of the same size before the capture
 * sizes it). */
sb_status sb_bandflux_vjp(sb_ctx *ctx, const sb_batch *batch, const float *cotangent, float *grad,
                          float *flux_out, float *jac_out, float *chi2_out, void *hip_stream);

/* Wait for the context's work on hip_stream and report the sticky device
 * flags (SB_ERR_RANGE if any result was turned into NaN since the last call);
 * clears them.  Synchronises hip_stream. */
sb_status sb_device_check(sb_ctx *ctx, void *hip_stream);

/* ---------------------------------------------------------------- fit server
 * Continuous batching of light-curve fits (the paper's optimisation example):
 * each request is one supernova with z given and (t0, x0, x1, c) free, fitted by
 * cfg.fit_iters Levenberg-Marquardt damped Gauss-Newton iterations on
 * (t0, ln x0, x1, c) with weights 1/sigma^2, lambda0 = cfg.lm_lambda0, x10 on a
 * rejected step and /10 on an accepted one, lambda kept in [1e-9, 1e9].
 * A server thread admits queued requests while device slots and the byte budget
 * allow, runs cfg.iters_per_tick iterations of every resident fit per launch,
 * and retires finished fits; requests that arrive while others run join the next
 * launch.  Per-supernova state stays on the device between launches.  A fit's
 * result does not depend on which other fits share its launches. */
typedef struct {
  int32_t n_obs;             /* 1..cfg.max_obs_per_fit */
  const float *t;            /* host [n_obs], copied at submit */
  const int32_t *band;       /* host [n_obs] */
  const float *data, *sigma; /* host [n_obs], sigma > 0 */
  float z;                   /* fixed */
  float t0, x0, x1, c;       /* starting point, x0 > 0 */
  uint32_t free_mask;        /* parameters the fit varies: an OR of SB_FREE_*; 0 means SB_FREE_ALL.
                                The others stay at their starting values (the LM system is solved
                                over the free parameters only).  Other bits: SB_ERR_ARG. */
  int32_t has_bounds;        /* nonzero: lower/upper bound (t0, x0, x1, c) (SB_SOLVER_LBFGSB only,
                                else SB_ERR_ARG); +-inf for none, an x0 lower bound <= 0 is none,
                                an x0 upper bound must be > 0; lower <= upper.  A start outside
                                the box starts from its projection onto it. */
  float lower[4], upper[4];
} sb_fit_request;

enum { SB_FREE_T0 = 1, SB_FREE_X0 = 2, SB_FREE_X1 = 4, SB_FREE_C = 8, SB_FREE_ALL = 15 };

typedef struct {
  sb_status status;          /* SB_OK, SB_PENDING, SB_CANCELLED, SB_FIT_DIVERGED */
  float z, t0, x0, x1, c;    /* fitted parameters (z as given) */
  float chi2;                /* at the fitted parameters */
  int32_t iters;             /* LM iterations run */
  int32_t n_accept;          /* accepted steps */
  double t_submit, t_admit, t_done;  /* host monotonic clock, seconds */
} sb_fit_result;

/* Queue a request; never waits for the GPU.  SB_ERR_ARG for a malformed request
 * (sizes, band ids, non-finite values), SB_ERR_BUDGET if it alone exceeds the
 * byte budget.  *ticket identifies the result. */
sb_status sb_fit_submit(sb_ctx *ctx, const sb_fit_request *req, uint64_t *ticket);

/* SB_PENDING while the fit runs; otherwise fills *out, forgets the ticket and
 * returns SB_OK (out->status carries the fit's own status). */
sb_status sb_fit_poll(sb_ctx *ctx, uint64_t ticket, sb_fit_result *out);

/* Like sb_fit_poll but blocks up to timeout_s seconds (SB_PENDING on timeout). */
sb_status sb_fit_wait(sb_ctx *ctx, uint64_t ticket, double timeout_s, sb_fit_result *out);

/* Cancel a queued or running fit; its result becomes SB_CANCELLED. */
sb_status sb_fit_cancel(sb_ctx *ctx, uint64_t ticket);

/* ------------------------------------------------------------ batch fits
 * The same fit as the server's, run over a whole batch of supernovae already on
 * the device (throughput rather than latency: one call fits every light curve of
 * a survey batch).  Fit f has observations [fit_offsets[f], fit_offsets[f+1]) of
 * the CSR arrays t, band, data, inv_sigma2 (all device, as in sb_batch),
 * fixed redshift z[f], start (t0[f], x0[f] > 0, x1[f], c[f]) and free_mask[f]
 * (SB_FREE_* bits, 0 = all; the array may be NULL: all free).  The call enqueues
 * ceil(cfg.fit_iters / cfg.iters_per_tick) launches (at least one) on
 * hip_stream, each running cfg.iters_per_tick iterations of every fit, with each
 * fit's state kept in device scratch between launches; a fit's result is
 * bitwise the same whichever other fits share the call.  Malformed device
 * inputs (band ids, CSR offsets, band windows off the surface) give NaN results
 * and the sticky flags of sb_device_check. */
typedef struct {
  int32_t n_fit, n_obs;
  const float *z, *t0, *x0, *x1, *c;   /* device [n_fit] */
  const uint32_t *free_mask;           /* device [n_fit] or NULL */
  const float *t;                      /* device [n_obs] */
  const int32_t *band;                 /* device [n_obs] */
  const int32_t *fit_offsets;          /* device CSR [n_fit + 1] */
  const float *data, *inv_sigma2;      /* device [n_obs] */
  const float *lower, *upper;          /* device [n_fit][4] bounds of (t0, x0, x1, c) or NULL (none);
                                          SB_SOLVER_LBFGSB only (else SB_ERR_ARG); as in sb_fit_request,
                                          a fit whose bounds are malformed ends SB_FIT_DIVERGED */
} sb_fit_batch_desc;

/* One fit's result (device array [n_fit] written by the last launch). */
typedef struct {
  float t0, x0, x1, c;       /* fitted parameters (a held one as given) */
  float chi2;                /* at the fitted parameters */
  int32_t status;            /* SB_OK or SB_FIT_DIVERGED */
  int32_t iters;             /* iterations run */
  int32_t n_accept;          /* accepted steps */
} sb_fit_out;

/* Fits every supernova of the batch (see above).  The per-fit state scratch
 * (cfg-independent, about 400 bytes per fit) is allocated stream-ordered for the
 * call and released after its last launch.  Asynchronous; out must stay valid
 * until the stream reaches the end of the call's work.  SB_ERR_ARG for NULL
 * pointers or sizes; n_fit = 0 does nothing. */
sb_status sb_fit_batch(sb_ctx *ctx, const sb_fit_batch_desc *batch, sb_fit_out *out, void *hip_stream);

/* The same batch fit for callers that cannot allocate (code under HIP graph
 * capture, serving loops that must not call hipMalloc): identical results to
 * sb_fit_batch, with the per-fit state in a fixed device array that the library
 * holds on each GPU it runs on until the process ends (SB_FIT_NOALLOC_MAX fits,
 * about 400 bytes each, 3.2 MB).  It calls no allocation routine.  n_fit above
 * SB_FIT_NOALLOC_MAX is SB_ERR_ARG.  Every call on one GPU uses the same array:
 * calls whose work overlaps on a GPU (different streams, or different contexts
 * on the same device) race and must be serialised by the caller. */
#define SB_FIT_NOALLOC_MAX 8192
sb_status sb_fit_batch_noalloc(sb_ctx *ctx, const sb_fit_batch_desc *batch, sb_fit_out *out, void *hip_stream);

/* ------------------------------------------------------------ nested sampling
 * The paper's nested-sampling example (section "Implementation", the example
 * scripts): Skilling's nested sampling of one light curve's posterior, with
 * ln L(theta) = log_norm - chi2(theta)/2 over an observation table on the device
 * (t, band, data, inv_sigma2 [n_obs]) and independent priors on z, t0, x0, x1, c.
 * N live points; each iteration the lowest ln L becomes a dead point with prior
 * mass X_i = exp(-i/N) and log weight ln(X_{i-1} - X_i), and is replaced by a
 * draw from the prior restricted to L > L*; ln Z and the information H
 * accumulate; the run stops after max_iter dead points, at max_evals likelihood
 * evaluations, or when ln(Z + L_max X) - ln Z < dlogz; the live points then join
 * with ln weight ln(X_final / N).  Constrained draws: uniform in the unit cube
 * inside the live points' box widened by `enlarge` about its centre, mapped by
 * the prior transform, evaluated `batch` at a time by one broadcast chi-square
 * launch; candidates above L* are kept in draw order for the following
 * iterations.  Draw n's unit-cube coordinates are Philox4x64-10 outputs (counter
 * (n, d div 4, 0, 0), key (seed, 0x5A17BF1A5A17BF1A), output d mod 4, mapped to
 * ((x >> 11) + 1/2) 2^-53); draws 0..N-1 are the initial live points.  A sample
 * whose band windows leave the surface has ln L = -inf (and sets the range flag).
 * Synchronous: the host loop waits on hip_stream for every batch. */
enum { SB_PRIOR_FIXED = 0, SB_PRIOR_UNIFORM = 1, SB_PRIOR_LOG_UNIFORM = 2 };
typedef struct {
  int32_t kind;              /* fixed: value a; uniform on [a, b]; log-uniform on [a, b], 0 < a < b */
  double a, b;
} sb_prior;
typedef struct {
  sb_prior prior[5];         /* z, t0, x0, x1, c */
  int32_t n_live;            /* >= 2 */
  int32_t batch;             /* candidates per device evaluation, >= 1 */
  int64_t max_iter;          /* dead points at most (the dead_* outputs hold this many rows) */
  int64_t max_evals;         /* likelihood evaluations at most */
  double dlogz;              /* stopping tolerance on ln Z (0: run to max_iter or max_evals) */
  double enlarge;            /* box widening factor, >= 1 */
  uint64_t seed;             /* first key word of the draws */
  double log_norm;           /* constant of ln L */
} sb_ns_config;
typedef struct {
  double logz, logz_err, information;   /* ln Z, sqrt(H / N), H */
  int64_t n_iter, n_eval, n_batches;
  int32_t stopped_on_evals;
} sb_ns_summary;

/* Outputs are host arrays owned by the caller, each may be NULL: dead_theta
 * [max_iter][5], dead_logl, dead_logw, dead_draw [max_iter] (rows 0..n_iter-1
 * written); live_theta [n_live][5], live_logl, live_logw [n_live]. */
sb_status sb_nested_sampling(sb_ctx *ctx, const sb_ns_config *cfg, int32_t n_obs, const float *t, const int32_t *band,
                             const float *data, const float *inv_sigma2, double *dead_theta, double *dead_logl,
                             double *dead_logw, int64_t *dead_draw, double *live_theta, double *live_logl,
                             double *live_logw, sb_ns_summary *out, void *hip_stream);

/* Host-only: one Philox4x64-10 block (the draws' generator), for checking it. */
void sb_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);

/* ------------------------------------------------------------ peak probes
 * Micro-benchmarks of the rates a roofline is quoted against (the MI355X
 * datasheet gives 157.3 TFLOP/s vector FP32 with packed FP32 and 8 TB/s of
 * HBM), for the caller to time on the device at hand: one launch, on the
 * current device and hip_stream, of a kernel whose work is known exactly; *work
 * receives its FLOPs or bytes.
 *   SB_PROBE_FMA_F32   n workgroups of 256 threads; each thread runs 16
 *                      independent chains of `iters` FP32 fused multiply-adds
 *                      x <- x a + b (chain j starts at j; a = 1023/1024,
 *                      b = 1/1024), unpacked like every kernel of this library,
 *                      and writes the sum of its chains to dst[thread] (device
 *                      float [n * 256]); work = 2 * n * 256 * 16 * iters flops.
 *   SB_PROBE_LDS_READ  n workgroups of 256 threads; each fills a 16 KiB LDS table
 *                      of float4 T[i] = (i, i + 1/4, i + 1/2, i + 3/4) and reads
 *                      all of it `iters` times over (thread t, sweep k: entries
 *                      (t xor (k mod 256)) + 256 r, r = 0..3, conflict free), writing
 *                      the sum of the components it read to dst[thread] (device
 *                      float [n * 256]); work = n * iters * 16384 bytes.
 *   SB_PROBE_COPY      copies n bytes (a multiple of 16) from device src to dst with
 *                      non-temporal 128-bit loads and stores, one per thread;
 *                      work = 2 n bytes (read + write).
 * SB_ERR_ARG for an unknown kind, n < 1, iters < 1 (FMA, LDS), n above 2^23
 * workgroups (FMA, LDS), a NULL buffer or one not 16-byte aligned. */
enum { SB_PROBE_FMA_F32 = 0, SB_PROBE_LDS_READ = 1, SB_PROBE_COPY = 2 };
sb_status sb_peak_probe(int32_t kind, int64_t n, int32_t iters, const void *src, void *dst, double *work,
                        void *hip_stream);

typedef struct {
  int64_t submitted, admitted, completed, cancelled, rejected;
  int64_t ticks;               /* server launches */
  int32_t queue_depth;         /* waiting for admission */
  int32_t active_slots;        /* resident on the device */
  int64_t bytes_in_use, budget_bytes;
  double busy_seconds;         /* host time with at least one fit resident */
  int64_t slot_ticks;          /* fits run, summed over launches (slot_ticks / ticks: mean fits per launch) */
  int64_t latency_hist[SB_LATENCY_BINS];  /* completed fits by submit-to-done latency: bin k counts
                                             [2^k, 2^(k+1)) microseconds; bin 0 also everything below,
                                             the last bin everything above */
} sb_stats_t;

sb_status sb_stats(sb_ctx *ctx, sb_stats_t *out);

const char *sb_status_string(sb_status st);
const char *sb_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SALTBF_H */
