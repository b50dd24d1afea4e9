/*
 * ep_tv.h -- C ABI of the MI355X (gfx950) EP-TV image-restoration library.
 *
 * What it computes (Yao, McLaughlin, Altmann, "Fast Scalable Image Restoration
 * using Total Variation Priors and Expectation Propagation", arXiv 2110.01585):
 * Gaussian approximations Q(x) = N(mu, diag v) of the posterior of an image x
 * observed as y = H x + n, n ~ N(0, xi I) (Sec. II-A, Eq. (1)), under the
 * anisotropic l1-TV prior prod exp(-lambda |x_i - x_j|) over 4-neighbour pairs
 * (Sec. II-B, Eq. (L1_TV)).  EP keeps five diagonal Gaussian factors
 * (Sec. III-A): q_{x,0} for the likelihood and q_{x,k}, k = 1..4, one per colour
 * class V_k of pixel pairs (Fig. 1, Eq. (prior1)).  One sweep is Algorithm 1's
 * loop body: likelihood-site update (Eqs. (tilted_P_1), (update_q0_x)), then for
 * each V_k all pairs in parallel (Eqs. (marginal_tilted_un), (update_qk_x)), with
 * damping and the negative-variance clamp (Sec. III-C).  With EM on, lambda is
 * replaced after every sweep by N / a_bar_u (Algorithm 2, Eq.
 * (3rd_alternative_a0)), N = number of pixels.
 *
 * Conventions shared by every entry point:
 *  - Return value: int32 status, 0 = OK, > 0 = warning, < 0 = error (EP_TV_*).
 *    No C++ exception crosses this boundary.  After an error, ep_tv_last_error()
 *    on the same context returns a message.
 *  - "device pointer" = memory on the GPU the context was created on (e.g. a
 *    torch tensor's data_ptr()); "host pointer" = ordinary CPU memory.
 *  - The caller owns every buffer it passes.  The library never frees caller
 *    memory and never keeps a caller pointer beyond the call, except the
 *    workspace given to ep_tv_create, which must stay alive and untouched by the
 *    caller until ep_tv_destroy.
 *  - Images are row-major, dense, float32: pixel (r, c) of an H x W image is
 *    element r * W + c.  (EP_TV_OP_GAUSS_CS observations are M floats.)  Pixel arrays passed per instance are given as a host
 *    array of n_problems device pointers.
 *  - All GPU work is enqueued on the HIP stream given to ep_tv_create.  Calls
 *    documented as "asynchronous" return before the GPU has finished; calls
 *    that return host-visible results synchronise that stream.
 *  - A context is not thread-safe; use one per host thread.
 */
#ifndef EP_TV_H
#define EP_TV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  EP_TV_OK = 0,
  EP_TV_W_NOT_CONVERGED = 1,   /* ep_tv_solve hit max_sweeps before the tolerance */
  EP_TV_W_WARM_FALLBACK = 2,   /* a warm start was rejected and a cold start used */
  EP_TV_E_ARG = -1,            /* invalid argument (sizes, xi <= 0, damping, NULL) */
  EP_TV_E_OOM = -2,            /* workspace smaller than ep_tv_workspace_bytes() */
  EP_TV_E_HIP = -3,            /* a HIP runtime call failed */
  EP_TV_E_NONFINITE = -4,      /* NaN/Inf detected in the EP state */
  EP_TV_E_STATE = -5,          /* call out of order (e.g. solve before observation) */
  EP_TV_E_DIVERGED = -6        /* EP diverged: after a likelihood-site update the mean of the
                                  global approximation exceeded 1e3 times the scale of the
                                  pixel-space observation (max(range, max |.|) of y, or of H^T y
                                  for the transform operators) at some pixel.  EP has no
                                  convergence guarantee (Sec. III); the spectral variance
                                  estimator can run away on small images with sparse masks,
                                  where RBMC (EP_TV_VAR_RBMC) does not */
};

/* Degradation operator H (Sec. II-A, cases (i)-(iii)). */
enum {
  EP_TV_OP_IDENTITY = 0,       /* denoising: H = I */
  EP_TV_OP_BLUR_PERIODIC = 1,  /* deconvolution: periodic 2-D convolution with given taps */
  EP_TV_OP_DFT_MASK = 2,       /* CS: subset of orthonormal 2-D DFT coefficients */
  EP_TV_OP_HADAMARD_MASK = 3,  /* CS: subset of orthonormal 2-D Walsh-Hadamard coefficients,
                                  Paley order along each axis (Sec. II-A case (iii), Sec. V).
                                  DFT and Hadamard: power-of-two sides in [4, 4096] */
  EP_TV_OP_GAUSS_CS = 4        /* CS: a dense M x N sensing matrix (e.g. Gaussian i.i.d.,
                                  Sec. II-A case (iii), Sec. V) acting on the image flattened
                                  row-major.  The likelihood site's mean and variances come
                                  from the Woodbury identity (Sec. III-C: H^T H of rank M < N),
                                  in FP64 on the matrix cores; N = height*width <= 65536,
                                  M in [1, 32768] */
};

/* Image boundary for the pixel-pair graph.  FREE: pairs inside the image only;
 * PERIODIC: wrap-around pairs added (requires even height and width). */
enum { EP_TV_BND_FREE = 0, EP_TV_BND_PERIODIC = 1 };

/* Pixel-difference factor phi(x_i - x_j) of the TV prior (Sec. II-B):
 *   L1:   exp(-lambda |u|)                                    (Eq. (L1_TV));
 *   MOG2: omega N(u; 0, s1^2) + (1 - omega) N(u; 0, s2^2)     (Eq. (MoG2_TV_prior));
 *   BG:   omega N(u; 0, s^2) + (1 - omega) delta(u)           (Eq. (BG_TV)).
 * EM of the hyperparameters (Algorithm 2) is defined for L1 only; every
 * instance of a context uses the same kind. */
enum { EP_TV_PRIOR_L1 = 0, EP_TV_PRIOR_MOG2 = 1, EP_TV_PRIOR_BG = 2 };

/* One restoration problem.  Host pointers inside are read (copied) by
 * ep_tv_create only. */
typedef struct {
  int32_t height, width;       /* image size, each in [1, 16384] */
  int32_t op;                  /* EP_TV_OP_* */
  int32_t boundary;            /* EP_TV_BND_* */
  const float* blur_taps;      /* host, blur_h * blur_w row-major, odd sizes <= 17, centred:
                                  (Hx)(r,c) = sum_ab taps[a][b] x(r-a+blur_h/2, c-b+blur_w/2) */
  int32_t blur_h, blur_w;
  const uint8_t* dft_mask;     /* host, height*width, nonzero = coefficient observed (DFT_MASK:
                                  frequency (r, c); HADAMARD_MASK: Paley-ordered Walsh functions
                                  (r, c) of the rows and columns); the constant coefficient
                                  (0, 0) is always treated as observed */
  double noise_var;            /* xi > 0, variance of each real observation (DFT: of Re and Im) */
  double lambda0;              /* > 0: lambda (fixed, or the EM starting value) */
  double damping;              /* in (0, 1]: weight of the new site value in the damped update */
  double cg_tol;               /* CG relative residual ||r||/||b|| for the likelihood site; 0 = 1e-8 */
  int32_t cg_max_iters;        /* CG iteration cap per likelihood-site update; 0 = 50 */
  int32_t cg_precond;          /* EP_TV_PRECOND_*: CG preconditioner of the likelihood site */
  double cg_reduce;            /* in [0, 1): also stop a likelihood-site CG once its residual
                                  has fallen by this factor from where the solve started
                                  (inexact solves while EP is far from its fixed point; the
                                  cg_tol floor still holds near it).  0 = solve to cg_tol, as
                                  every earlier sweep's result then follows the exact-solve
                                  trajectory */
  int32_t prior;               /* EP_TV_PRIOR_*; lambda0 is the L1 lambda (still checked > 0
                                  for the mixtures, which do not use it) */
  int32_t var_estimator;       /* EP_TV_VAR_*: estimator of diag Cov of the likelihood site's
                                  tilted distribution (non-identity operators) */
  double prior_omega;          /* MOG2 / BG: omega in (0, 1] */
  double prior_s1sq;           /* MOG2: s1^2 > 0; BG: s^2 > 0 */
  double prior_s2sq;           /* MOG2: s2^2 > 0; BG: unused */
  int32_t rbmc_samples;        /* EP_TV_VAR_RBMC: samples Ns in [1, 64]; otherwise ignored */
  int32_t noise_map;           /* 1: non-i.i.d. noise, one variance per pixel, given by
                                  ep_tv_set_noise_variance (EP_TV_OP_IDENTITY only; Sec. III-C
                                  notes that the likelihood factor stays exact for denoising:
                                  q_{x,0} = N(y, diag(xi_i))); 0: i.i.d. noise of variance
                                  noise_var (which then only sets the range of valid inputs) */
  const float* sense_matrix;   /* EP_TV_OP_GAUSS_CS: host, sense_rows x (height*width),
                                  row-major; copied by ep_tv_create */
  int32_t sense_rows;          /* EP_TV_OP_GAUSS_CS: M */
  int32_t reserved;            /* 0 */
} ep_tv_problem;

/* Estimators of diag Cov_{P_0}, the tilted variances of the likelihood site
 * (Sec. III-C, Eq. (tilted_P_1); exact for H = I, where the choice is moot).
 *  SPECTRAL: the cavity precision replaced by its mean d: the covariance is then
 *    diagonal in the operator's transform basis with constant diagonal
 *    c = mean_w 1/(|H(w)|^2/xi + d), and the site precision is 1/c - d at every
 *    pixel.  Exact at constant cavity; one reduction per sweep.  On small images
 *    with sparse masks it can make EP diverge (EP_TV_E_DIVERGED).
 *  RBMC: the simple Rao-Blackwellised Monte Carlo estimator (Siden, Lindgren,
 *    Bolin, Villani 2018) the paper names for general H: with Q = H^T H/xi +
 *    diag(tau_c), v_i = 1/Q_ii + (1/Q_ii^2) mean_s (sum_{j!=i} Q_ij x_j^(s))^2
 *    over Ns samples x^(s) ~ N(0, Q^{-1}), each one CG solve of Q x = z with
 *    z = H^T e1/sqrt(xi) + sqrt(tau_c) e2 (perturbation-optimisation).  The
 *    white noise (e1, e2) is an input (ep_tv_set_rbmc_noise), fixed for the
 *    run, so EP converges to a fixed point of one estimator realisation.
 *    Unbiased, v_i >= 1/Q_ii; costs Ns extra CG solves per sweep; sweeps are
 *    launched one by one (EP_TV_OPT_GRAPH does not apply). */
enum { EP_TV_VAR_SPECTRAL = 0, EP_TV_VAR_RBMC = 1 };

/* Preconditioner of the likelihood-site CG.  CIRCULANT is (H^T H / xi + d I)^{-1}
 * with d the mean cavity precision, applied by FFT; it needs power-of-two sizes
 * in [4, 4096] and one FFT pipeline per instance, so JACOBI (the inverse
 * diagonal) suits batches of many small instances.  AUTO = CIRCULANT where the
 * sizes allow, else JACOBI. */
enum { EP_TV_PRECOND_AUTO = 0, EP_TV_PRECOND_JACOBI = 1, EP_TV_PRECOND_CIRCULANT = 2 };

/* Per-instance statistics (host struct filled by ep_tv_solve / ep_tv_get_stats). */
typedef struct {
  int32_t sweeps_done;         /* sweeps run on this instance since the last (re)initialisation */
  int32_t cg_iters_last;       /* CG iterations of the last likelihood-site update */
  int32_t cg_iters_total;      /* CG iterations since the last (re)initialisation */
  int32_t clamp_count;         /* site updates whose precision was clamped (Sec. III-C) */
  int32_t status;              /* EP_TV_OK, EP_TV_W_NOT_CONVERGED or an error code */
  int32_t converged;           /* 1 once the convergence rule of ep_tv_solve held */
  double lambda;               /* current lambda */
  double a_bar_u;              /* sum over the last sweep's edges of the tilted E|u| */
  double max_dmu_rel;          /* last sweep: max |mu_t - mu_{t-1}| / (max y - min y) */
  double max_dv_rel;           /* last sweep: max |v_t / v_{t-1} - 1| */
  double elapsed_ms;           /* wall time of the ep_tv_solve call (same for all instances) */
  double lik_precision;        /* last likelihood-site precision gamma (non-identity operators) */
  double cavity_precision_mean;/* mean cavity precision d_bar of the last likelihood-site update */
  double cg_rel_residual;      /* ||r|| / ||b|| at the end of the last CG solve */
  int32_t cold_restarts;       /* automatic cold restarts of ep_tv_solve (0 or 1) */
  int32_t reserved_;
} ep_tv_stats;

typedef struct ep_tv_ctx ep_tv_ctx;

/* Library version string (static storage). */
const char* ep_tv_version(void);

/* Bytes of device workspace a context for these problems needs (host out-param).
 * p: host array of n_problems descriptors, n_problems in [1, 4096]. */
int ep_tv_workspace_bytes(const ep_tv_problem* p, int32_t n_problems, size_t* bytes);

/* Create a context for n_problems independent instances solved together (one
 * batch; each instance keeps its own lambda, convergence flag and statistics).
 * d_workspace: device pointer, >= ep_tv_workspace_bytes() bytes, 256-byte aligned,
 *   owned by the caller, used exclusively by this context until ep_tv_destroy.
 * hip_stream: hipStream_t to enqueue on (NULL = default stream).
 * out: receives the context.  Validates every descriptor (EP_TV_E_ARG). */
int ep_tv_create(const ep_tv_problem* p, int32_t n_problems, void* d_workspace,
                 size_t ws_bytes, void* hip_stream, ep_tv_ctx** out);

/* Set the observations and (re)initialise every instance cold, as in the
 * initialisation line of Algorithm 1: q_{x,0} = N(H^T y, xi I) (for H = I or
 * blur, y itself), TV sites with variance 1e8 where a pair of V_k covers the
 * pixel, flat (0, 0) elsewhere; lambda = lambda0.  Asynchronous.
 * d_y: host array of n_problems device pointers.  IDENTITY/BLUR: height*width
 *   floats.  DFT_MASK: height*width complex values as interleaved (re, im)
 *   float pairs, the orthonormal 2-D DFT coefficients of x plus noise; entries
 *   off the mask are ignored.  HADAMARD_MASK: height*width floats, the
 *   orthonormal 2-D Walsh coefficients of x plus noise, Paley order (entry
 *   (u, v) belongs to the u-th row and v-th column Walsh functions); entries
 *   off the mask are ignored.  The data is copied; the caller may reuse y. */
int ep_tv_set_observation(ep_tv_ctx* ctx, const float* const* d_y);

/* White noise of the RBMC estimator (instances with var_estimator = RBMC),
 * required before the first sweep of such a context and kept until it is set
 * again.  d_noise: host array of n_problems device pointers (NULL for instances
 * without RBMC), each rbmc_samples * (K + H*W) floats: for every sample s, e1
 * in the observation layout of ep_tv_set_observation (K = H*W floats; for
 * DFT_MASK K = 2*H*W, interleaved (re, im), both parts N(0, 1)), then e2 (H*W
 * floats, pixel space), all standard normal draws of the caller.  The data is
 * copied (as H^T e1 and e2); the sample solutions restart from zero.
 * Asynchronous. */
int ep_tv_set_rbmc_noise(ep_tv_ctx* ctx, const float* const* d_noise);

/* Per-pixel noise variances of the instances with noise_map = 1 (required before
 * their first sweep).  d_var: host array of n_problems device pointers (NULL
 * for the other instances), each height*width floats > 0 (row-major).  The
 * data is copied (as precisions); if an observation is set, every instance is
 * re-initialised cold.  Asynchronous. */
int ep_tv_set_noise_variance(ep_tv_ctx* ctx, const float* const* d_var);

/* Re-run the cold initialisation with the stored observations.  Asynchronous. */
int ep_tv_init_cold(ep_tv_ctx* ctx);

/* Warm start from a predicted posterior N(mu_hat, diag var_hat) per instance
 * (e.g. the network of ep_tv_net.h).  The sites are set so that the global
 * approximation of Eq. (Q_x_final) equals the prediction: for H = I the
 * likelihood site keeps its exact value (1/xi, y/xi) and the remaining
 * precision (at least 1e-8 per class) and eta are split equally over the colour
 * classes covering the pixel; for the other operators precision and eta are
 * split equally over the likelihood site and the covering classes.  Uncovered
 * classes stay (0, 0).  The first sweep then updates the likelihood site too.
 * lambda_scale > 0 sets lambda_0 = lambda_scale * (N / a_x)^lambda_power, where
 * a_x is the sum over all pairs of E|x_i - x_j| under the prediction (option 1
 * of the approximations of a_0, Sec. IV-B; lambda_scale = lambda_power = 1 is
 * that option as is; other values correct its bias, e.g. as calibrated on
 * training data); lambda_scale <= 0 keeps lambda0 of the problem descriptor.
 * lambda_power must be > 0.
 * d_mu_hat, d_var_hat: host arrays of n_problems device pointers, height*width
 * floats each.  An instance whose prediction holds a non-finite value or a
 * variance <= 0 starts cold instead, and the call returns
 * EP_TV_W_WARM_FALLBACK.  Synchronises the stream. */
int ep_tv_init_warm(ep_tv_ctx* ctx, const float* const* d_mu_hat, const float* const* d_var_hat,
                    double lambda_scale, double lambda_power);

/* Run n_sweeps sweeps of Algorithm 1 on every active instance; with em_enabled,
 * lambda <- N / a_bar_u after every sweep (the fast EP-EM of Algorithm 2, one EP
 * iteration per EM iteration).  Asynchronous; no host synchronisation. */
int ep_tv_run(ep_tv_ctx* ctx, int32_t n_sweeps, int32_t em_enabled);

/* One iteration of Algorithm 2: n_ep_sweeps sweeps of Algorithm 1 at the
 * current lambda, then lambda <- N / a_bar_u from the last of those sweeps.
 * lambda_out: host array of n_problems doubles receiving the new lambdas, or NULL
 * (then the call is asynchronous). */
int ep_tv_em_step(ep_tv_ctx* ctx, int32_t n_ep_sweeps, double* lambda_out);

/* Sweep until every instance has converged or max_sweeps sweeps were run, then
 * write the marginals.  Convergence rule, checked after every sweep on the GPU:
 *   max|mu_t - mu_{t-1}| <= tol * (max y - min y)  and  max|v_t/v_{t-1} - 1| <= 10 tol
 *   and, with EM, |lambda_t / lambda_{t-1} - 1| <= tol.
 * A converged instance is frozen (no further sweeps).  tol <= 0 runs exactly
 * max_sweeps sweeps.  d_mean, d_var: host arrays of n_problems device pointers
 * (height*width floats each) or NULL to skip.  stats: host array of n_problems
 * or NULL.  Synchronises the stream.  Returns EP_TV_W_NOT_CONVERGED if any
 * instance did not converge (tol > 0), EP_TV_E_NONFINITE on NaN/Inf,
 * EP_TV_E_DIVERGED when the divergence rule held.  A failed instance is frozen
 * (its stats status says which).  An instance started from ep_tv_init_warm or
 * ep_tv_set_sites that goes non-finite or diverges is re-initialised cold once,
 * automatically, and keeps sweeping within max_sweeps; if it then converges,
 * its status is EP_TV_W_WARM_FALLBACK and so is the return value (when nothing
 * worse happened).  Failures are detected every 8 sweeps. */
int ep_tv_solve(ep_tv_ctx* ctx, int32_t max_sweeps, double tol, int32_t em_enabled,
                float* const* d_mean, float* const* d_var, ep_tv_stats* stats);

/* Write mu = eta/tau and v = 1/tau of the global approximation (Eq. (Q_x_final))
 * for every instance.  Asynchronous.  Arguments as in ep_tv_solve. */
int ep_tv_marginals(ep_tv_ctx* ctx, float* const* d_mean, float* const* d_var);

/* Copy the five sites out (checkpoint).  d_out: host array of n_problems device
 * pointers, each 10*height*width floats, planar in the order
 * tau_0, eta_0, tau_1, eta_1, ..., tau_4, eta_4 (natural parameters:
 * tau = 1/variance, eta = mean/variance).  Asynchronous. */
int ep_tv_get_sites(ep_tv_ctx* ctx, float* const* d_out);

/* Restore the five sites (resume) in the layout of ep_tv_get_sites, and the
 * lambdas (host array of n_problems doubles, or NULL to keep them).  Resets the
 * convergence flags and sweep counters.  Asynchronous. */
int ep_tv_set_sites(ep_tv_ctx* ctx, const float* const* d_in, const double* lambda);

/* Current per-instance statistics into a host array of n_problems.  Synchronises. */
int ep_tv_get_stats(ep_tv_ctx* ctx, ep_tv_stats* stats);

/* The tilted-moment step of the TV-site update on its own (Sec. III-C, Eq.
 * (marginal_tilted_un) with the l1-TV factor of Eq. (L1_TV)), exposed so its
 * device arithmetic can be checked in isolation.  For each of n differences
 * u ~ N(u; m[i], s[i]) exp(-lambda |u|) it writes rho[i] = 1 - Var/s[i],
 * delta[i] = E[u] - m[i] and eabs[i] = E|u|.  All arrays are device pointers of
 * n floats, s[i] > 0, lambda >= 0.  hip_stream as in ep_tv_create.
 * Asynchronous. */
int ep_tv_tilted_moments(int32_t n, const float* d_m, const float* d_s, float lambda,
                         float* d_rho, float* d_delta, float* d_eabs, void* hip_stream);

/* The same for any factor kind (Sec. III-C with Eqs. (L1_TV), (MoG2_TV_prior),
 * (BG_TV)): prior = EP_TV_PRIOR_*, theta a host array of its hyperparameters
 * ({lambda}, {omega, s1^2, s2^2} or {omega, s^2}, validated as in ep_tv_problem).
 * For the mixtures eabs is written as 0 (E|u| serves only the L1 EM).
 * Asynchronous. */
int ep_tv_tilted_moments_prior(int32_t prior, const double* theta, int32_t n, const float* d_m,
                               const float* d_s, float* d_rho, float* d_delta, float* d_eabs,
                               void* hip_stream);

/* Diagnostic copy of the likelihood-site working planes of one instance with
 * a non-identity operator (Eqs. (tilted_P_1), (update_q0_x)): d_out (device,
 * 10*height*width floats, planar) receives, in order, E (the CG iterate),
 * tau_c and eta_c (cavity of site 0), b = H^T y / xi + eta_c, the CG residual r,
 * the preconditioned residual z, |H(w)|^2 (frequency (r, c) at pixel (r, c)),
 * the two search-direction buffers and the last product q = A p.  Returns
 * EP_TV_E_ARG for an identity-operator instance.
 * Asynchronous. */
int ep_tv_get_lik_planes(ep_tv_ctx* ctx, int32_t instance, float* d_out);

/* Kernel timing for measurement.  With timing enabled, HIP events are recorded
 * on the context's stream around every launch of the fused TV sweep kernel and
 * around every likelihood-site update (its CG solve and site kernels), and
 * their durations are accumulated.  ep_tv_set_timing(ctx, 1) also clears the
 * totals.  ep_tv_get_timing synchronises and fills a host struct. */
typedef struct {
  double sweep_ms;             /* total GPU time of TV sweep kernel launches */
  int32_t sweep_launches;
  double lik_ms;               /* total GPU time of likelihood-site updates */
  int32_t lik_updates;
  double apply_ms;             /* total GPU time of the products with A inside CG (for blur
                                  instances with separable taps: the H^T H kernel alone) */
  int32_t apply_launches;
  double precond_ms;           /* total GPU time of the real-transform preconditioner of the
                                  circulant-preconditioned CG (with the fused x, r update) */
  int32_t precond_launches;
  /* single kernels of the likelihood-site update (every launch of each): the
   * three passes of the real 2-D transform (forward row pass with the fused
   * x, r update; column pass with the filter; inverse row pass with the r.z,
   * r.r partials), the per-instance finishing (reduction) kernels, and the
   * remaining element-wise kernels (cavity and right-hand side, spectral sum,
   * CG start, Jacobi steps, site update) */
  double rf_fwd_ms;  int32_t rf_fwd_launches;
  double rf_filt_ms; int32_t rf_filt_launches;
  double rf_inv_ms;  int32_t rf_inv_launches;
  double fin_ms;     int32_t fin_launches;
  double lik_other_ms; int32_t lik_other_launches;
  /* EP_TV_OP_GAUSS_CS: the FP64 GEMM launches of the Woodbury moments (S = xi I
   * + H D^-1 H^T, the Cholesky trailing updates, the blocked triangular solve)
   * and their floating-point operations */
  double dgemm_ms;   int32_t dgemm_launches;
  double dgemm_flops;
} ep_tv_timing;

int ep_tv_set_timing(ep_tv_ctx* ctx, int32_t enable);
int ep_tv_get_timing(ep_tv_ctx* ctx, ep_tv_timing* out);

/* Launch options of a context.
 *  EP_TV_OPT_GRAPH (0/1, default 0): run sweeps by replaying captured HIP
 *    graphs instead of launching kernel by kernel.  The sequences (likelihood
 *    head + CG iterations, further CG iterations, site update + TV sweep +
 *    finalisation; for identity operators, 8 whole sweeps) are captured on a
 *    private stream at first use and replayed on the context's stream; the
 *    results are identical to direct launches.  ep_tv_run / ep_tv_solve use it;
 *    ep_tv_em_step and timing always launch directly.
 *  EP_TV_OPT_TILE_ROWS (even, >= 2): rows per tile of the TV sweep (every
 *    tile is 124 interior columns wide).  Smaller heights than the workspace was
 *    sized for (the smaller of 8 and the initial height) return EP_TV_E_ARG.
 * Both synchronise the stream. */
enum { EP_TV_OPT_GRAPH = 1, EP_TV_OPT_TILE_ROWS = 2, EP_TV_OPT_EM_OPTION = 3, EP_TV_OPT_PERSISTENT = 4 };
/*  EP_TV_OPT_EM_OPTION (1, 2 or 3, default 3): the approximation of a_0 in the
 *    EM update lambda = N / a_0 (Sec. IV): 3 = Eq. (3rd_alternative_a0), the
 *    sum over the sweep's edges of the tilted E|u_n|; 2 = Eq. (eq:au), E|u_n|
 *    under Q(u_n) = N(m_bar_n, S_bar_n), the Gaussian with the tilted moments;
 *    1 = Eq. (eq:ax), E|x_i - x_j| under the global Q(x) after the sweep
 *    (an extra pass over the sites).  The paper adopts option 3; 1 and 2 are
 *    there to compare the estimates of lambda (its Fig. 4).
 *  EP_TV_OPT_PERSISTENT (0 or 1, default 0): launch the fused TV sweep as one
 *    resident grid (as many workgroups as the device holds at once) whose
 *    workgroups take the tile blocks of all instances in a fixed round-robin
 *    order, instead of one workgroup per tile block.  Results are bit-identical
 *    either way (no workgroup depends on another). */
int ep_tv_set_option(ep_tv_ctx* ctx, int32_t option, int64_t value);
int ep_tv_get_option(ep_tv_ctx* ctx, int32_t option, int64_t* value);

/* Autotuner of the TV-sweep tile height: times the sweep kernel (repeats
 * launches per candidate, HIP events, on the context's stream and current
 * state, which it leaves unchanged) for the even tile heights 8, 10, 12, 14, 16,
 * 18, 20, 24, 28, 32, 40, 48, 64, 96 and 128 rows (heights that give the same
 * tiling as a smaller one are skipped; heights that are not a power of two let
 * the tile count fit a whole number of rounds of resident waves), keeps the
 * fastest for this context and records it for later contexts with the same set
 * of image sizes in this process (ep_tv_workspace_bytes and ep_tv_create then
 * start from it).  Needs an observation.  Synchronises.  out (host) may be NULL. */
typedef struct {
  int32_t tile_rows;           /* chosen height */
  int32_t candidates;          /* entries used in rows / ms */
  int32_t rows[16];
  double ms[16];               /* mean sweep-kernel time per candidate */
  double best_ms;              /* time of the chosen height */
  double default_ms;           /* time of the height in use before tuning */
} ep_tv_tune_result;
int ep_tv_autotune(ep_tv_ctx* ctx, int32_t repeats, ep_tv_tune_result* out);

/* Denoising without any allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same computation as ep_tv_create for one
 * EP_TV_OP_IDENTITY instance (l1 prior, lambda0 = lambda), ep_tv_set_observation,
 * ep_tv_run(n_sweeps, em_enabled) and ep_tv_marginals, run on the same kernels,
 * with every working buffer in a 24 MiB device array of the library (one per GPU,
 * held until the process ends) instead of a caller workspace.  It calls no
 * allocating routine, host or device.
 * height, width: in [1, 512] (EP_TV_E_ARG beyond); boundary: EP_TV_BND_*;
 * noise_var > 0, lambda > 0, damping in (0, 1], n_sweeps >= 0.
 * d_y: device, height*width floats (read); d_mean, d_var: device, height*width
 * floats each (written).  hip_stream as in ep_tv_create.  Asynchronous.
 * Calls on one GPU share its array: calls that overlap on one GPU (other
 * streams or threads) race and give wrong results. */
int ep_tv_denoise_noalloc(int32_t height, int32_t width, int32_t boundary, double noise_var,
                          double lambda, double damping, int32_t n_sweeps, int32_t em_enabled,
                          const float* d_y, float* d_mean, float* d_var, void* hip_stream);

/* Message for the last error on this context ("" if none).  Static to the ctx. */
const char* ep_tv_last_error(const ep_tv_ctx* ctx);

/* Destroy the context.  Frees only what the library allocated for itself. */
void ep_tv_destroy(ep_tv_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* EP_TV_H */
