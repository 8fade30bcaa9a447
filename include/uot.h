/*
 * uot.h - C ABI of libuot.so: entropic KL-unbalanced optimal transport on AMD Instinct
 * MI355X (gfx950), plain Sinkhorn and translation-invariant (TI) Sinkhorn.
 *
 * Method: Sejourne, Vialard, Peyre, "Faster Unbalanced Optimal Transport: Translation
 * invariant Sinkhorn and 1-D Frank-Wolfe", AISTATS 2022.
 *
 * Problem (Sec. 1, eq. primal-uot-kl, with D_phi = rho KL):
 *   UOT(alpha, beta) = inf_{pi >= 0} <pi, C> + eps KL(pi | alpha x beta)
 *                      + rho1 KL(pi 1 | alpha) + rho2 KL(pi^T 1 | beta)
 * and its dual (eq. dual-uot-kl), UOT = sup_{f,g} F_eps(f, g) with
 *   F_eps(f, g) = rho1 <alpha, 1 - e^{-f/rho1}> + rho2 <beta, 1 - e^{-g/rho2}>
 *                 - eps <alpha x beta, e^{(f + g - C)/eps} - 1>.
 * The optimal plan is pi_ij = alpha_i beta_j exp((f_i + g_j - C_ij)/eps).
 *
 * Conventions shared by every entry point
 *  - All array pointers are DEVICE pointers (memory returned by hipMalloc or a PyTorch
 *    CUDA/HIP tensor) unless the comment says (host). The caller owns all memory; the
 *    library never frees or retains a caller pointer after the call returns.
 *  - Arrays are float32, dense and row-major unless stated; sizes are element counts.
 *  - `stream` is a hipStream_t (NULL = the default stream). Work is ordered on it.
 *  - Scalars eps, rho1, rho2, p are double in the ABI and are rounded once to the
 *    working precision on the device; masses, lambda*, convergence tests and the dual
 *    value are accumulated in double precision.
 *  - Errors are reported by return code only (no exceptions, no abort). Arguments that
 *    can be checked on the host are validated before any launch; then outputs are left
 *    untouched. Weight arrays are checked on the device by the first kernel of a call
 *    (negative, NaN or infinite weights, or a zero total mass, give UOT_ERR_INVALID and
 *    leave the caller's outputs untouched).
 *  - Workspace: every call that needs scratch memory takes `workspace` and its size
 *    `workspace_bytes`. Query the size with uot_workspace_bytes(). A NULL workspace makes
 *    the call allocate (and free) its own with hipMalloc; a non-NULL workspace smaller
 *    than required gives UOT_ERR_WORKSPACE. The workspace must not be shared by calls
 *    that may run concurrently.
 *  - Calls that return a host value (info, value) synchronise `stream` before returning.
 *  - Two calls on different streams with different workspaces may run concurrently; the
 *    library keeps no global mutable state besides a per-device kernel-shape cache that
 *    is guarded by a mutex.
 */
#ifndef UOT_H_
#define UOT_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  UOT_OK = 0,
  UOT_ERR_INVALID = 1,   /* bad argument (sizes, pointers, eps/rho/p, weights)             */
  UOT_ERR_HIP = 2,       /* a HIP runtime call failed (message in uot_last_error())        */
  UOT_ERR_NUMERIC = 3,   /* non-finite potentials or value were produced                   */
  UOT_ERR_WORKSPACE = 4  /* workspace too small                                             */
} uot_status;

typedef enum {
  UOT_COST_DENSE = 0,    /* C given as a stored matrix                                      */
  UOT_COST_POINTS = 1    /* C_ij = ||x_i - y_j||_2^p evaluated on the fly                   */
} uot_cost_kind;

/*
 * Cost description (Sec. 1: C in R^{n x m}, or C_ij = d(x_i, y_j)^p built from points).
 *  kind = UOT_COST_DENSE:  C points to n rows of ldc floats (row-major, ldc >= m); only
 *                          the first m entries of each row are read. x, y, d, p unused.
 *  kind = UOT_COST_POINTS: x is [n, d], y is [m, d] (row-major float32), 1 <= d <= 64,
 *                          p >= 1 (p = 2 is the squared Euclidean cost and takes the
 *                          fastest path). C and ldc unused.
 *                          Accuracy of p = 2: by default the solvers' softmins evaluate
 *                          the exponent in the expanded form |x|^2 + |y|^2 - 2<x, y> on
 *                          points centred on their common mean (matrix cores), whose
 *                          float32 rounding is about E = 2^-24 (d + 4) (max|x - mu| +
 *                          max|y - mu|)^2 per softmin in potential units, i.e.
 *                          delta = E log2(e) / eps in the exponent. The solvers switch to
 *                          direct differences x - y (vector ALU, as uot_set_points_kernel(4))
 *                          by themselves where that rounding could reach the 1e-5 relative
 *                          accuracy of the potentials: delta > 3e-4 and
 *                          E min(max_iter, 1 / (1 - k1 k2)) / min(|f|_inf, |g|_inf) > 3e-5,
 *                          with k_i = rho_i / (eps + rho_i) and the norms read after the
 *                          first iteration. A solve to a tolerance (tol > 0, no Anderson
 *                          extrapolation, KL entropy) then keeps the expanded form while its
 *                          change is above max(100 tol, E) (or until that change stops
 *                          falling near that point) and finishes in the direct form from
 *                          those potentials; any other solve restarts in the direct
 *                          form (uot_info.points_form says which form ran). uot_dual_value takes
 *                          the direct form for p = 2; the backward and the marginals form the
 *                          exponent in double precision.
 * n (size of alpha, the "source" side) and m (size of beta) are >= 1.
 */
typedef struct {
  int32_t kind;
  int32_t n, m, d;
  const float *C;
  int64_t ldc;
  const float *x;
  const float *y;
  double p;
} uot_cost;

/*
 * Solver parameters.
 *  eps > 0         entropic regularisation (Sec. 1)
 *  rho1, rho2 > 0  KL penalty weights on the first and second marginal (finite)
 *  max_iter >= 1   iteration cap; one iteration = one g-update then one f-update (Sec. 3)
 *  tol >= 0        stop at the first iteration t with t % check_every == 0 and
 *                  max(||f_t - f_{t-1}||_inf, ||g_t - g_{t-1}||_inf) < tol, measured on
 *                  the reported (translated) potentials; tol = 0 runs exactly max_iter
 *  check_every>=1  period of the convergence test
 *  warm_start      0: start from f_0 = 0; 1: read the starting f_0 from the f argument
 *                  (for TI the start is the translation-invariant potential fb_0; passing
 *                  the f returned by an earlier TI call resumes that run)
 */
typedef struct {
  double eps, rho1, rho2;
  int32_t max_iter;
  double tol;
  int32_t check_every;
  int32_t warm_start;
} uot_params;

/* Per-call report (host). */
typedef struct {
  int32_t iters;        /* iterations run                                                  */
  int32_t converged;    /* 1 if the tol test passed, else 0 (max_iter reached or tol = 0)  */
  double last_change;   /* the change measured at the last iteration (inf after one)       */
  double lambda;        /* TI: lambda*(fb, gb) of Prop. 2 at the last iterate; plain: 0    */
  int32_t points_form;  /* p = 2 points cost: the exponent form the softmins used, 0 the
                           expanded form on centred points, 1 direct differences (see
                           uot_set_points_kernel), 2 the expanded form and then direct
                           differences to the tolerance (iters counts both); -1 for other
                           costs                                                            */
} uot_info;

enum {
  UOT_WS_SOLVE = 0,     /* uot_sinkhorn, uot_ti_sinkhorn                                   */
  UOT_WS_DUAL = 1,      /* uot_dual_value                                                  */
  UOT_WS_PLAN = 2,      /* uot_plan_apply (size independent of k up to k = 64)             */
  UOT_WS_BACKWARD = 3,  /* uot_backward                                                    */
  UOT_WS_ANDERSON = 4   /* uot_sinkhorn_anderson, uot_ti_sinkhorn_anderson (any k <= 8)    */
};

/* Workspace bytes needed by the entry point `which` for this cost (0 on invalid input). */
size_t uot_workspace_bytes(const uot_cost *cost, int32_t which);

/*
 * Plain (F-) Sinkhorn of Sec. 3 for rho KL penalties: alternate exact maximisation of
 * F_eps, in the log domain:
 *   g_j <- rho2/(eps+rho2) * Smin_alpha^eps(C_{:,j} - f)
 *   f_i <- rho1/(eps+rho1) * Smin_beta^eps(C_{i,:} - g)
 * with Smin_w^eps(h) = -eps log sum_k w_k exp(-h_k/eps) (the softmin of Sec. 3) and the
 * KL anisotropic prox x -> rho/(eps+rho) x.
 *  alpha [n], beta [m]: nonnegative weights (zero weights allowed; a zero weight removes
 *                       its point from every sum), any total masses > 0.
 *  f [n]: in (if warm_start) / out; g [m]: out. The dual potentials of the last iterate.
 *  info (host, may be NULL): iterations, convergence flag, last change.
 */
uot_status uot_sinkhorn(const uot_cost *cost, const float *alpha, const float *beta,
                        const uot_params *params, float *f, float *g, void *workspace,
                        size_t workspace_bytes, uot_info *info, void *stream);

/*
 * Translation-invariant (H-) Sinkhorn of Sec. 3 (Prop. 4) for general rho1, rho2 (App. B,
 * eq. general-iter-h-sink): alternate maximisation of H_eps(fb, gb) = sup_lambda
 * F_eps(fb + lambda, gb - lambda), each half-step a softmin followed by the KL prox and a
 * scalar translation computed from the tilted mass <alpha, e^{-fb/rho1}> (resp. beta).
 * Same arguments and conventions as uot_sinkhorn. The returned f, g are the translated
 * potentials Phi(fb, gb) = (fb + lambda*, gb - lambda*) with lambda* of Prop. 2, i.e. the
 * F-potentials, which converge to the same unique optimum as plain Sinkhorn.
 */
uot_status uot_ti_sinkhorn(const uot_cost *cost, const float *alpha, const float *beta,
                           const uot_params *params, float *f, float *g, void *workspace,
                           size_t workspace_bytes, uot_info *info, void *stream);

/* Anderson extrapolation settings (see uot_sinkhorn_anderson). */
typedef struct {
  int32_t k;          /* iterations per extrapolation = residuals in the mix, 2 <= k <= 8     */
  double r;           /* regularisation added to the Gram matrix, finite and > 0             */
  int32_t normalize;  /* 0: the appendix's form, G = U^T U; 1: G = U^T U / ||U^T U||_F       */
} uot_anderson;

/*
 * Plain or translation-invariant Sinkhorn with Anderson extrapolation (appendix on
 * combining Sinkhorn with Anderson acceleration). The iterated variable x is f for plain
 * Sinkhorn and fb for TI; one iteration T maps x to the next x through a g-step and an
 * f-step as in uot_sinkhorn / uot_ti_sinkhorn. From x_0, k iterations give x_1 .. x_k, the
 * residuals u_i = x_{i+1} - x_i form U, and, with G = U^T U,
 *   c = (G + r I)^{-1} 1 / (1^T (G + r I)^{-1} 1),   x <- sum_i c_i x_{i+1},
 * after which the next k iterations start from the extrapolated x. No extrapolation
 * follows the last iteration (max_iter), and the change of the first iteration after an
 * extrapolation is +inf, so the stopping test always compares two plain iterates. The
 * paper's experiment uses k = 4, r = 1e-7. With acc->normalize = 1, G is divided by its
 * Frobenius norm before r is added, which makes r relative to the residuals: with the
 * appendix's form a fixed r turns the weights into a plain average once the residuals are
 * small against sqrt(r), so the extrapolation stops helping near the optimum (on the 1-D
 * measures of Sec. 3 with k = 4, r = 1e-7: TI 110 iterations to a change below 1e-6 with
 * the appendix's form, as many as without extrapolation, against 20 normalised).
 * Arguments and conventions as uot_sinkhorn (params.warm_start gives x_0 = f for plain
 * Sinkhorn and fb = f for TI); acc (host) holds k, r and normalize, and k outside 2..8, r
 * not finite and > 0, or normalize not 0 or 1 give UOT_ERR_INVALID. The workspace is UOT_WS_ANDERSON's (the iterates of one
 * cycle, k + 1 vectors of n floats, beside the solver's own). A Gram system that cannot be
 * solved (non-finite entries) ends the solve with UOT_ERR_NUMERIC.
 */
uot_status uot_sinkhorn_anderson(const uot_cost *cost, const float *alpha, const float *beta,
                                 const uot_params *params, const uot_anderson *acc, float *f,
                                 float *g, void *workspace, size_t workspace_bytes,
                                 uot_info *info, void *stream);
uot_status uot_ti_sinkhorn_anderson(const uot_cost *cost, const float *alpha, const float *beta,
                                    const uot_params *params, const uot_anderson *acc, float *f,
                                    float *g, void *workspace, size_t workspace_bytes,
                                    uot_info *info, void *stream);

/* Marginal penalties and Sinkhorn variant of uot_sinkhorn_phi. */
enum {
  UOT_ENTROPY_KL = 0,    /* rho KL: phi*(x) = rho (e^{x/rho} - 1)                              */
  UOT_ENTROPY_BERG = 1   /* Berg: phi(x) = rho (x - 1 - log x), phi*(x) = -rho log(1 - x/rho)  */
};
enum {
  UOT_SINKHORN_F = 0,    /* alternate maximisation of F_eps (plain Sinkhorn)                  */
  UOT_SINKHORN_G = 1     /* alternate maximisation of G_eps(fb, gb, lambda) (G-Sinkhorn)       */
};
typedef struct {
  int32_t entropy;  /* UOT_ENTROPY_*, the same for both marginals (rho1, rho2 may differ)       */
  int32_t variant;  /* UOT_SINKHORN_*                                                          */
} uot_phi;

/*
 * Sinkhorn for a smooth entropy phi* (Sec. 3): the F-Sinkhorn updates with the dual update
 * U_i(S) = -aprox_{phi_i*}(-S), the root h of e^{(h - S)/eps} = phi_i*'(-h), i.e.
 *   g <- U_2(Smin_alpha^eps(C - f)),   f <- U_1(Smin_beta^eps(C - g))
 * (KL: U(S) = rho/(eps + rho) S, which is uot_sinkhorn; Berg: h > -rho solving
 * e^{(h - S)/eps} = rho / (rho + h), by Newton's method in log(rho + h), per point). The
 * G-Sinkhorn variant alternates maximisation of G_eps(fb, gb, lambda) = F_eps(fb + lambda,
 * gb - lambda) over gb, fb and lambda; equivalently, each iteration is the F-iteration above
 * from f = fb + lambda followed by the translation (f, g) -> (f + l*, g - l*) with
 * l* = lambda*(f, g), the root of <alpha, phi1*'(-f - l)> = <beta, phi2*'(-g + l)> (closed
 * form of Prop. 2 for KL; a bracketed Newton iteration over the potentials for Berg). The
 * reported f, g are the F-potentials (fb + lambda, gb - lambda); info->lambda is G's
 * lambda_t = lambda*(fb_t, gb_t), the sum of those steps (0 for F). Arguments and
 * conventions as uot_sinkhorn (warm_start gives f_0 = fb_0, lambda_0 = 0);
 * phi (host): entropy and variant, anything else gives UOT_ERR_INVALID. Workspace
 * UOT_WS_SOLVE.
 */
uot_status uot_sinkhorn_phi(const uot_cost *cost, const float *alpha, const float *beta,
                            const uot_params *params, const uot_phi *phi, float *f, float *g,
                            void *workspace, size_t workspace_bytes, uot_info *info,
                            void *stream);

/*
 * Dual value F_eps(f, g) of eq. (dual-uot-kl), which equals UOT(alpha, beta) at the
 * optimal potentials. m(pi) is obtained from one row-softmin pass over C:
 * m(pi) = sum_i alpha_i exp((f_i - Smin_beta^eps(C_{i,:} - g))/eps).
 *  f [n], g [m]: potentials; value (host): result. Synchronises the stream.
 */
uot_status uot_dual_value(const uot_cost *cost, const float *alpha, const float *beta, double eps,
                          double rho1, double rho2, const float *f, const float *g, void *workspace,
                          size_t workspace_bytes, double *value, void *stream);

/*
 * Plan application with pi_ij = alpha_i beta_j exp((f_i + g_j - C_ij)/eps), pi never stored:
 *  transpose = 0: out[i, c] = sum_j pi_ij V[j, c],  V is [m, k] (leading dim ldv >= k),
 *                 out is [n, k] (leading dim ldout >= k)
 *  transpose = 1: out[j, c] = sum_i pi_ij V[i, c],  V is [n, k], out is [m, k]
 * 1 <= k <= 64. V = NULL means a column of ones (k must be 1): the marginals pi 1 and
 * pi^T 1 of Sec. 1. Each output row is computed with its own running max of the exponent,
 * so pi V is exact up to rounding even where individual entries of e^{f+g-C} overflow.
 * One pass over the cost per 16 columns of V, one exp2 per entry, V applied on the float32
 * matrix cores: points costs up to dimension 16 through the backward's kernel (exponent in
 * double precision), stored costs with the float32 exponent of the stored-cost softmins.
 * Points costs above dimension 16 (and every cost under uot_set_grad_kernel(1)) take a
 * float32 exponent with two exp2 per entry and 4 columns per pass.
 */
uot_status uot_plan_apply(const uot_cost *cost, const float *alpha, const float *beta, double eps,
                          const float *f, const float *g, int32_t transpose, const float *V,
                          int32_t k, int64_t ldv, float *out, int64_t ldout, void *workspace,
                          size_t workspace_bytes, void *stream);

/*
 * Envelope-theorem gradients of UOT = sup F_eps at the given (converged) potentials,
 * each multiplied by grad_out (the partial derivatives of eq. dual-uot-kl, pi recomputed
 * tile by tile and never stored):
 *   dalpha_i = rho1 (1 - e^{-f_i/rho1}) - eps (sum_j beta_j e^{(f_i+g_j-C_ij)/eps} - m(beta))
 *   dbeta_j  = rho2 (1 - e^{-g_j/rho2}) - eps (sum_i alpha_i e^{(f_i+g_j-C_ij)/eps} - m(alpha))
 *   dx_i     = sum_j pi_ij p ||x_i - y_j||^{p-2} (x_i - y_j)     (points cost only)
 *   dy_j     = sum_i pi_ij p ||x_i - y_j||^{p-2} (y_j - x_i)     (points cost only)
 * (the gradient of ||x - y||^p is taken as 0 at x = y).
 * dx [n, d], dy [m, d], dalpha [n], dbeta [m]: outputs; any may be NULL (dx, dy must be
 * NULL for a dense cost).
 */
uot_status uot_backward(const uot_cost *cost, const float *alpha, const float *beta, double eps,
                        double rho1, double rho2, const float *f, const float *g, double grad_out,
                        float *dx, float *dy, float *dalpha, float *dbeta, void *workspace,
                        size_t workspace_bytes, void *stream);

/*
 * uot_backward without any allocation, for callers that cannot allocate (code under HIP
 * graph capture, tight serving or training loops, harnesses that forbid hipMalloc): the same
 * kernels and results as uot_backward, with its workspace taken from a scratch array of
 * UOT_NOALLOC_BYTES (96 MiB) that the library keeps in device memory on every GPU it runs on,
 * from the library's load until the process ends. The array's address on a device is looked
 * up on the first call made with that device current. The call allocates nothing: no
 * hipMalloc, hipFree or host allocation, and no kernel timing (uot_profile_* does not apply).
 *  - Limit: a problem whose UOT_WS_BACKWARD workspace (uot_workspace_bytes) exceeds
 *    UOT_NOALLOC_BYTES gives UOT_ERR_WORKSPACE before any launch; with points that is above
 *    n = m = 228,000 at D = 3 and above n = m = 70,000 at D = 16.
 *  - The array keeps the last call's contents; each call writes every scratch value it reads,
 *    so nothing has to start cleared.
 *  - Every call on one GPU uses that GPU's one array: calls that overlap on one GPU (other
 *    streams, other host threads) race on it and must be serialised by the caller.
 * Arguments, outputs and error behaviour otherwise as uot_backward.
 */
#define UOT_NOALLOC_BYTES ((size_t)96 << 20)
uot_status uot_backward_noalloc(const uot_cost *cost, const float *alpha, const float *beta,
                                double eps, double rho1, double rho2, const float *f,
                                const float *g, double grad_out, float *dx, float *dy,
                                float *dalpha, float *dbeta, void *stream);

/* Per-problem outcome of uot_ti_sinkhorn_batched (the status array). */
enum {
  UOT_BATCH_CONVERGED = 0,  /* the tol test passed                                           */
  UOT_BATCH_MAX_ITER = 1,   /* max_iter reached first (or tol = 0)                           */
  UOT_BATCH_INVALID = 2,    /* bad weights (negative, NaN, inf, zero mass) or eps/rho <= 0    */
  UOT_BATCH_NUMERIC = 3     /* non-finite potentials                                          */
};

/*
 * Many independent KL-UOT problems with point costs, solved together by translation-
 * invariant Sinkhorn (Sec. 3, Prop. 4 / App. B), each to its own convergence. Problem b
 * owns points [offN[b], offN[b+1]) of x/alpha/f and [offM[b], offM[b+1]) of y/beta/g
 * (every problem has at least one point on each side).
 *  B >= 1; offN, offM (host) [B+1], offN[0] = offM[0] = 0, nondecreasing.
 *  d in [1, 8]; p >= 1 (p = 2: squared Euclidean cost; otherwise ||x - y||^p).
 *  x [offN[B], d], y [offM[B], d], alpha [offN[B]], beta [offM[B]] (device, float32).
 *  eps, rho1, rho2 (device, double) [B]: per-problem parameters (> 0, finite).
 *  max_iter, tol, check_every: as in uot_params, applied to every problem; a problem stops
 *  at its own first passing check (or at max_iter) while the others continue.
 *  f [offN[B]], g [offM[B]] (device, out): the translated potentials of each problem.
 *  iters, status (device, int32 [B], out): iterations run and UOT_BATCH_* outcome.
 * p = 2: each problem whose expanded-form rounding E (as for uot_cost, from its own spread)
 * satisfies E log2(e) / eps_b <= 3e-4 takes its exponents in the expanded form; the others
 * through the differences x - y.
 * All problems advance together one half-step per kernel launch; a wave takes one chunk of
 * targets of one problem at a time (up to 256, 128 or 64 targets, or 64 targets against a
 * range of the sources, by a work-item plan tuned per size signature) from a shared
 * counter over the problems still running, so the work follows the active problems as they
 * converge. A chunk of iterations
 * is captured once as a HIP graph and replayed until every problem has stopped.
 * Returns UOT_OK when every problem has an outcome (check the status array); bad host
 * arguments give UOT_ERR_INVALID before any launch.
 */
uot_status uot_ti_sinkhorn_batched(int32_t B, const int64_t *offN, const int64_t *offM, int32_t d,
                                   double p, const float *x, const float *y, const float *alpha,
                                   const float *beta, const double *eps, const double *rho1,
                                   const double *rho2, int32_t max_iter, double tol,
                                   int32_t check_every, float *f, float *g, int32_t *iters,
                                   int32_t *status, void *workspace, size_t workspace_bytes,
                                   void *stream);

/*
 * Frank-Wolfe for unregularised (eps = 0) KL-UOT between 1-D measures (Sec. 4), for B
 * independent problems at once. Problem b owns the points [offN[b], offN[b+1]) of x/alpha/f
 * and [offM[b], offM[b+1]) of y/beta/g; its supports must be sorted ascending. The method
 * is Frank-Wolfe on H_0(fb, gb) = sup_lambda F_0(fb + lambda, gb - lambda) over fb (+) gb <= C,
 * C_ij = |x_i - y_j|^p, from (0, 0): each iteration forms the gradient of H_0, the tilted
 * histograms alpha e^{-(fb + l)/rho1} and beta e^{-(gb - l)/rho2} with l = lambda*(fb, gb)
 * (Prop. 2; equal masses), takes the linear oracle (r, s) = the dual solution of balanced
 * 1-D OT between them (the monotone coupling; its walk's cells are tight), and steps
 * (fb, gb) <- (1 - gamma)(fb, gb) + gamma (r, s) with gamma = 2/(2 + t) (line_search = 0) or
 * the maximiser of H_0 on the segment (line_search = 1). The Frank-Wolfe gap
 * <grad H_0, (r, s) - (fb, gb)> bounds H_0* - H_0(fb, gb); an iteration whose gap is <= tol
 * (tol > 0) ends that problem before its step, otherwise it runs max_iter iterations.
 *  B >= 1; offN, offM (host) [B+1] as in uot_ti_sinkhorn_batched.
 *  x [offN[B]], y [offM[B]], alpha [offN[B]], beta [offM[B]] (device, float32).
 *  rho1, rho2 (device, double) [B]; p >= 1 (host).
 *  f [offN[B]], g [offM[B]] (device, out): the reported potentials (fb + l*, gb - l*).
 *  iters (device, int32 [B], out): iterations run (linear-oracle calls); gap (device,
 *  double [B], out): the last gap; status (device, int32 [B], out): UOT_BATCH_* (INVALID:
 *  unsorted support, bad weights or penalties; its f, g are NaN).
 * Everything runs in double precision; one workgroup owns one problem at a time and runs all
 * of its iterations in one launch. Workspace: uot_fw1d_workspace_bytes.
 */
uot_status uot_fw1d_batched(int32_t B, const int64_t *offN, const int64_t *offM, const float *x,
                            const float *y, const float *alpha, const float *beta,
                            const double *rho1, const double *rho2, double p, int32_t line_search,
                            int32_t max_iter, double tol, float *f, float *g, int32_t *iters,
                            double *gap, int32_t *status, void *workspace,
                            size_t workspace_bytes, void *stream);

/* Workspace bytes of uot_fw1d_batched (offN, offM on the host); 0 on invalid input. */
size_t uot_fw1d_workspace_bytes(int32_t B, const int64_t *offN, const int64_t *offM);

/*
 * Unregularised 1-D unbalanced barycenters (Sec. 5) of K measures, for B independent problems:
 * Frank-Wolfe on the translation-invariant multi-marginal dual
 *   H(fb) = sup_{sum_k lambda_k = 0} sum_k <alpha_k, w_k rho (1 - e^{-(fb_k + lambda_k)/(w_k rho)})>
 * over fb_0 (+) ... (+) fb_{K-1} <= C, C(z) = min_b sum_k w_k (z_k - b)^2 (squared distance;
 * b = sum w_k z_k / sum w_k, the barycentric map), with the closed-form lambda* of the KL
 * setting (q_k = log <alpha_k, e^{-fb_k/(w_k rho)}>, lambda_k = w_k rho q_k - w_k/sum_j w_j *
 * sum_j w_j rho q_j), from fb = 0 with step 2/(2 + t). The linear oracle is the balanced
 * multi-marginal walk between the tilted histograms (the measure with the least remaining
 * mass advances; the first on ties), whose visited tuples are tight.
 *  B >= 1, 2 <= K <= 16; off (host) [B*K + 1]: measure k of problem b is the point range
 *  [off[b*K + k], off[b*K + k + 1]) (at least one point), supports sorted ascending.
 *  x, alpha [off[B*K]] (device, float32); w [B*K] (device, double, > 0); rho [B] (device,
 *  double, > 0).
 *  f [off[B*K]] (device, out): the reported potentials fb_k + lambda_k.
 *  bary_x, bary_w (device, out): problem b's barycenter, the barycentric points and masses of
 *  the tuples of the balanced plan between its final tilted marginals (those marginals are
 *  the plan's marginals at the optimum), off[(b+1)K] - off[bK] - K + 1 entries starting at
 *  off[bK] - bK + b.
 *  iters, gap, status (device, [B], out): as in uot_fw1d_batched.
 * Double precision; one workgroup per problem, all iterations in one launch.
 */
uot_status uot_fw1d_barycenter(int32_t B, int32_t K, const int64_t *off, const float *x,
                               const float *alpha, const double *w, const double *rho,
                               int32_t max_iter, double tol, float *f, float *bary_x,
                               float *bary_w, int32_t *iters, double *gap, int32_t *status,
                               void *workspace, size_t workspace_bytes, void *stream);

/* Workspace bytes of uot_fw1d_barycenter (off on the host); 0 on invalid input. */
size_t uot_fw1d_barycenter_workspace_bytes(int32_t B, int32_t K, const int64_t *off);

/* Workspace bytes of uot_ti_sinkhorn_batched (offN, offM on the host); 0 on invalid input. */
size_t uot_batched_workspace_bytes(int32_t B, const int64_t *offN, const int64_t *offM, int32_t d);

/*
 * Work-item plan of uot_ti_sinkhorn_batched, process-wide (for tests and benchmarks; the plan
 * only changes how targets are grouped into work items, i.e. the order of the per-problem
 * partial sums). Items come at four levels: up to 256 targets (level 0, four per lane), 128
 * (level 1, two per lane), 64 (level 2, one per lane), and level 3: the chunks of level 2
 * with their sources split into ranges of 512, one item per range, whose per-target partial
 * sums the last of them to finish merges.
 *  0 = automatic and autotuned: a plan starts at one level and moves to a finer one once the
 *      busier side has at most tau x (resident waves) active items. For each size signature
 *      (device, B, d, check_every, tol > 0 and the log2 sizes of sum N, sum M, max N, max M)
 *      the first nine calls each run one candidate of
 *      {level 0 throughout; 0 then 1 at tau = 2; 0 then 1 at tau = 8; level 1 throughout;
 *       1 then 2 at tau = 2; 1 then 2 at tau = 8; level 2 throughout; 1 then 3 at tau = 2;
 *       1 then 3 at tau = 0.5}, timed on the host, and later calls take the fastest;
 *  1 = level 0 throughout, 2 = level 1 throughout, 3 = level 0 for the first chunk of
 *  iterations and level 1 after it, 4 = level 2 throughout, 5 = level 3 throughout.
 * Returns the previous setting, or -1 for an unknown value (nothing changes). Must not be
 * changed while a batched solve runs.
 */
int32_t uot_batched_set_plan(int32_t plan);

/* The item levels and switch threshold of the calling thread's last uot_ti_sinkhorn_batched
 * call under the automatic plan (host outputs, may be NULL); returns 1, or 0 (and -1 levels)
 * after another plan or before any call. */
int32_t uot_batched_last_plan(int32_t *start_level, int32_t *end_level, double *threshold);

/* Forgets every autotuned plan of the automatic batched plan (thread-safe). */
void uot_batched_autotune_reset(void);

/*
 * Load statistics of uot_ti_sinkhorn_batched, process-wide (for benchmarks): while enabled,
 * each solve records one row per chunk of iterations (and one for the start), kept until the
 * next solve; uot_batched_trace_read copies up to max_rows rows of 9 doubles (host memory)
 * and returns the number of rows of the last solve:
 *   chunk index, fine plan (0/1), problems running, active work items of the g- and f-steps,
 *   sum of N_p M_p over the running problems, wave time on work items during the chunk and
 *   the chunk's duration (both in ticks of the GPU's constant-rate clock, s_memrealtime), and
 *   the waves resident in one launch. busy / (duration x resident waves) is the fraction of
 *   the chip's wave slots that did work. The counters cost two clock reads per work item.
 */
void uot_batched_trace_enable(int32_t on);
int32_t uot_batched_trace_read(double *rows, int32_t max_rows);

/*
 * Kernel timing, for benchmarks (off by default). uot_profile_enable(period): 0 disables;
 * period >= 1 times every period-th softmin launch of uot_sinkhorn / uot_ti_sinkhorn
 * (counted process-wide) with start/stop HIP events attached to the kernel dispatch itself
 * (hipExtLaunchKernel: no extra commands in the stream), and accumulates its duration, with
 * the number of cost entries it processed, per kernel kind: 0 = points-cost softmin on the
 * matrix cores or the expanded form, 1 = stored-cost column softmin, 2 = stored-cost row
 * softmin, 3 = the one-pass kernel of uot_backward and of the marginals of uot_plan_apply
 * (points costs; its launches count towards the same period), 4 = points-cost softmin on
 * direct differences (p = 2 direct form, other p). Reading the events back
 * synchronises with the timed launches when the event ring (512 pairs) wraps, so a period
 * above 1 keeps a long solve asynchronous (an odd period samples both half-steps).
 * Thread-safe (a mutex guards the counters).
 *  uot_profile_read returns the number of timed launches of `kind` (-1 for a bad kind) and
 *  writes the summed milliseconds and summed entries (host pointers, may be NULL).
 */
void uot_profile_enable(int32_t period);
void uot_profile_reset(void);
int64_t uot_profile_read(int32_t kind, double *total_ms, double *total_entries);

/*
 * Issue-rate probes, for benchmarks: the chip-wide throughput of one instruction kind on the
 * current device, the rates behind the rooflines of the softmin (v_exp_f32, bf16 MFMA), the
 * backward (double and float32 FMAs, double and float32 MFMAs) and the batched kernels. Each
 * lane (vector kinds) or wave (matrix-core kinds) runs independent dependency chains of the
 * instruction (8, or 4 for bf16; 8 waves resident per SIMD); one untimed launch, then one
 * launch timed with HIP events on `stream`. Writes to *ops_per_s (host) lane-operations per
 * second for the vector kinds, flop/s for the matrix-core kinds (v_mfma_f64_16x16x4_f64,
 * v_mfma_f32_16x16x4_f32, v_mfma_f32_32x32x16_bf16: 2 M N K flops per instruction).
 * Allocates and frees a small device buffer; synchronises `stream`.
 * UOT_ERR_INVALID for an unknown kind or a NULL output, UOT_ERR_HIP on a runtime error.
 */
typedef enum {
  UOT_PROBE_EXP2 = 0,
  UOT_PROBE_FMA32 = 1,
  UOT_PROBE_FMA64 = 2,
  UOT_PROBE_MFMA_F64 = 3,
  UOT_PROBE_MFMA_F32 = 4,
  UOT_PROBE_MFMA_BF16 = 5
} uot_probe_kind;
uot_status uot_probe_rate(int32_t kind, double *ops_per_s, void *stream);

/*
 * Implementation of the squared-Euclidean (p = 2) points softmin, process-wide:
 * 0 = default (3 up to dimension 16, 2 above), 1 = vector ALU, 2 = matrix cores on the
 * float32 exponent, 3 = matrix cores on the exponent split into bf16 pieces (three per
 * float32 value, float32 accuracy; dimensions up to 16, 2 above); these evaluate the
 * exponent in the expanded form (see the accuracy note at uot_cost). 4 = vector ALU on the
 * differences x - y, as for p != 2: no expanded-form rounding, at a fraction of the speed
 * (the solvers and uot_dual_value; the backward, the marginals and the plan products up to
 * dimension 16 form their exponents in double precision whatever this setting).
 * Returns the previous setting, or -1 for an unknown value (then nothing changes). All
 * compute the same softmin; the switch must not be changed while calls are running.
 */
int32_t uot_set_points_kernel(int32_t variant);

/*
 * Implementation of the backward's per-entry pass (uot_backward, uot_backward_noalloc and
 * the marginals of uot_plan_apply, points costs) for dimensions 1 to 16, process-wide:
 * 0 = default, matrix cores (double-precision MFMA inner products, float32 MFMA gradient
 * sums), 1 = vector ALU. Other dimensions always take the vector ALU. Both form the same
 * exponents in double precision and the same sums in float32 (in another order). Returns the
 * previous setting, or -1 for an unknown value (then nothing changes); must not be changed
 * while calls are running.
 */
int32_t uot_set_grad_kernel(int32_t variant);

/*
 * Kernel-shape autotuning, process-wide, on by default: the first solve (uot_sinkhorn,
 * uot_ti_sinkhorn and their variants) of a shape with at least 2^20 cost entries per
 * half-step times its own first half-step's softmin with several source-split counts (the
 * resident-block capacity scaled by 0.5, 0.75, 1, 1.5, 2) and keeps the fastest for that
 * device, record form, dimension, target and source counts and side; later calls and
 * uot_dual_value take the kept shape. The split count changes only the order in which partial
 * sums merge (float32 rounding). uot_set_autotune(0) uses the untuned shape everywhere (same
 * results in every process); returns the previous setting. Thread-safe.
 */
int32_t uot_set_autotune(int32_t on);

/* Static description of a status code. */
const char *uot_status_string(uot_status s);

/* Text of the last error raised on the calling thread ("" if none). */
const char *uot_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* UOT_H_ */
