/*
 * FP64 CPU oracle for entropic KL-unbalanced optimal transport
 * (Sejourne, Vialard, Peyre, "Faster Unbalanced Optimal Transport:
 * Translation invariant Sinkhorn and 1-D Frank-Wolfe", AISTATS 2022).
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do. It shares no code with the GPU path.
 *
 * Written to be checked by eye against the paper: every quantity is the plain
 * definition, evaluated in double precision with std libm exp/log, a
 * log-sum-exp with an explicit max, no blocking, no fusion, no fast-math.
 * OpenMP only splits independent outer loops (one row or one column each).
 *
 * Notation (Sec. 1 and Sec. 3 of the paper):
 *   Smin_w^s(h)  = -s log sum_k w_k exp(-h_k / s)            (softmin)
 *   k1 = rho1/(eps+rho1), k2 = rho2/(eps+rho2)               (KL anisotropic prox)
 *   tau1 = rho1/(rho1+rho2), tau2 = rho2/(rho1+rho2)         (Prop. 3)
 * Weights enter as log-weights; a zero weight (log = -inf) drops its term from
 * every sum (the nu_i = 0 convention of the Csiszar divergence, Sec. 1).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Threads of the OpenMP loops below (timing the oracle on one or all host cores). */
void or_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int or_max_threads(void) { return omp_get_max_threads(); }

typedef struct {
  int n, m, d;          /* n source points (alpha), m target points (beta), point dimension */
  const double *C;      /* dense cost, row-major n x m with leading dimension ldc; NULL => points */
  long ldc;
  const double *x;      /* points mode: x [n, d] row-major */
  const double *y;      /* points mode: y [m, d] row-major */
  double p;             /* points mode: C_ij = ||x_i - y_j||_2^p */
} or_cost;

/* Cost entry C_ij (Sec. 1: C_ij = d(x_i, y_j)^p when built from points). */
static double or_c(const or_cost *k, int i, int j) {
  if (k->C) return k->C[(long)i * k->ldc + j];
  double s = 0.0;
  for (int t = 0; t < k->d; ++t) {
    double u = k->x[(long)i * k->d + t] - k->y[(long)j * k->d + t];
    s += u * u;
  }
  if (k->p == 2.0) return s;
  return pow(sqrt(s), k->p);
}

/* log sum_k exp(v_k) over entries with v_k > -inf; -inf if there are none. */
static double or_lse(int n, const double *v) {
  double mx = -INFINITY;
  for (int k = 0; k < n; ++k)
    if (v[k] > mx) mx = v[k];
  if (mx == -INFINITY) return -INFINITY;
  double acc = 0.0;
  for (int k = 0; k < n; ++k)
    if (v[k] > -INFINITY) acc += exp(v[k] - mx);
  return mx + log(acc);
}

/* Softmin of Sec. 3 on a vector: Smin_w^s(h) = -s log sum_k w_k exp(-h_k/s). */
double or_smin_vec(int n, const double *logw, const double *h, double s) {
  double *v = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  for (int k = 0; k < n; ++k) v[k] = (logw[k] == -INFINITY) ? -INFINITY : logw[k] - h[k] / s;
  double r = -s * or_lse(n, v);
  free(v);
  return r;
}

/* Column softmin (g-side half-step): out_j = Smin_alpha^eps(C_{:,j} - h)
 *   = -eps log sum_i alpha_i exp((h_i - C_ij)/eps),  j = 0..m-1. */
void or_smin_cols(const or_cost *k, const double *loga, const double *h, double eps, double *out) {
  const int n = k->n, m = k->m;
#pragma omp parallel
  {
    double *v = (double *)malloc(sizeof(double) * (size_t)n);
#pragma omp for schedule(static)
    for (int j = 0; j < m; ++j) {
      for (int i = 0; i < n; ++i)
        v[i] = (loga[i] == -INFINITY) ? -INFINITY : loga[i] + (h[i] - or_c(k, i, j)) / eps;
      out[j] = -eps * or_lse(n, v);
    }
    free(v);
  }
}

/* Row softmin (f-side half-step): out_i = Smin_beta^eps(C_{i,:} - h)
 *   = -eps log sum_j beta_j exp((h_j - C_ij)/eps),  i = 0..n-1. */
void or_smin_rows(const or_cost *k, const double *logb, const double *h, double eps, double *out) {
  const int n = k->n, m = k->m;
#pragma omp parallel
  {
    double *v = (double *)malloc(sizeof(double) * (size_t)m);
#pragma omp for schedule(static)
    for (int i = 0; i < n; ++i) {
      for (int j = 0; j < m; ++j)
        v[j] = (logb[j] == -INFINITY) ? -INFINITY : logb[j] + (h[j] - or_c(k, i, j)) / eps;
      out[i] = -eps * or_lse(m, v);
    }
    free(v);
  }
}

static double sup_diff(int n, const double *a, const double *b) {
  double r = 0.0;
  for (int k = 0; k < n; ++k) {
    double u = fabs(a[k] - b[k]);
    if (u > r) r = u;
  }
  return r;
}

/* Optimal translation lambda*(fb, gb) of Prop. 2, written through softmins:
 * lambda* = tau1 * Smin_beta^rho2(gb) - tau2 * Smin_alpha^rho1(fb). */
double or_lambda_star(int n, int m, const double *loga, const double *logb, const double *fb,
                      const double *gb, double rho1, double rho2) {
  const double tau1 = rho1 / (rho1 + rho2), tau2 = rho2 / (rho1 + rho2);
  return tau1 * or_smin_vec(m, logb, gb, rho2) - tau2 * or_smin_vec(n, loga, fb, rho1);
}

/*
 * Sinkhorn solver.
 *   ti = 0: F-Sinkhorn (Sec. 3): g <- k2 Smin_alpha^eps(C - f), then f <- k1 Smin_beta^eps(C - g).
 *           The g-update uses rho2 and the f-update rho1 (first-order conditions of F_eps in g and f).
 *   ti = 1: H-Sinkhorn, general rho1, rho2 (App. B, derivation of Prop. 4, eq. general-iter-h-sink):
 *           gh = k2 Smin_alpha^eps(C - fb) - eps*rho2/((eps+rho2)(rho1+rho2)) Smin_alpha^rho1(fb)
 *           gb = gh + kg/(1-kg) Smin_beta^rho2(gh),   kg = eps*rho1/((eps+rho2)(rho1+rho2))
 *           fh = k1 Smin_beta^eps(C - gb) - eps*rho1/((eps+rho1)(rho1+rho2)) Smin_beta^rho2(gb)
 *           fb = fh + kf/(1-kf) Smin_alpha^rho1(fh),  kf = eps*rho2/((eps+rho1)(rho1+rho2))
 *           and reports Phi(fb, gb) = (fb + lambda*, gb - lambda*) (Sec. 1 / App. B map Phi).
 * One iteration = g-step then f-step; f starts at 0 unless warm_start (f then holds f_0,
 * or fb_0 for ti = 1). After each iteration t the change
 *   delta_t = max(||f_t - f_{t-1}||_inf, ||g_t - g_{t-1}||_inf)
 * is computed on the reported (translated) potentials; if tol > 0 the solver stops at the
 * first t with t % check_every == 0 and delta_t < tol. delta_1 uses g_0 = the g the first
 * half-step would see as "previous": it is defined as +inf.
 * Optional histories (NULL to skip): hist_delta[max_iter], hist_f[max_iter*n], hist_g[max_iter*m].
 * Returns the number of iterations run; writes f, g, *lambda_out (0 for ti = 0), *last_delta.
 */
/* Working state of one solve: log-weights, parameters and the potentials being iterated. */
typedef struct {
  const or_cost *k;
  const double *loga, *logb;
  double eps, rho1, rho2;
  int ti;
  double *fb, *gb, *S;  /* f, g (plain) or fb, gb (TI); S: softmin scratch of max(n, m) */
} or_state;

/* One iteration, g-step then f-step, from s->fb (see the formulas above). Leaves the new
 * fb, gb in s and writes the reported potentials: fr, gr = (f, g) for plain Sinkhorn and
 * Phi(fb, gb) = (fb + lambda*, gb - lambda*) for TI. Returns lambda* (0 for plain). */
static double or_iterate(or_state *s, double *fr, double *gr) {
  const or_cost *k = s->k;
  const int n = k->n, m = k->m;
  const double eps = s->eps, rho1 = s->rho1, rho2 = s->rho2;
  const double k1 = rho1 / (eps + rho1), k2 = rho2 / (eps + rho2);
  double *fb = s->fb, *gb = s->gb, *S = s->S;
  double lam = 0.0;
  if (!s->ti) {
    or_smin_cols(k, s->loga, fb, eps, S);
    for (int j = 0; j < m; ++j) gb[j] = k2 * S[j];
    or_smin_rows(k, s->logb, gb, eps, S);
    for (int i = 0; i < n; ++i) fb[i] = k1 * S[i];
    memcpy(fr, fb, sizeof(double) * (size_t)n);
    memcpy(gr, gb, sizeof(double) * (size_t)m);
  } else {
    const double cg = eps * rho2 / ((eps + rho2) * (rho1 + rho2));
    const double kg = eps * rho1 / ((eps + rho2) * (rho1 + rho2));
    const double cf = eps * rho1 / ((eps + rho1) * (rho1 + rho2));
    const double kf = eps * rho2 / ((eps + rho1) * (rho1 + rho2));
    double sA = or_smin_vec(n, s->loga, fb, rho1);
    or_smin_cols(k, s->loga, fb, eps, S);
    for (int j = 0; j < m; ++j) gb[j] = k2 * S[j] - cg * sA;          /* gh */
    double tg = kg / (1.0 - kg) * or_smin_vec(m, s->logb, gb, rho2);
    for (int j = 0; j < m; ++j) gb[j] += tg;                          /* gb */
    double sB = or_smin_vec(m, s->logb, gb, rho2);
    or_smin_rows(k, s->logb, gb, eps, S);
    for (int i = 0; i < n; ++i) fb[i] = k1 * S[i] - cf * sB;          /* fh */
    double tf = kf / (1.0 - kf) * or_smin_vec(n, s->loga, fb, rho1);
    for (int i = 0; i < n; ++i) fb[i] += tf;                          /* fb */
    lam = or_lambda_star(n, m, s->loga, s->logb, fb, gb, rho1, rho2);
    for (int i = 0; i < n; ++i) fr[i] = fb[i] + lam;
    for (int j = 0; j < m; ++j) gr[j] = gb[j] - lam;
  }
  return lam;
}

int or_sinkhorn(const or_cost *k, const double *alpha, const double *beta, double eps, double rho1,
                double rho2, int ti, int max_iter, double tol, int check_every, int warm_start,
                double *f, double *g, double *lambda_out, double *last_delta, double *hist_delta,
                double *hist_f, double *hist_g) {
  const int n = k->n, m = k->m;
  double *loga = (double *)malloc(sizeof(double) * (size_t)n);
  double *logb = (double *)malloc(sizeof(double) * (size_t)m);
  for (int i = 0; i < n; ++i) loga[i] = log(alpha[i]);
  for (int j = 0; j < m; ++j) logb[j] = log(beta[j]);
  double *fb = (double *)malloc(sizeof(double) * (size_t)n);  /* f (plain) or fb (TI) */
  double *gb = (double *)malloc(sizeof(double) * (size_t)m);
  double *S = (double *)malloc(sizeof(double) * (size_t)(n > m ? n : m));
  double *fo = (double *)malloc(sizeof(double) * (size_t)n);  /* reported f, previous iteration */
  double *go = (double *)malloc(sizeof(double) * (size_t)m);
  double *fr = (double *)malloc(sizeof(double) * (size_t)n);  /* reported f, this iteration */
  double *gr = (double *)malloc(sizeof(double) * (size_t)m);
  for (int i = 0; i < n; ++i) fb[i] = warm_start ? f[i] : 0.0;
  for (int j = 0; j < m; ++j) gb[j] = 0.0;
  or_state st = {k, loga, logb, eps, rho1, rho2, ti, fb, gb, S};
  double lam = 0.0, delta = INFINITY;
  int t = 0;
  for (t = 1; t <= max_iter; ++t) {
    lam = or_iterate(&st, fr, gr);
    if (t == 1) {
      delta = INFINITY;
    } else {
      double a = sup_diff(n, fr, fo), b = sup_diff(m, gr, go);
      delta = a > b ? a : b;
    }
    if (hist_delta) hist_delta[t - 1] = delta;
    if (hist_f) memcpy(hist_f + (size_t)(t - 1) * n, fr, sizeof(double) * (size_t)n);
    if (hist_g) memcpy(hist_g + (size_t)(t - 1) * m, gr, sizeof(double) * (size_t)m);
    memcpy(fo, fr, sizeof(double) * (size_t)n);
    memcpy(go, gr, sizeof(double) * (size_t)m);
    if (tol > 0 && check_every > 0 && t % check_every == 0 && delta < tol) break;
  }
  if (t > max_iter) t = max_iter;
  memcpy(f, fo, sizeof(double) * (size_t)n);
  memcpy(g, go, sizeof(double) * (size_t)m);
  if (lambda_out) *lambda_out = ti ? lam : 0.0;
  if (last_delta) *last_delta = delta;
  free(loga); free(logb); free(fb); free(gb); free(S); free(fo); free(go); free(fr); free(gr);
  return t;
}

/*
 * Anderson extrapolation (appendix "Combining Sinkhorn with Anderson acceleration").
 * X holds K + 1 iterates of a map T, row k = x_k (length n), with x_{k+1} = T(x_k). The
 * residuals u_k = x_{k+1} - x_k (k < K) form U = [u_0 .. u_{K-1}]. With G = U^T U, the
 * appendix's regularised closed form is
 *   c = (G + r I)^{-1} 1 / (1^T (G + r I)^{-1} 1),
 * the minimiser of c^T (G + r I) c over 1^T c = 1 (normalize = 0). normalize = 1 is a
 * variant: G is first divided by its Frobenius norm (left as is when that norm is 0), so
 * that r is relative to the scale of the residuals. The extrapolated point is
 * out = sum_k c_k x_{k+1}, the combination of the images T(x_k). Writes c[K] and out[n];
 * returns 0, or -1 (c, out untouched) if G + r I is singular.
 */
int or_anderson_mix(int n, int K, const double *X, double r, int normalize, double *c,
                    double *out) {
  double G[16][16], z[16];
  if (K < 1 || K > 16) return -1;
  for (int a = 0; a < K; ++a)
    for (int b = 0; b < K; ++b) {
      double sum = 0.0;
      for (int i = 0; i < n; ++i) {
        const double ua = X[(size_t)(a + 1) * n + i] - X[(size_t)a * n + i];
        const double ub = X[(size_t)(b + 1) * n + i] - X[(size_t)b * n + i];
        sum += ua * ub;
      }
      G[a][b] = sum;
    }
  double fro = 0.0;
  for (int a = 0; a < K; ++a)
    for (int b = 0; b < K; ++b) fro += G[a][b] * G[a][b];
  fro = sqrt(fro);
  for (int a = 0; a < K; ++a) {
    if (normalize && fro > 0.0)
      for (int b = 0; b < K; ++b) G[a][b] /= fro;
    G[a][a] += r;
    z[a] = 1.0;
  }
  /* (G + r I) z = 1 by Gaussian elimination with partial pivoting */
  for (int p = 0; p < K; ++p) {
    int piv = p;
    for (int a = p + 1; a < K; ++a)
      if (fabs(G[a][p]) > fabs(G[piv][p])) piv = a;
    if (G[piv][p] == 0.0) return -1;
    if (piv != p) {
      for (int b = 0; b < K; ++b) { const double t = G[p][b]; G[p][b] = G[piv][b]; G[piv][b] = t; }
      const double t = z[p]; z[p] = z[piv]; z[piv] = t;
    }
    for (int a = p + 1; a < K; ++a) {
      const double l = G[a][p] / G[p][p];
      for (int b = p; b < K; ++b) G[a][b] -= l * G[p][b];
      z[a] -= l * z[p];
    }
  }
  for (int p = K - 1; p >= 0; --p) {
    double v = z[p];
    for (int b = p + 1; b < K; ++b) v -= G[p][b] * z[b];
    z[p] = v / G[p][p];
  }
  double zs = 0.0;
  for (int a = 0; a < K; ++a) zs += z[a];
  if (zs == 0.0 || !isfinite(zs)) return -1;
  for (int a = 0; a < K; ++a) c[a] = z[a] / zs;
  for (int i = 0; i < n; ++i) {
    double v = 0.0;
    for (int a = 0; a < K; ++a) v += c[a] * X[(size_t)(a + 1) * n + i];
    out[i] = v;
  }
  return 0;
}

/*
 * Anderson-accelerated Sinkhorn: the solver above (plain for ti = 0, TI for ti = 1) whose
 * iterated variable x = f (plain) or fb (TI) is extrapolated every K iterations. From x_0,
 * K iterations give x_1 .. x_K; after iteration t with t % K == 0 (and t < max_iter, and
 * the stopping test not met) x is replaced by or_anderson_mix(x_0 .. x_K) and the next cycle
 * starts from it (its g-step recomputes g); normalize selects the form of the mix (see
 * or_anderson_mix). The change delta_t is measured as in
 * or_sinkhorn, except that it is +inf at the first iteration after an extrapolation. K = 1
 * extrapolates to x_1 itself, i.e. reproduces or_sinkhorn's iterates. If the mix fails
 * (singular system) the cycle ends without extrapolation. Returns the iterations run.
 */
int or_sinkhorn_anderson(const or_cost *k, const double *alpha, const double *beta, double eps,
                         double rho1, double rho2, int ti, int K, double r, int normalize,
                         int max_iter,
                         double tol, int check_every, int warm_start, double *f, double *g,
                         double *lambda_out, double *last_delta, double *hist_delta) {
  const int n = k->n, m = k->m;
  if (K < 1 || K > 16) return -1;
  double *loga = (double *)malloc(sizeof(double) * (size_t)n);
  double *logb = (double *)malloc(sizeof(double) * (size_t)m);
  for (int i = 0; i < n; ++i) loga[i] = log(alpha[i]);
  for (int j = 0; j < m; ++j) logb[j] = log(beta[j]);
  double *fb = (double *)malloc(sizeof(double) * (size_t)n);
  double *gb = (double *)malloc(sizeof(double) * (size_t)m);
  double *S = (double *)malloc(sizeof(double) * (size_t)(n > m ? n : m));
  double *fo = (double *)malloc(sizeof(double) * (size_t)n);
  double *go = (double *)malloc(sizeof(double) * (size_t)m);
  double *fr = (double *)malloc(sizeof(double) * (size_t)n);
  double *gr = (double *)malloc(sizeof(double) * (size_t)m);
  double *X = (double *)malloc(sizeof(double) * (size_t)(K + 1) * n);  /* x_0 .. x_K */
  double *xe = (double *)malloc(sizeof(double) * (size_t)n);
  double c[16];
  for (int i = 0; i < n; ++i) fb[i] = warm_start ? f[i] : 0.0;
  for (int j = 0; j < m; ++j) gb[j] = 0.0;
  memcpy(X, fb, sizeof(double) * (size_t)n);
  or_state st = {k, loga, logb, eps, rho1, rho2, ti, fb, gb, S};
  double lam = 0.0, delta = INFINITY;
  int fresh = 0, t = 0;
  for (t = 1; t <= max_iter; ++t) {
    lam = or_iterate(&st, fr, gr);
    const int kc = (t - 1) % K + 1;
    memcpy(X + (size_t)kc * n, fb, sizeof(double) * (size_t)n);
    if (t == 1 || fresh) {
      delta = INFINITY;
    } else {
      double a = sup_diff(n, fr, fo), b = sup_diff(m, gr, go);
      delta = a > b ? a : b;
    }
    fresh = 0;
    if (hist_delta) hist_delta[t - 1] = delta;
    memcpy(fo, fr, sizeof(double) * (size_t)n);
    memcpy(go, gr, sizeof(double) * (size_t)m);
    if (tol > 0 && check_every > 0 && t % check_every == 0 && delta < tol) break;
    if (kc == K && t < max_iter) {
      if (or_anderson_mix(n, K, X, r, normalize, c, xe) == 0) {
        memcpy(fb, xe, sizeof(double) * (size_t)n);
        fresh = 1;
      }
      memcpy(X, fb, sizeof(double) * (size_t)n);
    }
  }
  if (t > max_iter) t = max_iter;
  memcpy(f, fo, sizeof(double) * (size_t)n);
  memcpy(g, go, sizeof(double) * (size_t)m);
  if (lambda_out) *lambda_out = ti ? lam : 0.0;
  if (last_delta) *last_delta = delta;
  free(loga); free(logb); free(fb); free(gb); free(S); free(fo); free(go); free(fr); free(gr);
  free(X); free(xe);
  return t;
}

/*
 * Generic entropies (Sec. 3, the phi* of the dual; the Berg entropy of the experiments of
 * Sec. 3): div = 0 is rho KL, phi*(x) = rho (e^{x/rho} - 1); div = 1 is the Berg entropy
 * phi(x) = rho (x - 1 - log x), phi*(x) = -rho log(1 - x/rho) for x < rho.
 * phi*'(x): KL e^{x/rho}; Berg rho / (rho - x) (+inf for x >= rho).
 */
double or_phistar_prime(int div, double rho, double x) {
  if (div == 0) return exp(x / rho);
  return x < rho ? rho / (rho - x) : INFINITY;
}

double or_phistar(int div, double rho, double x) {
  if (div == 0) return rho * (exp(x / rho) - 1.0);
  return x < rho ? -rho * log(1.0 - x / rho) : INFINITY;
}

/*
 * The dual update of one potential from its softmin S (Sec. 3): g = -aprox_{phi*}(-S), the
 * minimiser y of eps e^{(-S - y)/eps} + phi*(y) negated; its optimality condition reads
 *   e^{(g - S)/eps} = phi*'(-g).
 * KL: g = rho/(eps + rho) S. Berg: (g - S)/eps = log rho - log(rho + g) on g > -rho, whose
 * left minus right side increases from -inf to +inf; solved by bisection on (-rho, max(S, 0)]
 * until the bracket stops shrinking.
 */
double or_dual_update(int div, double rho, double eps, double S) {
  if (div == 0) return rho / (eps + rho) * S;
  double lo = -rho, hi = S > 0.0 ? S : 0.0;
  for (int it = 0; it < 2000; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    const double h = (mid - S) / eps + log(rho + mid) - log(rho);
    if (h > 0.0) hi = mid; else lo = mid;
  }
  return 0.5 * (lo + hi);
}

/*
 * Optimal translation lambda*(fb, gb) for a generic entropy (Prop. on the existence of
 * lambda*): the root of <alpha, phi1*'(-fb - lambda)> = <beta, phi2*'(-gb + lambda)>.
 * KL: the closed form of Prop. 2. Berg: the left side decreases from +inf to 0 and the right
 * side increases from 0 to +inf on (-rho1 - min fb, rho2 + min gb) (minima over positive
 * weights): bisection until the bracket stops shrinking.
 */
double or_lambda_star_div(int div, int n, int m, const double *alpha, const double *beta,
                          const double *fb, const double *gb, double rho1, double rho2) {
  if (div == 0) {
    double *la = (double *)malloc(sizeof(double) * (size_t)n);
    double *lb = (double *)malloc(sizeof(double) * (size_t)m);
    for (int i = 0; i < n; ++i) la[i] = log(alpha[i]);
    for (int j = 0; j < m; ++j) lb[j] = log(beta[j]);
    const double r = or_lambda_star(n, m, la, lb, fb, gb, rho1, rho2);
    free(la); free(lb);
    return r;
  }
  double fmin = INFINITY, gmin = INFINITY;
  for (int i = 0; i < n; ++i) if (alpha[i] > 0.0 && fb[i] < fmin) fmin = fb[i];
  for (int j = 0; j < m; ++j) if (beta[j] > 0.0 && gb[j] < gmin) gmin = gb[j];
  double lo = -rho1 - fmin, hi = rho2 + gmin;
  for (int it = 0; it < 2000; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    double a = 0.0, b = 0.0;
    for (int i = 0; i < n; ++i)
      if (alpha[i] > 0.0) a += alpha[i] * or_phistar_prime(1, rho1, -fb[i] - mid);
    for (int j = 0; j < m; ++j)
      if (beta[j] > 0.0) b += beta[j] * or_phistar_prime(1, rho2, -gb[j] + mid);
    if (a > b) lo = mid; else hi = mid;
  }
  return 0.5 * (lo + hi);
}

/*
 * Dual value F_eps(f, g) = -<alpha, phi1*(-f)> - <beta, phi2*(-g)> - eps (m(pi) - m(alpha) m(beta))
 * for a generic entropy (eq. dual-uot with its phi*; for KL it equals or_dual_value).
 */
double or_dual_value_div(const or_cost *k, const double *alpha, const double *beta, double eps,
                         double rho1, double rho2, int div, const double *f, const double *g) {
  const int n = k->n, m = k->m;
  double a = 0.0, b = 0.0, ma = 0.0, mb = 0.0;
  for (int i = 0; i < n; ++i) { if (alpha[i] > 0.0) a += alpha[i] * or_phistar(div, rho1, -f[i]); ma += alpha[i]; }
  for (int j = 0; j < m; ++j) { if (beta[j] > 0.0) b += beta[j] * or_phistar(div, rho2, -g[j]); mb += beta[j]; }
  double mpi = 0.0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < m; ++j) mpi += alpha[i] * beta[j] * exp((f[i] + g[j] - or_c(k, i, j)) / eps);
  return -a - b - eps * (mpi - ma * mb);
}

/*
 * F-Sinkhorn (variant 0) or G-Sinkhorn (variant 1) of Sec. 3 for a generic entropy div:
 *   F: g_{t+1} = U2(Smin_alpha^eps(C - f_t)),  f_{t+1} = U1(Smin_beta^eps(C - g_{t+1}))
 *   G: gb_{t+1} = U2(Smin_alpha^eps(C - fb_t - lambda_t)) + lambda_t,
 *      fb_{t+1} = U1(Smin_beta^eps(C - gb_{t+1} + lambda_t)) - lambda_t,
 *      lambda_{t+1} = lambda*(fb_{t+1}, gb_{t+1}),
 *      reported (f, g) = (fb + lambda, gb - lambda)
 * with U_i(S) = or_dual_update(div, rho_i, eps, S) (the g-update uses rho2, the f-update
 * rho1) and, for G, the +-lambda_t outside the prox (maximising G_eps(fb, gb, lambda) =
 * F_eps(fb + lambda, gb - lambda) in gb at fixed fb + lambda). From f = fb = 0, lambda = 0;
 * change and stopping rule as or_sinkhorn. Returns the iterations run.
 */
int or_sinkhorn_div(const or_cost *k, const double *alpha, const double *beta, double eps,
                    double rho1, double rho2, int div, int variant, int max_iter, double tol,
                    int check_every, double *f, double *g, double *lambda_out, double *last_delta) {
  const int n = k->n, m = k->m;
  double *loga = (double *)malloc(sizeof(double) * (size_t)n);
  double *logb = (double *)malloc(sizeof(double) * (size_t)m);
  for (int i = 0; i < n; ++i) loga[i] = log(alpha[i]);
  for (int j = 0; j < m; ++j) logb[j] = log(beta[j]);
  double *fb = (double *)calloc((size_t)n, sizeof(double));
  double *gb = (double *)calloc((size_t)m, sizeof(double));
  double *S = (double *)malloc(sizeof(double) * (size_t)(n > m ? n : m));
  double *h = (double *)malloc(sizeof(double) * (size_t)(n > m ? n : m));
  double *fo = (double *)malloc(sizeof(double) * (size_t)n);
  double *go = (double *)malloc(sizeof(double) * (size_t)m);
  double lam = 0.0, delta = INFINITY;
  int t;
  for (t = 1; t <= max_iter; ++t) {
    const double l = variant ? lam : 0.0;
    for (int i = 0; i < n; ++i) h[i] = fb[i] + l;
    or_smin_cols(k, loga, h, eps, S);
    for (int j = 0; j < m; ++j) gb[j] = or_dual_update(div, rho2, eps, S[j]) + l;
    for (int j = 0; j < m; ++j) h[j] = gb[j] - l;
    or_smin_rows(k, logb, h, eps, S);
    for (int i = 0; i < n; ++i) fb[i] = or_dual_update(div, rho1, eps, S[i]) - l;
    if (variant) lam = or_lambda_star_div(div, n, m, alpha, beta, fb, gb, rho1, rho2);
    double d = 0.0;
    for (int i = 0; i < n; ++i) {
      const double v = fb[i] + lam;
      if (t > 1 && fabs(v - fo[i]) > d) d = fabs(v - fo[i]);
      fo[i] = v;
    }
    for (int j = 0; j < m; ++j) {
      const double v = gb[j] - lam;
      if (t > 1 && fabs(v - go[j]) > d) d = fabs(v - go[j]);
      go[j] = v;
    }
    delta = t > 1 ? d : INFINITY;
    if (tol > 0 && check_every > 0 && t % check_every == 0 && delta < tol) break;
  }
  if (t > max_iter) t = max_iter;
  memcpy(f, fo, sizeof(double) * (size_t)n);
  memcpy(g, go, sizeof(double) * (size_t)m);
  if (lambda_out) *lambda_out = lam;
  if (last_delta) *last_delta = delta;
  free(loga); free(logb); free(fb); free(gb); free(S); free(h); free(fo); free(go);
  return t;
}

/*
 * ---------------------------------------------------------------------------------------
 * 1-D Frank-Wolfe for unregularised KL-UOT (eps = 0), Sec. 4.
 * ---------------------------------------------------------------------------------------
 * Balanced 1-D OT between sorted supports x[0..n) and y[0..m) (ascending) with weights a, b
 * of equal total mass and cost C_ij = |x_i - y_j|^p, p >= 1: the monotone (north-west
 * corner) coupling walks the cells of the n x m grid from (0, 0), at each cell moving mass
 * min(remaining of row i, remaining of column j); a row that runs out first (or ties) moves
 * the walk down, otherwise right; the last row or column absorbs what is left. Dual
 * potentials from complementary slackness along the walk: r_0 = 0, s_0 = C_00, and each
 * cell (i, j) entered is tight, r_i + s_j = C_ij (entering row i at column j sets r_i,
 * entering column j at row i sets s_j). For costs with the Monge property (|x - y|^p, p >= 1)
 * this pair is dual feasible, r_i + s_j <= C_ij everywhere.
 * Writes r[n], s[m]; if cells != NULL also the walk: cells[2k], cells[2k+1] = (i, j) and
 * mass[k] for its n + m - 1 cells. Returns the transport cost sum_k mass_k C(cell_k).
 */
static double or_c1d(double x, double y, double p) { return pow(fabs(x - y), p); }

double or_solve_ot_1d(int n, int m, const double *x, const double *y, const double *a,
                      const double *b, double p, double *r, double *s, int *cells, double *mass) {
  int i = 0, j = 0, k = 0;
  double ra = a[0], rb = b[0], cost = 0.0;
  r[0] = 0.0;
  s[0] = or_c1d(x[0], y[0], p);
  while (1) {
    const int last_i = i == n - 1, last_j = j == m - 1;
    double moved;
    int down;
    if (last_i && last_j) { moved = ra > rb ? ra : rb; down = -1; }
    else if (last_j) { moved = ra; down = 1; }           /* the last column takes the row   */
    else if (last_i) { moved = rb; down = 0; }           /* the last row takes the column   */
    else if (ra <= rb) { moved = ra; down = 1; }
    else { moved = rb; down = 0; }
    if (moved < 0.0) moved = 0.0;
    if (cells) { cells[2 * k] = i; cells[2 * k + 1] = j; mass[k] = moved; }
    cost += moved * or_c1d(x[i], y[j], p);
    ++k;
    if (down < 0) break;
    if (down) {
      rb -= moved;
      ++i;
      ra = a[i];
      r[i] = or_c1d(x[i], y[j], p) - s[j];
    } else {
      ra -= moved;
      ++j;
      rb = b[j];
      s[j] = or_c1d(x[i], y[j], p) - r[i];
    }
  }
  return cost;
}

/*
 * H_0 for KL (Sec. 4 applies F-W to H_0 = sup_lambda F_0(fb + lambda, gb - lambda)): with
 * A = <alpha, e^{-fb/rho1}>, B = <beta, e^{-gb/rho2}>, the maximising lambda is
 * rho1 rho2/(rho1 + rho2) log(A/B) (Prop. 2), and
 *   H_0 = rho1 m(alpha) + rho2 m(beta) - (rho1 + rho2) A^{tau1} B^{tau2}.
 * Computed here as F_0 at (fb + lambda*, gb - lambda*), its definition.
 */
double or_h0(int n, int m, const double *alpha, const double *beta, const double *fb,
             const double *gb, double rho1, double rho2, double *lambda_out) {
  double A = 0.0, B = 0.0;
  for (int i = 0; i < n; ++i) A += alpha[i] * exp(-fb[i] / rho1);
  for (int j = 0; j < m; ++j) B += beta[j] * exp(-gb[j] / rho2);
  const double lam = rho1 * rho2 / (rho1 + rho2) * (log(A) - log(B));
  double v = 0.0;
  for (int i = 0; i < n; ++i) v += rho1 * alpha[i] * (1.0 - exp(-(fb[i] + lam) / rho1));
  for (int j = 0; j < m; ++j) v += rho2 * beta[j] * (1.0 - exp(-(gb[j] - lam) / rho2));
  if (lambda_out) *lambda_out = lam;
  return v;
}

/*
 * Frank-Wolfe on H_0 over {fb (+) gb <= C} (Sec. 4, KL): from (fb, gb) = (0, 0), each
 * iteration t = 0, 1, ... forms the tilted histograms (the gradient of H_0, Prop. on
 * lambda*) at = alpha e^{-(fb + l)/rho1}, bt = beta e^{-(gb - l)/rho2}, l = lambda*(fb, gb),
 * which have equal masses; takes the linear maximisation oracle (r, s) = the dual solution
 * of balanced 1-D OT between (x, at) and (y, bt) (or_solve_ot_1d, after scaling both to mass
 * 1); the Frank-Wolfe gap <at, r - fb> + <bt, s - gb> (>= H_0* - H_0(fb, gb)); and steps
 * (fb, gb) <- (1 - gamma)(fb, gb) + gamma (r, s) with gamma = 2/(2 + t) (line_search = 0) or
 * the maximiser of H_0 on the segment, gamma in [0, 1] (line_search = 1; H_0 along the
 * segment is concave, found by bisection on the sign of its derivative to the last bit).
 * An iteration is one oracle call and, unless its gap is <= tol (tol > 0), one step; the
 * loop ends at such an iteration or after max_iter iterations. Writes the reported
 * potentials (fb + lambda*, gb - lambda*) and returns the iterations run; *gap_out is the
 * last gap. hist_gap[max_iter] (optional) receives every gap.
 */
int or_fw_1d(int n, int m, const double *x, const double *y, const double *alpha,
             const double *beta, double rho1, double rho2, double p, int line_search,
             int max_iter, double tol, double *f, double *g, double *gap_out, double *hist_gap) {
  double *fb = (double *)calloc((size_t)n, sizeof(double));
  double *gb = (double *)calloc((size_t)m, sizeof(double));
  double *at = (double *)malloc(sizeof(double) * (size_t)n);
  double *bt = (double *)malloc(sizeof(double) * (size_t)m);
  double *r = (double *)malloc(sizeof(double) * (size_t)n);
  double *s = (double *)malloc(sizeof(double) * (size_t)m);
  double *ft = (double *)malloc(sizeof(double) * (size_t)n);
  double *gt = (double *)malloc(sizeof(double) * (size_t)m);
  double gap = INFINITY, lam = 0.0;
  int t;
  for (t = 0; t < max_iter; ++t) {
    or_h0(n, m, alpha, beta, fb, gb, rho1, rho2, &lam);
    double ma = 0.0, mb = 0.0;
    for (int i = 0; i < n; ++i) { at[i] = alpha[i] * exp(-(fb[i] + lam) / rho1); ma += at[i]; }
    for (int j = 0; j < m; ++j) { bt[j] = beta[j] * exp(-(gb[j] - lam) / rho2); mb += bt[j]; }
    gap = 0.0;
    {
      double *an = ft, *bn = gt;  /* scratch: histograms scaled to mass 1 */
      for (int i = 0; i < n; ++i) an[i] = at[i] / ma;
      for (int j = 0; j < m; ++j) bn[j] = bt[j] / mb;
      or_solve_ot_1d(n, m, x, y, an, bn, p, r, s, NULL, NULL);
    }
    for (int i = 0; i < n; ++i) gap += at[i] * (r[i] - fb[i]);
    for (int j = 0; j < m; ++j) gap += bt[j] * (s[j] - gb[j]);
    if (hist_gap) hist_gap[t] = gap;
    if (tol > 0.0 && gap <= tol) break;
    double gamma;
    if (!line_search) {
      gamma = 2.0 / (2.0 + t);
    } else {
      /* derivative of H_0 along the segment at gamma: with l* at the point,
       * dH/dgamma = <at(gamma), r - fb> + <bt(gamma), s - gb> (envelope theorem) */
      double lo = 0.0, hi = 1.0;
      for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        for (int i = 0; i < n; ++i) ft[i] = (1.0 - mid) * fb[i] + mid * r[i];
        for (int j = 0; j < m; ++j) gt[j] = (1.0 - mid) * gb[j] + mid * s[j];
        double l2;
        or_h0(n, m, alpha, beta, ft, gt, rho1, rho2, &l2);
        double d = 0.0;
        for (int i = 0; i < n; ++i) d += alpha[i] * exp(-(ft[i] + l2) / rho1) * (r[i] - fb[i]);
        for (int j = 0; j < m; ++j) d += beta[j] * exp(-(gt[j] - l2) / rho2) * (s[j] - gb[j]);
        if (d > 0.0) lo = mid; else hi = mid;
      }
      gamma = 0.5 * (lo + hi);
    }
    for (int i = 0; i < n; ++i) fb[i] = (1.0 - gamma) * fb[i] + gamma * r[i];
    for (int j = 0; j < m; ++j) gb[j] = (1.0 - gamma) * gb[j] + gamma * s[j];
  }
  or_h0(n, m, alpha, beta, fb, gb, rho1, rho2, &lam);
  for (int i = 0; i < n; ++i) f[i] = fb[i] + lam;
  for (int j = 0; j < m; ++j) g[j] = gb[j] - lam;
  if (gap_out) *gap_out = gap;
  free(fb); free(gb); free(at); free(bt); free(r); free(s); free(ft); free(gt);
  return t < max_iter ? t + 1 : max_iter;
}

/*
 * ---------------------------------------------------------------------------------------
 * 1-D unbalanced barycenters by Frank-Wolfe on the translation-invariant multi-marginal
 * dual (Sec. 5), squared distance ground cost.
 * ---------------------------------------------------------------------------------------
 * Multi-marginal cost of one tuple (z_0 .. z_{K-1}): min_b sum_k w_k (z_k - b)^2, attained
 * at the barycentric map b = sum_k w_k z_k / sum_k w_k.
 */
static double or_mm_cost(int K, const double *w, const double *z, double *bary) {
  double sw = 0.0, sz = 0.0;
  for (int k = 0; k < K; ++k) { sw += w[k]; sz += w[k] * z[k]; }
  const double b = sz / sw;
  double c = 0.0;
  for (int k = 0; k < K; ++k) c += w[k] * (z[k] - b) * (z[k] - b);
  if (bary) *bary = b;
  return c;
}

/*
 * Balanced multi-marginal OT in 1-D between K measures with sorted supports x_k (offsets
 * off[0..K]) and weights a of equal masses: the walk starts at the first point of every
 * measure; at each step the measure with the least remaining mass among those not at their
 * last point (the first such k on ties) advances, the current tuple receiving that mass and
 * every measure's remainder dropping by it; when all are at their last point the final
 * tuple takes what is left. Every visited tuple is tight: f_{0,0} = C(first tuple), the
 * other f_{k,0} = 0, and a measure entering point i sets f_{k,i} = C(tuple) minus the other
 * potentials of the tuple. Writes f[off[K]] and, optionally, the support and mass of each
 * visited tuple (off[K] - K + 1 of them: its barycentric point and mass). Returns the total
 * transport cost.
 */
double or_solve_mot_1d(int K, const int64_t *off, const double *x, const double *a,
                       const double *w, double *f, double *bary_x, double *bary_m) {
  int idx[64];
  double rem[64], z[64];
  if (K < 1 || K > 64) return NAN;
  for (int k = 0; k < K; ++k) {
    idx[k] = 0;
    rem[k] = a[off[k]];
    z[k] = x[off[k]];
    f[off[k]] = 0.0;
  }
  double b;
  f[off[0]] = or_mm_cost(K, w, z, &b);
  double cost = 0.0;
  int t = 0;
  while (1) {
    int p = -1;
    for (int k = 0; k < K; ++k)
      if (idx[k] < off[k + 1] - off[k] - 1 && (p < 0 || rem[k] < rem[p])) p = k;
    const double c = or_mm_cost(K, w, z, &b);
    if (p < 0) {  /* every measure at its last point: the final tuple takes the rest */
      double mv = 0.0;
      for (int k = 0; k < K; ++k) if (rem[k] > mv) mv = rem[k];
      cost += mv * c;
      if (bary_x) { bary_x[t] = b; bary_m[t] = mv; }
      break;
    }
    const double mv = rem[p] > 0.0 ? rem[p] : 0.0;
    cost += mv * c;
    if (bary_x) { bary_x[t] = b; bary_m[t] = mv; }
    ++t;
    for (int k = 0; k < K; ++k) rem[k] -= mv;
    idx[p] += 1;
    const int64_t e = off[p] + idx[p];
    z[p] = x[e];
    rem[p] = a[e];
    double others = 0.0;
    for (int k = 0; k < K; ++k) if (k != p) others += f[off[k] + idx[k]];
    f[e] = or_mm_cost(K, w, z, NULL) - others;
  }
  return cost;
}

/*
 * Optimal translation of the multi-marginal dual (Prop. for the KL setting in Sec. 5): with
 * q_k = log <a_k, e^{-fb_k / (w_k rho)}>, lambda_k = w_k rho q_k - w_k / sum_j w_j *
 * sum_j w_j rho q_j (so sum_k lambda_k = 0).
 */
void or_mm_lambda(int K, const int64_t *off, const double *a, const double *fb, const double *w,
                  double rho, double *lam) {
  double sw = 0.0, sq = 0.0, q[64];
  for (int k = 0; k < K; ++k) {
    double s = 0.0;
    for (int64_t i = off[k]; i < off[k + 1]; ++i) s += a[i] * exp(-fb[i] / (w[k] * rho));
    q[k] = log(s);
    sw += w[k];
    sq += w[k] * rho * q[k];
  }
  for (int k = 0; k < K; ++k) lam[k] = w[k] * rho * q[k] - w[k] / sw * sq;
}

/* The multi-marginal dual F(f) = sum_k <a_k, w_k rho (1 - e^{-f_k / (w_k rho)})> (KL). */
double or_mm_dual(int K, const int64_t *off, const double *a, const double *f, const double *w,
                  double rho) {
  double v = 0.0;
  for (int k = 0; k < K; ++k)
    for (int64_t i = off[k]; i < off[k + 1]; ++i)
      v += a[i] * w[k] * rho * (1.0 - exp(-f[i] / (w[k] * rho)));
  return v;
}

/*
 * Frank-Wolfe on H(fb) = sup_{sum lambda = 0} F(fb + lambda) over fb_0 (+) ... (+) fb_{K-1} <= C
 * (Sec. 5), from fb = 0: each iteration takes lambda* (or_mm_lambda), the gradient of H =
 * the tilted histograms a_k e^{-(fb_k + lambda_k)/(w_k rho)} (equal masses), the linear
 * oracle = the balanced multi-marginal dual between them (or_solve_mot_1d after scaling to
 * mass 1), the gap sum_k <at_k, r_k - fb_k>, and the step 2/(2 + t). An iteration whose
 * gap is <= tol (tol > 0) ends the loop before its step. Writes the reported potentials
 * fb_k + lambda_k, and the barycenter: the support and masses of the balanced plan between
 * the final tilted marginals (off[K] - K + 1 entries; masses in the units of the inputs).
 * Returns the iterations run.
 */
int or_fw_barycenter(int K, const int64_t *off, const double *x, const double *a,
                     const double *w, double rho, int max_iter, double tol, double *f,
                     double *bary_x, double *bary_m, double *gap_out) {
  const int64_t tot = off[K];
  double *fb = (double *)calloc((size_t)tot, sizeof(double));
  double *at = (double *)malloc(sizeof(double) * (size_t)tot);
  double *an = (double *)malloc(sizeof(double) * (size_t)tot);
  double *r = (double *)malloc(sizeof(double) * (size_t)tot);
  double lam[64], mass[64];
  double gap = INFINITY;
  int t;
  for (t = 0; t < max_iter; ++t) {
    or_mm_lambda(K, off, a, fb, w, rho, lam);
    for (int k = 0; k < K; ++k) {
      mass[k] = 0.0;
      for (int64_t i = off[k]; i < off[k + 1]; ++i) {
        at[i] = a[i] * exp(-(fb[i] + lam[k]) / (w[k] * rho));
        mass[k] += at[i];
      }
      for (int64_t i = off[k]; i < off[k + 1]; ++i) an[i] = at[i] / mass[k];
    }
    or_solve_mot_1d(K, off, x, an, w, r, NULL, NULL);
    gap = 0.0;
    for (int64_t i = 0; i < tot; ++i) gap += at[i] * (r[i] - fb[i]);
    if (tol > 0.0 && gap <= tol) break;
    const double gamma = 2.0 / (2.0 + t);
    for (int64_t i = 0; i < tot; ++i) fb[i] = (1.0 - gamma) * fb[i] + gamma * r[i];
  }
  or_mm_lambda(K, off, a, fb, w, rho, lam);
  double m0 = 0.0;
  for (int k = 0; k < K; ++k) {
    mass[k] = 0.0;
    for (int64_t i = off[k]; i < off[k + 1]; ++i) {
      f[i] = fb[i] + lam[k];
      at[i] = a[i] * exp(-f[i] / (w[k] * rho));
      mass[k] += at[i];
    }
    for (int64_t i = off[k]; i < off[k + 1]; ++i) an[i] = at[i] / mass[k];
  }
  m0 = mass[0];
  if (bary_x) {
    or_solve_mot_1d(K, off, x, an, w, r, bary_x, bary_m);
    for (int64_t e = 0; e < tot - K + 1; ++e) bary_m[e] *= m0;
  }
  if (gap_out) *gap_out = gap;
  free(fb); free(at); free(an); free(r);
  return t < max_iter ? t + 1 : max_iter;
}

/* Plan entry pi_ij = alpha_i beta_j exp((f_i + g_j - C_ij)/eps) (primal-dual link of the dual problem). */
static double or_pi(const or_cost *k, const double *alpha, const double *beta, double eps,
                    const double *f, const double *g, int i, int j) {
  if (alpha[i] == 0.0 || beta[j] == 0.0) return 0.0;
  return alpha[i] * beta[j] * exp((f[i] + g[j] - or_c(k, i, j)) / eps);
}

/* Plan application: transpose = 0: out[i, c] = sum_j pi_ij V[j, c]  (V is m x kc, out n x kc);
 *                   transpose = 1: out[j, c] = sum_i pi_ij V[i, c]  (V is n x kc, out m x kc).
 * With V = ones this gives the marginals pi_1 = pi 1 and pi_2 = pi^T 1 (Sec. 1). */
void or_plan_apply(const or_cost *k, const double *alpha, const double *beta, double eps,
                   const double *f, const double *g, int transpose, const double *V, int kc,
                   double *out) {
  const int n = k->n, m = k->m;
  if (!transpose) {
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
      for (int c = 0; c < kc; ++c) out[(long)i * kc + c] = 0.0;
      for (int j = 0; j < m; ++j) {
        double p = or_pi(k, alpha, beta, eps, f, g, i, j);
        for (int c = 0; c < kc; ++c) out[(long)i * kc + c] += p * V[(long)j * kc + c];
      }
    }
  } else {
#pragma omp parallel for schedule(static)
    for (int j = 0; j < m; ++j) {
      for (int c = 0; c < kc; ++c) out[(long)j * kc + c] = 0.0;
      for (int i = 0; i < n; ++i) {
        double p = or_pi(k, alpha, beta, eps, f, g, i, j);
        for (int c = 0; c < kc; ++c) out[(long)j * kc + c] += p * V[(long)i * kc + c];
      }
    }
  }
}

/* Total plan mass m(pi) = sum_ij pi_ij. */
static double or_plan_mass(const or_cost *k, const double *alpha, const double *beta, double eps,
                           const double *f, const double *g) {
  const int n = k->n, m = k->m;
  double tot = 0.0;
#pragma omp parallel for reduction(+ : tot) schedule(static)
  for (int i = 0; i < n; ++i) {
    double r = 0.0;
    for (int j = 0; j < m; ++j) r += or_pi(k, alpha, beta, eps, f, g, i, j);
    tot += r;
  }
  return tot;
}

/* Dual functional F_eps of eq. (dual-uot-kl) for rho KL penalties, with
 * -phi*(-f) = rho (1 - exp(-f/rho)) (the KL conjugate, as written in the proof of Prop. 3):
 * F = rho1 <alpha, 1 - e^{-f/rho1}> + rho2 <beta, 1 - e^{-g/rho2}> - eps (m(pi) - m(alpha) m(beta)). */
double or_dual_value(const or_cost *k, const double *alpha, const double *beta, double eps,
                     double rho1, double rho2, const double *f, const double *g) {
  const int n = k->n, m = k->m;
  double a = 0.0, b = 0.0, ma = 0.0, mb = 0.0;
  for (int i = 0; i < n; ++i) { a += alpha[i] * (1.0 - exp(-f[i] / rho1)); ma += alpha[i]; }
  for (int j = 0; j < m; ++j) { b += beta[j] * (1.0 - exp(-g[j] / rho2)); mb += beta[j]; }
  double mpi = or_plan_mass(k, alpha, beta, eps, f, g);
  return rho1 * a + rho2 * b - eps * (mpi - ma * mb);
}

/* Generalised KL(mu | nu) = sum mu log(mu/nu) - m(mu) + m(nu) (Sec. 1), with 0 log 0 = 0;
 * +inf when some nu_i = 0 < mu_i. */
static double or_kl(int n, const double *mu, const double *nu) {
  double r = 0.0;
  for (int k = 0; k < n; ++k) {
    if (mu[k] > 0.0) {
      if (nu[k] == 0.0) return INFINITY;
      r += mu[k] * log(mu[k] / nu[k]);
    }
    r += nu[k] - mu[k];
  }
  return r;
}

/* Primal objective of eq. (primal-uot-kl) at the plan built from (f, g):
 * P(pi) = <pi, C> + eps KL(pi | alpha x beta) + rho1 KL(pi_1 | alpha) + rho2 KL(pi_2 | beta). */
double or_primal_value(const or_cost *k, const double *alpha, const double *beta, double eps,
                       double rho1, double rho2, const double *f, const double *g) {
  const int n = k->n, m = k->m;
  double *p1 = (double *)calloc((size_t)n, sizeof(double));
  double *p2 = (double *)calloc((size_t)m, sizeof(double));
  double lin = 0.0, klpi = 0.0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < m; ++j) {
      double ab = alpha[i] * beta[j];
      double p = or_pi(k, alpha, beta, eps, f, g, i, j);
      p1[i] += p;
      p2[j] += p;
      lin += p * or_c(k, i, j);
      if (p > 0.0) klpi += p * log(p / ab);
      klpi += ab - p;
    }
  double r = lin + eps * klpi + rho1 * or_kl(n, p1, alpha) + rho2 * or_kl(m, p2, beta);
  free(p1); free(p2);
  return r;
}

/* Translation-invariant functional H_eps of Prop. 3 (eq. dual-form-hell). */
double or_h_value(const or_cost *k, const double *alpha, const double *beta, double eps,
                  double rho1, double rho2, const double *fb, const double *gb) {
  const int n = k->n, m = k->m;
  const double tau1 = rho1 / (rho1 + rho2), tau2 = rho2 / (rho1 + rho2);
  double ma = 0.0, mb = 0.0, A = 0.0, B = 0.0;
  for (int i = 0; i < n; ++i) { ma += alpha[i]; A += alpha[i] * exp(-fb[i] / rho1); }
  for (int j = 0; j < m; ++j) { mb += beta[j]; B += beta[j] * exp(-gb[j] / rho2); }
  double mpi = or_plan_mass(k, alpha, beta, eps, fb, gb);
  return rho1 * ma + rho2 * mb - eps * (mpi - ma * mb) - (rho1 + rho2) * pow(A, tau1) * pow(B, tau2);
}

/*
 * Envelope-theorem gradients of UOT = sup F_eps at optimal (f, g), each scaled by gout:
 *   dUOT/dalpha_i = rho1 (1 - e^{-f_i/rho1}) - eps (sum_j beta_j e^{(f_i+g_j-C_ij)/eps} - m(beta))
 *   dUOT/dbeta_j  = rho2 (1 - e^{-g_j/rho2}) - eps (sum_i alpha_i e^{(f_i+g_j-C_ij)/eps} - m(alpha))
 *   dUOT/dx_i     = sum_j pi_ij grad_x c(x_i, y_j),  dUOT/dy_j = sum_i pi_ij grad_y c(x_i, y_j)
 * with c = ||x - y||^p, grad_x c = p ||x-y||^{p-2} (x - y) (taken as 0 at x = y).
 * These are the partial derivatives of eq. (dual-uot-kl) in (alpha, beta, C), as the
 * envelope argument of Prop. 1 uses them. Any output pointer may be NULL.
 */
void or_gradients(const or_cost *k, const double *alpha, const double *beta, double eps, double rho1,
                  double rho2, const double *f, const double *g, double gout, double *dx, double *dy,
                  double *dalpha, double *dbeta) {
  const int n = k->n, m = k->m, d = k->d;
  double ma = 0.0, mb = 0.0;
  for (int i = 0; i < n; ++i) ma += alpha[i];
  for (int j = 0; j < m; ++j) mb += beta[j];
  if (dalpha) {
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
      double s = 0.0;
      for (int j = 0; j < m; ++j)
        if (beta[j] != 0.0) s += beta[j] * exp((f[i] + g[j] - or_c(k, i, j)) / eps);
      dalpha[i] = gout * (rho1 * (1.0 - exp(-f[i] / rho1)) - eps * (s - mb));
    }
  }
  if (dbeta) {
#pragma omp parallel for schedule(static)
    for (int j = 0; j < m; ++j) {
      double s = 0.0;
      for (int i = 0; i < n; ++i)
        if (alpha[i] != 0.0) s += alpha[i] * exp((f[i] + g[j] - or_c(k, i, j)) / eps);
      dbeta[j] = gout * (rho2 * (1.0 - exp(-g[j] / rho2)) - eps * (s - ma));
    }
  }
  if (k->C) return; /* dense cost: no point gradients */
  if (dx) {
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
      for (int t = 0; t < d; ++t) dx[(long)i * d + t] = 0.0;
      for (int j = 0; j < m; ++j) {
        double p = or_pi(k, alpha, beta, eps, f, g, i, j);
        double s = 0.0;
        for (int t = 0; t < d; ++t) {
          double u = k->x[(long)i * d + t] - k->y[(long)j * d + t];
          s += u * u;
        }
        double w = (k->p == 2.0) ? 2.0 : (s > 0.0 ? k->p * pow(sqrt(s), k->p - 2.0) : 0.0);
        for (int t = 0; t < d; ++t)
          dx[(long)i * d + t] += gout * p * w * (k->x[(long)i * d + t] - k->y[(long)j * d + t]);
      }
    }
  }
  if (dy) {
#pragma omp parallel for schedule(static)
    for (int j = 0; j < m; ++j) {
      for (int t = 0; t < d; ++t) dy[(long)j * d + t] = 0.0;
      for (int i = 0; i < n; ++i) {
        double p = or_pi(k, alpha, beta, eps, f, g, i, j);
        double s = 0.0;
        for (int t = 0; t < d; ++t) {
          double u = k->x[(long)i * d + t] - k->y[(long)j * d + t];
          s += u * u;
        }
        double w = (k->p == 2.0) ? 2.0 : (s > 0.0 ? k->p * pow(sqrt(s), k->p - 2.0) : 0.0);
        for (int t = 0; t < d; ++t)
          dy[(long)j * d + t] += gout * p * w * (k->y[(long)j * d + t] - k->x[(long)i * d + t]);
      }
    }
  }
}
