// Frank-Wolfe for unregularised 1-D KL-UOT (Sec. 4), many independent problems: one
// workgroup owns one problem at a time and runs all of its iterations (problems never
// interact, so no grid-wide synchronisation is needed). Everything is double precision.
//
// One iteration on (fb, gb):
//  * A = <alpha, e^{-fb/rho1}>, B = <beta, e^{-gb/rho2}> (log-sum-exp); lambda* =
//    rho1 rho2/(rho1 + rho2) log(A/B) (Prop. 2); the gradient of H_0 is the pair of tilted
//    histograms alpha e^{-(fb + lambda*)/rho1}, beta e^{-(gb - lambda*)/rho2}, of common mass
//    Mt = A e^{-lambda*/rho1}; normalised, they are alpha e^{-fb/rho1}/A and beta e^{-gb/rho2}/B.
//  * Linear oracle = balanced 1-D OT between the sorted supports with those weights, solved by
//    the monotone coupling. With the inclusive CDFs Ac, Bc, the coupling's walk steps down
//    from cell (i, j) iff Ac_i <= Bc_j, so row i + 1 starts at column #{j : Bc_j < Ac_i} and
//    column j + 1 at row #{i : Ac_i <= Bc_j}: the co-ranks of a merge of Ac and Bc in which
//    rows go first on ties (merge path: one binary search per thread, then a sequential
//    merge of its share). The walk's cells are tight, so r_{i+1} - r_i =
//    C(i+1, j_{i+1}) - C(i, j_{i+1}) and s_{j+1} - s_j = C(i_{j+1}, j+1) - C(i_{j+1}, j):
//    prefix sums from r_0 = 0, s_0 = C(0, 0).
//  * Gap = Mt (<at, r - fb> + <bt, s - gb>) with the normalised histograms; stop if <= tol.
//  * Step gamma = 2/(2 + t), or the maximiser of H_0 on the segment: H_0 = const -
//    (rho1 + rho2) a^{tau1} b^{tau2} (a, b: A and B along the segment), so gamma minimises the
//    convex psi = tau1 log a + tau2 log b on [0, 1], by Newton's method on psi' inside a
//    shrinking bracket.
#include <cfloat>

#include "uot_batched.h"
#include "uot_internal.h"

namespace uot {
namespace {

constexpr int kFwThreads = 256;

__device__ __forceinline__ double cost1d(double x, double y, double p) {
  const double d = fabs(x - y);
  return p == 2.0 ? d * d : (p == 1.0 ? d : pow(d, p));
}

// Block-wide reductions over NT threads (broadcast to every thread).
template <int NT = kFwThreads>
__device__ double fw_sum(double v) {
  constexpr int kFwWaves = NT / 64;
  __shared__ double sh[kFwWaves];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = sh[0];
#pragma unroll
  for (int k = 1; k < kFwWaves; ++k) s += sh[k];
  __syncthreads();
  return s;
}
template <int NT = kFwThreads>
__device__ double fw_max(double v) {
  constexpr int kFwWaves = NT / 64;
  __shared__ double sh[kFwWaves];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = sh[0];
#pragma unroll
  for (int k = 1; k < kFwWaves; ++k) s = fmax(s, sh[k]);
  __syncthreads();
  return s;
}
template <int NT = kFwThreads>
__device__ int fw_min_int(int v) {
  constexpr int kFwWaves = NT / 64;
  __shared__ int sh[kFwWaves];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  int s = sh[0];
#pragma unroll
  for (int k = 1; k < kFwWaves; ++k) s = min(s, sh[k]);
  __syncthreads();
  return s;
}

// Online log-sum-exp triple over one side: running max m and sums of e^{v - m} times
// (1, u, u^2); merged across the block. Returns log S0 and the ratios S1/S0, S2/S0.
struct Lse3 {
  double m = -INFINITY, s0 = 0.0, s1 = 0.0, s2 = 0.0;
  __device__ void add(double v, double u) {
    if (v == -INFINITY) return;
    if (v > m) {
      const double c = exp(m - v);
      s0 *= c; s1 *= c; s2 *= c;
      m = v;
    }
    const double e = exp(v - m);
    s0 += e; s1 += e * u; s2 += e * u * u;
  }
  template <int NT = kFwThreads>
  __device__ void reduce(double &logs0, double &r1, double &r2) {
    const double M = fw_max<NT>(m);
    const double c = (m == -INFINITY) ? 0.0 : exp(m - M);
    const double t0 = fw_sum<NT>(s0 * c), t1 = fw_sum<NT>(s1 * c), t2 = fw_sum<NT>(s2 * c);
    logs0 = M + log(t0);
    r1 = t1 / t0;
    r2 = t2 / t0;
  }
};

// In-place inclusive prefix sum of v[0..n) by the block: each thread owns a contiguous
// chunk; the chunk totals are scanned within each wave by lane shuffles and across the
// waves through LDS.
template <int NT = kFwThreads>
__device__ void fw_scan(double *v, int n) {
  constexpr int kFwWaves = NT / 64;
  __shared__ double sh[kFwWaves];
  const int chunk = (n + NT - 1) / NT;
  const int i0 = min(n, (int)threadIdx.x * chunk), i1 = min(n, i0 + chunk);
  double s = 0.0;
  for (int i = i0; i < i1; ++i) s += v[i];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double inc = s;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const double up = __shfl_up(inc, o, 64);
    if (lane >= o) inc += up;
  }
  if (lane == 63) sh[wave] = inc;
  __syncthreads();
  double run = inc - s;  // exclusive prefix within the wave
  for (int w = 0; w < wave; ++w) run += sh[w];
  for (int i = i0; i < i1; ++i) {
    run += v[i];
    v[i] = run;
  }
  __syncthreads();
}

// K values reduced together (one LDS exchange and two barriers for all of them; each value
// is summed, or maximised, in the same order as fw_sum / fw_max would).
template <int K, int NT = kFwThreads>
__device__ void fw_sum_k(double (&v)[K]) {
  constexpr int kW = NT / 64;
  __shared__ double sh[K][kW];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1)
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] += __shfl_xor(v[k], o, 64);
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int k = 0; k < K; ++k) sh[k][threadIdx.x >> 6] = v[k];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double t = sh[k][0];
#pragma unroll
    for (int w = 1; w < kW; ++w) t += sh[k][w];
    v[k] = t;
  }
  __syncthreads();
}
template <int K, int NT = kFwThreads>
__device__ void fw_max_k(double (&v)[K]) {
  constexpr int kW = NT / 64;
  __shared__ double sh[K][kW];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1)
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = fmax(v[k], __shfl_xor(v[k], o, 64));
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int k = 0; k < K; ++k) sh[k][threadIdx.x >> 6] = v[k];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double t = sh[k][0];
#pragma unroll
    for (int w = 1; w < kW; ++w) t = fmax(t, sh[k][w]);
    v[k] = t;
  }
  __syncthreads();
}

// Lse3::reduce of two sides at once (same arithmetic, four barriers instead of sixteen).
__device__ void lse3_reduce2(const Lse3 &a, const Lse3 &b, double &la, double &a1, double &a2,
                             double &lb, double &b1, double &b2) {
  double M[2] = {a.m, b.m};
  fw_max_k<2>(M);
  const double ca = (a.m == -INFINITY) ? 0.0 : exp(a.m - M[0]);
  const double cb = (b.m == -INFINITY) ? 0.0 : exp(b.m - M[1]);
  double S[6] = {a.s0 * ca, a.s1 * ca, a.s2 * ca, b.s0 * cb, b.s1 * cb, b.s2 * cb};
  fw_sum_k<6>(S);
  la = M[0] + log(S[0]);
  a1 = S[1] / S[0];
  a2 = S[2] / S[0];
  lb = M[1] + log(S[3]);
  b1 = S[4] / S[3];
  b2 = S[5] / S[3];
}

// fw_scan of two arrays at once (one LDS exchange).
__device__ void fw_scan2(double *v, int n, double *u, int m) {
  constexpr int kW = kFwThreads / 64;
  __shared__ double sh[2][kW];
  const int cv = (n + kFwThreads - 1) / kFwThreads, cu = (m + kFwThreads - 1) / kFwThreads;
  const int i0 = min(n, (int)threadIdx.x * cv), i1 = min(n, i0 + cv);
  const int j0 = min(m, (int)threadIdx.x * cu), j1 = min(m, j0 + cu);
  double sv = 0.0, su = 0.0;
  for (int i = i0; i < i1; ++i) sv += v[i];
  for (int j = j0; j < j1; ++j) su += u[j];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double iv = sv, iu = su;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const double pv = __shfl_up(iv, o, 64), pu = __shfl_up(iu, o, 64);
    if (lane >= o) {
      iv += pv;
      iu += pu;
    }
  }
  if (lane == 63) {
    sh[0][wave] = iv;
    sh[1][wave] = iu;
  }
  __syncthreads();
  double rv = iv - sv, ru = iu - su;  // exclusive prefixes within the wave
  for (int w = 0; w < wave; ++w) {
    rv += sh[0][w];
    ru += sh[1][w];
  }
  for (int i = i0; i < i1; ++i) {
    rv += v[i];
    v[i] = rv;
  }
  for (int j = j0; j < j1; ++j) {
    ru += u[j];
    u[j] = ru;
  }
  __syncthreads();
}

// Number of Ac elements among the first k merged elements (rows first on ties).
__device__ int fw_corank(int k, const double *Ac, int n, const double *Bc, int m) {
  int lo = max(0, k - m), hi = min(k, n);
  while (lo < hi) {
    const int a = (lo + hi) >> 1, b = k - a;
    if (b > 0 && a < n && Bc[b - 1] >= Ac[a]) lo = a + 1; else hi = a;
  }
  return lo;
}

struct FwArgs {
  int B;
  const int64_t *offN, *offM;  // device [B + 1]
  const float *x, *y, *alpha, *beta;
  const double *rho1, *rho2;
  double p;
  int line_search, max_iter;
  double tol;
  double *fb, *gb, *Ac, *Bc, *r, *s;  // [N] / [M] per problem at the problem's offsets
  float *f, *g;
  int32_t *iters;
  double *gap;
  int32_t *status;
};

// Validation of one problem: sorted supports, finite nonnegative weights with positive
// masses, finite positive penalties.
__device__ bool fw_valid(const FwArgs &a, int64_t o1, int n, int64_t o2, int m, double r1,
                         double r2) {
  int bad = 0;
  double ma = 0.0, mb = 0.0;
  for (int i = threadIdx.x; i < n; i += kFwThreads) {
    const float w = a.alpha[o1 + i];
    if (!(w >= 0.0f) || !isfinite(w)) bad = 1;
    ma += w;
    if (i + 1 < n && !(a.x[o1 + i] <= a.x[o1 + i + 1])) bad = 1;
  }
  for (int j = threadIdx.x; j < m; j += kFwThreads) {
    const float w = a.beta[o2 + j];
    if (!(w >= 0.0f) || !isfinite(w)) bad = 1;
    mb += w;
    if (j + 1 < m && !(a.y[o2 + j] <= a.y[o2 + j + 1])) bad = 1;
  }
  ma = fw_sum(ma);
  mb = fw_sum(mb);
  bad = -fw_min_int(-bad);
  return !bad && ma > 0.0 && mb > 0.0 && isfinite(r1) && isfinite(r2) && r1 > 0.0 && r2 > 0.0;
}

__global__ __launch_bounds__(kFwThreads) void k_fw1d(FwArgs a) {
  __shared__ double sgam;
  for (int prob = blockIdx.x; prob < a.B; prob += gridDim.x) {
    const int64_t o1 = a.offN[prob], o2 = a.offM[prob];
    const int n = (int)(a.offN[prob + 1] - o1), m = (int)(a.offM[prob + 1] - o2);
    const double r1 = a.rho1[prob], r2 = a.rho2[prob], p = a.p;
    const double tau1 = r1 / (r1 + r2), tau2 = r2 / (r1 + r2);
    const float *x = a.x + o1, *y = a.y + o2, *al = a.alpha + o1, *be = a.beta + o2;
    double *fb = a.fb + o1, *gb = a.gb + o2, *Ac = a.Ac + o1, *Bc = a.Bc + o2;
    double *r = a.r + o1, *s = a.s + o2;
    if (!fw_valid(a, o1, n, o2, m, r1, r2)) {
      for (int i = threadIdx.x; i < n; i += kFwThreads) a.f[o1 + i] = NAN;
      for (int j = threadIdx.x; j < m; j += kFwThreads) a.g[o2 + j] = NAN;
      if (threadIdx.x == 0) {
        a.status[prob] = kBatchInvalid;
        a.iters[prob] = 0;
        a.gap[prob] = NAN;
      }
      __syncthreads();
      continue;
    }
    for (int i = threadIdx.x; i < n; i += kFwThreads) fb[i] = 0.0;
    for (int j = threadIdx.x; j < m; j += kFwThreads) gb[j] = 0.0;
    __syncthreads();
    double gap = INFINITY;
    int t = 0;
    for (; t < a.max_iter; ++t) {
      // log A, log B, lambda*
      Lse3 la, lb;
      for (int i = threadIdx.x; i < n; i += kFwThreads) {
        const double w = al[i];
        la.add(w > 0.0 ? log(w) - fb[i] / r1 : -INFINITY, 0.0);
      }
      for (int j = threadIdx.x; j < m; j += kFwThreads) {
        const double w = be[j];
        lb.add(w > 0.0 ? log(w) - gb[j] / r2 : -INFINITY, 0.0);
      }
      double LA, LB, dummy1, dummy2, dummy3, dummy4;
      lse3_reduce2(la, lb, LA, dummy1, dummy2, LB, dummy3, dummy4);
      const double lam = r1 * r2 / (r1 + r2) * (LA - LB);
      const double logmt = LA - lam / r1;  // log of the common tilted mass
      // normalised tilted histograms, then their CDFs
      for (int i = threadIdx.x; i < n; i += kFwThreads) {
        const double w = al[i];
        Ac[i] = w > 0.0 ? exp(log(w) - fb[i] / r1 - LA) : 0.0;
      }
      for (int j = threadIdx.x; j < m; j += kFwThreads) {
        const double w = be[j];
        Bc[j] = w > 0.0 ? exp(log(w) - gb[j] / r2 - LB) : 0.0;
      }
      __syncthreads();
      fw_scan2(Ac, n, Bc, m);
      // the walk of the monotone coupling by merge path (co-ranks of the merge: each thread
      // takes a share of the diagonals); where row i + 1 starts at column j it writes the
      // oracle's potential step r_{i+1} - r_i = C(i+1, j) - C(i, j), where column j + 1
      // starts at row i, s_{j+1} - s_j = C(i, j+1) - C(i, j)
      {
        const int total = n + m;
        const int per = (total + kFwThreads - 1) / kFwThreads;
        const int d0 = min(total, (int)threadIdx.x * per), d1 = min(total, d0 + per);
        int ai = fw_corank(d0, Ac, n, Bc, m), bi = d0 - ai;
        for (int d = d0; d < d1; ++d) {
          if (ai < n && (bi >= m || Ac[ai] <= Bc[bi])) {
            if (ai + 1 < n) {
              const int j = min(bi, m - 1);
              r[ai + 1] = cost1d(x[ai + 1], y[j], p) - cost1d(x[ai], y[j], p);
            }
            ++ai;
          } else {
            if (bi + 1 < m) {
              const int i = min(ai, n - 1);
              s[bi + 1] = cost1d(x[i], y[bi + 1], p) - cost1d(x[i], y[bi], p);
            }
            ++bi;
          }
        }
        if (threadIdx.x == 0) {
          r[0] = 0.0;
          s[0] = cost1d(x[0], y[0], p);
        }
      }
      __syncthreads();
      fw_scan2(r, n, s, m);
      // Frank-Wolfe gap with the gradient pair (normalised histograms times the mass)
      double gp = 0.0;
      for (int i = threadIdx.x; i < n; i += kFwThreads)
        gp += (Ac[i] - (i > 0 ? Ac[i - 1] : 0.0)) * (r[i] - fb[i]);
      for (int j = threadIdx.x; j < m; j += kFwThreads)
        gp += (Bc[j] - (j > 0 ? Bc[j - 1] : 0.0)) * (s[j] - gb[j]);
      gap = exp(logmt) * fw_sum(gp);
      if (a.tol > 0.0 && gap <= a.tol) break;
      double gamma = 2.0 / (2.0 + t);
      if (a.line_search) {
        // psi(gamma) = tau1 log a + tau2 log b along fb + gamma (r - fb), gb + gamma (s - gb):
        // psi' = tau1 <u>_a + tau2 <u>_b, psi'' = tau1 var_a(u) + tau2 var_b(u) with
        // u = -(r - fb)/rho1 on the f side (-(s - gb)/rho2 on the g side) and <.>_a the
        // average under the weights alpha e^{-f_gamma/rho1} (likewise b). psi' < 0: H_0 still
        // increases at gamma.
        auto derivs = [&](double gm, double &d1, double &d2) {
          Lse3 pa, pb;
          for (int i = threadIdx.x; i < n; i += kFwThreads) {
            const double w = al[i], dl = r[i] - fb[i];
            pa.add(w > 0.0 ? log(w) - (fb[i] + gm * dl) / r1 : -INFINITY, -dl / r1);
          }
          for (int j = threadIdx.x; j < m; j += kFwThreads) {
            const double w = be[j], dl = s[j] - gb[j];
            pb.add(w > 0.0 ? log(w) - (gb[j] + gm * dl) / r2 : -INFINITY, -dl / r2);
          }
          double l0, a1, a2, m0, b1, b2;
          lse3_reduce2(pa, pb, l0, a1, a2, m0, b1, b2);
          d1 = tau1 * a1 + tau2 * b1;
          d2 = tau1 * (a2 - a1 * a1) + tau2 * (b2 - b1 * b1);
        };
        double d1, d2;
        derivs(0.0, d1, d2);
        if (!(d1 < 0.0)) {
          gamma = 0.0;  // no ascent along the segment
        } else {
          derivs(1.0, d1, d2);
          if (d1 <= 0.0) {
            gamma = 1.0;
          } else {
            double lo = 0.0, hi = 1.0, gm = 0.5;
            for (int it = 0; it < 100; ++it) {
              derivs(gm, d1, d2);
              if (d1 < 0.0) lo = gm; else hi = gm;
              double ng = d2 > 0.0 ? gm - d1 / d2 : 0.5 * (lo + hi);
              if (!(ng > lo && ng < hi)) ng = 0.5 * (lo + hi);
              const bool stop = d1 == 0.0 || !(fabs(ng - gm) > 1e-15) || !(hi - lo > 1e-15);
              gm = ng;
              if (stop) break;
            }
            gamma = gm;
          }
        }
      }
      if (threadIdx.x == 0) sgam = gamma;
      __syncthreads();
      gamma = sgam;
      for (int i = threadIdx.x; i < n; i += kFwThreads) fb[i] = (1.0 - gamma) * fb[i] + gamma * r[i];
      for (int j = threadIdx.x; j < m; j += kFwThreads) gb[j] = (1.0 - gamma) * gb[j] + gamma * s[j];
      __syncthreads();
    }
    const int run = t < a.max_iter ? t + 1 : a.max_iter;
    // reported potentials (fb + lambda*, gb - lambda*)
    Lse3 la, lb;
    for (int i = threadIdx.x; i < n; i += kFwThreads) {
      const double w = al[i];
      la.add(w > 0.0 ? log(w) - fb[i] / r1 : -INFINITY, 0.0);
    }
    for (int j = threadIdx.x; j < m; j += kFwThreads) {
      const double w = be[j];
      lb.add(w > 0.0 ? log(w) - gb[j] / r2 : -INFINITY, 0.0);
    }
    double LA, LB, u1, u2, u3, u4;
    lse3_reduce2(la, lb, LA, u1, u2, LB, u3, u4);
    const double lam = r1 * r2 / (r1 + r2) * (LA - LB);
    bool finite = true;
    for (int i = threadIdx.x; i < n; i += kFwThreads) {
      const double v = fb[i] + lam;
      finite = finite && isfinite(v);
      a.f[o1 + i] = (float)v;
    }
    for (int j = threadIdx.x; j < m; j += kFwThreads) {
      const double v = gb[j] - lam;
      finite = finite && isfinite(v);
      a.g[o2 + j] = (float)v;
    }
    const int allfinite = fw_min_int(finite ? 1 : 0);
    if (threadIdx.x == 0) {
      a.iters[prob] = run;
      a.gap[prob] = gap;
      a.status[prob] = !allfinite ? kBatchNumeric
                       : (a.tol > 0.0 && gap <= a.tol) ? kBatchConverged
                                                       : kBatchMaxIter;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------------------
// Unbalanced 1-D barycenters (Sec. 5): Frank-Wolfe on the translation-invariant
// multi-marginal dual, squared distance ground cost, one workgroup per problem of K measures.
// The linear oracle is the balanced multi-marginal walk: at each step the measure with the
// least remaining mass (the first on ties) advances, i.e. measure k leaves its point i at
// the level Ac_k[i] of its normalised CDF, and the events happen in the order of these levels
// (ties: smaller k first). At the event (k, i) the other measures stand at their co-ranks:
// #{i' : Ac_j[i'] <= level} for j < k and #{i' : Ac_j[i'] < level} for j > k. Every visited
// tuple is tight, so f_{k,i+1} - f_{k,i} = C(tuple after) - C(tuple before): prefix sums per
// measure from f_{0,0} = C(first tuple), f_{k,0} = 0.
// ---------------------------------------------------------------------------------------
constexpr int kBaryMaxK = kBaryMaxMeasures;

struct BaryArgs {
  int B, K;
  const int64_t *off;   // device [B*K + 1]: measure m = b*K + k owns [off[m], off[m+1])
  const float *x, *alpha;
  const double *w;      // [B*K]
  const double *rho;    // [B]
  int max_iter;
  double tol;
  double *fb, *Ac, *r;  // per point
  float *f;             // per point (out)
  float *bx, *bw;       // per problem [off[(b+1)K] - off[bK] - K + 1] at offset off[bK] - bK + b
  int32_t *iters;
  double *gap;
  int32_t *status;
};

// Number of entries of the sorted a[0..n) that are < v (strict) or <= v.
__device__ __forceinline__ int count_below(const double *a, int n, double v, bool inclusive) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (inclusive ? a[mid] <= v : a[mid] < v) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// Tuple costs for the squared distance: C(z) = sum_k w_k (z_k - b)^2 with the barycentric
// point b = sum_k w_k z_k / sw, i.e. C = sum_k w_k z_k^2 - (sum_k w_k z_k)^2 / sw. Moving one
// entry z_k by d changes it by w_k d (2 z_k + d - (2 S1 + w_k d) / sw), S1 = sum_k w_k z_k
// before the move; the walk needs only S1 per event, no per-tuple arrays.
__device__ __forceinline__ double move_cost(double wk, double zk, double d, double s1, double sw) {
  return wk * d * (2.0 * zk + d - (2.0 * s1 + wk * d) / sw);
}

template <int NT>
__global__ __launch_bounds__(NT) void k_fw_bary(BaryArgs a) {
  __shared__ double q[kBaryMaxK], lam[kBaryMaxK], wsh[kBaryMaxK];
  __shared__ int cur_sh[kBaryMaxK * NT];
  __shared__ int64_t o[kBaryMaxK + 1];
  const int K = a.K;
  for (int prob = blockIdx.x; prob < a.B; prob += gridDim.x) {
    const int m0 = prob * K;
    if (threadIdx.x <= K) o[threadIdx.x] = a.off[m0 + threadIdx.x];
    if (threadIdx.x < K) wsh[threadIdx.x] = a.w[m0 + threadIdx.x];
    __syncthreads();
    const double rho = a.rho[prob];
    double sw = 0.0;
    for (int k = 0; k < K; ++k) sw += wsh[k];
    // the first tuple (every measure at its first point): its cost and barycentric point
    double first_cost = 0.0, first_b = 0.0;
    for (int k = 0; k < K; ++k) first_b += wsh[k] * (double)a.x[o[k]];
    first_b /= sw;
    for (int k = 0; k < K; ++k) {
      const double u = (double)a.x[o[k]] - first_b;
      first_cost += wsh[k] * u * u;
    }
    const int64_t base = o[0];
    const int64_t tot = o[K] - base;
    float *bx = a.bx + (base - m0 + prob), *bw = a.bw + (base - m0 + prob);
    const int T = (int)(tot - K);  // events; T + 1 visited tuples
    // validation: sorted supports, finite nonnegative weights, positive masses and penalties
    int bad = !(rho > 0.0) || !isfinite(rho);
    for (int k = 0; k < K; ++k) bad |= !(wsh[k] > 0.0) || !isfinite(wsh[k]);
    for (int64_t e = threadIdx.x; e < tot; e += NT) {
      const int64_t g = base + e;
      const float v = a.alpha[g];
      if (!(v >= 0.0f) || !isfinite(v)) bad = 1;
      int k = 0;
      while (g >= o[k + 1]) ++k;
      if (g + 1 < o[k + 1] && !(a.x[g] <= a.x[g + 1])) bad = 1;
    }
    for (int k = 0; k < K; ++k) {
      double mk = 0.0;
      for (int64_t g = o[k] + threadIdx.x; g < o[k + 1]; g += NT) mk += a.alpha[g];
      mk = fw_sum<NT>(mk);
      bad |= !(mk > 0.0);
    }
    bad = -fw_min_int<NT>(-bad);
    if (bad) {
      for (int64_t e = threadIdx.x; e < tot; e += NT) a.f[base + e] = NAN;
      if (threadIdx.x == 0) { a.status[prob] = kBatchInvalid; a.iters[prob] = 0; a.gap[prob] = NAN; }
      __syncthreads();
      continue;
    }
    double *fb = a.fb + base, *Ac = a.Ac + base, *r = a.r + base;
    for (int64_t e = threadIdx.x; e < tot; e += NT) fb[e] = 0.0;
    __syncthreads();

    // q_k = log <alpha_k, e^{-fb_k/(w_k rho)}> and lambda* (closed form); then Ac = the
    // normalised tilted CDFs. Returns log of the common tilted mass.
    auto tilt = [&]() -> double {
      for (int k = 0; k < K; ++k) {
        Lse3 l;
        const double sc = 1.0 / (wsh[k] * rho);
        for (int64_t g = o[k] + threadIdx.x; g < o[k + 1]; g += NT) {
          const double v = a.alpha[g];
          l.add(v > 0.0 ? log(v) - fb[g - base] * sc : -INFINITY, 0.0);
        }
        double lq, u1, u2;
        l.reduce<NT>(lq, u1, u2);
        if (threadIdx.x == 0) q[k] = lq;
      }
      __syncthreads();
      double sq = 0.0;
      for (int k = 0; k < K; ++k) sq += wsh[k] * rho * q[k];
      if (threadIdx.x < K) lam[threadIdx.x] = wsh[threadIdx.x] * rho * q[threadIdx.x] - wsh[threadIdx.x] / sw * sq;
      for (int k = 0; k < K; ++k) {
        const double sc = 1.0 / (wsh[k] * rho);
        for (int64_t g = o[k] + threadIdx.x; g < o[k + 1]; g += NT) {
          const double v = a.alpha[g];
          Ac[g - base] = v > 0.0 ? exp(log(v) - fb[g - base] * sc - q[k]) : 0.0;
        }
      }
      __syncthreads();
      for (int k = 0; k < K; ++k) fw_scan<NT>(Ac + (o[k] - base), (int)(o[k + 1] - o[k]));
      return q[0] - lam[0] / (wsh[0] * rho);
    };

    // the walk: potentials into r (oracle mode) or the barycenter (plan mode). Each thread
    // takes a contiguous run of points; along a run within one measure the levels do not
    // decrease, so the co-ranks in the other measures are found by one binary search at the
    // run's first event and then by forward steps.
    auto walk = [&](bool plan) {
      const int64_t chunk = (tot + NT - 1) / NT;
      const int64_t e0 = min(tot, (int64_t)threadIdx.x * chunk), e1 = min(tot, e0 + chunk);
      // forward cursors of this thread's run, one per measure, in LDS (column per thread)
      int *cur = cur_sh + threadIdx.x;
      int curk = -1, k = 0;
      for (int64_t e = e0; e < e1; ++e) {
        const int64_t g = base + e;
        while (g >= o[k + 1]) ++k;
        const int i = (int)(g - o[k]);
        const int nk = (int)(o[k + 1] - o[k]);
        if (i == 0 && !plan) r[e] = k == 0 ? first_cost : 0.0;
        if (i + 1 >= nk) continue;  // the last point never leaves
        const double lev = Ac[e];
        const double xk = a.x[g];
        double s1 = wsh[k] * xk;  // sum_j w_j z_j of the tuple before the event
        int pos = i;
        for (int jj = 0; jj < K; ++jj) {
          if (jj == k) continue;
          const int nj = (int)(o[jj + 1] - o[jj]);
          const double *aj = Ac + (o[jj] - base);
          int c;
          if (k != curk) {
            c = count_below(aj, nj, lev, jj < k);
          } else {
            c = cur[jj * NT];
            if (jj < k) { while (c < nj && aj[c] <= lev) ++c; }
            else { while (c < nj && aj[c] < lev) ++c; }
          }
          cur[jj * NT] = c;
          // clamped: a level at or past a measure's total (rounding, trailing zero weights)
          // leaves it at its last point, and keeps pos inside [0, T)
          const int cc = min(c, nj - 1);
          pos += cc;
          s1 += wsh[jj] * (double)a.x[o[jj] + cc];
        }
        curk = k;
        const double d = (double)a.x[g + 1] - xk;
        if (!plan) {
          r[e + 1] = move_cost(wsh[k], xk, d, s1, sw);
        } else {
          // the barycentric point of the tuple after the event at merged position pos
          bx[pos + 1] = (float)((s1 + wsh[k] * d) / sw);
          r[pos] = lev;  // the event's level (r is free in plan mode)
        }
      }
      __syncthreads();
    };

    double gap = INFINITY;
    int t = 0;
    for (; t < a.max_iter; ++t) {
      const double logmt = tilt();
      walk(false);
      for (int k = 0; k < K; ++k) fw_scan<NT>(r + (o[k] - base), (int)(o[k + 1] - o[k]));
      double gp = 0.0;
      for (int64_t e = threadIdx.x; e < tot; e += NT) {
        const int64_t g = base + e;
        int k = 0;
        while (g >= o[k + 1]) ++k;
        const double an = Ac[e] - (g > o[k] ? Ac[e - 1] : 0.0);
        gp += an * (r[e] - fb[e]);
      }
      gap = exp(logmt) * fw_sum<NT>(gp);
      if (a.tol > 0.0 && gap <= a.tol) break;
      const double gamma = 2.0 / (2.0 + t);
      for (int64_t e = threadIdx.x; e < tot; e += NT) fb[e] = (1.0 - gamma) * fb[e] + gamma * r[e];
      __syncthreads();
    }
    const int run = t < a.max_iter ? t + 1 : a.max_iter;
    // reported potentials and the barycenter of the final tilted marginals
    const double logmt = tilt();
    const double mt = exp(logmt);
    bool finite = true;
    for (int64_t e = threadIdx.x; e < tot; e += NT) {
      const int64_t g = base + e;
      int k = 0;
      while (g >= o[k + 1]) ++k;
      const double v = fb[e] + lam[k];
      finite = finite && isfinite(v);
      a.f[g] = (float)v;
    }
    if (threadIdx.x == 0) bx[0] = (float)first_b;
    walk(true);
    // masses: tuple tt lies between the events tt - 1 and tt (levels 0 and 1 at the ends)
    for (int tt = threadIdx.x; tt <= T; tt += NT) {
      const double hi = tt < T ? fmin(r[tt], 1.0) : 1.0;
      const double lo = tt > 0 ? fmin(r[tt - 1], 1.0) : 0.0;
      bw[tt] = (float)(fmax(hi - lo, 0.0) * mt);
    }
    __syncthreads();
    const int allfinite = fw_min_int<NT>(finite ? 1 : 0);
    if (threadIdx.x == 0) {
      a.iters[prob] = run;
      a.gap[prob] = gap;
      a.status[prob] = !allfinite ? kBatchNumeric
                       : (a.tol > 0.0 && gap <= a.tol) ? kBatchConverged : kBatchMaxIter;
    }
    __syncthreads();
  }
}

}  // namespace

hipError_t launch_fw_bary(const BaryLaunch &l, hipStream_t s) {
  if (l.K < 2 || l.K > kBaryMaxK) return hipErrorInvalidValue;
  BaryArgs a;
  a.B = l.B;
  a.K = l.K;
  a.off = l.off;
  a.x = l.x;
  a.alpha = l.alpha;
  a.w = l.w;
  a.rho = l.rho;
  a.max_iter = l.max_iter;
  a.tol = l.tol;
  a.fb = l.fb;
  a.Ac = l.Ac;
  a.r = l.r;
  a.f = l.f;
  a.bx = l.bx;
  a.bw = l.bw;
  a.iters = l.iters;
  a.gap = l.gap;
  a.status = l.status;
  const int grid = l.B < l.max_blocks ? l.B : l.max_blocks;
  // 1024 threads (the whole CU; 66.5 KB of LDS with the cursor columns) per problem when
  // there are no more problems than CUs (max_blocks is twice the CU count): the walk's runs
  // are four times shorter and its memory waits spread over 16 waves.
  if (l.B <= l.max_blocks / 2)
    hipLaunchKernelGGL(k_fw_bary<1024>, dim3(grid > 0 ? grid : 1), dim3(1024), 0, s, a);
  else
    hipLaunchKernelGGL(k_fw_bary<kFwThreads>, dim3(grid > 0 ? grid : 1), dim3(kFwThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_fw1d(const FwLaunch &l, hipStream_t s) {
  FwArgs a;
  a.B = l.B;
  a.offN = l.offN;
  a.offM = l.offM;
  a.x = l.x;
  a.y = l.y;
  a.alpha = l.alpha;
  a.beta = l.beta;
  a.rho1 = l.rho1;
  a.rho2 = l.rho2;
  a.p = l.p;
  a.line_search = l.line_search;
  a.max_iter = l.max_iter;
  a.tol = l.tol;
  a.fb = l.fb;
  a.gb = l.gb;
  a.Ac = l.Ac;
  a.Bc = l.Bc;
  a.r = l.r;
  a.s = l.s;
  a.f = l.f;
  a.g = l.g;
  a.iters = l.iters;
  a.gap = l.gap;
  a.status = l.status;
  const int grid = l.B < l.max_blocks ? l.B : l.max_blocks;
  hipLaunchKernelGGL(k_fw1d, dim3(grid > 0 ? grid : 1), dim3(kFwThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace uot
