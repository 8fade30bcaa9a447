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
constexpr int kFwWaves = kFwThreads / 64;

__device__ __forceinline__ double cost1d(double x, double y, double p) {
  const double d = fabs(x - y);
  return p == 2.0 ? d * d : (p == 1.0 ? d : pow(d, p));
}

// Block-wide reductions (broadcast to every thread).
__device__ double fw_sum(double v) {
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
__device__ double fw_max(double v) {
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
__device__ int fw_min_int(int v) {
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
  __device__ void reduce(double &logs0, double &r1, double &r2) {
    const double M = fw_max(m);
    const double c = (m == -INFINITY) ? 0.0 : exp(m - M);
    const double t0 = fw_sum(s0 * c), t1 = fw_sum(s1 * c), t2 = fw_sum(s2 * c);
    logs0 = M + log(t0);
    r1 = t1 / t0;
    r2 = t2 / t0;
  }
};

// In-place inclusive prefix sum of v[0..n) by the block: each thread owns a contiguous
// chunk; the chunk totals are scanned within each wave by lane shuffles and across the
// waves through LDS.
__device__ void fw_scan(double *v, int n) {
  __shared__ double sh[kFwWaves];
  const int chunk = (n + kFwThreads - 1) / kFwThreads;
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
  int *jst, *ist;                      // row start columns [N], column start rows [M]
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
    int *jst = a.jst + o1, *ist = a.ist + o2;
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
      double LA, LB, dummy1, dummy2;
      la.reduce(LA, dummy1, dummy2);
      lb.reduce(LB, dummy1, dummy2);
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
      fw_scan(Ac, n);
      fw_scan(Bc, m);
      // co-ranks of the merge: start column of each row, start row of each column
      {
        const int total = n + m;
        const int per = (total + kFwThreads - 1) / kFwThreads;
        const int d0 = min(total, (int)threadIdx.x * per), d1 = min(total, d0 + per);
        int ai = fw_corank(d0, Ac, n, Bc, m), bi = d0 - ai;
        for (int d = d0; d < d1; ++d) {
          if (ai < n && (bi >= m || Ac[ai] <= Bc[bi])) {
            if (ai + 1 < n) jst[ai + 1] = min(bi, m - 1);
            ++ai;
          } else {
            if (bi + 1 < m) ist[bi + 1] = min(ai, n - 1);
            ++bi;
          }
        }
      }
      __syncthreads();
      // potentials of the oracle: prefix sums of cost differences along the walk
      for (int i = threadIdx.x; i < n; i += kFwThreads) {
        if (i == 0) { r[0] = 0.0; continue; }
        const int j = jst[i];
        r[i] = cost1d(x[i], y[j], p) - cost1d(x[i - 1], y[j], p);
      }
      for (int j = threadIdx.x; j < m; j += kFwThreads) {
        if (j == 0) { s[0] = cost1d(x[0], y[0], p); continue; }
        const int i = ist[j];
        s[j] = cost1d(x[i], y[j], p) - cost1d(x[i], y[j - 1], p);
      }
      __syncthreads();
      fw_scan(r, n);
      fw_scan(s, m);
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
          pa.reduce(l0, a1, a2);
          pb.reduce(m0, b1, b2);
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
    double LA, LB, u1, u2;
    la.reduce(LA, u1, u2);
    lb.reduce(LB, u1, u2);
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

}  // namespace

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
  a.jst = l.jst;
  a.ist = l.ist;
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
