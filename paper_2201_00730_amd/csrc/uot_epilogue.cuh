// Device helpers shared by the epilogue kernels and the fused softmin kernels: log-sum-exp
// merges, block reductions, centred coordinates, source records and the scalar reduction of
// a half-step (tilted masses, TI translations, lambda*, change, convergence test).
#pragma once

#include <cfloat>

#include "uot_internal.h"

namespace uot {

// Log-sum-exp pair (max, sum of exp(v - max)) merge; (-inf, 0) is the neutral element.
static __device__ __forceinline__ void lse_merge(double &m, double &s, double mo, double so) {
  const double mn = fmax(m, mo);
  if (mn == -INFINITY) { m = mn; s = 0.0; return; }
  s = s * exp(m - mn) + so * exp(mo - mn);
  m = mn;
}

// Block-wide reduction over 256 threads of a log-sum-exp pair (mm, ms), meaning ms e^mm with
// (-inf, 0) neutral, and of a (max, min) range. Maxima and minima go first (lane shuffles,
// then the four wave results through LDS); the sums are then rescaled to the block maximum,
// so the pair costs one exp per thread rather than one per merge level.
static __device__ void block_reduce_part(double &mm, double &ms, double &dmx, double &dmn) {
  constexpr int kWaves = kBlock / 64;
  __shared__ double s[4][kWaves];
  double m = mm, x = dmx, n = dmn;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    m = fmax(m, __shfl_xor(m, o, 64));
    x = fmax(x, __shfl_xor(x, o, 64));
    n = fmin(n, __shfl_xor(n, o, 64));
  }
  const int w = threadIdx.x >> 6;
  const bool lead = (threadIdx.x & 63) == 0;
  if (lead) { s[0][w] = m; s[1][w] = x; s[2][w] = n; }
  __syncthreads();
  m = s[0][0]; x = s[1][0]; n = s[2][0];
#pragma unroll
  for (int k = 1; k < kWaves; ++k) {
    m = fmax(m, s[0][k]);
    x = fmax(x, s[1][k]);
    n = fmin(n, s[2][k]);
  }
  double v = (mm == -INFINITY) ? 0.0 : ms * exp(mm - m);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if (lead) s[3][w] = v;
  __syncthreads();
  double sum = s[3][0];
#pragma unroll
  for (int k = 1; k < kWaves; ++k) sum += s[3][k];
  __syncthreads();
  mm = m;
  ms = sum;
  dmx = x;
  dmn = n;
}

static __device__ double block_sum(double v) {
  __shared__ double s[kBlock];
  const int t = threadIdx.x;
  s[t] = v;
  __syncthreads();
  for (int off = kBlock / 2; off > 0; off >>= 1) {
    if (t < off) s[t] += s[t + off];
    __syncthreads();
  }
  const double r = s[0];
  __syncthreads();
  return r;
}

// Log2-sum over the split partials of one target: M + log2(sum_p l_p 2^{m_p - M}).
static __device__ __forceinline__ double combine_lse2(const float2 *part, int nsplit, int nt, int t) {
  float M = -FLT_MAX;
  for (int p = 0; p < nsplit; ++p) M = fmaxf(M, part[(size_t)p * nt + t].x);
  double L = 0.0;
  for (int p = 0; p < nsplit; ++p) {
    const float2 q = part[(size_t)p * nt + t];
    L += (double)q.y * exp2((double)q.x - (double)M);
  }
  return (double)M + log2(L);
}

// Centred coordinates of one target (as the softmin kernels form them) and their squared norm.
template <int D>
static __device__ __forceinline__ double centred(const float *pts, int d, int t, const double *mu,
                                          float *yc) {
  double n2 = 0.0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    yc[k] = k < d ? pts[(size_t)t * d + k] - (float)mu[k] : 0.0f;
    n2 += (double)yc[k] * (double)yc[k];
  }
  return n2;
}

// Writes the source record of point t with stored potential hf (see rec_stride).
template <int D, int MODE>
static __device__ __forceinline__ void write_record(float *rec, int t, const float *yc, double yn2,
                                             float hf, float w, double sc) {
  const double lw2 = w > 0.0f ? log2((double)w) : -INFINITY;
  float *rp = rec + (size_t)t * rec_stride(MODE, D);
  if constexpr (MODE == kSqEuc) {
#pragma unroll
    for (int k = 0; k < D; ++k) rp[k] = (float)(2.0 * sc * (double)yc[k]);
    rp[D] = (float)(sc * (double)hf + lw2 - sc * yn2);
#pragma unroll
    for (int k = D + 1; k < rec_stride(MODE, D); ++k) rp[k] = 0.0f;  // padding read by MFMA
  } else if constexpr (MODE == kSqEucMx) {
    constexpr int KP = mx_slots(D);
    __bf16 up[D][3], bp[3];
#pragma unroll
    for (int k = 0; k < D; ++k) split3((float)(2.0 * sc * (double)yc[k]), up[k][0], up[k][1], up[k][2]);
    split3((float)(sc * (double)hf + lw2 - sc * yn2), bp[0], bp[1], bp[2]);
    auto slot = [&](int e) -> unsigned {
      const __bf16 v = e < 6 * D ? up[e / 6][mx_piece_u(e % 6)]
                       : e < 6 * D + 3 ? bp[e - 6 * D]
                       : e < 6 * D + 5 ? (__bf16)1.0f : (__bf16)0.0f;
      return (unsigned)__builtin_bit_cast(unsigned short, v);
    };
    unsigned *wp = reinterpret_cast<unsigned *>(rp);
#pragma unroll
    for (int e = 0; e < KP; e += 2) wp[e / 2] = slot(e) | (slot(e + 1) << 16);
  } else if constexpr (MODE == kPower) {
#pragma unroll
    for (int k = 0; k < D; ++k) rp[k] = yc[k];
    rp[D] = (float)(sc * (double)hf + lw2);
#pragma unroll
    for (int k = D + 1; k < rec_stride(MODE, D); ++k) rp[k] = 0.0f;
  } else {
    rp[0] = (float)(sc * (double)hf + lw2);
  }
}

// The early-exit flag is read by softmin blocks while the side reduction may write it, so
// both sides access it atomically (relaxed: a stale read only costs the reader's work).
static __device__ __forceinline__ int32_t get_done(const int32_t *done) {
  return __hip_atomic_load(done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
static __device__ __forceinline__ void set_done(SolveState *st, int32_t v) {
  __hip_atomic_store(&st->done, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The dual update of one potential with the Berg entropy (Sec. 3, g = -aprox_{phi*}(-S)):
// h > -rho solving e^{(h - S)/eps} = rho / (rho + h). In w = log(rho + h) the equation is
// q(w) = (e^w - rho - S)/eps + w - log rho = 0 with q convex, increasing and q' >= 1, so
// Newton's method converges from any start (past the first step, from above and
// monotonically); the KL update rho/(eps + rho) S, kept inside the domain, is the start.
static __device__ double berg_update(double S, double rho, double eps) {
  const double lr = log(rho);
  double w = log(fmax(rho + rho / (eps + rho) * S, 0.5 * rho));
  for (int it = 0; it < 100; ++it) {
    const double e = exp(w);
    const double step = ((e - rho - S) / eps + w - lr) / (e / eps + 1.0);
    w -= step;
    if (!(fabs(step) > 1e-15 * fmax(1.0, fabs(w)))) break;
  }
  return exp(w) - rho;
}

// Block-wide sums (s0, s1) and minima (m0, m1) over NT threads, broadcast to every thread.
template <int NT>
static __device__ void block_sum2(double &s0, double &s1) {
  constexpr int kWaves = NT / 64;
  __shared__ double sh[2][kWaves];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    s0 += __shfl_xor(s0, o, 64);
    s1 += __shfl_xor(s1, o, 64);
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) { sh[0][w] = s0; sh[1][w] = s1; }
  __syncthreads();
  s0 = sh[0][0];
  s1 = sh[1][0];
#pragma unroll
  for (int k = 1; k < kWaves; ++k) { s0 += sh[0][k]; s1 += sh[1][k]; }
  __syncthreads();
}
template <int NT>
static __device__ void block_min2(double &m0, double &m1) {
  constexpr int kWaves = NT / 64;
  __shared__ double sh[2][kWaves];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    m0 = fmin(m0, __shfl_xor(m0, o, 64));
    m1 = fmin(m1, __shfl_xor(m1, o, 64));
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) { sh[0][w] = m0; sh[1][w] = m1; }
  __syncthreads();
  m0 = sh[0][0];
  m1 = sh[1][0];
#pragma unroll
  for (int k = 1; k < kWaves; ++k) { m0 = fmin(m0, sh[0][k]); m1 = fmin(m1, sh[1][k]); }
  __syncthreads();
}

// Adds w rho / (rho + p + s l) and its derivative in l to (D, dD) for the entries of one side
// (s = +1 for f, -1 for g, which enters D with a minus sign); four independent entries per
// step keep several divisions in flight.
template <int NT>
static __device__ void berg_terms(const float *pot, const float *w, int n, double rho, double l,
                                  double sgn, double &D, double &dD) {
  int i = threadIdx.x;
  for (; i + 3 * NT < n; i += 4 * NT) {
    double q[4], ww[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      ww[u] = w[i + u * NT];
      q[u] = rho / (rho + (double)pot[i + u * NT] + sgn * l);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (ww[u] > 0.0) {
        D += sgn * ww[u] * q[u];
        dD -= ww[u] * q[u] * q[u] / rho;
      }
  }
  for (; i < n; i += NT) {
    const double ww = w[i];
    if (ww > 0.0) {
      const double q = rho / (rho + (double)pot[i] + sgn * l);
      D += sgn * ww * q;
      dD -= ww * q * q / rho;
    }
  }
}

// lambda*(f, g) with the Berg entropy (the maximiser of G_eps in lambda, whose first-order
// condition equates the tilted masses): the root of
//   D(l) = sum_i a_i rho1 / (rho1 + f_i + l) - sum_j b_j rho2 / (rho2 + g_j - l),
// which decreases on (-rho1 - min f, rho2 + min g) (minima over positive weights). Newton
// steps from `start`, inside a bracket that every evaluation shrinks (a step leaving it is
// replaced by bisection). Run by a whole block of NT threads; every thread gets the result.
template <int NT>
static __device__ double berg_lambda(const ReduceArgs &a, double start) {
  double fmn = INFINITY, gmn = INFINITY;
  for (int i = threadIdx.x; i < a.nf; i += NT)
    if (a.w_f[i] > 0.0f) fmn = fmin(fmn, (double)a.pot_f[i]);
  for (int j = threadIdx.x; j < a.ng; j += NT)
    if (a.w_g[j] > 0.0f) gmn = fmin(gmn, (double)a.pot_g[j]);
  block_min2<NT>(fmn, gmn);
  double lo = -a.rho1 - fmn, hi = a.rho2 + gmn;
  double lam = (start > lo && start < hi) ? start : 0.5 * (lo + hi);
  for (int it = 0; it < 200; ++it) {
    double D = 0.0, dD = 0.0;
    berg_terms<NT>(a.pot_f, a.w_f, a.nf, a.rho1, lam, 1.0, D, dD);
    berg_terms<NT>(a.pot_g, a.w_g, a.ng, a.rho2, lam, -1.0, D, dD);
    block_sum2<NT>(D, dD);
    if (D > 0.0) lo = lam; else hi = lam;
    double nl = lam - D / dD;
    if (!(nl > lo && nl < hi)) nl = 0.5 * (lo + hi);
    const bool stop = D == 0.0 || !(fabs(nl - lam) > 1e-15 * fmax(1.0, fabs(lam)));
    lam = nl;
    if (stop) break;
  }
  return lam;
}

// Reduces the block partials of a half-step (or of the start) into the scalar state; run by
// one block of kBlock threads. Thread 0 writes the results.
static __device__ void reduce_scalars(const ReduceArgs &a) {
  SolveState *st = a.st;
  // this thread's partials: maxima first, then the mass sums rescaled to their maximum
  double mm = -INFINITY, ms = 0.0, dmx = -INFINITY, dmn = INFINITY;
  for (int b = threadIdx.x; b < a.nb; b += kBlock) {
    const BlockPart q = a.bparts[b];
    mm = fmax(mm, q.mass_max);
    dmx = fmax(dmx, q.dmax);
    dmn = fmin(dmn, q.dmin);
  }
  if (mm > -INFINITY)
    for (int b = threadIdx.x; b < a.nb; b += kBlock) {
      const BlockPart q = a.bparts[b];
      if (q.mass_max > -INFINITY) ms += q.mass_sum * exp(q.mass_max - mm);
    }
  block_reduce_part(mm, ms, dmx, dmn);
  if (threadIdx.x != 0) return;
  const double L = (mm == -INFINITY) ? -INFINITY : mm + log(ms);  // log of the tilted mass
  if (a.kind == kReduceInit) {
    st->iter = 0;
    st->tau_f = st->tau_g = st->lambda = 0.0;
    st->off_f_prev = st->off_g_prev = 0.0;
    st->gdiff_max = st->gdiff_min = 0.0;
    st->delta = INFINITY;
    st->sA = -a.rho1 * L;  // Smin_alpha^rho1(f_0)
    st->sB = 0.0;
    if (!st->pos_a || !st->pos_b) st->error |= kErrWeights;
    set_done(st, st->error ? 1 : 0);
  } else if (a.kind == kReduceRestart) {
    st->sA = -a.rho1 * L;  // Smin_alpha^rho1 of the extrapolated x, stored untranslated
    st->tau_f = 0.0;
  } else if (a.kind == kReduceG) {
    const double sBhat = -a.rho2 * L;  // Smin_beta^rho2(ghat)
    const double tg = a.ti ? a.kappa_t / (1.0 - a.kappa_t) * sBhat : 0.0;
    st->tau_g = tg;
    st->sB = sBhat + tg;
    st->gdiff_max = dmx;
    st->gdiff_min = dmn;
  } else {
    const double sAhat = -a.rho1 * L;  // Smin_alpha^rho1(fhat)
    double tf = 0.0, lam = 0.0;
    if (a.ti) {
      tf = a.kappa_t / (1.0 - a.kappa_t) * sAhat;
      st->sA = sAhat + tf;
      lam = a.tau1 * st->sB - a.tau2 * st->sA;  // Prop. 2 through softmins
    } else {
      st->sA = sAhat;
      // G-Sinkhorn: the stored pair is the F-update from the last reported f; its optimal
      // translation lambda*(stored f, stored g) (Prop. 2 for KL) moves the reported pair, and
      // G's own lambda_t = lambda*(fb_t, gb_t) advances by the same amount
      // (Berg: computed by k_berg_lambda after the f-step's combine)
      if (a.gvar) lam = a.entropy == kEntropyBerg ? st->lam_step : a.tau1 * st->sB - a.tau2 * sAhat;
    }
    // the next g-step reads the stored f translated by tau_f: TI's translation, or G's step
    st->tau_f = a.gvar ? lam : tf;
    if (a.tau_out) *a.tau_out = tf;
    st->lambda = a.gvar ? st->lambda + lam : lam;
    const double off_f = tf + lam, off_g = st->tau_g - lam;
    const int it = st->iter + 1;
    st->iter = it;
    double delta = INFINITY;
    if (it > 1 && !st->fresh) {
      const double cf = off_f - st->off_f_prev, cg = off_g - st->off_g_prev;
      const double df = fmax(dmx + cf, -(dmn + cf));
      const double dg = fmax(st->gdiff_max + cg, -(st->gdiff_min + cg));
      delta = fmax(df, dg);
    }
    st->delta = delta;
    st->fresh = 0;
    st->off_f_prev = off_f;
    st->off_g_prev = off_g;
    if (!isfinite(off_f) || !isfinite(off_g) || isnan(delta)) st->error |= kErrNumeric;
    if (st->error)
      set_done(st, 1);
    else if (a.tol > 0.0 && a.check_every > 0 && it % a.check_every == 0 && delta < a.tol)
      set_done(st, 1);
  }
}

// Merges the split partials of targets [t_begin, t_begin + kBlock / LANES) (LANES threads per
// target), applies the half-step epilogue (KL prox and TI translation, App. B) and writes the
// new potentials and source records; sets this thread's contribution to the block's
// (tilted-mass log-sum-exp, potential-change range) partial. Returns false, having written
// nothing, once the solve is done.
template <int D, int MODE, int LANES>
static __device__ bool combine_range(const CombineArgs &a, int t_begin, double &mm, double &ms,
                                     double &dmx, double &dmn) {
  const int sub = threadIdx.x % LANES;
  const int t = t_begin + threadIdx.x / LANES;
  const int tc = t < a.nt ? t : a.nt - 1;
  // Everything the epilogue reads, the early-exit flag included, is loaded first, so that
  // its latency overlaps the merge.
  const int32_t done = get_done(&a.st->done);
  const float w = a.w[tc];
  const float old = a.pot[tc];
  const double tau_src = a.ep.src_is_x ? a.st->tau_f : a.st->tau_g;
  const double s_src = a.ep.src_is_x ? a.st->sA : a.st->sB;
  float yc[D > 0 ? D : 1];
  double yn2 = 0.0;
  if constexpr (MODE != kDense) yn2 = centred<D>(a.tgt, a.d, tc, a.st->mu, yc);
  // log2-sum over the split partials: M + log2(sum_p l_p 2^{m_p - M}), one pass, the loads of
  // a batch of 8 partials issued together (this merge is latency bound)
  constexpr int kBatch = 8;
  float M = -FLT_MAX, L = 0.0f;
  for (int p0 = sub; p0 < a.nsplit; p0 += kBatch * LANES) {
    float2 q[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int p = p0 + u * LANES;
      q[u] = p < a.nsplit ? a.part[(size_t)p * a.nt + tc] : make_float2(-FLT_MAX, 0.0f);
    }
    float nm = M;
#pragma unroll
    for (int u = 0; u < kBatch; ++u) nm = fmaxf(nm, q[u].x);
    float acc = L * __builtin_amdgcn_exp2f(M - nm);
#pragma unroll
    for (int u = 0; u < kBatch; ++u) acc += q[u].y * __builtin_amdgcn_exp2f(q[u].x - nm);
    M = nm;
    L = acc;
  }
#pragma unroll
  for (int o = 1; o < LANES; o <<= 1) {
    const float Mo = __shfl_xor(M, o, LANES), Lo = __shfl_xor(L, o, LANES);
    const float nm = fmaxf(M, Mo);
    L = L * __builtin_amdgcn_exp2f(M - nm) + Lo * __builtin_amdgcn_exp2f(Mo - nm);
    M = nm;
  }
  if (done) return false;  // the same flag for the whole block
  mm = -INFINITY;
  ms = 0.0;
  dmx = -INFINITY;
  dmn = INFINITY;
  if (sub == 0 && t < a.nt) {
    double lse2 = (double)M + log2((double)L);
    if constexpr (is_sq(MODE)) lse2 -= a.sc * yn2;
    const double S = -lse2 / a.sc;  // softmin over the stored source potential
    const double hnew = a.ep.entropy == kEntropyBerg
                            ? berg_update(S - tau_src, a.ep.rho_t, a.eps)
                            : a.ep.k_t * (S - tau_src) - a.ep.c_t * s_src;
    const float hf = (float)hnew;
    a.pot[t] = hf;
    if (a.snap) a.snap[t] = hf;
    dmx = dmn = (double)hf - (double)old;
    write_record<D, MODE>(a.rec_out, t, yc, yn2, hf, w, a.sc);
    if (w > 0.0f) { mm = log((double)w) - (double)hf / a.ep.rho_t; ms = 1.0; }
    if (!isfinite(hnew)) atomicOr(&a.st->error, kErrNumeric);
  }
  return true;
}

// combine_range over one block's targets, then the block partial into bparts[tile].
template <int D, int MODE, int LANES>
static __device__ void combine_block(const CombineArgs &a, int t_begin, int tile) {
  double mm, ms, dmx, dmn;
  if (!combine_range<D, MODE, LANES>(a, t_begin, mm, ms, dmx, dmn)) return;
  block_reduce_part(mm, ms, dmx, dmn);
  if (threadIdx.x == 0) a.bparts[tile] = BlockPart{mm, ms, dmx, dmn};
}

}  // namespace uot
