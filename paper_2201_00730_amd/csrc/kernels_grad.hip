// Envelope gradients and plan marginals of a points cost, one pass over the sources per
// side, one exp2 per entry (gfx950).
//
// Targets t are the points of one side, sources s those of the other; both are centred by the
// common mean mu (t' = t - mu, s' = s - mu; the cost is translation invariant). With
// sc = log2(e)/eps and b_s = sc h_s + log2 w_s the plan entry is
//   pi_ts = w_t 2^{sc h_t} 2^{e_ts},   e_ts = b_s - sc C_ts,   C_ts = ||t' - s'||^p,
// its row sum pi1_t = w_t 2^{sc h_t} sum_s 2^{e_ts}, and the gradient of <pi, C> in t (the
// envelope theorem applied to the dual, Sec. 1)
//   sum_s pi_ts c'(||t - s||) (t - s),   c'(r) (t - s) = p r^{p-2} (t - s)  (0 at t = s).
// Per (source split, target) the kernel accumulates, relative to a reference r_t,
//   l_t = sum_s q_ts,  lw_t = sum_s q_ts w_ts,  a_tk = sum_s q_ts w_ts s'_k,   q_ts = 2^{e_ts - r_t},
// with w = 1 for p = 2 (the factor p = 2 is applied by the combine) and p d2^{(p-2)/2}
// otherwise; the combine forms the gradient t'_k lw_t - a_tk in double precision.
//
// Precision. A plan entry moves by a factor 2^{delta} when its exponent moves by delta, and
// sc C_ts reaches several hundred (D = 16, eps = 0.05: sc ~ 29, C ~ 15..40 on the entries that
// carry the plan), so a float32 exponent would leave ~1e-5 relative error in each entry. The
// exponent is therefore formed in double precision, where float32 and double run at the same
// vector rate on this chip: d2 = |t'|^2 + |s'|^2 - 2 <t', s'> (D double FMAs; its cancellation
// costs 2^-53 of the norms), then e - r_t in double, and only that difference, a number of
// order one on the entries that matter, is rounded to float32 for the exp2. For p != 2 the
// cost d2^{p/2} is taken in double as well.
//
// Reference. Each lane keeps a running reference r_t per target, an integer-valued float
// raised to ceil(e) whenever a source brings a larger exponent, so rescaling the
// sums is a multiplication by a power of two (exact), and the entries that carry the sum have
// e - r_t in [-few, 0] whatever the potentials, which keeps the float32 rounding of e - r_t
// small where it matters. The combine takes the references exactly.
//
// Two implementations of this pass: k_grad_mfma (dimension buckets up to 16, the default;
// inner products and gradient sums on the matrix cores) and k_grad_partial (every bucket;
// vector ALU). In k_grad_partial each lane owns R targets (coordinates in double,
// accumulators in float, all in registers); the sources of one split are uniform across the
// wave and read with scalar loads.
#include <atomic>
#include <cfloat>

#include "uot_internal.h"

namespace uot {
namespace {

__device__ __forceinline__ float fexp2(float x) { return __builtin_amdgcn_exp2f(x); }

template <int D>
constexpr int grad_targets_per_lane() {
  return D <= 8 ? 4 : (D <= 16 ? 2 : 1);
}

template <int D>
__global__ __launch_bounds__(256) void k_grad_records(GradRecordArgs a) {
  const int s = blockIdx.x * 256 + threadIdx.x;
  if (s >= a.n + kGradPadRows) return;
  double *r = a.rec + (size_t)s * grad_rec_stride(D);
  float *rf = reinterpret_cast<float *>(r + D + 2);
  if (s >= a.n) {  // padding: no mass
#pragma unroll
    for (int k = 0; k < D; ++k) {
      r[k] = 0.0;
      rf[k] = 0.0f;
    }
    r[D] = 0.0;
    r[D + 1] = -INFINITY;
    return;
  }
  double nn = 0.0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const double v = k < a.d ? (double)a.pts[(size_t)s * a.d + k] - a.mu[k] : 0.0;
    r[k] = v;
    rf[k] = (float)v;
    nn = fma(v, v, nn);
  }
  r[D] = nn;
  const float w = a.w[s];
  r[D + 1] = w > 0.0f ? a.sc * (double)a.pot[s] + log2((double)w) : -INFINITY;
}

// Cost ||t' - s'||^p from the squared distance, in double precision.
template <bool P2>
__device__ __forceinline__ double cost_of(double d2, double half_p) {
  if constexpr (P2) {
    return d2;
  } else {
    const double dd = d2 > 0.0 ? d2 : 0.0;
    if (half_p == 0.5) return sqrt(dd);
    return dd > 0.0 ? exp2(half_p * log2(dd)) : 0.0;
  }
}

// Gradient weight p d2^{(p-2)/2} = p C / d2 (0 at t = s); 1 for p = 2.
template <bool P2>
__device__ __forceinline__ float weight_of(double d2, double cst, float p) {
  if constexpr (P2) {
    return 1.0f;
  } else {
    const float df = (float)d2;
    return df > 0.0f ? p * (float)cst * __builtin_amdgcn_rcpf(df) : 0.0f;
  }
}

template <int D, int R, bool GRAD, bool P2>
__global__ __launch_bounds__(256) void k_grad_partial(GradArgs a) {
  constexpr int SD = grad_rec_stride(D);
  constexpr int PS = grad_part_stride(GRAD ? D : 0);
  constexpr int NA = GRAD ? D : 1;
  const int t0 = blockIdx.x * (256 * R) + threadIdx.x;
  const double sc = a.sc, half_p = a.half_p;
  const float p = a.p;

  double y[R][D];
  double yn[R];
  float ref[R], l[R], lw[R], acc[R][NA];
  bool valid[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int t = t0 + r * 256;
    valid[r] = t < a.nt;
    const int tc = valid[r] ? t : a.nt - 1;
    double nn = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      y[r][k] = k < a.d ? (double)a.tgt[(size_t)tc * a.d + k] - a.mu[k] : 0.0;
      nn = fma(y[r][k], y[r][k], nn);
    }
    yn[r] = nn;
    ref[r] = -FLT_MAX;  // an integer-valued float
    l[r] = 0.0f;
    lw[r] = 0.0f;
#pragma unroll
    for (int k = 0; k < NA; ++k) acc[r][k] = 0.0f;
  }
  const int s0 = blockIdx.y * a.split_len;
  const int s1 = min(a.ns, s0 + a.split_len);

  // squared distance of target r to the source at rp (two FMA chains)
  auto dist2 = [&](int r, const double *rp) -> double {
    double d0 = 0.0, d1 = 0.0;
#pragma unroll
    for (int k = 0; k + 1 < D; k += 2) {
      d0 = fma(y[r][k], rp[k], d0);
      d1 = fma(y[r][k + 1], rp[k + 1], d1);
    }
    if constexpr (D % 2 == 1) d0 = fma(y[r][D - 1], rp[D - 1], d0);
    return fma(-2.0, d0 + d1, yn[r] + rp[D]);
  };

  // One source per step: its record (D + 2 doubles, D floats) stays in scalar registers.
  for (int s = s0; s < s1; ++s) {
    const double *rp = a.rec + (size_t)s * SD;
    const float *rf = reinterpret_cast<const float *>(rp + D + 2);
    const double bs = rp[D + 1];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const double d2 = dist2(r, rp);
      const double cst = cost_of<P2>(d2, half_p);
      const double e = fma(-sc, cst, bs);
      if (e > (double)ref[r]) {  // a new maximum: raise the reference to ceil(e)
        const float mc = ceilf((float)e);
        if (mc > ref[r]) {
          const float scale = fexp2(ref[r] - mc);  // a power of two (or 0 from -FLT_MAX)
          l[r] *= scale;
          if constexpr (GRAD) {
            lw[r] *= scale;
#pragma unroll
            for (int k = 0; k < D; ++k) acc[r][k] *= scale;
          }
          ref[r] = mc;
        }
      }
      const float q = fexp2((float)(e - (double)ref[r]));
      l[r] += q;
      if constexpr (GRAD) {
        const float qw = P2 ? q : q * weight_of<P2>(d2, cst, p);
        if constexpr (!P2) lw[r] += qw;
#pragma unroll
        for (int k = 0; k < D; ++k) acc[r][k] = fmaf(qw, rf[k], acc[r][k]);
      }
    }
  }

#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int t = t0 + r * 256;
    if (!valid[r]) continue;
    float *o = a.part + ((size_t)blockIdx.y * a.nt + t) * PS;
    o[0] = l[r] > 0.0f ? ref[r] : -FLT_MAX;
    o[1] = l[r];
    if constexpr (GRAD) {
      o[2] = P2 ? l[r] : lw[r];
#pragma unroll
      for (int k = 0; k < D; ++k) o[3 + k] = acc[r][k];
    }
  }
}

// Merges the split partials of each target (double precision) and writes what was asked:
//   rowsum_t = sum_s w_s e^{(h_t + h_s - C_ts)/eps} = 2^{sc h_t + M} sum,
//   marg_t   = w_t rowsum_t                                   (the plan marginal pi1_t),
//   dw_t     = gout (rho (1 - e^{-h_t/rho}) - eps (rowsum_t - mass_other))   (d/d w_t),
//   dpts_tk  = gout w_t 2^{sc h_t + M} pfac (t'_k lw - a_k)   (d/d t_k),
// with pfac = 2 for p = 2 (the kernel's weight is 1 there) and 1 otherwise.
template <int DC>
__global__ __launch_bounds__(256) void k_grad_combine(GradCombineArgs a) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= a.nt) return;
  constexpr int ps = grad_part_stride(DC);
  constexpr int NA = DC > 0 ? DC : 1;
  float M = -FLT_MAX;
  for (int q = 0; q < a.nsplit; ++q) M = fmaxf(M, a.part[((size_t)q * a.nt + t) * ps]);
  double sum = 0.0, lw = 0.0, acc[NA];
#pragma unroll
  for (int k = 0; k < NA; ++k) acc[k] = 0.0;
  for (int q = 0; q < a.nsplit; ++q) {
    const float *o = a.part + ((size_t)q * a.nt + t) * ps;
    if (o[1] == 0.0f) continue;
    const double f = exp2((double)o[0] - (double)M);
    sum += f * (double)o[1];
    if constexpr (DC > 0) {
      lw += f * (double)o[2];
#pragma unroll
      for (int k = 0; k < DC; ++k) acc[k] += f * (double)o[3 + k];
    }
  }
  const double h = (double)a.h_t[t];
  const double base = sum > 0.0 ? exp2(a.sc * h + (double)M) : 0.0;  // 2^{sc h_t + M}
  const double rowsum = base * sum;
  const double wt = (double)a.w_t[t];
  if (a.marg) a.marg[(size_t)t * a.marg_stride] = (float)(wt * rowsum);
  if (a.dw) {
    const double v = a.rho * (-expm1(-h / a.rho)) - a.eps * (rowsum - *a.mass_other);
    a.dw[t] = (float)(a.gout * v);
  }
  if constexpr (DC > 0) {
    if (a.apply_out) {  // payload pass: (pi V)_tc = w_t 2^{sc h_t + M} sum_s q_ts V_sc
      const double fac = wt * base;
#pragma unroll
      for (int k = 0; k < DC; ++k)
        if (k < a.d) a.apply_out[(size_t)t * a.ldout + k] = (float)(fac * acc[k]);
    }
    if (a.dpts) {
      const double fac = wt > 0.0 ? a.gout * wt * base * a.pfac : 0.0;
#pragma unroll
      for (int k = 0; k < DC; ++k)
        if (k < a.d) {
          const double tk = (double)a.tgt[(size_t)t * a.d + k] - a.mu[k];
          a.dpts[(size_t)t * a.d + k] = (float)(fac * fma(tk, lw, -acc[k]));
        }
    }
  }
}

// Matrix-core form of k_grad_partial for coordinate buckets up to 16 (p = 2 or not). Per
// 16-source step and 16-target group a wave forms the 256 inner products <s', t'> with
// ceil(D/4) double-precision MFMAs (v_mfma_f64_16x16x4_f64, coordinates past D zero: the
// same FP64 products and sums as the vector form, in another order), evaluates exponents
// and exp2 on the vector ALU, and
// accumulates the gradient sums a_tk = sum_s q_ts w_ts s'_k with four float32 MFMAs
// (v_mfma_f32_16x16x4_f32) whose A operand is the q tile just computed. Operand layouts of
// these 16x16x4 instructions (checked on the device): A[i][k] in lane i + 16 k and B[k][j] in
// lane j + 16 k for both; the result D[i][j] sits in lane j + 16 (i % 4), element i / 4, for
// the double-precision one and in lane j + 16 (i / 4), element i % 4, for the float32 one.
// With sources as the rows of the inner-product tile, lane j + 16 c holds the entries
// (target j, sources c + 4 r, r = 0..3): element r is the A operand (k = c) of the q-tile
// MFMA over sources 4 r .. 4 r + 3, so no data moves between the two products.
// All four lanes of a target (c = 0..3) share one integer-valued reference, raised together
// (a max over the lane quarter) so the MFMA sums over c add entries of one scale.
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kMfmaGroups = 4;  // 16-target groups per wave: 256 targets per block

template <int D>
constexpr bool grad_uses_mfma() {
  return D <= 16;
}

// PAY: a payload pass of the plan application (GRAD true): the B operand of the q-tile MFMAs
// is V[s, col] (col < vcols, zero past the last source) and the entries carry no weight.
template <int D, bool GRAD, bool P2, bool PAY = false>
__global__ __launch_bounds__(256) void k_grad_mfma(GradArgs a) {
  static_assert(D <= 16, "coordinate bucket must be at most 16");
  static_assert(GRAD || !PAY, "a payload pass accumulates");
  constexpr int SD = grad_rec_stride(D);
  constexpr int PS = PAY ? grad_part_stride(16) : grad_part_stride(GRAD ? D : 0);
  constexpr int KS = (D + 3) / 4;
  constexpr int G = kMfmaGroups;
  const int lane = threadIdx.x & 63;
  const int col = lane & 15, qr = lane >> 4;
  const int tw = blockIdx.x * (4 * G * 16) + (threadIdx.x >> 6) * (G * 16);
  const double sc = a.sc, half_p = a.half_p, sc2 = 2.0 * a.sc;
  const float p = a.p;

  double tb[G][KS], yn[G], base[G];  // base: -r_t, plus -sc |t'|^2 for p = 2
  float ref[G], l[G], lw[G];
  f32x4 acc[G];
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const int t = tw + 16 * g + col;
    const int tc = t < a.nt ? t : a.nt - 1;
    const float *tp = a.tgt + (size_t)tc * a.d;
    double nn = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      const double v = k < a.d ? (double)tp[k] - a.mu[k] : 0.0;
      nn = fma(v, v, nn);
    }
    yn[g] = P2 ? -sc * nn : nn;  // p = 2: the target's share of the exponent
#pragma unroll
    for (int j = 0; j < KS; ++j) {
      const int k = 4 * j + qr;
      tb[g][j] = k < a.d ? (double)tp[k] - a.mu[k] : 0.0;
    }
    ref[g] = -FLT_MAX;
    base[g] = (P2 ? yn[g] : 0.0) + (double)FLT_MAX;
    l[g] = 0.0f;
    lw[g] = 0.0f;
    acc[g] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  }
  const int s0 = blockIdx.y * a.split_len;
  const int s1 = min(a.ns, s0 + a.split_len);

  // Operands of one 16-source step: the inner products' A operand (source sb + col,
  // coordinates 4 j + qr) and this lane's four entries per group (sources sb + qr + 4 i:
  // |s'|^2, b_s, and coordinate col for the gradient sums), loaded one step ahead. Split
  // lengths are multiples of 16, so only the last split ends inside a step, and the padding
  // records after the last source (b = -inf, zero coordinates) complete that step.
  struct Step {
    double av[KS], sn[4], bs[4];
    float sv[4];
  };
  auto load_step = [&](int sb, Step &st) {
    const double *ra = a.rec + (size_t)(sb + col) * SD;
    const double *rb = a.rec + (size_t)(sb + qr) * SD;
#pragma unroll
    for (int j = 0; j < KS; ++j) st.av[j] = (4 * j + 4 > D && 4 * j + qr >= D) ? 0.0 : ra[4 * j + qr];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const double *rp = rb + 4 * i * SD;
      if constexpr (SD % 2 == 0 && D % 2 == 0) {  // |s'|^2, b_s: one 16-byte aligned load
        const double2 nb = *reinterpret_cast<const double2 *>(rp + D);
        st.sn[i] = nb.x;
        st.bs[i] = nb.y;
      } else {
        st.sn[i] = rp[D];
        st.bs[i] = rp[D + 1];
      }
      if constexpr (PAY) {
        const int si = sb + qr + 4 * i;
        st.sv[i] = (col < a.vcols && si < a.ns) ? a.V[(size_t)si * a.ldv + col] : 0.0f;
      } else if constexpr (GRAD) {
        st.sv[i] = col < D ? reinterpret_cast<const float *>(rp + D + 2)[col] : 0.0f;
      }
    }
  };
  const int last = s0 + (s1 - 1 - s0) / 16 * 16;  // first source of the last step
  Step cur;
  if (s0 < s1) load_step(s0, cur);
  for (int sb = s0; sb < s1; sb += 16) {
    Step nxt;
    load_step(min(sb + 16, last), nxt);  // the last step loads itself again (in bounds)
    const double(&av)[KS] = cur.av;
    const double(&sn)[4] = cur.sn;
    const double(&bs)[4] = cur.bs;
    const float(&sv)[4] = cur.sv;
    double cb[4];  // p = 2: the source's share b_s - sc |s'|^2, common to the groups
#pragma unroll
    for (int i = 0; i < 4; ++i) cb[i] = P2 ? fma(-sc, sn[i], bs[i]) : 0.0;
#pragma unroll
    for (int g = 0; g < G; ++g) {
      f64x4 dd = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int j = 0; j < KS; ++j) dd = __builtin_amdgcn_mfma_f64_16x16x4f64(av[j], tb[g][j], dd, 0, 0, 0);
      // exponents relative to the reference, e - r_t, in double; rounded to float32 for
      // the test against 0 and for exp2
      double er[4], d2[4], cst[4];
      float ef[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        if constexpr (P2) {  // e - r = (b_s - sc |s'|^2) + (-sc |t'|^2 - r) + 2 sc <s', t'>
          er[i] = fma(sc2, dd[i], cb[i] + base[g]);
        } else {
          d2[i] = fma(-2.0, dd[i], yn[g] + sn[i]);
          cst[i] = cost_of<P2>(d2[i], half_p);
          er[i] = fma(-sc, cst[i], bs[i] + base[g]);
        }
        ef[i] = (float)er[i];
      }
      const bool up = fmaxf(fmaxf(ef[0], ef[1]), fmaxf(ef[2], ef[3])) > 0.0f;
      if (__builtin_amdgcn_ballot_w64(up)) {  // raise the quarter's shared reference
        double ea[4];  // absolute exponents (e - r_t + r_t would cancel for r_t = -FLT_MAX)
#pragma unroll
        for (int i = 0; i < 4; ++i) ea[i] = P2 ? fma(sc2, dd[i], cb[i] + yn[g]) : fma(-sc, cst[i], bs[i]);
        const double m = fmax(fmax(ea[0], ea[1]), fmax(ea[2], ea[3]));
        float mc = up ? ceilf((float)m) : ref[g];
        mc = fmaxf(mc, __shfl_xor(mc, 16));
        mc = fmaxf(mc, __shfl_xor(mc, 32));
        const float nr = fmaxf(mc, ref[g]);
        const float scale = fexp2(ref[g] - nr);  // a power of two (or 0 from -FLT_MAX)
        ref[g] = nr;
        base[g] = (P2 ? yn[g] : 0.0) - (double)nr;
        l[g] *= scale;
        if constexpr (GRAD) {
          lw[g] *= scale;
#pragma unroll
          for (int i = 0; i < 4; ++i) acc[g][i] *= __shfl(scale, 4 * qr + i);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {  // recomputed: the old reference may be -FLT_MAX
          er[i] = P2 ? fma(sc2, dd[i], cb[i] + base[g]) : fma(-sc, cst[i], bs[i] + base[g]);
          ef[i] = (float)er[i];
        }
      }
      float q[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) q[i] = fexp2(ef[i]);
      l[g] += (q[0] + q[1]) + (q[2] + q[3]);
      if constexpr (GRAD) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const float qw = (P2 || PAY) ? q[i] : q[i] * weight_of<P2>(d2[i], cst[i], p);
          if constexpr (!P2 && !PAY) lw[g] += qw;
          acc[g] = __builtin_amdgcn_mfma_f32_16x16x4f32(qw, sv[i], acc[g], 0, 0, 0);
        }
      }
    }
    cur = nxt;
  }

#pragma unroll
  for (int g = 0; g < G; ++g) {
    float lt = l[g] + __shfl_xor(l[g], 16);
    lt += __shfl_xor(lt, 32);
    float lwt = lw[g];
    if constexpr (GRAD && !P2 && !PAY) {
      lwt += __shfl_xor(lwt, 16);
      lwt += __shfl_xor(lwt, 32);
    }
    const int t = tw + 16 * g + col;
    if (qr == 0 && t < a.nt) {
      float *o = a.part + ((size_t)blockIdx.y * a.nt + t) * PS;
      o[0] = lt > 0.0f ? ref[g] : -FLT_MAX;
      o[1] = lt;
      if constexpr (GRAD) o[2] = (P2 || PAY) ? lt : lwt;
    }
    if constexpr (GRAD) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int ti = tw + 16 * g + 4 * qr + i;
        if (ti < a.nt && col < (PAY ? 16 : D)) a.part[((size_t)blockIdx.y * a.nt + ti) * PS + 3 + col] = acc[g][i];
      }
    }
  }
}

// Plan application to a payload on a stored cost: the loop of k_grad_mfma's payload pass with
// the inner-product MFMAs replaced by the cost entries themselves. Lane (col, qr) takes, per
// 16-source step, sources sb + 4 qr + i (i = 0..3: four consecutive entries of a row of C
// when the targets are its rows); element i is the A operand (k = qr) of the q-tile MFMA over
// sources sb + 4 k + i, whose B operand V[sb + 4 qr + i][col] the same lane loads.
template <bool TRANS>
__global__ __launch_bounds__(256) void k_dense_payload(DensePayloadArgs a) {
  constexpr int G = kMfmaGroups;
  constexpr int PS = grad_part_stride(16);
  const int lane = threadIdx.x & 63;
  const int col = lane & 15, qr = lane >> 4;
  const int tw = blockIdx.x * (4 * G * 16) + (threadIdx.x >> 6) * (G * 16);
  const float sc = a.sc;
  float ref[G], l[G];
  f32x4 acc[G];
  int tcl[G];
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const int t = tw + 16 * g + col;
    tcl[g] = t < a.nt ? t : a.nt - 1;
    ref[g] = -FLT_MAX;
    l[g] = 0.0f;
    acc[g] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  }
  const int s0 = blockIdx.y * a.split_len;
  const int s1 = min(a.ns, s0 + a.split_len);
  for (int sb = s0; sb < s1; sb += 16) {
    float bs[4], sv[4];
    bool ok[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int si = sb + 4 * qr + i;
      ok[i] = si < s1;
      bs[i] = ok[i] ? a.rec[si] : -INFINITY;
      sv[i] = (ok[i] && col < a.vcols) ? a.V[(size_t)si * a.ldv + col] : 0.0f;
    }
    const bool row4 = !TRANS && a.vec4 && ok[3];  // this lane's four entries in one 16-byte load
#pragma unroll
    for (int g = 0; g < G; ++g) {
      float cv[4];
      if (row4) {
        const float4 c4 = *reinterpret_cast<const float4 *>(a.C + (size_t)tcl[g] * a.ldc + sb + 4 * qr);
        cv[0] = c4.x;
        cv[1] = c4.y;
        cv[2] = c4.z;
        cv[3] = c4.w;
      } else {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int si = sb + 4 * qr + i;
          cv[i] = ok[i] ? (TRANS ? a.C[(size_t)si * a.ldc + tcl[g]] : a.C[(size_t)tcl[g] * a.ldc + si]) : 0.0f;
        }
      }
      float e[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) e[i] = fmaf(-sc, cv[i], bs[i]);
      const float m = fmaxf(fmaxf(e[0], e[1]), fmaxf(e[2], e[3]));
      const bool up = m > ref[g];
      if (__builtin_amdgcn_ballot_w64(up)) {  // raise the quarter's shared reference
        float mc = up ? ceilf(m) : ref[g];
        mc = fmaxf(mc, __shfl_xor(mc, 16));
        mc = fmaxf(mc, __shfl_xor(mc, 32));
        const float nr = fmaxf(mc, ref[g]);
        const float scale = fexp2(ref[g] - nr);
        ref[g] = nr;
        l[g] *= scale;
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[g][i] *= __shfl(scale, 4 * qr + i);
      }
      float q[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) q[i] = fexp2(e[i] - ref[g]);
      l[g] += (q[0] + q[1]) + (q[2] + q[3]);
#pragma unroll
      for (int i = 0; i < 4; ++i) acc[g] = __builtin_amdgcn_mfma_f32_16x16x4f32(q[i], sv[i], acc[g], 0, 0, 0);
    }
  }
#pragma unroll
  for (int g = 0; g < G; ++g) {
    float lt = l[g] + __shfl_xor(l[g], 16);
    lt += __shfl_xor(lt, 32);
    const int t = tw + 16 * g + col;
    if (qr == 0 && t < a.nt) {
      float *o = a.part + ((size_t)blockIdx.y * a.nt + t) * PS;
      o[0] = lt > 0.0f ? ref[g] : -FLT_MAX;
      o[1] = lt;
      o[2] = lt;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int ti = tw + 16 * g + 4 * qr + i;
      if (ti < a.nt) a.part[((size_t)blockIdx.y * a.nt + ti) * PS + 3 + col] = acc[g][i];
    }
  }
}

template <int D>
hipError_t records_for(const GradRecordArgs &a, hipStream_t s) {
  hipLaunchKernelGGL((k_grad_records<D>), dim3((a.n + kGradPadRows + 255) / 256), dim3(256), 0, s, a);
  return hipGetLastError();
}

// Backward kernel choice for buckets up to 16: 0 the matrix-core form (also the plan
// application's payload passes), 1 the vector form (the plan application then takes the
// float32-exponent apply kernel).
std::atomic<int> g_grad_variant{0};

template <int D, bool GRAD, bool P2>
hipError_t grad_for(const GradArgs &a, hipStream_t s, const LaunchTiming *t) {
  if constexpr (grad_uses_mfma<D>()) {
    if (g_grad_variant.load(std::memory_order_relaxed) == 0) {
      dim3 grid((a.nt + 64 * kMfmaGroups - 1) / (64 * kMfmaGroups), a.nsplit);
      if (a.V != nullptr) {
        if constexpr (GRAD) return launch_timed(k_grad_mfma<D, true, P2, true>, grid, dim3(256), s, t, a);
        return hipErrorInvalidValue;
      }
      return launch_timed(k_grad_mfma<D, GRAD, P2>, grid, dim3(256), s, t, a);
    }
  }
  if (a.V != nullptr) return hipErrorInvalidValue;  // payload passes: matrix-core buckets only
  constexpr int R = grad_targets_per_lane<D>();
  dim3 grid((a.nt + 256 * R - 1) / (256 * R), a.nsplit);
  return launch_timed(k_grad_partial<D, R, GRAD, P2>, grid, dim3(256), s, t, a);
}

template <int D>
hipError_t grad_for_mode(const GradArgs &a, hipStream_t s, const LaunchTiming *t) {
  const bool p2 = a.half_p == 1.0;
  if (a.grad) return p2 ? grad_for<D, true, true>(a, s, t) : grad_for<D, true, false>(a, s, t);
  return p2 ? grad_for<D, false, true>(a, s, t) : grad_for<D, false, false>(a, s, t);
}

template <int DC>
hipError_t combine_for(const GradCombineArgs &a, hipStream_t s) {
  hipLaunchKernelGGL((k_grad_combine<DC>), dim3((a.nt + 255) / 256), dim3(256), 0, s, a);
  return hipGetLastError();
}

#define UOT_GRAD_BUCKETS(FN, DD, ...)               \
  switch (DD) {                                     \
    case 1: return FN<1>(__VA_ARGS__);              \
    case 2: return FN<2>(__VA_ARGS__);              \
    case 3: return FN<3>(__VA_ARGS__);              \
    case 4: return FN<4>(__VA_ARGS__);              \
    case 5: return FN<5>(__VA_ARGS__);              \
    case 6: return FN<6>(__VA_ARGS__);              \
    case 7: return FN<7>(__VA_ARGS__);              \
    case 8: return FN<8>(__VA_ARGS__);              \
    case 12: return FN<12>(__VA_ARGS__);            \
    case 16: return FN<16>(__VA_ARGS__);            \
    case 24: return FN<24>(__VA_ARGS__);            \
    case 32: return FN<32>(__VA_ARGS__);            \
    case 48: return FN<48>(__VA_ARGS__);            \
    case 64: return FN<64>(__VA_ARGS__);            \
    default: break;                                 \
  }

}  // namespace

hipError_t launch_dense_payload(const DensePayloadArgs &a, hipStream_t s) {
  if (a.vcols < 1 || a.vcols > 16 || a.split_len % 16 != 0) return hipErrorInvalidValue;
  dim3 grid((a.nt + 64 * kMfmaGroups - 1) / (64 * kMfmaGroups), a.nsplit);
  if (a.trans)
    hipLaunchKernelGGL(k_dense_payload<true>, grid, dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(k_dense_payload<false>, grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

bool grad_payload_supported(int d) {
  return dim_bucket(d) <= 16 && g_grad_variant.load(std::memory_order_relaxed) == 0;
}

int grad_source_align(int d) {
  const int b = dim_bucket(d);
  return b <= 16 && g_grad_variant.load(std::memory_order_relaxed) == 0 ? 16 : 1;
}

int grad_targets_per_block(int d) {
  const int b = dim_bucket(d);
  if (b <= 16 && g_grad_variant.load(std::memory_order_relaxed) == 0)
    return 64 * kMfmaGroups;
  return 256 * (b <= 8 ? 4 : (b <= 16 ? 2 : 1));
}

hipError_t launch_grad_records(const GradRecordArgs &a, hipStream_t s) {
  UOT_GRAD_BUCKETS(records_for, dim_bucket(a.d), a, s)
  return hipErrorInvalidValue;
}

hipError_t launch_grad_partial(const GradArgs &a, hipStream_t s, const LaunchTiming *t) {
  UOT_GRAD_BUCKETS(grad_for_mode, dim_bucket(a.d), a, s, t)
  return hipErrorInvalidValue;
}

hipError_t launch_grad_combine(const GradCombineArgs &a, hipStream_t s) {
  if (a.apply_out != nullptr) return a.d <= 16 ? combine_for<16>(a, s) : hipErrorInvalidValue;
  if (a.dpts == nullptr) return combine_for<0>(a, s);
  UOT_GRAD_BUCKETS(combine_for, dim_bucket(a.d), a, s)
  return hipErrorInvalidValue;
}

}  // namespace uot

extern "C" int32_t uot_set_grad_kernel(int32_t variant) {
  if (variant < 0 || variant > 1) return -1;
  return uot::g_grad_variant.exchange(variant);
}
