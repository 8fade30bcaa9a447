// Batched translation-invariant Sinkhorn for many independent KL-UOT problems with point
// costs (gfx950).
//
// Problems are packed back to back (CSR offsets offN/offM). One half-step of every active
// problem is one launch of k_batched_half: each wave repeatedly takes a work item (problem
// p, a chunk of <= 256 targets of p) from a dynamic counter over the compacted list of active
// items, computes the softmin of its targets over all sources of p (one target per lane for
// items of <= 64 targets, two up to 128, four above; the sources staged 64 at a time through
// the wave's LDS slice and read back uniformly across the wave; one exp2 per entry against a
// per-target reference, the target's log-sum-exp of its previous half-step), applies the KL
// prox and TI translation of App. B, writes the new potentials and source records, and
// leaves its item partials (tilted mass log-sum-exp, potential-change range). The last wave to finish an item of p (an atomic ticket, no waiting) reduces p's
// partials into p's scalars: the translation tau, Smin of the new side, and after an f-step
// lambda* (Prop. 2), the change of the reported potentials and the convergence flag.
// k_batched_compact rebuilds the active item lists between chunks of iterations.
//
// Same base-2 conventions as the single-problem kernels: sc_p = log2(e)/eps_p and records
//   u_s = x_s - mu_p,  b_s = sc_p h_s + log2 w_s,  exponent v_ts = b_s - sc_p ||u_s - (y_t - mu_p)||^p
// where mu_p is the common mean of problem p's two clouds. For p = 2 the coordinates are
// stored scaled by sqrt(sc_p) (targets scaled the same way), so v_ts = b_s - ||u'_s - y'_t||^2
// is a chain of FMAs starting from b_s: one multiplication fewer per entry, and the same
// rounding (each scaled coordinate is rounded once, as the unscaled one was). The cost is always taken through the
// differences (p = 2 included: ||.||^2 as is), so the float32 rounding of an exponent is
// relative to its entry's own cost; the expanded form |x|^2 + |y|^2 - 2<x, y> would carry an
// absolute rounding of the clouds' squared spread, which at small eps is not small against
// the potentials.
#include <cfloat>
#include <type_traits>

#include "uot_batched.h"

namespace uot {
namespace {

constexpr int kTile = 8;

__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float fast_log2(float x) { return __builtin_amdgcn_logf(x); }

// Wave-wide reductions (all 64 lanes participate).
__device__ __forceinline__ double wave_max(double v) {
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ double wave_min(double v) {
  for (int o = 32; o >= 1; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ void wave_lse(double &m, double &s) {
  for (int o = 32; o >= 1; o >>= 1) {
    const double mo = __shfl_xor(m, o, 64), so = __shfl_xor(s, o, 64);
    const double mn = fmax(m, mo);
    if (mn == -INFINITY) {
      s = 0.0;
    } else {
      s = s * exp(m - mn) + so * exp(mo - mn);
    }
    m = mn;
  }
}

// TI coefficients of a half-step whose targets have penalty rho_t and sources rho_s.
struct HalfCoef {
  double k_t, c_t, kappa_t;
};
__device__ __forceinline__ HalfCoef half_coef(double eps, double rho_t, double rho_s) {
  HalfCoef c;
  c.k_t = rho_t / (eps + rho_t);
  c.c_t = eps * rho_t / ((eps + rho_t) * (rho_s + rho_t));
  c.kappa_t = eps * rho_s / ((eps + rho_t) * (rho_s + rho_t));
  return c;
}

template <int D>
__device__ __forceinline__ void write_rec(float *rp, const float *yc, float hf, float w, double sc) {
  const double lw2 = w > 0.0f ? log2((double)w) : -INFINITY;
  const double b = sc * (double)hf + lw2;
  double n2 = 0.0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    rp[k] = yc[k];
    n2 = fma((double)yc[k], (double)yc[k], n2);
  }
  rp[D] = (float)b;
#pragma unroll
  for (int k = D + 1; k < batched_rec_stride(D); ++k) rp[k] = 0.0f;
  if constexpr (batched_has_expanded_slot(D)) rp[D + 1] = (float)(b - n2);
}

// Reduces problem p's item partials of the half-step just finished (one wave). Not inlined:
// it runs once per problem and half-step, and inlined it would raise the register count of
// the whole softmin kernel.
__device__ __noinline__ void reduce_problem(const BatchedArgs &a, int p, bool g_step) {
  BatchState &st = a.state[p];
  const int i0 = g_step ? a.pitem_g[p] : a.pitem_f[p];
  const int i1 = g_step ? a.pitem_g[p + 1] : a.pitem_f[p + 1];
  const BlockPart *parts = g_step ? a.part_g : a.part_f;
  double mm = -INFINITY, ms = 0.0, dmx = -INFINITY, dmn = INFINITY;
  const int lane = threadIdx.x & 63;
  for (int i = i0 + lane; i < i1; i += 64) {
    const BlockPart q = parts[i];
    const double mn = fmax(mm, q.mass_max);
    if (mn != -INFINITY) ms = ms * exp(mm - mn) + q.mass_sum * exp(q.mass_max - mn);
    mm = mn;
    dmx = fmax(dmx, q.dmax);
    dmn = fmin(dmn, q.dmin);
  }
  wave_lse(mm, ms);
  dmx = wave_max(dmx);
  dmn = wave_min(dmn);
  if (lane != 0) return;
  const double eps = a.eps[p], r1 = a.rho1[p], r2 = a.rho2[p];
  const double L = (mm == -INFINITY) ? -INFINITY : mm + log(ms);
  if (g_step) {
    const HalfCoef c = half_coef(eps, r2, r1);
    const double sBhat = -r2 * L;
    const double tg = c.kappa_t / (1.0 - c.kappa_t) * sBhat;
    st.tau_g = tg;
    st.sB = sBhat + tg;
    st.gdiff_max = dmx;
    st.gdiff_min = dmn;
  } else {
    const HalfCoef c = half_coef(eps, r1, r2);
    const double sAhat = -r1 * L;
    const double tf = c.kappa_t / (1.0 - c.kappa_t) * sAhat;
    st.tau_f = tf;
    st.sA = sAhat + tf;
    const double tau1 = r1 / (r1 + r2), tau2 = r2 / (r1 + r2);
    const double lam = tau1 * st.sB - tau2 * st.sA;
    st.lambda = lam;
    const double off_f = tf + lam, off_g = st.tau_g - lam;
    const int it = st.iter + 1;
    st.iter = it;
    double delta = INFINITY;
    if (it > 1) {
      const double cf = off_f - st.off_f_prev, cg = off_g - st.off_g_prev;
      delta = fmax(fmax(dmx + cf, -(dmn + cf)), fmax(st.gdiff_max + cg, -(st.gdiff_min + cg)));
    }
    st.delta = delta;
    st.off_f_prev = off_f;
    st.off_g_prev = off_g;
    if (!isfinite(off_f) || !isfinite(off_g) || isnan(delta)) st.status = kBatchNumeric;
    if (st.status != kBatchRunning) {
      st.done = 1;
    } else if (a.tol > 0.0 && it % a.check_every == 0 && delta < a.tol) {
      st.status = kBatchConverged;
      st.done = 1;
    } else if (it >= a.max_iter) {
      st.status = kBatchMaxIter;
      st.done = 1;
    }
  }
}

// One work item of a half-step: targets it.y .. it.y + it.z - 1 of problem p, lane l taking
// targets it.y + l + 64 r for r < R (R = 1, 2, 4 for items of at most 64, 128, 256 targets), so that
// each source record read feeds R targets per lane. Softmin over all sources of p, epilogue,
// item partials, and the problem's reduction by the last wave to finish one of its items.
// SPLIT (R = 1): the softmin over sources it2.x .. it2.x + it2.y - 1 of p only; the item
// publishes its per-target (max, sum), and the last item of its group (slots it2.z ..
// it2.z + it2.w - 1, counted at it2.z) merges the group's partials and runs the epilogue;
// the others leave an empty item partial.
template <int D, bool SQ, int R, bool SPLIT = false>
__device__ __forceinline__ void batched_item(const BatchedArgs &a, int g_step, const int4 it,
                                             float *stage, const int4 it2 = make_int4(0, 0, 0, 1)) {
  static_assert(!SPLIT || R == 1, "split items hold one target per lane");
  const int lane = threadIdx.x & 63;
  const int64_t *off_t = g_step ? a.offM : a.offN;
  const int64_t *off_s = g_step ? a.offN : a.offM;
  const float *tpts = g_step ? a.y : a.x;
  const float *tw = g_step ? a.beta : a.alpha;
  float *tpot = g_step ? a.pot_y : a.pot_x;
  float *trec = g_step ? a.rec_y : a.rec_x;
  const float *srec = g_step ? a.rec_x : a.rec_y;
  BlockPart *parts = g_step ? a.part_g : a.part_f;
  int *ticket = g_step ? a.ticket_g : a.ticket_f;
  const int *pitem = g_step ? a.pitem_g : a.pitem_f;
  constexpr int SD = batched_rec_stride(D);
  const int p = it.x;
  BatchState &st = a.state[p];
  const double scd = 1.4426950408889634074 / a.eps[p];
  const float sc = (float)scd;
  const float ssc = SQ ? (float)sqrt(scd) : 1.0f;  // coordinate scale of the p = 2 records
  const int64_t tb = off_t[p];
  const double *mu = a.mu + (size_t)p * kBatchMaxDim;
  float yc[R][D];
  bool valid[R];
  int64_t tg[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    valid[r] = lane + 64 * r < it.z;
    tg[r] = tb + it.y + (valid[r] ? lane + 64 * r : 0);
#pragma unroll
    for (int k = 0; k < D; ++k) yc[r][k] = k < a.d ? (tpts[tg[r] * a.d + k] - (float)mu[k]) * ssc : 0.0f;
  }
  // softmin over all sources of p (a split item: its range of them)
  const int64_t s0 = SPLIT ? off_s[p] + it2.x : off_s[p];
  const int64_t s1 = SPLIT ? s0 + it2.y : off_s[p + 1];
  float m[R], l[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    m[r] = -FLT_MAX;
    l[r] = 0.0f;
  }
  const float half_p = a.half_p;
  auto expo = [&](const float *rp, int r) -> float {
    if constexpr (SQ) {  // b_s - ||u'_s - y'_t||^2 on scaled coordinates
      float v = rp[D];
#pragma unroll
      for (int k = 0; k < D; ++k) {
        const float u = rp[k] - yc[r][k];
        v = fmaf(-u, u, v);
      }
      return v;
    } else {
      float d2 = 0.0f;
#pragma unroll
      for (int k = 0; k < D; ++k) {
        const float u = rp[k] - yc[r][k];
        d2 = fmaf(u, u, d2);
      }
      const float c = half_p == 0.5f ? __builtin_sqrtf(d2) : fast_exp2(half_p * fast_log2(d2));
      return fmaf(-sc, c, rp[D]);
    }
  };
  // The passes over the sources. They walk the sources in chunks of 64: each lane loads one
  // record of the next chunk (a coalesced load of the whole chunk per wave, in flight while
  // the wave works on the current chunk), stores it in the wave's LDS slice, and the wave
  // reads the records back one source at a time (the same address in every lane: an LDS
  // broadcast). Only this wave touches its slice, and a wave's LDS accesses complete in
  // program order, so the slice needs no block barrier.
  auto walk = [&](auto &&body) {
    constexpr int SV = SD / 4;  // float4 per record
    const float4 *gs = reinterpret_cast<const float4 *>(srec);
    float4 *st4 = reinterpret_cast<float4 *>(stage);
    float4 pre[SV];
    auto fetch = [&](int64_t c0) {
      const int64_t si = c0 + lane;
#pragma unroll
      for (int v = 0; v < SV; ++v) pre[v] = si < s1 ? gs[si * SV + v] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    };
    fetch(s0);
    for (int64_t c0 = s0; c0 < s1; c0 += 64) {
      const int cnt = s1 - c0 < 64 ? (int)(s1 - c0) : 64;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int v = 0; v < SV; ++v) st4[lane * SV + v] = pre[v];
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      if (c0 + 64 < s1) fetch(c0 + 64);
      // tiles of kTile sources, then the remaining ones singly
      int j = 0;
      for (; j + kTile <= cnt; j += kTile) body(stage + j * SD, std::integral_constant<int, kTile>());
      for (; j < cnt; ++j) body(stage + j * SD, std::integral_constant<int, 1>());
    }
  };
  // The expanded form of the p = 2 exponent (problems whose rounding rule allows it): with
  // the record's second offset a_s = b_s - ||u'_s||^2, v_ts - c = (a_s - (||y'_t||^2 + c))
  // + sum_k u'_sk (2 y'_tk), one subtraction and D FMAs.
  constexpr bool kExp = SQ && batched_has_expanded_slot(D);
  float y2[kExp ? R : 1][kExp ? D : 1], yn2[kExp ? R : 1];
  if constexpr (kExp) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      float n2 = 0.0f;
#pragma unroll
      for (int k = 0; k < D; ++k) {
        y2[r][k] = 2.0f * yc[r][k];
        n2 = fmaf(yc[r][k], yc[r][k], n2);
      }
      yn2[r] = n2;
    }
  }
  // v_ts - c[r] in the chosen form (c: the reference, or 0 for the maximum pass)
  auto vshift = [&](auto ex, const float *rp, int r, float c) -> float {
    if constexpr (decltype(ex)::value && kExp) {
      float v = rp[D + 1] - c;
#pragma unroll
      for (int k = 0; k < D; ++k) v = fmaf(rp[k], y2[r][k], v);
      return v;
    } else {
      return expo(rp, r) - c;
    }
  };
  // sum_pass: ls[r] = sum_s 2^{v_s - ref[r]}
  auto sum_pass = [&](auto ex, const float (&ref)[R], float (&ls)[R]) {
    float c[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      ls[r] = 0.0f;
      c[r] = (decltype(ex)::value && kExp) ? yn2[kExp ? r : 0] + ref[r] : ref[r];
    }
    walk([&](const float *rp, auto nk) {
#pragma unroll
      for (int k = 0; k < decltype(nk)::value; ++k)
#pragma unroll
        for (int r = 0; r < R; ++r) ls[r] += fast_exp2(vshift(ex, rp + k * SD, r, c[r]));
    });
  };
  // max_pass: mx[r] = max(max_s v_s, -FLT_MAX) (finite, so that v - mx is never NaN)
  auto max_pass = [&](auto ex, float (&mx)[R]) {
    float c[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      mx[r] = -FLT_MAX;
      c[r] = (decltype(ex)::value && kExp) ? yn2[kExp ? r : 0] : 0.0f;
    }
    walk([&](const float *rp, auto nk) {
#pragma unroll
      for (int k = 0; k < decltype(nk)::value; ++k)
#pragma unroll
        for (int r = 0; r < R; ++r) mx[r] = fmaxf(mx[r], vshift(ex, rp + k * SD, r, c[r]));
    });
  };
  // running_max_pass: one pass with a running maximum per target (the split items, whose
  // partials are merged by maximum); the sum is rescaled once per tile that raises it.
  auto running_max_pass = [&](float (&mr)[R], float (&lr)[R]) {
    walk([&](const float *rp, auto nk) {
      constexpr int NK = decltype(nk)::value;
      float v[NK][R];
#pragma unroll
      for (int k = 0; k < NK; ++k)
#pragma unroll
        for (int r = 0; r < R; ++r) v[k][r] = expo(rp + k * SD, r);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        float mt = v[0][r];
#pragma unroll
        for (int k = 1; k < NK; ++k) mt = fmaxf(mt, v[k][r]);
        const float mn = fmaxf(mr[r], mt);
        float acc = lr[r] * fast_exp2(mr[r] - mn);
#pragma unroll
        for (int k = 0; k < NK; ++k) acc += fast_exp2(v[k][r] - mn);
        lr[r] = acc;
        mr[r] = mn;
      }
    });
  };

  if constexpr (!SPLIT) {
    // Fixed reference per target: the log-sum-exp of its last softmin. Each entry costs one
    // exp2 of v - ref and one add (no running maximum, no rescale); the sum shows whether
    // the reference was close: inside [2^-64, 2^64] every term is finite and the terms
    // flushed below 2^-126 are under 2^-62 of the sum. Otherwise (and on the first
    // half-step) a pass over the sources finds each target's maximum, which becomes the
    // reference of a second summing pass (its sum is then in [1, sources]).
    const float *lref = g_step ? a.lref_y : a.lref_x;
    bool have = true;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      m[r] = valid[r] ? lref[tg[r]] : 0.0f;
      have = have && __builtin_isfinite(m[r]);
    }
    auto passes = [&](auto ex) {
      bool ok = false;
      if (__all(have)) {
        sum_pass(ex, m, l);
        ok = true;
#pragma unroll
        for (int r = 0; r < R; ++r) ok = ok && (!valid[r] || (l[r] >= 0x1p-64f && l[r] <= 0x1p64f));
        ok = __all(ok);
      }
      if (!ok) {
        max_pass(ex, m);
        sum_pass(ex, m, l);
      }
    };
    if (kExp && st.expanded)  // the problem's form (the same for the whole wave)
      passes(std::true_type());
    else
      passes(std::false_type());
  } else {
    running_max_pass(m, l);
  }
  if constexpr (SPLIT) {
    float2 *spart = g_step ? a.spart_g : a.spart_f;
    int *gtick = g_step ? a.gtick_g : a.gtick_f;
    spart[(size_t)it.w * 64 + lane] = make_float2(m[0], l[0]);
    int glast = 0;
    if (lane == 0) {
      parts[it.w] = BlockPart{-INFINITY, 0.0, -INFINITY, INFINITY};  // empty unless last
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      glast = (atomicAdd(&gtick[it2.z], 1) == it2.w - 1) ? 1 : 0;
    }
    glast = __shfl(glast, 0, 64);
    if (!glast) {  // the problem's arrival only
      int last = 0;
      if (lane == 0) {
        const int nitems = pitem[p + 1] - pitem[p];
        last = (atomicAdd(&ticket[p], 1) == nitems - 1) ? 1 : 0;
      }
      last = __shfl(last, 0, 64);
      if (last) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        reduce_problem(a, p, g_step != 0);
        if (lane == 0) ticket[p] = 0;
      }
      return;
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // the group's partials
    float mt = -FLT_MAX, lt = 0.0f;
    for (int j = it2.z; j < it2.z + it2.w; ++j) {
      const float2 q = spart[(size_t)j * 64 + lane];
      const float mn = fmaxf(mt, q.x);
      lt = lt * fast_exp2(mt - mn) + q.y * fast_exp2(q.x - mn);
      mt = mn;
    }
    m[0] = mt;
    l[0] = lt;
    if (lane == 0) gtick[it2.z] = 0;  // every member has arrived
  }
  // epilogue: KL prox and TI translation (App. B), records of the new potential (the
  // problem's parameters are read only now, so that they are not held through the passes)
  const double eps = a.eps[p], r1 = a.rho1[p], r2 = a.rho2[p];
  const HalfCoef cf = g_step ? half_coef(eps, r2, r1) : half_coef(eps, r1, r2);
  const double tau_src = g_step ? st.tau_f : st.tau_g;
  const double s_src = g_step ? st.sA : st.sB;
  const double rho_t = g_step ? r2 : r1;
  double mm = -INFINITY, ms = 0.0, dmx = -INFINITY, dmn = INFINITY;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (!valid[r]) continue;
    const double lse2 = (double)m[r] + log2((double)l[r]);
    (g_step ? a.lref_y : a.lref_x)[tg[r]] = (float)lse2;
    const double S = -lse2 / scd;
    const double hnew = cf.k_t * (S - tau_src) - cf.c_t * s_src;
    const float hf = (float)hnew;
    const float old = tpot[tg[r]];
    tpot[tg[r]] = hf;
    const double dh = (double)hf - (double)old;
    dmx = fmax(dmx, dh);
    dmn = fmin(dmn, dh);
    const float w = tw[tg[r]];
    // the record's coordinates never change (written by k_batched_init): only its offsets
    const double lw2 = w > 0.0f ? log2((double)w) : -INFINITY;
    trec[(size_t)tg[r] * SD + D] = (float)(scd * (double)hf + lw2);
    if constexpr (kExp) {  // the expanded form's offset b - ||y'||^2 (as write_rec forms it)
      double n2 = 0.0;
#pragma unroll
      for (int k = 0; k < D; ++k) n2 = fma((double)yc[r][k], (double)yc[r][k], n2);
      trec[(size_t)tg[r] * SD + D + 1] = (float)(scd * (double)hf + lw2 - n2);
    }
    if (w > 0.0f) {
      const double v = log((double)w) - (double)hf / rho_t;
      if (v > mm) {
        ms = ms * exp(mm - v) + 1.0;
        mm = v;
      } else {
        ms += exp(v - mm);
      }
    }
    if (!isfinite(hnew)) st.status = kBatchNumeric;
    // one target's FP64 chain at a time: interleaving the R chains would multiply the
    // registers the whole kernel is allocated
    __builtin_amdgcn_sched_barrier(0);
  }
  wave_lse(mm, ms);
  dmx = wave_max(dmx);
  dmn = wave_min(dmn);
  int last = 0;
  if (lane == 0) {
    parts[it.w] = BlockPart{mm, ms, dmx, dmn};
    // release only: an acquire here would invalidate this XCD's L2 (and the source records
    // the other waves on it are reading) after every item
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const int nitems = pitem[p + 1] - pitem[p];
    last = (atomicAdd(&ticket[p], 1) == nitems - 1) ? 1 : 0;
  }
  last = __shfl(last, 0, 64);
  if (last) {
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // the other items' partials and records
    reduce_problem(a, p, g_step != 0);
    if (lane == 0) ticket[p] = 0;
  }
}

// One half-step for every active problem. g_step: targets y (beta, rho2), sources x.
// SPL: the split item level (items of <= 64 targets, some with a source range; its own
// kernel, so the registers of the other levels' kernel stay as they are).
template <int D, bool SQ, bool SPL>
__global__ __launch_bounds__(256) void k_batched_half(BatchedArgs a, int g_step) {
  const int lane = threadIdx.x & 63;
  const int nact = g_step ? *a.nact_g : *a.nact_f;
  const int *act = g_step ? a.act_g : a.act_f;
  const int4 *items = g_step ? a.items_g : a.items_f;
  int *ctr = g_step ? a.ctr_g : a.ctr_f;
  // each wave's staging slice for the source records of its items (64 records)
  __shared__ float4 s_stage[4][64 * batched_rec_stride(D) / 4];
  float *stage = reinterpret_cast<float *>(s_stage[threadIdx.x >> 6]);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    // the other side's counter is idle during this launch: reset it for the next one
    if (g_step) *a.ctr_f = 0; else *a.ctr_g = 0;
  }

  unsigned long long busy = 0;
  for (;;) {
    int item = 0;
    if (lane == 0) item = atomicAdd(ctr, 1);
    item = __shfl(item, 0, 64);
    if (item >= nact) break;
    const int4 it = items[act[item]];  // (problem, first target, count, slot)
    if (a.state[it.x].done) continue;  // finished by an earlier half-step (compaction is periodic)
    const unsigned long long t0 = a.stats ? __builtin_amdgcn_s_memrealtime() : 0ull;
    if constexpr (SPL) {
      const int4 it2 = (g_step ? a.items2_g : a.items2_f)[act[item]];
      if (it2.w > 1)
        batched_item<D, SQ, 1, true>(a, g_step, it, stage, it2);
      else
        batched_item<D, SQ, 1>(a, g_step, it, stage);
    } else if (it.z > 128)
      batched_item<D, SQ, 4>(a, g_step, it, stage);
    else if (it.z > 64)
      batched_item<D, SQ, 2>(a, g_step, it, stage);
    else
      batched_item<D, SQ, 1>(a, g_step, it, stage);
    if (a.stats) busy += __builtin_amdgcn_s_memrealtime() - t0;
  }
  if (a.stats && lane == 0 && busy) atomicAdd(&a.stats->busy, busy);
}

// Rebuilds the active item lists (items of problems not done), resets the work counters,
// and counts the problems still running. One block.
__global__ __launch_bounds__(1024) void k_batched_compact(BatchedArgs a) {
  __shared__ int s_ng, s_nf, s_run;
  __shared__ double s_work[1024];
  if (threadIdx.x == 0) { s_ng = 0; s_nf = 0; s_run = 0; }
  __syncthreads();
  double work = 0.0;
  for (int p = threadIdx.x; p < a.B; p += blockDim.x)
    if (!a.state[p].done) {
      atomicAdd(&s_run, 1);
      work += (double)(a.offN[p + 1] - a.offN[p]) * (double)(a.offM[p + 1] - a.offM[p]);
    }
  if (a.stats) {
    s_work[threadIdx.x] = work;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
      if (threadIdx.x < o) s_work[threadIdx.x] += s_work[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      a.stats->work = s_work[0];
      a.stats->t_compact = __builtin_amdgcn_s_memrealtime();
    }
  }
  for (int i = threadIdx.x; i < a.n_items_g; i += blockDim.x)
    if (!a.state[a.items_g[i].x].done) a.act_g[atomicAdd(&s_ng, 1)] = i;
  for (int i = threadIdx.x; i < a.n_items_f; i += blockDim.x)
    if (!a.state[a.items_f[i].x].done) a.act_f[atomicAdd(&s_nf, 1)] = i;
  __syncthreads();
  if (threadIdx.x == 0) {
    *a.nact_g = s_ng;
    *a.nact_f = s_nf;
    *a.running = s_run;
    *a.ctr_g = 0;
    *a.ctr_f = 0;
  }
}

// Per problem (one block each): common mean of its clouds, weight checks, zero potentials,
// records of both sides from zero potentials, and the initial scalars (Smin_alpha^rho1(0)).
template <int D>
__global__ __launch_bounds__(256) void k_batched_init(BatchedArgs a) {
  const int p = blockIdx.x;
  __shared__ double sh[256];
  __shared__ int s_bad, s_pa, s_pb;
  const int64_t n0 = a.offN[p], n1 = a.offN[p + 1], m0 = a.offM[p], m1 = a.offM[p + 1];
  if (threadIdx.x == 0) { s_bad = 0; s_pa = 0; s_pb = 0; }
  __syncthreads();
  double *mu = a.mu + (size_t)p * kBatchMaxDim;
  for (int k = 0; k < kBatchMaxDim; ++k) {
    double s = 0.0;
    if (k < a.d) {
      for (int64_t i = n0 + threadIdx.x; i < n1; i += 256) s += (double)a.x[i * a.d + k];
      for (int64_t j = m0 + threadIdx.x; j < m1; j += 256) s += (double)a.y[j * a.d + k];
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) mu[k] = (k < a.d) ? sh[0] / (double)((n1 - n0) + (m1 - m0)) : 0.0;
    __syncthreads();
  }
  const double eps = a.eps[p], r1 = a.rho1[p];
  const double scd = 1.4426950408889634074 / eps;
  const float ssc = a.half_p == 1.0f ? (float)sqrt(scd) : 1.0f;  // p = 2: scaled coordinates
  constexpr int SD = batched_rec_stride(D);
  // x side (alpha) and y side (beta): zero potentials and records; tilted mass of alpha;
  // the largest |x - mu|^2 and |y - mu|^2 (the rounding of the expanded exponent form)
  double mm = -INFINITY, ms = 0.0;
  double r2max[2] = {0.0, 0.0};
  for (int side = 0; side < 2; ++side) {
    const int64_t b0 = side == 0 ? n0 : m0, b1 = side == 0 ? n1 : m1;
    const float *pts = side == 0 ? a.x : a.y;
    const float *w = side == 0 ? a.alpha : a.beta;
    float *pot = side == 0 ? a.pot_x : a.pot_y;
    float *rec = side == 0 ? a.rec_x : a.rec_y;
    float *lref = side == 0 ? a.lref_x : a.lref_y;
    for (int64_t i = b0 + threadIdx.x; i < b1; i += 256) {
      lref[i] = __builtin_nanf("");  // no reference yet: the first softmin finds its maximum
      const float wi = w[i];
      if (!(wi >= 0.0f) || isinf(wi)) s_bad = 1;
      if (wi > 0.0f) { if (side == 0) s_pa = 1; else s_pb = 1; }
      float yc[D];
      double r2 = 0.0;
#pragma unroll
      for (int k = 0; k < D; ++k) {
        const double u = k < a.d ? (double)pts[i * a.d + k] - mu[k] : 0.0;
        r2 = fma(u, u, r2);
        yc[k] = k < a.d ? (pts[i * a.d + k] - (float)mu[k]) * ssc : 0.0f;
      }
      r2max[side] = fmax(r2max[side], r2);
      pot[i] = 0.0f;
      write_rec<D>(rec + (size_t)i * SD, yc, 0.0f, wi, scd);
      if (side == 0 && wi > 0.0f) {
        const double v = log((double)wi);
        const double mn = fmax(mm, v);
        ms = ms * exp(mm - mn) + exp(v - mn);
        mm = mn;
      }
    }
  }
  // block log-sum-exp of the alpha terms, block maxima of the squared radii
  __shared__ double sm[256], ss[256], sr[2][256];
  sm[threadIdx.x] = mm;
  ss[threadIdx.x] = ms;
  sr[0][threadIdx.x] = r2max[0];
  sr[1][threadIdx.x] = r2max[1];
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      const double m_a = sm[threadIdx.x], m_b = sm[threadIdx.x + o];
      const double mn = fmax(m_a, m_b);
      if (mn != -INFINITY)
        ss[threadIdx.x] = ss[threadIdx.x] * exp(m_a - mn) + ss[threadIdx.x + o] * exp(m_b - mn);
      sm[threadIdx.x] = mn;
      sr[0][threadIdx.x] = fmax(sr[0][threadIdx.x], sr[0][threadIdx.x + o]);
      sr[1][threadIdx.x] = fmax(sr[1][threadIdx.x], sr[1][threadIdx.x + o]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    BatchState &st = a.state[p];
    const double L = sm[0] == -INFINITY ? -INFINITY : sm[0] + log(ss[0]);
    st.sA = -r1 * L;
    st.sB = 0.0;
    st.tau_f = st.tau_g = st.lambda = 0.0;
    st.off_f_prev = st.off_g_prev = 0.0;
    st.gdiff_max = st.gdiff_min = 0.0;
    st.delta = INFINITY;
    st.iter = 0;
    const double e = a.eps[p], q1 = a.rho1[p], q2 = a.rho2[p];
    const bool bad_par = !(e > 0.0) || !isfinite(e) || !(q1 > 0.0) || !isfinite(q1) ||
                         !(q2 > 0.0) || !isfinite(q2);
    const bool bad = s_bad || !s_pa || !s_pb || bad_par;
    st.status = bad ? kBatchInvalid : kBatchRunning;
    st.done = bad ? 1 : 0;
    // p = 2: the expanded exponent where its float32 rounding, E = 2^-24 (d + 4) (max|x - mu|
    // + max|y - mu|)^2 in potential units, is small against eps (the single-problem solvers'
    // rule, its first condition alone)
    const double span = sqrt(sr[0][0]) + sqrt(sr[1][0]);
    const double E = 0x1p-24 * (double)(a.d + 4) * span * span;
    st.expanded = (batched_has_expanded_slot(D) && a.half_p == 1.0f &&
                   E * 1.4426950408889634074 / e <= kBatchFormDelta) ? 1 : 0;
    a.ticket_g[p] = 0;
    a.ticket_f[p] = 0;
  }
}

// Reported potentials f = fhat + tau_f + lambda, g = ghat + tau_g - lambda, per problem;
// iteration counts and statuses.
__global__ __launch_bounds__(256) void k_batched_finalize(BatchedArgs a, float *f, float *g,
                                                           int32_t *iters, int32_t *status) {
  const int64_t totN = a.offN[a.B], totM = a.offM[a.B];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < totN + totM; i += stride) {
    const bool xs = i < totN;
    const int64_t j = xs ? i : i - totN;
    const int64_t *off = xs ? a.offN : a.offM;
    int lo = 0, hi = a.B - 1;  // problem p with off[p] <= j < off[p + 1]
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (off[mid] <= j) lo = mid; else hi = mid - 1;
    }
    const BatchState &st = a.state[lo];
    if (xs) f[j] = (float)((double)a.pot_x[j] + st.tau_f + st.lambda);
    else g[j] = (float)((double)a.pot_y[j] + st.tau_g - st.lambda);
  }
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < a.B; p += stride) {
    iters[p] = a.state[p].iter;
    status[p] = a.state[p].status;
  }
}

template <int D, bool SPL>
hipError_t launch_half_sp(const BatchedArgs &a, int g_step, int blocks, hipStream_t s) {
  if (a.half_p == 1.0f)
    hipLaunchKernelGGL((k_batched_half<D, true, SPL>), dim3(blocks), dim3(256), 0, s, a, g_step);
  else
    hipLaunchKernelGGL((k_batched_half<D, false, SPL>), dim3(blocks), dim3(256), 0, s, a, g_step);
  return hipGetLastError();
}

template <int D>
hipError_t launch_half_t(const BatchedArgs &a, int g_step, int blocks, hipStream_t s) {
  if (a.items2_g != nullptr) return launch_half_sp<D, true>(a, g_step, blocks, s);
  return launch_half_sp<D, false>(a, g_step, blocks, s);
}

template <int D>
hipError_t launch_init_t(const BatchedArgs &a, hipStream_t s) {
  hipLaunchKernelGGL((k_batched_init<D>), dim3(a.B), dim3(256), 0, s, a);
  return hipGetLastError();
}

template <int D>
int half_occupancy_t(const BatchedArgs &a) {
  int nb = 0;
  const hipError_t e = a.half_p == 1.0f
      ? (a.items2_g != nullptr
             ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batched_half<D, true, true>, 256, 0)
             : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batched_half<D, true, false>, 256, 0))
      : (a.items2_g != nullptr
             ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batched_half<D, false, true>, 256, 0)
             : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batched_half<D, false, false>, 256, 0));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return nb;
}

#define UOT_BATCH_DISPATCH(FN, ...)            \
  do {                                         \
    switch (a.d) {                             \
      case 1: return FN<1>(__VA_ARGS__);       \
      case 2: return FN<2>(__VA_ARGS__);       \
      case 3: return FN<3>(__VA_ARGS__);       \
      case 4: return FN<4>(__VA_ARGS__);       \
      case 5: return FN<5>(__VA_ARGS__);       \
      case 6: return FN<6>(__VA_ARGS__);       \
      case 7: return FN<7>(__VA_ARGS__);       \
      case 8: return FN<8>(__VA_ARGS__);       \
    }                                          \
  } while (0)

}  // namespace

hipError_t launch_batched_half(const BatchedArgs &a, int g_step, int blocks, hipStream_t s) {
  UOT_BATCH_DISPATCH(launch_half_t, a, g_step, blocks, s);
  return hipErrorInvalidValue;
}

hipError_t launch_batched_init(const BatchedArgs &a, hipStream_t s) {
  UOT_BATCH_DISPATCH(launch_init_t, a, s);
  return hipErrorInvalidValue;
}

int batched_half_blocks_per_cu(const BatchedArgs &a) {
  UOT_BATCH_DISPATCH(half_occupancy_t, a);
  return 0;
}

hipError_t launch_batched_compact(const BatchedArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_batched_compact, dim3(1), dim3(1024), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_batched_finalize(const BatchedArgs &a, float *f, float *g, int32_t *iters,
                                   int32_t *status, hipStream_t s) {
  hipLaunchKernelGGL(k_batched_finalize, dim3(1024), dim3(256), 0, s, a, f, g, iters, status);
  return hipGetLastError();
}

}  // namespace uot
