// Envelope gradients and plan marginals of a points cost, one pass over the sources per
// side, one exp2 per entry (gfx950).
//
// Targets t are the points of one side, sources s those of the other, with source records
// (x_s - mu, b_s = sc h_s + log2 w_s) and sc = log2(e)/eps. The plan entry is
//   pi_ts = w_t 2^{sc h_t} 2^{e_ts},   e_ts = b_s - sc C_ts,   C_ts = ||t - s||^p,
// its row sum pi1_t = w_t 2^{sc h_t} sum_s 2^{e_ts}, and the gradient of <pi, C> in t (the
// envelope theorem applied to the dual, Sec. 1)
//   sum_s pi_ts c'(||t - s||) (t - s),   c'(r) (t - s) = p r^{p-2} (t - s)  (0 at t = s).
// Per (source split, target) the kernel accumulates, relative to a reference r_t,
//   l_t = sum_s 2^{e_ts - r_t},   acc_tk = sum_s 2^{e_ts - r_t} w(d2) (t_k - s_k),
// with w = 1 for p = 2 (the factor p = 2 is applied by the combine) and p d2^{(p-2)/2}
// otherwise. The exponent is taken through the differences t - s, so its float32 rounding is
// relative to the entry's own cost, not to the spread of the clouds.
//
// Reference. With gradients requested, r_t starts at -sc h_t / k_t: at the optimum the
// target's potential is the KL prox of its softmin, h_t = k_t Smin(C_t - h_s) (Sec. 3), so
// this is log2 sum_s 2^{e_ts} and each entry costs one exp2 and no rescaling. A wave in
// which some lane's sum leaves [2^-64, 2^64] (potentials far from the optimum) redoes its
// split with a running maximum raised once per tile of sources. Without gradients (row sums
// only) the running maximum is used from the start (one max per entry is cheap there).
//
// Work split: each lane owns R targets (coordinates and accumulators in registers); the
// sources of one split are uniform across the wave and read with scalar loads.
#include <cfloat>

#include "uot_internal.h"

namespace uot {
namespace {

__device__ __forceinline__ float fexp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float flog2(float x) { return __builtin_amdgcn_logf(x); }

constexpr float kSumLo = 0x1p-64f, kSumHi = 0x1p64f;

template <int D>
constexpr int grad_targets_per_lane() {
  return D <= 8 ? 4 : (D <= 16 ? 2 : 1);
}

// Sources per tile of the running-maximum loop.
constexpr int kTile = 4;

template <int D, int R, bool GRAD>
__global__ __launch_bounds__(256) void k_grad_partial(GradArgs a) {
  constexpr int SD = rec_stride(kPower, D);
  constexpr int PS = grad_part_stride(GRAD ? D : 0);
  const int t0 = blockIdx.x * (256 * R) + threadIdx.x;
  const float sc = a.sc, half_p = a.half_p, p = a.p;
  const float gexp = 0.5f * (p - 2.0f);

  float y[R][D];
  float ref[R];
  bool valid[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int t = t0 + r * 256;
    valid[r] = t < a.nt;
    const int tc = valid[r] ? t : a.nt - 1;
#pragma unroll
    for (int k = 0; k < D; ++k)
      y[r][k] = k < a.d ? a.tgt[(size_t)tc * a.d + k] - (float)a.mu[k] : 0.0f;
    ref[r] = (float)(-(double)sc * (double)a.h_t[tc] * a.inv_k);
  }
  const int s0 = blockIdx.y * a.split_len;
  const int s1 = min(a.ns, s0 + a.split_len);

  auto cost = [&](float d2) -> float {
    if (half_p == 1.0f) return d2;
    if (half_p == 0.5f) return __builtin_sqrtf(d2);
    return fexp2(half_p * flog2(d2));
  };
  auto weight = [&](float d2) -> float {
    if (half_p == 1.0f) return 1.0f;
    return d2 > 0.0f ? p * fexp2(gexp * flog2(d2)) : 0.0f;
  };

  float l[R], acc[R][GRAD ? D : 1];
  auto clear = [&]() {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      l[r] = 0.0f;
#pragma unroll
      for (int k = 0; k < (GRAD ? D : 1); ++k) acc[r][k] = 0.0f;
    }
  };
  clear();

  bool fast = GRAD;
  if constexpr (GRAD) {
    // one exp2 per entry against the reference of the optimum
    for (int s = s0; s < s1; ++s) {
      const float *rp = a.rec + (size_t)s * SD;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        float diff[D];
        float d2 = 0.0f;
#pragma unroll
        for (int k = 0; k < D; ++k) {
          diff[k] = y[r][k] - rp[k];
          d2 = fmaf(diff[k], diff[k], d2);
        }
        const float q = fexp2(fmaf(-sc, cost(d2), rp[D] - ref[r]));
        l[r] += q;
        const float qw = q * weight(d2);
#pragma unroll
        for (int k = 0; k < D; ++k) acc[r][k] = fmaf(qw, diff[k], acc[r][k]);
      }
    }
    bool bad = false;
#pragma unroll
    for (int r = 0; r < R; ++r) bad |= valid[r] && !(l[r] >= kSumLo && l[r] <= kSumHi);
    fast = !__any(bad);
  }

  if (!fast) {
    // running maximum, raised once per tile of kTile sources
    clear();
#pragma unroll
    for (int r = 0; r < R; ++r) ref[r] = -FLT_MAX;
    for (int s = s0; s < s1; s += kTile) {
      const int ns = min(kTile, s1 - s);
      float e[kTile][R];
#pragma unroll
      for (int j = 0; j < kTile; ++j) {
        const float *rp = a.rec + (size_t)(s + (j < ns ? j : 0)) * SD;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          float d2 = 0.0f;
#pragma unroll
          for (int k = 0; k < D; ++k) {
            const float u = y[r][k] - rp[k];
            d2 = fmaf(u, u, d2);
          }
          e[j][r] = j < ns ? fmaf(-sc, cost(d2), rp[D]) : -INFINITY;
        }
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        float mt = e[0][r];
#pragma unroll
        for (int j = 1; j < kTile; ++j) mt = fmaxf(mt, e[j][r]);
        const float mn = fmaxf(ref[r], mt);
        const float scale = fexp2(ref[r] - mn);
        l[r] *= scale;
        if constexpr (GRAD) {
#pragma unroll
          for (int k = 0; k < D; ++k) acc[r][k] *= scale;
        }
        ref[r] = mn;
      }
#pragma unroll
      for (int j = 0; j < kTile; ++j) {
        if (j >= ns) break;
        const float *rp = a.rec + (size_t)(s + j) * SD;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const float q = fexp2(e[j][r] - ref[r]);
          l[r] += q;
          if constexpr (GRAD) {
            float diff[D];
            float d2 = 0.0f;
#pragma unroll
            for (int k = 0; k < D; ++k) {
              diff[k] = y[r][k] - rp[k];
              d2 = fmaf(diff[k], diff[k], d2);
            }
            const float qw = q * weight(d2);
#pragma unroll
            for (int k = 0; k < D; ++k) acc[r][k] = fmaf(qw, diff[k], acc[r][k]);
          }
        }
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
#pragma unroll
      for (int k = 0; k < D; ++k) o[2 + k] = acc[r][k];
    }
  }
}

// Merges the split partials of each target (double precision) and writes what was asked:
//   rowsum_t = sum_s w_s e^{(h_t + h_s - C_ts)/eps} = 2^{sc h_t + M} sum,
//   marg_t   = w_t rowsum_t                                   (the plan marginal pi1_t),
//   dw_t     = gout (rho (1 - e^{-h_t/rho}) - eps (rowsum_t - mass_other))   (d/d w_t),
//   dpts_tk  = gout w_t 2^{sc h_t + M} pfac acc_k              (d/d t_k),
// with pfac = 2 for p = 2 (the kernel's weight is 1 there) and 1 otherwise.
template <int DC>
__global__ __launch_bounds__(256) void k_grad_combine(GradCombineArgs a) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= a.nt) return;
  constexpr int ps = grad_part_stride(DC);
  float M = -FLT_MAX;
  for (int q = 0; q < a.nsplit; ++q) M = fmaxf(M, a.part[((size_t)q * a.nt + t) * ps]);
  double sum = 0.0, acc[DC > 0 ? DC : 1];
#pragma unroll
  for (int k = 0; k < (DC > 0 ? DC : 1); ++k) acc[k] = 0.0;
  for (int q = 0; q < a.nsplit; ++q) {
    const float *o = a.part + ((size_t)q * a.nt + t) * ps;
    if (o[1] == 0.0f) continue;
    const double f = exp2((double)o[0] - (double)M);
    sum += f * (double)o[1];
    if constexpr (DC > 0) {
#pragma unroll
      for (int k = 0; k < DC; ++k) acc[k] += f * (double)o[2 + k];
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
    if (a.dpts) {
      const double fac = wt > 0.0 ? a.gout * wt * base * a.pfac : 0.0;
#pragma unroll
      for (int k = 0; k < DC; ++k)
        if (k < a.d) a.dpts[(size_t)t * a.d + k] = (float)(fac * acc[k]);
    }
  }
}

template <int D, bool GRAD>
hipError_t grad_for(const GradArgs &a, hipStream_t s, const LaunchTiming *t) {
  constexpr int R = grad_targets_per_lane<D>();
  dim3 grid((a.nt + 256 * R - 1) / (256 * R), a.nsplit);
  return launch_timed(k_grad_partial<D, R, GRAD>, grid, dim3(256), s, t, a);
}

template <int D>
hipError_t grad_for_mode(const GradArgs &a, hipStream_t s, const LaunchTiming *t) {
  return a.grad ? grad_for<D, true>(a, s, t) : grad_for<D, false>(a, s, t);
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

int grad_targets_per_block(int d) {
  const int b = dim_bucket(d);
  return 256 * (b <= 8 ? 4 : (b <= 16 ? 2 : 1));
}

hipError_t launch_grad_partial(const GradArgs &a, hipStream_t s, const LaunchTiming *t) {
  UOT_GRAD_BUCKETS(grad_for_mode, dim_bucket(a.d), a, s, t)
  return hipErrorInvalidValue;
}

hipError_t launch_grad_combine(const GradCombineArgs &a, hipStream_t s) {
  if (a.dpts == nullptr) return combine_for<0>(a, s);
  UOT_GRAD_BUCKETS(combine_for, dim_bucket(a.d), a, s)
  return hipErrorInvalidValue;
}

}  // namespace uot
