// Points-cost softmin partials on the VALU (gfx950).
//
// For every target t and every split of the sources, one pass computes the log2-domain
// running pair (max m_t, sum l_t) of 2^{v_ts}, where v_ts is the exponent of the softmin
// of Sec. 3 written in base 2:
//   kSqEuc: v_ts = b_s + <u_s, y_t>,   u_s = 2 sc (x_s - mu),  b_s = sc h_s + log2 w_s - sc |x_s - mu|^2
//           (the target term -sc |y_t - mu|^2 is added by the combine kernel)
//   kPower: v_ts = b_s - sc ||x_s - y_t||^p,   b_s = sc h_s + log2 w_s
// with sc = log2(e)/eps, so that Smin_w^eps(C_{:,t} - h) = -(LSE2_t)/sc.
//
// Work split: each thread owns R targets (its lanes' coordinates stay in registers); the
// sources of one split are uniform across the wave and are read with scalar loads. Sources
// are taken 8 at a time: the 8 x R exponents are formed, the running max is raised once per
// tile, and each entry then costs one exp2.
#include <cfloat>

#include "uot_internal.h"

namespace uot {
namespace {

constexpr int kTile = 8;

__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float fast_log2(float x) { return __builtin_amdgcn_logf(x); }

template <int MODE>
__device__ __forceinline__ float cost_pow(float d2, float half_p) {
  // ||x - y||^p from the squared distance: p = 1 takes a square root, otherwise
  // 2^{(p/2) log2 d2} (d2 = 0 gives log2 = -inf and the power 0).
  if (half_p == 0.5f) return __builtin_sqrtf(d2);
  return fast_exp2(half_p * fast_log2(d2));
}

template <int D, int MODE, int R>
__global__ __launch_bounds__(256) void k_points_partial(PointsArgs a) {
  if (a.done != nullptr && *a.done) return;
  constexpr int SD = rec_stride(MODE, D);
  const int t0 = blockIdx.x * (256 * R) + threadIdx.x;

  float y[R][D];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int t = t0 + r * 256;
    const int tc = t < a.nt ? t : a.nt - 1;
#pragma unroll
    for (int d = 0; d < D; ++d)
      y[r][d] = d < a.d ? a.tgt[(size_t)tc * a.d + d] - (float)a.mu[d] : 0.0f;
  }

  float m[R], l[R];
#pragma unroll
  for (int r = 0; r < R; ++r) { m[r] = -FLT_MAX; l[r] = 0.0f; }

  const int s0 = blockIdx.y * a.split_len;
  const int s1 = min(a.ns, s0 + a.split_len);
  const float sc = a.sc, half_p = a.half_p;

  auto exponent = [&](const float *rp, int r) -> float {
    if constexpr (MODE == kSqEuc) {
      float acc = rp[D];
#pragma unroll
      for (int d = 0; d < D; ++d) acc = fmaf(rp[d], y[r][d], acc);
      return acc;
    } else {
      float d2 = 0.0f;
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const float u = rp[d] - y[r][d];
        d2 = fmaf(u, u, d2);
      }
      return fmaf(-sc, cost_pow<MODE>(d2, half_p), rp[D]);
    }
  };

  int s = s0;
  for (; s + kTile <= s1; s += kTile) {
    float v[kTile][R];
#pragma unroll
    for (int k = 0; k < kTile; ++k) {
      const float *rp = a.rec + (size_t)(s + k) * SD;
#pragma unroll
      for (int r = 0; r < R; ++r) v[k][r] = exponent(rp, r);
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      float mt = v[0][r];
#pragma unroll
      for (int k = 1; k < kTile; ++k) mt = fmaxf(mt, v[k][r]);
      const float mn = fmaxf(m[r], mt);
      float acc = l[r] * fast_exp2(m[r] - mn);
#pragma unroll
      for (int k = 0; k < kTile; ++k) acc += fast_exp2(v[k][r] - mn);
      l[r] = acc;
      m[r] = mn;
    }
  }
  for (; s < s1; ++s) {
    const float *rp = a.rec + (size_t)s * SD;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const float v = exponent(rp, r);
      const float mn = fmaxf(m[r], v);
      l[r] = l[r] * fast_exp2(m[r] - mn) + fast_exp2(v - mn);
      m[r] = mn;
    }
  }

#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int t = t0 + r * 256;
    if (t < a.nt) a.part[(size_t)blockIdx.y * a.nt + t] = make_float2(m[r], l[r]);
  }
}

template <int D>
constexpr int targets_per_thread() {
  return D <= 4 ? 4 : (D <= 8 ? 2 : 1);
}

template <int D, int MODE>
hipError_t launch_bucket(const PointsArgs &a, hipStream_t st) {
  constexpr int R = targets_per_thread<D>();
  dim3 grid((a.nt + 256 * R - 1) / (256 * R), a.nsplit);
  hipLaunchKernelGGL((k_points_partial<D, MODE, R>), grid, dim3(256), 0, st, a);
  return hipGetLastError();
}

template <int MODE>
hipError_t launch_mode(const PointsArgs &a, hipStream_t st) {
  switch (dim_bucket(a.d)) {
    case 1: return launch_bucket<1, MODE>(a, st);
    case 2: return launch_bucket<2, MODE>(a, st);
    case 3: return launch_bucket<3, MODE>(a, st);
    case 4: return launch_bucket<4, MODE>(a, st);
    case 5: return launch_bucket<5, MODE>(a, st);
    case 6: return launch_bucket<6, MODE>(a, st);
    case 7: return launch_bucket<7, MODE>(a, st);
    case 8: return launch_bucket<8, MODE>(a, st);
    case 12: return launch_bucket<12, MODE>(a, st);
    case 16: return launch_bucket<16, MODE>(a, st);
    case 24: return launch_bucket<24, MODE>(a, st);
    case 32: return launch_bucket<32, MODE>(a, st);
    case 48: return launch_bucket<48, MODE>(a, st);
    case 64: return launch_bucket<64, MODE>(a, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

int points_targets_per_block(int mode, int d) {
  (void)mode;
  const int b = dim_bucket(d);
  return 256 * (b <= 4 ? 4 : (b <= 8 ? 2 : 1));
}

hipError_t launch_points_partial(int mode, const PointsArgs &a, hipStream_t st) {
  if (mode == kSqEuc) return launch_mode<kSqEuc>(a, st);
  if (mode == kPower) return launch_mode<kPower>(a, st);
  return hipErrorInvalidValue;
}

}  // namespace uot
