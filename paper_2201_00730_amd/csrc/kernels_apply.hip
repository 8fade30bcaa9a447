// Plan application with the plan recomputed on the fly (gfx950).
//
// For each target t, with source offsets a_s = sc h_s + log2 w_s (sc = log2(e)/eps):
//   e_ts = a_s - sc C_ts,   pi_ts = w_t 2^{sc h_t} 2^{e_ts},   out_tc = sum_s pi_ts V_sc.
// One pass keeps a running max of e_ts per target and rescales its accumulators, so no
// entry of pi is ever formed in overflowing range. Sources are split across blocks and the
// per-split (max, sum, accumulators) records are merged by a second kernel. Accumulators
// are taken 4 output columns per launch. Dense costs are read as C[t, s] (targets = rows)
// or C[s, t] (targets = columns). (The marginals and the envelope gradients take the
// one-exp pass of kernels_grad.hip.)
#include <cfloat>

#include "uot_internal.h"

namespace uot {
namespace {

constexpr int kKV = 4;                 // accumulator columns per launch
constexpr int kRecF = 2 + kKV;         // floats per partial record: max, sum, acc[4]

__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float fast_log2(float x) { return __builtin_amdgcn_logf(x); }

struct ApplyLaunch {
  ApplyArgs a;
  const float *src_off;  // a_s [ns]
  int c0, kv;            // output columns [c0, c0 + kv)
  int split_len, nsplit;
  float *part;           // [nsplit, nt, kRecF]
};

template <int D, int MODE>
__global__ __launch_bounds__(256) void k_apply_partial(ApplyLaunch L) {
  const ApplyArgs &a = L.a;
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= a.nt) return;
  float yt[D > 0 ? D : 1];
  if constexpr (MODE != kDense) {
#pragma unroll
    for (int k = 0; k < D; ++k) yt[k] = k < a.d ? a.tgt[(size_t)t * a.d + k] - (float)a.mu[k] : 0.0f;
  }
  const float sc = a.sc;
  const float half_p = (float)(0.5 * a.p);
  float m = -FLT_MAX, l = 0.0f, acc[kKV];
#pragma unroll
  for (int c = 0; c < kKV; ++c) acc[c] = 0.0f;
  const int s0 = blockIdx.y * L.split_len;
  const int s1 = min(a.ns, s0 + L.split_len);
  for (int s = s0; s < s1; ++s) {
    float cst, d2 = 0.0f;
    float diff[D > 0 ? D : 1];
    if constexpr (MODE == kDense) {
      cst = a.transpose ? a.C[(size_t)s * a.ldc + t] : a.C[(size_t)t * a.ldc + s];
    } else {
#pragma unroll
      for (int k = 0; k < D; ++k) {
        const float xs = k < a.d ? a.src[(size_t)s * a.d + k] - (float)a.mu[k] : 0.0f;
        diff[k] = yt[k] - xs;
        d2 = fmaf(diff[k], diff[k], d2);
      }
      if (MODE == kSqEuc) cst = d2;
      else cst = (half_p == 0.5f) ? __builtin_sqrtf(d2) : fast_exp2(half_p * fast_log2(d2));
    }
    const float e = fmaf(-sc, cst, L.src_off[s]);
    const float mn = fmaxf(m, e);
    const float scale = fast_exp2(m - mn);
    const float pe = fast_exp2(e - mn);
    l = l * scale + pe;
#pragma unroll
    for (int c = 0; c < kKV; ++c) {
      const float v = c < L.kv ? a.V[(size_t)s * a.ldv + L.c0 + c] : 0.0f;
      acc[c] = acc[c] * scale + pe * v;
    }
    m = mn;
  }
  float *o = L.part + ((size_t)blockIdx.y * a.nt + t) * kRecF;
  o[0] = m;
  o[1] = l;
#pragma unroll
  for (int c = 0; c < kKV; ++c) o[2 + c] = acc[c];
}

__global__ __launch_bounds__(256) void k_apply_combine(ApplyLaunch L) {
  const ApplyArgs &a = L.a;
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= a.nt) return;
  float M = -FLT_MAX;
  for (int p = 0; p < L.nsplit; ++p) M = fmaxf(M, L.part[((size_t)p * a.nt + t) * kRecF]);
  double acc[kKV] = {0.0, 0.0, 0.0, 0.0};
  for (int p = 0; p < L.nsplit; ++p) {
    const float *q = L.part + ((size_t)p * a.nt + t) * kRecF;
    const double sc = exp2((double)q[0] - (double)M);
#pragma unroll
    for (int c = 0; c < kKV; ++c) acc[c] += sc * (double)q[2 + c];
  }
  // pi_ts factor of the target: w_t 2^{sc h_t} 2^{M}
  const double wt = (double)a.w_t[t];
  const double fac = wt > 0.0 ? wt * exp2((double)a.sc * (double)a.h_t[t] + (double)M) : 0.0;
  for (int c = 0; c < L.kv; ++c)
    a.out[(size_t)t * a.ldout + L.c0 + c] = (float)(fac * acc[c]);
}

template <int D, int MODE>
hipError_t apply_for(const ApplyLaunch &L, hipStream_t s) {
  dim3 grid((L.a.nt + 255) / 256, L.nsplit);
  hipLaunchKernelGGL((k_apply_partial<D, MODE>), grid, dim3(256), 0, s, L);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_apply_combine, dim3((L.a.nt + 255) / 256), dim3(256), 0, s, L);
  return hipGetLastError();
}

hipError_t apply_dispatch(const ApplyLaunch &L, hipStream_t s) {
  const int mode = L.a.mode;
  if (mode == kDense) return apply_for<0, kDense>(L, s);
  const int b = dim_bucket(L.a.d);
#define UOT_APPLY_CASE(DD)                                              \
  case DD:                                                              \
    return mode == kSqEuc ? apply_for<DD, kSqEuc>(L, s) : apply_for<DD, kPower>(L, s);
  switch (b) {
    UOT_APPLY_CASE(1) UOT_APPLY_CASE(2) UOT_APPLY_CASE(3) UOT_APPLY_CASE(4)
    UOT_APPLY_CASE(5) UOT_APPLY_CASE(6) UOT_APPLY_CASE(7) UOT_APPLY_CASE(8)
    UOT_APPLY_CASE(12) UOT_APPLY_CASE(16) UOT_APPLY_CASE(24) UOT_APPLY_CASE(32)
    UOT_APPLY_CASE(48) UOT_APPLY_CASE(64)
  }
#undef UOT_APPLY_CASE
  return hipErrorInvalidValue;
}

// Source offsets a_s = sc h_s + log2 w_s.
__global__ __launch_bounds__(256) void k_src_offsets(const float *h, const float *w, int n, float sc,
                                                     float *out) {
  const int s = blockIdx.x * 256 + threadIdx.x;
  if (s >= n) return;
  const float ws = w[s];
  out[s] = ws > 0.0f ? (float)((double)sc * (double)h[s] + log2((double)ws)) : -INFINITY;
}

__global__ __launch_bounds__(1024) void k_sum(const float *w, int n, double *out) {
  __shared__ double s[1024];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 1024) acc += (double)w[i];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 512; off > 0; off >>= 1) {
    if (threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = s[0];
}

}  // namespace

// Scratch layout: source offsets [round_up(ns, 64)] floats, then the split partials.
size_t apply_partial_bytes(int nt, int ns) {
  const int split = ns < 256 ? ns : 256;
  const int nsplit = (ns + split - 1) / split;
  const size_t off_floats = (size_t)((ns + 63) / 64) * 64;
  return (off_floats + (size_t)nsplit * (size_t)nt * kRecF) * sizeof(float);
}

// scratch: at least apply_partial_bytes(nt, ns) bytes.
hipError_t launch_apply_with_scratch(const ApplyArgs &a, void *scratch, hipStream_t s) {
  ApplyLaunch L;
  L.a = a;
  float *src_off = reinterpret_cast<float *>(scratch);
  const int split = a.ns < 256 ? a.ns : 256;
  L.split_len = split;
  L.nsplit = (a.ns + split - 1) / split;
  L.part = src_off + ((a.ns + 63) / 64) * 64;
  L.src_off = src_off;
  hipLaunchKernelGGL(k_src_offsets, dim3((a.ns + 255) / 256), dim3(256), 0, s, a.h_s, a.w_s, a.ns,
                     a.sc, src_off);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (a.V == nullptr) return hipErrorInvalidValue;
  const int ncols = a.k;
  for (int c0 = 0; c0 < ncols; c0 += kKV) {
    L.c0 = c0;
    L.kv = (ncols - c0) < kKV ? (ncols - c0) : kKV;
    e = apply_dispatch(L, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_sum(const float *w, int n, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(1024), 0, s, w, n, out);
  return hipGetLastError();
}

}  // namespace uot
