// Stored-cost softmins (gfx950). Both directions stream C once per half-step, so the
// half-steps are bound by HBM bandwidth (4 bytes of C per entry); the arithmetic is one
// FMA, a max and one exp2 per entry. Exponents are in base 2 with sc = log2(e)/eps:
//   v_ts = a_s - sc C_ts,   a_s = sc h_s + log2 w_s  (the source record).
//
// Column direction (g-step, targets = columns j of row-major C): a thread owns 4 adjacent
// columns and walks down the rows of one split with float4 loads, so a wave reads 1 KiB of
// contiguous C per row; the row offsets a_i are uniform and come through scalar loads.
// Row direction (f-step, targets = rows): a wave owns kRowsPerWave rows and sweeps them
// together with float4 loads (lanes interleaved along the row), sharing each loaded chunk of
// the column offsets between them; the (max, sum) pairs are merged across lanes with
// shuffles. One row per wave: 16384^2 rows softmin 6.3 TB/s against 5.0 TB/s with four
// (more waves in flight; the offsets re-read per row stay in L2).
#include <cfloat>

#include "uot_epilogue.cuh"
#include "uot_internal.h"

namespace uot {
namespace {

constexpr int kRowTile = 8;
constexpr int kColsPerThread = 4;
constexpr int kRowsPerWave = 1;

__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }

typedef float f32x4 __attribute__((ext_vector_type(4)));

// Streaming (non-temporal) 16-byte load: C is read once per half-step.
__device__ __forceinline__ float4 load4_stream(const float *p) {
  const f32x4 v = __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(p));
  return make_float4(v.x, v.y, v.z, v.w);
}

// VEC4: C and ldc allow aligned float4 loads.
template <bool VEC4>
__global__ __launch_bounds__(256) void k_dense_cols_partial(DenseArgs a) {
  if (a.done != nullptr && get_done(a.done)) return;
  const int j0 = (blockIdx.x * 256 + threadIdx.x) * kColsPerThread;
  if (j0 >= a.m) return;
  const bool full = VEC4 && (j0 + kColsPerThread <= a.m);
  const int i0 = blockIdx.y * a.split_len;
  const int i1 = min(a.n, i0 + a.split_len);
  const float sc = a.sc;
  float m[kColsPerThread], l[kColsPerThread];
#pragma unroll
  for (int c = 0; c < kColsPerThread; ++c) { m[c] = -FLT_MAX; l[c] = 0.0f; }

  auto load_row = [&](int i, float *cv) {
    const float *row = a.C + (size_t)i * a.ldc + j0;
    if (full) {
      const float4 q = load4_stream(row);
      cv[0] = q.x; cv[1] = q.y; cv[2] = q.z; cv[3] = q.w;
    } else {
#pragma unroll
      for (int c = 0; c < kColsPerThread; ++c) cv[c] = (j0 + c < a.m) ? row[c] : 0.0f;
    }
  };

  int i = i0;
  for (; i + kRowTile <= i1; i += kRowTile) {
    float v[kRowTile][kColsPerThread];
#pragma unroll
    for (int k = 0; k < kRowTile; ++k) {
      float cv[kColsPerThread];
      load_row(i + k, cv);
      const float ai = a.rec[i + k];
#pragma unroll
      for (int c = 0; c < kColsPerThread; ++c) v[k][c] = fmaf(-sc, cv[c], ai);
    }
#pragma unroll
    for (int c = 0; c < kColsPerThread; ++c) {
      float mt = v[0][c];
#pragma unroll
      for (int k = 1; k < kRowTile; ++k) mt = fmaxf(mt, v[k][c]);
      const float mn = fmaxf(m[c], mt);
      float acc = l[c] * fast_exp2(m[c] - mn);
#pragma unroll
      for (int k = 0; k < kRowTile; ++k) acc += fast_exp2(v[k][c] - mn);
      l[c] = acc;
      m[c] = mn;
    }
  }
  for (; i < i1; ++i) {
    float cv[kColsPerThread];
    load_row(i, cv);
    const float ai = a.rec[i];
#pragma unroll
    for (int c = 0; c < kColsPerThread; ++c) {
      const float v = fmaf(-sc, cv[c], ai);
      const float mn = fmaxf(m[c], v);
      l[c] = l[c] * fast_exp2(m[c] - mn) + fast_exp2(v - mn);
      m[c] = mn;
    }
  }
  float2 *out = a.part + (size_t)blockIdx.y * a.m + j0;
#pragma unroll
  for (int c = 0; c < kColsPerThread; ++c)
    if (j0 + c < a.m) out[c] = make_float2(m[c], l[c]);
}

template <bool VEC4>
__global__ __launch_bounds__(256) void k_dense_rows(DenseArgs a) {
  if (a.done != nullptr && get_done(a.done)) return;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int row0 = (blockIdx.x * 4 + wave) * kRowsPerWave;
  if (row0 >= a.n) return;  // whole wave exits together
  const float sc = a.sc;
  float m[kRowsPerWave], l[kRowsPerWave];
#pragma unroll
  for (int r = 0; r < kRowsPerWave; ++r) { m[r] = -FLT_MAX; l[r] = 0.0f; }

  for (int c0 = lane * 4; c0 < a.m; c0 += 256) {
    const bool full = VEC4 && (c0 + 4 <= a.m);
    float bv[4];
    if (full) {
      const float4 q = *reinterpret_cast<const float4 *>(a.rec + c0);
      bv[0] = q.x; bv[1] = q.y; bv[2] = q.z; bv[3] = q.w;
    } else {
#pragma unroll
      for (int c = 0; c < 4; ++c) bv[c] = (c0 + c < a.m) ? a.rec[c0 + c] : -INFINITY;
    }
#pragma unroll
    for (int r = 0; r < kRowsPerWave; ++r) {
      const int row = row0 + r;
      if (row >= a.n) break;  // uniform across the wave
      const float *rp = a.C + (size_t)row * a.ldc + c0;
      float cv[4];
      if (full) {
        const float4 q = load4_stream(rp);
        cv[0] = q.x; cv[1] = q.y; cv[2] = q.z; cv[3] = q.w;
      } else {
#pragma unroll
        for (int c = 0; c < 4; ++c) cv[c] = (c0 + c < a.m) ? rp[c] : 0.0f;
      }
      float v[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) v[c] = fmaf(-sc, cv[c], bv[c]);
      const float mt = fmaxf(fmaxf(v[0], v[1]), fmaxf(v[2], v[3]));
      const float mn = fmaxf(m[r], mt);
      float acc = l[r] * fast_exp2(m[r] - mn);
#pragma unroll
      for (int c = 0; c < 4; ++c) acc += fast_exp2(v[c] - mn);
      l[r] = acc;
      m[r] = mn;
    }
  }
  // merge the per-lane (max, sum) pairs of each row across the wave
#pragma unroll
  for (int r = 0; r < kRowsPerWave; ++r) {
    float mm = m[r], ll = l[r];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      const float mo = __shfl_xor(mm, off, 64);
      const float lo = __shfl_xor(ll, off, 64);
      const float mn = fmaxf(mm, mo);
      ll = ll * fast_exp2(mm - mn) + lo * fast_exp2(mo - mn);
      mm = mn;
    }
    const int row = row0 + r;
    if (lane == 0 && row < a.n) a.part[row] = make_float2(mm, ll);
  }
}

}  // namespace

int dense_cols_per_block() { return 256 * kColsPerThread; }
int dense_rows_per_block() { return 4 * kRowsPerWave; }

hipError_t launch_dense_cols_partial(const DenseArgs &a, hipStream_t st, const LaunchTiming *t) {
  const bool vec = (reinterpret_cast<uintptr_t>(a.C) % 16 == 0) && (a.ldc % 4 == 0);
  dim3 grid((a.m + dense_cols_per_block() - 1) / dense_cols_per_block(), a.nsplit);
  return vec ? launch_timed(k_dense_cols_partial<true>, grid, dim3(256), st, t, a)
             : launch_timed(k_dense_cols_partial<false>, grid, dim3(256), st, t, a);
}

hipError_t launch_dense_rows(const DenseArgs &a, hipStream_t st, const LaunchTiming *t) {
  const bool vec = (reinterpret_cast<uintptr_t>(a.C) % 16 == 0) && (a.ldc % 4 == 0) &&
                   (reinterpret_cast<uintptr_t>(a.rec) % 16 == 0);
  dim3 grid((a.n + dense_rows_per_block() - 1) / dense_rows_per_block());
  return vec ? launch_timed(k_dense_rows<true>, grid, dim3(256), st, t, a)
             : launch_timed(k_dense_rows<false>, grid, dim3(256), st, t, a);
}

}  // namespace uot
