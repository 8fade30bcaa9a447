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

#include "uot_epilogue.cuh"
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


// ---------------------------------------------------------------------------------------
// Squared-Euclidean costs on the matrix cores. The base-2 exponent of entry (s, t), shifted
// by the running reference sigma_t of its target, is an augmented dot product plus a
// per-column constant,
//   v_ts - sigma_t = sum_{e < K} A_se B_et - sigma_t,
//   A_s = (u_s[0..D-1], b_s, 0...),   B_t = (y_t - mu, 1, 0...),
// a K = D+1 (rounded to even) contraction done by v_mfma_f32_32x32x2f32 with sources as the
// 32 rows and targets as the 32 columns of each output tile; -sigma_t enters as the
// accumulator input of the first k-slice (a register tile holding -sigma of each lane's
// column), so it costs no contraction depth. The VALU then does one exp2 and one add per
// entry. A_s comes from the source record; B_t is built in registers. Element e of k-slice ks
// for lane half h is e = KS*h + ks, so the KS elements a lane needs from one record are
// contiguous.
//
// Each lane owns one target column (lane % 32) and 16 source rows of every tile. sigma_t is
// shared by the two lanes of a column and is raised only when a tile's sum of 2^{v - sigma}
// exceeds 2^64 in either lane (or at the column's first tile); otherwise the exponents are
// used as they come out of the matrix core. The next tile's MFMAs are issued before the
// current tile's exps (software pipelining); an accumulator computed with an older sigma is
// corrected on the slow path.
// ---------------------------------------------------------------------------------------
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kMfmaWaves = 4;  // waves per block

template <int D>
struct MfmaShape {
  static constexpr int K = ((D + 1) + 1) / 2 * 2;  // augmented depth, even
  static constexpr int KS = K / 2;                  // k-slices of the 32x32x2 instruction
  static constexpr int SD = rec_stride(kSqEuc, D);
  static constexpr int EB = D;                      // element holding b_s (A) / 1 (B)
  static_assert(K <= SD, "record shorter than the contraction");
};

template <int D, int TJ, bool FUSE>
__global__ __launch_bounds__(256) void k_points_mfma(PointsArgs a, FusedTail fz) {
  if (a.done != nullptr && *a.done) return;
  using S = MfmaShape<D>;
  constexpr int KS = S::KS, SD = S::SD;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int col = lane & 31;
  const int h = lane >> 5;
  const int tbase = (blockIdx.x * kMfmaWaves + wave) * (32 * TJ);

  // B fragments: element e = KS*h + ks of (y - mu, 1, 0...)
  float bf[TJ][KS];
#pragma unroll
  for (int tj = 0; tj < TJ; ++tj) {
    const int t = tbase + tj * 32 + col;
    const bool valid = t < a.nt;
    const int tc = valid ? t : 0;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int e = KS * h + ks;
      const int ec = e < a.d ? e : 0;
      const float coord = a.tgt[(size_t)tc * a.d + ec] - (float)a.mu[ec];
      bf[tj][ks] = (e < D) ? ((valid && e < a.d) ? coord : 0.0f) : (e == S::EB ? 1.0f : 0.0f);
    }
  }

  const int s0 = blockIdx.y * a.split_len;
  const int s1 = min(a.ns, s0 + a.split_len);

  // A fragments of the tile starting at sb: record elements [KS*h, KS*h + KS) (in bounds since
  // K <= SD). Tiles end at s1 or at the padded end of the record array, whose pad records
  // carry b = -inf (weight 0), so no source needs a mask.
  auto load_a = [&](int sb, float *af) {
    const float *rp = a.rec + (size_t)(sb + col) * SD + KS * h;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) af[ks] = rp[ks];
  };
  float sig[TJ], l[TJ];  // running reference and sum of 2^{v - sig} (this lane's rows)
  bool started[TJ];
#pragma unroll
  for (int tj = 0; tj < TJ; ++tj) { sig[tj] = 0.0f; l[tj] = 0.0f; started[tj] = false; }

  // Re-centres column tile tj on its largest exponent and adds it (all lanes; exact for any
  // column). acc was computed with the current sig.
  auto recentre = [&](const f32x16 &acc, int tj) {
    float tm = acc[0];
#pragma unroll
    for (int r = 1; r < 16; ++r) tm = fmaxf(tm, acc[r]);
    tm = fmaxf(tm, __shfl_xor(tm, 32, 64));
    if (tm > -INFINITY) {
      const float delta = started[tj] ? fmaxf(tm, 0.0f) : tm;
      float t2 = 0.0f;
#pragma unroll
      for (int r = 0; r < 16; ++r) t2 += fast_exp2(acc[r] - delta);
      // first tile: no rescale (delta may be far below -126 and 0 * 2^{-delta} is NaN)
      l[tj] = started[tj] ? l[tj] * fast_exp2(-delta) + t2 : t2;
      sig[tj] += delta;
      started[tj] = true;
    }
  };

  // Tiles of 32 sources; the next tile's records are prefetched while this tile's exps run,
  // and the waves resident on the SIMD cover each other's matrix-core latency. The inner
  // loop is the fast path, where -sig (the accumulator input) is loop-invariant; a tile that
  // would overflow the sums, or a column not yet started, leaves it for recentre().
  float an[KS], ac[KS];
  load_a(s0, an);
  int sb = s0;
  while (sb < s1) {
    f32x16 nsig[TJ];
#pragma unroll
    for (int tj = 0; tj < TJ; ++tj)
#pragma unroll
      for (int r = 0; r < 16; ++r) nsig[tj][r] = -sig[tj];
    bool all_started = true;
#pragma unroll
    for (int tj = 0; tj < TJ; ++tj) all_started = all_started && __all(started[tj]);
    f32x16 acc[TJ];
    bool slow = false;
    for (; sb < s1; sb += 32) {
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) ac[ks] = an[ks];
      if (sb + 32 < s1) load_a(sb + 32, an);
#pragma unroll
      for (int tj = 0; tj < TJ; ++tj) {
        acc[tj] = __builtin_amdgcn_mfma_f32_32x32x2f32(ac[0], bf[tj][0], nsig[tj], 0, 0, 0);
#pragma unroll
        for (int ks = 1; ks < KS; ++ks)
          acc[tj] = __builtin_amdgcn_mfma_f32_32x32x2f32(ac[ks], bf[tj][ks], acc[tj], 0, 0, 0);
      }
      if (!all_started) { slow = true; break; }
      float ts[TJ];
      bool ok = true;
#pragma unroll
      for (int tj = 0; tj < TJ; ++tj) {
        float q0 = fast_exp2(acc[tj][0]), q1 = fast_exp2(acc[tj][1]);
        float q2 = fast_exp2(acc[tj][2]), q3 = fast_exp2(acc[tj][3]);
#pragma unroll
        for (int r = 4; r < 16; r += 4) {
          q0 += fast_exp2(acc[tj][r]);
          q1 += fast_exp2(acc[tj][r + 1]);
          q2 += fast_exp2(acc[tj][r + 2]);
          q3 += fast_exp2(acc[tj][r + 3]);
        }
        ts[tj] = (q0 + q1) + (q2 + q3);
        ok = ok && !__any(!(ts[tj] <= 0x1p64f));
      }
      if (!ok) { slow = true; break; }
#pragma unroll
      for (int tj = 0; tj < TJ; ++tj) l[tj] += ts[tj];
    }
    if (!slow) break;
#pragma unroll
    for (int tj = 0; tj < TJ; ++tj) recentre(acc[tj], tj);
    sb += 32;
  }

  // merge the two half-waves of each column (same sigma; sums add)
#pragma unroll
  for (int tj = 0; tj < TJ; ++tj) {
    const float lo = __shfl_xor(l[tj], 32, 64);
    const float ll = l[tj] + lo;
    const int t = tbase + tj * 32 + col;
    if (h == 0 && t < a.nt)
      a.part[(size_t)blockIdx.y * a.nt + t] = make_float2(ll > 0.0f ? sig[tj] : -FLT_MAX, ll);
  }

  if constexpr (FUSE) {
    // The last of the gridDim.y split blocks of this tile to arrive merges the tile; no block
    // waits for another.
    // Every wave waits for its own partial stores to complete before the barrier (the
    // barrier alone does not wait for them), so thread 0's release (L2 write-back) covers
    // the whole block. Only the last block acquires (L2 invalidate): an invalidate in every
    // block would evict the source records that the blocks still running stream.
    __shared__ int s_last;
    __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
    __syncthreads();
    if (threadIdx.x == 0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      const unsigned prev = atomicAdd(&fz.tile_ticket[blockIdx.x], 1u);
      s_last = (prev == gridDim.y - 1u) ? 1 : 0;
    }
    __syncthreads();
    if (!s_last) return;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (threadIdx.x == 0) fz.tile_ticket[blockIdx.x] = 0u;
    constexpr int kTileTargets = kMfmaWaves * 32 * TJ;
    combine_and_reduce<D, kSqEuc, 256 / kTileTargets>(fz.c, blockIdx.x * kTileTargets,
                                                      blockIdx.x, gridDim.x);
  }
}


template <int D, int TJ>
hipError_t launch_mfma_tj(const PointsArgs &a, const FusedTail *fz, hipStream_t st) {
  const int tpb = kMfmaWaves * 32 * TJ;
  dim3 grid((a.nt + tpb - 1) / tpb, a.nsplit);
  if (fz != nullptr)
    hipLaunchKernelGGL((k_points_mfma<D, TJ, true>), grid, dim3(64 * kMfmaWaves), 0, st, a, *fz);
  else
    hipLaunchKernelGGL((k_points_mfma<D, TJ, false>), grid, dim3(64 * kMfmaWaves), 0, st, a,
                       FusedTail{});
  return hipGetLastError();
}

template <int D>
hipError_t launch_mfma_bucket(const PointsArgs &a, const FusedTail *fz, hipStream_t st) {
  return mfma_tiles_per_wave() == 2 ? launch_mfma_tj<D, 2>(a, fz, st)
                                    : launch_mfma_tj<D, 1>(a, fz, st);
}

hipError_t launch_mfma(const PointsArgs &a, const FusedTail *fz, hipStream_t st) {
  switch (dim_bucket(a.d)) {
    case 1: return launch_mfma_bucket<1>(a, fz, st);
    case 2: return launch_mfma_bucket<2>(a, fz, st);
    case 3: return launch_mfma_bucket<3>(a, fz, st);
    case 4: return launch_mfma_bucket<4>(a, fz, st);
    case 5: return launch_mfma_bucket<5>(a, fz, st);
    case 6: return launch_mfma_bucket<6>(a, fz, st);
    case 7: return launch_mfma_bucket<7>(a, fz, st);
    case 8: return launch_mfma_bucket<8>(a, fz, st);
    case 12: return launch_mfma_bucket<12>(a, fz, st);
    case 16: return launch_mfma_bucket<16>(a, fz, st);
    case 24: return launch_mfma_bucket<24>(a, fz, st);
    case 32: return launch_mfma_bucket<32>(a, fz, st);
    case 48: return launch_mfma_bucket<48>(a, fz, st);
    case 64: return launch_mfma_bucket<64>(a, fz, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename Kern>
int occupancy_blocks(Kern kern) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, 256, 0) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return nb;
}

template <int D>
int points_blocks_per_cu_bucket(int mode) {
  if (mode == kSqEuc && g_points_variant != kPointsValu)
    return mfma_tiles_per_wave() == 2 ? occupancy_blocks(k_points_mfma<D, 2, true>)
                                      : occupancy_blocks(k_points_mfma<D, 1, true>);
  constexpr int R = targets_per_thread<D>();
  return mode == kSqEuc ? occupancy_blocks(k_points_partial<D, kSqEuc, R>)
                        : occupancy_blocks(k_points_partial<D, kPower, R>);
}

}  // namespace

int g_points_variant = kPointsAuto;

int points_blocks_per_cu(int mode, int d) {
  switch (dim_bucket(d)) {
    case 1: return points_blocks_per_cu_bucket<1>(mode);
    case 2: return points_blocks_per_cu_bucket<2>(mode);
    case 3: return points_blocks_per_cu_bucket<3>(mode);
    case 4: return points_blocks_per_cu_bucket<4>(mode);
    case 5: return points_blocks_per_cu_bucket<5>(mode);
    case 6: return points_blocks_per_cu_bucket<6>(mode);
    case 7: return points_blocks_per_cu_bucket<7>(mode);
    case 8: return points_blocks_per_cu_bucket<8>(mode);
    case 12: return points_blocks_per_cu_bucket<12>(mode);
    case 16: return points_blocks_per_cu_bucket<16>(mode);
    case 24: return points_blocks_per_cu_bucket<24>(mode);
    case 32: return points_blocks_per_cu_bucket<32>(mode);
    case 48: return points_blocks_per_cu_bucket<48>(mode);
    case 64: return points_blocks_per_cu_bucket<64>(mode);
    default: return 0;
  }
}

// 32-target column tiles per wave of the matrix-core kernel.
int mfma_tiles_per_wave() { return g_points_variant == kPointsMfma2 ? 2 : 1; }

bool points_uses_mfma(int mode, int d) {
  (void)d;
  if (mode != kSqEuc) return false;
  return g_points_variant != kPointsValu;
}

int points_targets_per_block(int mode, int d) {
  if (points_uses_mfma(mode, d)) return kMfmaWaves * 32 * mfma_tiles_per_wave();
  const int b = dim_bucket(d);
  return 256 * (b <= 4 ? 4 : (b <= 8 ? 2 : 1));
}

int points_fused_tiles(int nt) {
  const int tpb = kMfmaWaves * 32 * mfma_tiles_per_wave();
  return (nt + tpb - 1) / tpb;
}

hipError_t launch_points_fused(const PointsArgs &a, const FusedTail &f, hipStream_t st) {
  if (!points_uses_mfma(kSqEuc, a.d)) return hipErrorInvalidValue;
  return launch_mfma(a, &f, st);
}

int points_split_align(int mode, int d) { return points_uses_mfma(mode, d) ? 32 : 8; }

hipError_t launch_points_partial(int mode, const PointsArgs &a, hipStream_t st) {
  if (points_uses_mfma(mode, a.d)) return launch_mfma(a, nullptr, st);
  if (mode == kSqEuc) return launch_mode<kSqEuc>(a, st);
  if (mode == kPower) return launch_mode<kPower>(a, st);
  return hipErrorInvalidValue;
}

}  // namespace uot
