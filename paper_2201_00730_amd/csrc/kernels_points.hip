// Points-cost softmin partials (gfx950): vector-ALU kernels for any p, matrix-core kernels
// for p = 2 further below.
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
#include "uot_mx.cuh"

namespace uot {
namespace {

constexpr int kTile = 8;

__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float fast_log2(float x) { return __builtin_amdgcn_logf(x); }

template <bool P2>
__device__ __forceinline__ float cost_pow(float d2, float half_p) {
  // ||x - y||^p from the squared distance: p = 2 (compiled apart) is d2 itself, p = 1 takes
  // a square root, otherwise 2^{(p/2) log2 d2} (d2 = 0 gives log2 = -inf and the power 0).
  if constexpr (P2) {
    return d2;
  } else {
    if (half_p == 0.5f) return __builtin_sqrtf(d2);
    return fast_exp2(half_p * fast_log2(d2));
  }
}

template <int D, int MODE, int R, bool P2>
__global__ __launch_bounds__(256) void k_points_partial(PointsArgs a) {
  if (a.done != nullptr && get_done(a.done)) return;
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
      return fmaf(-sc, cost_pow<P2>(d2, half_p), rp[D]);
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
  return D <= 4 ? 4 : (D <= 16 ? 2 : 1);
}

template <int D, int MODE>
hipError_t launch_bucket(const PointsArgs &a, hipStream_t st, const LaunchTiming *t) {
  constexpr int R = targets_per_thread<D>();
  dim3 grid((a.nt + 256 * R - 1) / (256 * R), a.nsplit);
  if (MODE == kPower && a.half_p == 1.0f)
    return launch_timed(k_points_partial<D, MODE, R, true>, grid, dim3(256), st, t, a);
  return launch_timed(k_points_partial<D, MODE, R, false>, grid, dim3(256), st, t, a);
}

template <int MODE>
hipError_t launch_mode(const PointsArgs &a, hipStream_t st, const LaunchTiming *t) {
  switch (dim_bucket(a.d)) {
    case 1: return launch_bucket<1, MODE>(a, st, t);
    case 2: return launch_bucket<2, MODE>(a, st, t);
    case 3: return launch_bucket<3, MODE>(a, st, t);
    case 4: return launch_bucket<4, MODE>(a, st, t);
    case 5: return launch_bucket<5, MODE>(a, st, t);
    case 6: return launch_bucket<6, MODE>(a, st, t);
    case 7: return launch_bucket<7, MODE>(a, st, t);
    case 8: return launch_bucket<8, MODE>(a, st, t);
    case 12: return launch_bucket<12, MODE>(a, st, t);
    case 16: return launch_bucket<16, MODE>(a, st, t);
    case 24: return launch_bucket<24, MODE>(a, st, t);
    case 32: return launch_bucket<32, MODE>(a, st, t);
    case 48: return launch_bucket<48, MODE>(a, st, t);
    case 64: return launch_bucket<64, MODE>(a, st, t);
    default: return hipErrorInvalidValue;
  }
}


// ---------------------------------------------------------------------------------------
// Squared-Euclidean softmin on the matrix cores: the forms and the column loop are in
// uot_mx.cuh; this kernel gives each wave one 32-target column tile of one source split.
// ---------------------------------------------------------------------------------------
constexpr int kMfmaWaves = 4;  // waves per block
constexpr int kXcds = 8;       // accelerator complex dies of the MI355X (L2 per die)

// Centred coordinates of target t (zero beyond the true dimension and for t >= nt).
template <int D>
__device__ __forceinline__ void target_coords(const PointsArgs &a, int t, float (&yc)[D]) {
  const bool valid = t < a.nt;
  const int tc = valid ? t : 0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const int kc = k < a.d ? k : 0;
    const float v = a.tgt[(size_t)tc * a.d + kc] - (float)a.mu[kc];
    yc[k] = (valid && k < a.d) ? v : 0.0f;
  }
}

template <int D, typename Form>
__global__ __launch_bounds__(256) void k_points_mfma(PointsArgs a) {
  static_assert(kMfmaWaves * 64 == kBlock, "the side reduction runs on one whole block");
  constexpr int NJ = Form::NJ;
  typedef typename Form::Frag Frag;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int col = lane & 31;
  const int h = lane >> 5;
  // XCD-aware order: workgroups go to the 8 XCDs round-robin by id, so id b runs on XCD
  // b % 8; give XCD x the contiguous range x * per .. of the split-major (split, tile) pairs,
  // so each XCD's L2 holds the source records of about nsplit / 8 splits, not of all.
  const int ntiles = (a.nt + kMfmaWaves * 32 - 1) / (kMfmaWaves * 32);
  const int per = (int)(gridDim.x / kXcds);
  const int q = (int)(blockIdx.x % kXcds) * per + (int)(blockIdx.x / kXcds);
  const int pairs = ntiles * a.nsplit;
  if (q >= pairs) {
    // the first block past the pairs reduces the previous half-step (block-uniform branch)
    if (q == pairs && a.red_on && !get_done(&a.red.st->done)) reduce_scalars(a.red);
    return;
  }
  const int split = q / ntiles, tile = q - split * ntiles;
  const int t = (tile * kMfmaWaves + wave) * 32 + col;
  const int s0 = split * a.split_len;
  const int s1 = min(a.ns, s0 + a.split_len);

  // The first tile's records, the target coordinates and the early-exit flag are loaded
  // together, so the start costs one memory latency.
  Frag fa[NJ], bf[NJ];
  Form::load_a(a.rec + (size_t)s0 * Form::RS, col, h, fa);
  float yc[D];
  target_coords<D>(a, t, yc);
  const bool stop = a.done != nullptr && get_done(a.done);
  Form::build_b(yc, h, bf);
  if (stop) return;
  float sig, l;
  if constexpr (Form::kSigmaInB && Form::NJ >= 4)
    column_softmin_ahead2<Form>(a.rec, s0, s1, col, h, bf, fa, sig, l);
  else
    column_softmin<Form>(a.rec, s0, s1, col, h, bf, fa, sig, l);

  // merge the two half-waves of each column (same sigma; sums add)
  const float ll = l + __shfl_xor(l, 32, 64);
  if (h == 0 && t < a.nt)
    a.part[(size_t)split * a.nt + t] = make_float2(ll > 0.0f ? sig : -FLT_MAX, ll);
}

template <int D, typename Form>
hipError_t launch_mfma_form(const PointsArgs &a, hipStream_t st, const LaunchTiming *t) {
  constexpr int tpb = kMfmaWaves * 32;
  // (split, tile) pairs, one block each, plus the side-reduction block
  const int blocks = (a.nt + tpb - 1) / tpb * a.nsplit + (a.red_on ? 1 : 0);
  dim3 grid((blocks + kXcds - 1) / kXcds * kXcds);  // whole rounds over the XCDs
  return launch_timed(k_points_mfma<D, Form>, grid, dim3(64 * kMfmaWaves), st, t, a);
}

#define UOT_MFMA_BUCKETS_LO(FN, FORM, ...)         \
  switch (dim_bucket(a.d)) {                        \
    case 1: return FN<1, FORM<1>>(__VA_ARGS__);     \
    case 2: return FN<2, FORM<2>>(__VA_ARGS__);     \
    case 3: return FN<3, FORM<3>>(__VA_ARGS__);     \
    case 4: return FN<4, FORM<4>>(__VA_ARGS__);     \
    case 5: return FN<5, FORM<5>>(__VA_ARGS__);     \
    case 6: return FN<6, FORM<6>>(__VA_ARGS__);     \
    case 7: return FN<7, FORM<7>>(__VA_ARGS__);     \
    case 8: return FN<8, FORM<8>>(__VA_ARGS__);     \
    case 12: return FN<12, FORM<12>>(__VA_ARGS__);  \
    case 16: return FN<16, FORM<16>>(__VA_ARGS__);  \
    default: break;                                 \
  }
#define UOT_MFMA_BUCKETS_HI(FN, FORM, ...)         \
  switch (dim_bucket(a.d)) {                        \
    case 24: return FN<24, FORM<24>>(__VA_ARGS__);  \
    case 32: return FN<32, FORM<32>>(__VA_ARGS__);  \
    case 48: return FN<48, FORM<48>>(__VA_ARGS__);  \
    case 64: return FN<64, FORM<64>>(__VA_ARGS__);  \
    default: break;                                 \
  }

hipError_t launch_mfma_f32(const PointsArgs &a, hipStream_t st, const LaunchTiming *t) {
  UOT_MFMA_BUCKETS_LO(launch_mfma_form, F32Form, a, st, t)
  UOT_MFMA_BUCKETS_HI(launch_mfma_form, F32Form, a, st, t)
  return hipErrorInvalidValue;
}

hipError_t launch_mfma_bf16(const PointsArgs &a, hipStream_t st, const LaunchTiming *t) {
  UOT_MFMA_BUCKETS_LO(launch_mfma_form, Bf16Form, a, st, t)
  return hipErrorInvalidValue;
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

template <int D, typename Form>
int mfma_occupancy(const PointsArgs &a) {
  (void)a;
  return occupancy_blocks(k_points_mfma<D, Form>);
}

template <int D>
int valu_occupancy(int mode) {
  constexpr int R = targets_per_thread<D>();
  return mode == kSqEuc ? occupancy_blocks(k_points_partial<D, kSqEuc, R, false>)
                        : occupancy_blocks(k_points_partial<D, kPower, R, true>);
}

}  // namespace

int g_points_variant = kPointsAuto;

int points_record_mode(int mode, int d) {
  if (mode != kSqEuc) return mode;
  if (g_points_variant == kPointsDirect) return kPower;
  const bool bf16 = g_points_variant == kPointsAuto || g_points_variant == kPointsMfmaBf16;
  return (bf16 && dim_bucket(d) <= kMxMaxDim) ? kSqEucMx : kSqEuc;
}

bool points_uses_mfma(int mode, int d) {
  (void)d;
  return mode == kSqEucMx || (mode == kSqEuc && g_points_variant != kPointsValu);
}

int points_blocks_per_cu(int mode, int d) {
  PointsArgs a{};
  a.d = d;
  if (mode == kSqEucMx) {
    UOT_MFMA_BUCKETS_LO(mfma_occupancy, Bf16Form, a)
    return 0;
  }
  if (points_uses_mfma(mode, d)) {
    UOT_MFMA_BUCKETS_LO(mfma_occupancy, F32Form, a)
    UOT_MFMA_BUCKETS_HI(mfma_occupancy, F32Form, a)
    return 0;
  }
  switch (dim_bucket(d)) {
    case 1: return valu_occupancy<1>(mode);
    case 2: return valu_occupancy<2>(mode);
    case 3: return valu_occupancy<3>(mode);
    case 4: return valu_occupancy<4>(mode);
    case 5: return valu_occupancy<5>(mode);
    case 6: return valu_occupancy<6>(mode);
    case 7: return valu_occupancy<7>(mode);
    case 8: return valu_occupancy<8>(mode);
    case 12: return valu_occupancy<12>(mode);
    case 16: return valu_occupancy<16>(mode);
    case 24: return valu_occupancy<24>(mode);
    case 32: return valu_occupancy<32>(mode);
    case 48: return valu_occupancy<48>(mode);
    case 64: return valu_occupancy<64>(mode);
    default: return 0;
  }
}

int points_targets_per_block(int mode, int d) {
  if (points_uses_mfma(mode, d)) return kMfmaWaves * 32;
  const int b = dim_bucket(d);
  return 256 * (b <= 4 ? 4 : (b <= 16 ? 2 : 1));
}

int points_split_align(int mode, int d) { return points_uses_mfma(mode, d) ? 32 : 8; }

hipError_t launch_points_partial(int mode, const PointsArgs &a, hipStream_t st,
                                 const LaunchTiming *t) {
  if (mode == kSqEucMx) return launch_mfma_bf16(a, st, t);
  if (points_uses_mfma(mode, a.d)) return launch_mfma_f32(a, st, t);
  if (mode == kSqEuc) return launch_mode<kSqEuc>(a, st, t);
  if (mode == kPower) return launch_mode<kPower>(a, st, t);
  return hipErrorInvalidValue;
}

}  // namespace uot
