// Matrix-core column softmin of the squared-Euclidean cost (gfx950), used by the points
// softmin kernel.
//
// The base-2 exponent of entry (s, t), shifted
// by the running reference sigma_t of its target, is a contraction plus a per-column
// constant,
//   v_ts - sigma_t = sum_{e < K} A_se B_et - sigma_t,
// with sources as the 32 rows and targets as the 32 columns of each output tile. The VALU
// then does one exp2 and one add per entry. A_s comes from the source record, B_t is built in
// registers. Two forms:
//
//  - float32 (F32Form): A_s = (u_s, b_s, 0...), B_t = (y_t - mu, 1, 0...), K = D+1 rounded to
//    even, v_mfma_f32_32x32x2f32; -sigma_t enters as the accumulator input of the first
//    instruction (a register tile holding -sigma of each lane's column), so it costs no
//    contraction depth. Element e of k-slice j for lane half h is e = NJ*h + j.
//  - bf16-split (Bf16Form): the slots of mx_slots() (three bf16 pieces per float32 value, six
//    piece products per coordinate; -sigma_t in two slots of the contraction, so the
//    accumulator input is zero), v_mfma_f32_32x32x16_bf16, K = 16 per instruction. Lane
//    half h of instruction j holds slots 16j + 8h .. 16j + 8h + 7. The bf16 matrix cores run
//    beside the exp/add stream of the other waves, where the float32 ones take VALU cycles;
//    the split keeps the float32 accuracy of the exponent.
//
// Each lane owns one target column (lane % 32) and 16 source rows of every tile. sigma_t is
// shared by the two lanes of a column and is raised only when a tile's sum of 2^{v - sigma}
// exceeds 2^64 in either lane (or at the column's first tile); otherwise the exponents are
// used as they come out of the matrix core.
#pragma once

#include <cfloat>

#include "uot_internal.h"

namespace uot {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ float mx_exp2(float x) { return __builtin_amdgcn_exp2f(x); }

template <int D>
struct F32Form {
  static constexpr int K = ((D + 1) + 1) / 2 * 2;  // augmented depth, even
  static constexpr int NJ = K / 2;                  // instructions per tile
  static constexpr int RS = rec_stride(kSqEuc, D);  // record stride (floats)
  static constexpr bool kSigmaInB = false;          // -sigma enters as accumulator input
  static_assert(K <= RS, "record shorter than the contraction");
  typedef float Frag;

  static __device__ __forceinline__ float elem(const float (&yc)[D], int e) {
    return e < D ? yc[e] : (e == D ? 1.0f : 0.0f);
  }
  static __device__ __forceinline__ void build_b(const float (&yc)[D], int h, Frag (&b)[NJ]) {
#pragma unroll
    for (int j = 0; j < NJ; ++j) b[j] = h ? elem(yc, NJ + j) : elem(yc, j);
  }
  static __device__ __forceinline__ float representable(float sig) { return sig; }
  static __device__ __forceinline__ void set_sigma(Frag (&)[NJ], float, int) {}
  // record elements [NJ*h, NJ*h + NJ) of source row `col` of the tile at `tile`
  static __device__ __forceinline__ void load_a(const float *tile, int col, int h, Frag (&af)[NJ]) {
    const float *rp = tile + col * RS + NJ * h;
#pragma unroll
    for (int j = 0; j < NJ; ++j) af[j] = rp[j];
  }
  static __device__ __forceinline__ f32x16 mma(const Frag (&af)[NJ], const Frag (&b)[NJ],
                                               const f32x16 &c) {
    f32x16 acc = __builtin_amdgcn_mfma_f32_32x32x2f32(af[0], b[0], c, 0, 0, 0);
#pragma unroll
    for (int j = 1; j < NJ; ++j) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(af[j], b[j], acc, 0, 0, 0);
    return acc;
  }
};

template <int D>
struct Bf16Form {
  static constexpr int KP = mx_slots(D);
  static constexpr int NJ = KP / 16;                  // instructions per tile
  static constexpr int RS = rec_stride(kSqEucMx, D);  // record stride (floats)
  static constexpr bool kSigmaInB = true;             // -sigma in slots ES0, ES1
  static constexpr int ES0 = 6 * D + 3, ES1 = 6 * D + 4;
  typedef bf16x8 Frag;

  static __device__ __forceinline__ __bf16 elem(const __bf16 (&yp)[D][3], int e) {
    return e < 6 * D ? yp[e / 6][mx_piece_y(e % 6)] : (e < 6 * D + 3 ? (__bf16)1.0f : (__bf16)0.0f);
  }
  static __device__ __forceinline__ void build_b(const float (&yc)[D], int h, Frag (&b)[NJ]) {
    __bf16 yp[D][3];
#pragma unroll
    for (int k = 0; k < D; ++k) split3(yc[k], yp[k][0], yp[k][1], yp[k][2]);
#pragma unroll
    for (int j = 0; j < NJ; ++j)
#pragma unroll
      for (int i = 0; i < 8; ++i) b[j][i] = h ? elem(yp, 16 * j + 8 + i) : elem(yp, 16 * j + i);
  }
  // Nearest value at or below sig's two-piece rounding that the slots carry exactly:
  // -(s0 + s1) with s0 = bf16(-sig), s1 = bf16(-sig - s0) (the sum is exact in float32).
  static __device__ __forceinline__ float representable(float sig) {
    const __bf16 s0 = (__bf16)(-sig);
    const __bf16 s1 = (__bf16)(-sig - (float)s0);
    return -((float)s0 + (float)s1);
  }
  // Writes the pieces of -sig (sig representable) into the slots this lane half holds.
  static __device__ __forceinline__ void set_sigma(Frag (&b)[NJ], float sig, int h) {
    const __bf16 s0 = (__bf16)(-sig);
    const __bf16 s1 = (__bf16)(-sig - (float)s0);
#pragma unroll
    for (int j = 0; j < NJ; ++j)
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int e0 = 16 * j + i, e1 = e0 + 8;
        if (e0 == ES0 || e0 == ES1 || e1 == ES0 || e1 == ES1) {
          const int e = h ? e1 : e0;
          b[j][i] = e == ES0 ? s0 : (e == ES1 ? s1 : b[j][i]);
        }
      }
  }
  // slots [16j + 8h, 16j + 8h + 8) of source row `col` for every instruction j
  static __device__ __forceinline__ void load_a(const float *tile, int col, int h, Frag (&af)[NJ]) {
    const Frag *rp = reinterpret_cast<const Frag *>(tile + col * RS) + h;
#pragma unroll
    for (int j = 0; j < NJ; ++j) af[j] = rp[2 * j];
  }
  static __device__ __forceinline__ f32x16 mma(const Frag (&af)[NJ], const Frag (&b)[NJ],
                                               const f32x16 &c) {
    f32x16 acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[0], b[0], c, 0, 0, 0);
#pragma unroll
    for (int j = 1; j < NJ; ++j) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[j], b[j], acc, 0, 0, 0);
    return acc;
  }
};

// One wave's column softmin over the source records of `rec` in tiles of 32 from s0 while
// the tile start is below s1 (records past the real sources are weight-0 pads, b = -inf,
// up to a whole tile). Lane (col, h) owns
// target column col and returns the running reference sig and this lane's sum l of
// 2^{v - sig} over its 16 rows of every tile (the two lanes of a column share sig; their
// sums add). bf is the column's B fragment set (its sigma slots are rewritten); fa holds
// the records of the tile at s0 on entry (Form::load_a), so that the caller can issue that
// load together with its own.
template <typename Form>
__device__ __forceinline__ void column_softmin(const float *rec, int s0, int s1, int col, int h,
                                               typename Form::Frag (&bf)[Form::NJ],
                                               typename Form::Frag (&fa)[Form::NJ], float &sig,
                                               float &l) {
  constexpr int NJ = Form::NJ, RS = Form::RS;
  typedef typename Form::Frag Frag;
  auto load_a = [&](int sb, Frag (&af)[NJ]) { Form::load_a(rec + (size_t)sb * RS, col, h, af); };
  sig = 0.0f;
  l = 0.0f;
  bool started = false;
  // Re-centres the tile on its column maximum and adds it (all lanes; exact for any column).
  // acc was computed with the current sig.
  auto recentre = [&](const f32x16 &acc) {
    float tm = acc[0];
#pragma unroll
    for (int r = 1; r < 16; ++r) tm = fmaxf(tm, acc[r]);
    tm = fmaxf(tm, __shfl_xor(tm, 32, 64));
    if (tm > -INFINITY) {
      const float ns = Form::representable(sig + (started ? fmaxf(tm, 0.0f) : tm));
      const float delta = ns - sig;
      float t2 = 0.0f;
#pragma unroll
      for (int r = 0; r < 16; ++r) t2 += mx_exp2(acc[r] - delta);
      // first tile: no rescale (delta may be far below -126 and 0 * 2^{-delta} is NaN)
      l = started ? l * mx_exp2(-delta) + t2 : t2;
      sig = ns;
      started = true;
      Form::set_sigma(bf, sig, h);
    }
  };

  // Adds the tile in acc to l unless it would overflow the sum (wave-uniform answer).
  auto fast_add = [&](const f32x16 &acc) {
    float q0 = mx_exp2(acc[0]), q1 = mx_exp2(acc[1]);
    float q2 = mx_exp2(acc[2]), q3 = mx_exp2(acc[3]);
#pragma unroll
    for (int r = 4; r < 16; r += 4) {
      q0 += mx_exp2(acc[r]);
      q1 += mx_exp2(acc[r + 1]);
      q2 += mx_exp2(acc[r + 2]);
      q3 += mx_exp2(acc[r + 3]);
    }
    const float ts = (q0 + q1) + (q2 + q3);
    if (__any(!(ts <= 0x1p64f))) return false;
    l += ts;
    return true;
  };

  // The next tile's records are loaded into the fragments as soon as this tile's MFMAs have
  // read them, so the load overlaps this tile's exps (one buffer, no copies), and the waves
  // resident on the SIMD (eight at this register count) cover each other's latencies.
  // The inner loop is the fast path, where the accumulator input (-sig, F32Form) and the
  // B fragments (Bf16Form) are loop-invariant; a tile that would overflow the sum, or a
  // column not yet started, leaves it for recentre(), which may move sig.
  int sb = s0;
  while (sb < s1) {
    f32x16 cin;
#pragma unroll
    for (int r = 0; r < 16; ++r) cin[r] = Form::kSigmaInB ? 0.0f : -sig;
    const bool all_started = __all(started);
    f32x16 acc;
    bool slow = false;
    for (; sb < s1; sb += 32) {
      acc = Form::mma(fa, bf, cin);
      if (sb + 32 < s1) load_a(sb + 32, fa);
      if (!all_started || !fast_add(acc)) { slow = true; break; }
    }
    if (!slow) break;
    recentre(acc);
    sb += 32;
  }
}

// column_softmin with the records prefetched two tiles ahead, in two fragment sets that take
// the tiles in turn (no copies). For the bf16-split forms of larger D (four or more
// instructions per tile, 16 bytes per instruction and lane): their register count leaves
// two or three waves per SIMD, too few to cover a one-tile-ahead load with the other waves'
// work. Same arithmetic and tile order as column_softmin; the slow path (recentre) is
// taken tile by tile.
template <typename Form>
__device__ __forceinline__ void column_softmin_ahead2(const float *rec, int s0, int s1, int col,
                                                      int h, typename Form::Frag (&bf)[Form::NJ],
                                                      typename Form::Frag (&fa)[Form::NJ],
                                                      float &sig, float &l) {
  static_assert(Form::kSigmaInB, "the accumulator input is zero: sigma rides in B");
  constexpr int NJ = Form::NJ, RS = Form::RS;
  typedef typename Form::Frag Frag;
  auto load_a = [&](int sb, Frag (&af)[NJ]) { Form::load_a(rec + (size_t)sb * RS, col, h, af); };
  Frag fb[NJ];
  if (s0 + 32 < s1) load_a(s0 + 32, fb);
  sig = 0.0f;
  l = 0.0f;
  bool started = false;
  f32x16 zero;
#pragma unroll
  for (int r = 0; r < 16; ++r) zero[r] = 0.0f;
  auto recentre = [&](const f32x16 &acc) {
    float tm = acc[0];
#pragma unroll
    for (int r = 1; r < 16; ++r) tm = fmaxf(tm, acc[r]);
    tm = fmaxf(tm, __shfl_xor(tm, 32, 64));
    if (tm > -INFINITY) {
      const float ns = Form::representable(sig + (started ? fmaxf(tm, 0.0f) : tm));
      const float delta = ns - sig;
      float t2 = 0.0f;
#pragma unroll
      for (int r = 0; r < 16; ++r) t2 += mx_exp2(acc[r] - delta);
      l = started ? l * mx_exp2(-delta) + t2 : t2;
      sig = ns;
      started = true;
      Form::set_sigma(bf, sig, h);
    }
  };
  auto fast_add = [&](const f32x16 &acc) {
    float q0 = mx_exp2(acc[0]), q1 = mx_exp2(acc[1]);
    float q2 = mx_exp2(acc[2]), q3 = mx_exp2(acc[3]);
#pragma unroll
    for (int r = 4; r < 16; r += 4) {
      q0 += mx_exp2(acc[r]);
      q1 += mx_exp2(acc[r + 1]);
      q2 += mx_exp2(acc[r + 2]);
      q3 += mx_exp2(acc[r + 3]);
    }
    const float ts = (q0 + q1) + (q2 + q3);
    if (__any(!(ts <= 0x1p64f))) return false;
    l += ts;
    return true;
  };
  // one tile from the fragment set `cur`, which then receives the tile two ahead
  auto step = [&](Frag (&cur)[NJ], int sb) {
    const f32x16 acc = Form::mma(cur, bf, zero);
    if (sb + 64 < s1) load_a(sb + 64, cur);
    if (!__all(started) || !fast_add(acc)) recentre(acc);
  };
  for (int sb = s0; sb < s1; sb += 64) {
    step(fa, sb);
    if (sb + 32 >= s1) break;
    step(fb, sb + 32);
  }
}

}  // namespace uot
