// Issue-rate probes (gfx950): the chip-wide throughput of the vector instructions that the
// softmin, backward and batched kernels are built from, measured on the device that runs
// them, so the rooflines reported beside those kernels rest on this chip's rates and not on
// spec-sheet arithmetic alone.
//
// Each lane runs kChains independent dependency chains of one instruction kind for kSteps
// steps (the chains hide the instruction latency; 8 waves per SIMD are resident), and the
// launch is timed with HIP events around it after one untimed launch. The rate is
// lanes x chains x steps / time, in lane-operations per second, for the vector kinds, and
// waves x chains x steps x (2 M N K) / time, in flop/s, for the matrix-core kinds (each wave
// issues independent accumulations of one MFMA shape).
#include "uot.h"
#include "uot_internal.h"

namespace uot {
namespace {

constexpr int kChains = 8;
constexpr int kSteps = 2048;
constexpr int kProbeBlocks = 2048;  // 256 CUs x 8 waves per SIMD at 4 waves per block

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// Flops of one matrix-core instruction of a probe kind (0 for the vector kinds).
constexpr double mfma_flops(int kind) {
  return kind == UOT_PROBE_MFMA_F64 ? 2.0 * 16 * 16 * 4
         : kind == UOT_PROBE_MFMA_F32 ? 2.0 * 16 * 16 * 4
         : kind == UOT_PROBE_MFMA_BF16 ? 2.0 * 32 * 32 * 16 : 0.0;
}

template <int KIND>
__global__ __launch_bounds__(256) void k_probe(float *out, float seed) {
  const int tid = blockIdx.x * 256 + threadIdx.x;
  if constexpr (KIND == UOT_PROBE_MFMA_F64) {
    const double x = (double)seed + 1e-3 * (tid & 63), y = 1.0 - 1e-3 * (tid & 7);
    f64x4 acc[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc[c] = f64x4{0.0, 0.0, 0.0, 0.0};
    for (int i = 0; i < kSteps; ++i) {
#pragma unroll
      for (int c = 0; c < kChains; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, acc[c], 0, 0, 0);
    }
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
    out[tid] = (float)s;
  } else if constexpr (KIND == UOT_PROBE_MFMA_F32) {
    const float x = seed + 1e-3f * (float)(tid & 63), y = 1.0f - 1e-3f * (float)(tid & 7);
    f32x4 acc[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc[c] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    for (int i = 0; i < kSteps; ++i) {
#pragma unroll
      for (int c = 0; c < kChains; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(x, y, acc[c], 0, 0, 0);
    }
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
    out[tid] = s;
  } else if constexpr (KIND == UOT_PROBE_MFMA_BF16) {
    constexpr int C = kChains / 2;  // 16 accumulator registers per chain
    bf16x8 x, y;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      x[k] = (__bf16)(seed + 1e-2f * (float)((tid + k) & 7));
      y[k] = (__bf16)(1.0f - 1e-2f * (float)((tid + 3 * k) & 7));
    }
    f32x16 acc[C];
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[c][r] = 0.0f;
    for (int i = 0; i < kSteps; ++i) {
#pragma unroll
      for (int c = 0; c < C; ++c) acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x, y, acc[c], 0, 0, 0);
    }
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
      for (int r = 0; r < 16; ++r) s += acc[c][r];
    out[tid] = s;
  } else if constexpr (KIND == UOT_PROBE_FMA64) {
    double v[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) v[c] = (double)seed + 0.01 * (c + (tid & 7));
    const double a = 0.999, b = 0.001;
    for (int i = 0; i < kSteps; ++i) {
#pragma unroll
      for (int c = 0; c < kChains; ++c) v[c] = fma(v[c], a, b);
    }
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += v[c];
    out[tid] = (float)s;
  } else {
    float v[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) v[c] = seed + 0.01f * (float)(c + (tid & 7));
    const float a = 0.999f, b = 0.001f;
    for (int i = 0; i < kSteps; ++i) {
#pragma unroll
      for (int c = 0; c < kChains; ++c) {
        if constexpr (KIND == UOT_PROBE_EXP2)
          v[c] = __builtin_amdgcn_exp2f(-v[c]);  // stays in (0.5, 1]
        else
          v[c] = fmaf(v[c], a, b);
      }
    }
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += v[c];
    out[tid] = s;
  }
}

template <int KIND>
hipError_t probe_launch(float *out, hipStream_t s) {
  hipLaunchKernelGGL((k_probe<KIND>), dim3(kProbeBlocks), dim3(256), 0, s, out, 0.5f);
  return hipGetLastError();
}

hipError_t probe_dispatch(int kind, float *out, hipStream_t s) {
  switch (kind) {
    case UOT_PROBE_EXP2: return probe_launch<UOT_PROBE_EXP2>(out, s);
    case UOT_PROBE_FMA32: return probe_launch<UOT_PROBE_FMA32>(out, s);
    case UOT_PROBE_FMA64: return probe_launch<UOT_PROBE_FMA64>(out, s);
    case UOT_PROBE_MFMA_F64: return probe_launch<UOT_PROBE_MFMA_F64>(out, s);
    case UOT_PROBE_MFMA_F32: return probe_launch<UOT_PROBE_MFMA_F32>(out, s);
    case UOT_PROBE_MFMA_BF16: return probe_launch<UOT_PROBE_MFMA_BF16>(out, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace
}  // namespace uot

extern "C" uot_status uot_probe_rate(int32_t kind, double *ops_per_s, void *stream) {
  using namespace uot;
  if (kind < UOT_PROBE_EXP2 || kind > UOT_PROBE_MFMA_BF16 || ops_per_s == nullptr)
    return UOT_ERR_INVALID;
  hipStream_t s = static_cast<hipStream_t>(stream);
  float *out = nullptr;
  if (hipMalloc(&out, (size_t)kProbeBlocks * 256 * sizeof(float)) != hipSuccess) return UOT_ERR_HIP;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  uot_status st = UOT_ERR_HIP;
  if (hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess &&
      probe_dispatch(kind, out, s) == hipSuccess && hipEventRecord(e0, s) == hipSuccess &&
      probe_dispatch(kind, out, s) == hipSuccess && hipEventRecord(e1, s) == hipSuccess &&
      hipEventSynchronize(e1) == hipSuccess) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, e0, e1) == hipSuccess && ms > 0.0f) {
      const double f = mfma_flops(kind);
      const double chains = kind == UOT_PROBE_MFMA_BF16 ? kChains / 2 : kChains;
      *ops_per_s = f > 0.0 ? (double)kProbeBlocks * 4.0 * chains * kSteps * f / (ms * 1e-3)
                           : (double)kProbeBlocks * 256.0 * kChains * kSteps / (ms * 1e-3);
      st = UOT_OK;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(out);
  return st;
}
