// Anderson extrapolation of the iterated potential (appendix on combining Sinkhorn with
// Anderson acceleration): the Gram matrix of the residuals of one cycle, the regularised
// K x K solve and the mix. Iterates are stored in float with a double translation each
// (x_k = H[k] + taus[k]); everything else is double precision.
#include <cfloat>

#include "uot_epilogue.cuh"
#include "uot_internal.h"

namespace uot {
namespace {

constexpr int kGramTerms = kAndersonMaxK * (kAndersonMaxK + 1) / 2;
constexpr int kGramMaxBlocks = 1024;

// Residual products of one element: u_a u_b for b <= a < K, in packed lower-triangle order
// (a (a + 1) / 2 + b), with u_a = x_{a+1} - x_a.
__global__ __launch_bounds__(kBlock) void k_anderson_gram(AndersonArgs a) {
  if (get_done(&a.st->done)) return;
  double acc[kGramTerms];
#pragma unroll
  for (int e = 0; e < kGramTerms; ++e) acc[e] = 0.0;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < a.n; i += gridDim.x * kBlock) {
    double u[kAndersonMaxK];
    double prev = (double)a.H[i] + a.taus[0];
#pragma unroll
    for (int k = 0; k < kAndersonMaxK; ++k) {
      if (k < a.K) {
        const double x = (double)a.H[(size_t)(k + 1) * a.ldh + i] + a.taus[k + 1];
        u[k] = x - prev;
        prev = x;
      } else {
        u[k] = 0.0;
      }
    }
#pragma unroll
    for (int p = 0; p < kAndersonMaxK; ++p)
#pragma unroll
      for (int q = 0; q <= p; ++q) acc[p * (p + 1) / 2 + q] += u[p] * u[q];
  }
  constexpr int kWaves = kBlock / 64;
  __shared__ double red[kGramTerms][kWaves];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int e = 0; e < kGramTerms; ++e) {
    double v = acc[e];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (lane == 0) red[e][wave] = v;
  }
  __syncthreads();
  if (threadIdx.x < kGramTerms) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) s += red[threadIdx.x][w];
    a.gram[(size_t)blockIdx.x * kGramTerms + threadIdx.x] = s;
  }
}

// One block: sums the block Grams (G = U^T U), divides G by its Frobenius norm when
// a.normalize is set, adds r, solves (G + r I) z = 1 by Cholesky (G + r I is symmetric
// positive definite for r > 0) and writes c = z / sum(z). A system that does not factor
// (non-finite entries) is a numeric error that ends the solve.
__global__ __launch_bounds__(kBlock) void k_anderson_solve(AndersonArgs a, int nb) {
  if (get_done(&a.st->done)) return;
  __shared__ double gs[kGramTerms];
  if (threadIdx.x < kGramTerms) {
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += a.gram[(size_t)b * kGramTerms + threadIdx.x];
    gs[threadIdx.x] = s;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  const int K = a.K;
  double G[kAndersonMaxK][kAndersonMaxK];
  double fro = 0.0;
  for (int p = 0; p < K; ++p)
    for (int q = 0; q <= p; ++q) {
      const double v = gs[p * (p + 1) / 2 + q];
      G[p][q] = v;
      G[q][p] = v;
      fro += (p == q ? 1.0 : 2.0) * v * v;
    }
  fro = sqrt(fro);
  for (int p = 0; p < K; ++p) {
    if (a.normalize && fro > 0.0)
      for (int q = 0; q < K; ++q) G[p][q] /= fro;
    G[p][p] += a.r;
  }
  // Cholesky G = L L^T in place (lower triangle)
  bool ok = true;
  for (int j = 0; j < K && ok; ++j) {
    double d = G[j][j];
    for (int q = 0; q < j; ++q) d -= G[j][q] * G[j][q];
    if (!(d > 0.0) || !isfinite(d)) {
      ok = false;
      break;
    }
    const double ljj = sqrt(d);
    G[j][j] = ljj;
    for (int p = j + 1; p < K; ++p) {
      double v = G[p][j];
      for (int q = 0; q < j; ++q) v -= G[p][q] * G[j][q];
      G[p][j] = v / ljj;
    }
  }
  double z[kAndersonMaxK];
  double zs = 0.0;
  if (ok) {
    for (int p = 0; p < K; ++p) {  // L w = 1
      double v = 1.0;
      for (int q = 0; q < p; ++q) v -= G[p][q] * z[q];
      z[p] = v / G[p][p];
    }
    for (int p = K - 1; p >= 0; --p) {  // L^T z = w
      double v = z[p];
      for (int q = p + 1; q < K; ++q) v -= G[q][p] * z[q];
      z[p] = v / G[p][p];
    }
    for (int p = 0; p < K; ++p) zs += z[p];
    ok = isfinite(zs) && zs != 0.0;
  }
  if (!ok) {
    atomicOr(&a.st->error, kErrNumeric);
    set_done(a.st, 1);
    return;
  }
  for (int p = 0; p < K; ++p) a.c[p] = z[p] / zs;
  a.st->fresh = 1;
  *a.tau0 = 0.0;
}

// x = sum_k c_k x_{k+1}, written as the stored potential (untranslated) and as the first
// iterate of the next cycle.
__global__ __launch_bounds__(kBlock) void k_anderson_mix(AndersonArgs a) {
  if (get_done(&a.st->done)) return;
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= a.n) return;
  double v = 0.0;
  for (int k = 0; k < a.K; ++k)
    v += a.c[k] * ((double)a.H[(size_t)(k + 1) * a.ldh + i] + a.taus[k + 1]);
  const float xf = (float)v;
  a.pot[i] = xf;
  a.H0[i] = xf;
}

}  // namespace

int anderson_gram_blocks(int n) {
  const int nb = (n + kBlock - 1) / kBlock;
  return nb < kGramMaxBlocks ? (nb > 0 ? nb : 1) : kGramMaxBlocks;
}

size_t anderson_gram_bytes(int n) {
  return (size_t)anderson_gram_blocks(n) * kGramTerms * sizeof(double);
}

hipError_t launch_anderson(const AndersonArgs &a, hipStream_t s) {
  if (a.K < 2 || a.K > kAndersonMaxK || a.n < 1) return hipErrorInvalidValue;
  const int nb = anderson_gram_blocks(a.n);
  hipLaunchKernelGGL(k_anderson_gram, dim3(nb), dim3(kBlock), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_anderson_solve, dim3(1), dim3(kBlock), 0, s, a, nb);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_anderson_mix, dim3((a.n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

}  // namespace uot
