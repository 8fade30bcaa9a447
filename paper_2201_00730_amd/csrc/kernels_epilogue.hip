// O(N + M) kernels around the softmin passes: combine of split partials with the half-step
// epilogue (KL prox and TI translation), the single-block scalar reductions (tilted masses,
// lambda*, convergence test), source-record construction, input validation, centring of the
// point clouds, the final translation of the potentials and the dual-value / weight-gradient
// terms. Everything scalar is double precision.
#include <cfloat>

#include "uot_epilogue.cuh"

namespace uot {
namespace {

template <int D, int MODE>
__global__ __launch_bounds__(kBlock) void k_build_records(RecordArgs a) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  double mm = -INFINITY, ms = 0.0, dmx = 0.0, dmn = 0.0;
  if (t < a.n) {
    const double h = (a.pot ? (double)a.pot[t] : 0.0) + a.pot_off;
    const float hf = (float)h;
    if (a.pot_copy) a.pot_copy[t] = hf;
    float yc[D > 0 ? D : 1];
    double yn2 = 0.0;
    if constexpr (MODE != kDense) yn2 = centred<D>(a.pts, a.d, t, a.st->mu, yc);
    const float w = a.w[t];
    write_record<D, MODE>(a.rec, t, yc, yn2, hf, w, a.sc);
    if (w > 0.0f) { mm = log((double)w) - (double)hf / a.rho; ms = 1.0; }
  } else if (t < rec_count(a.n)) {
    // pad record: zero coordinates, weight 0
    float yc[D > 0 ? D : 1];
#pragma unroll
    for (int k = 0; k < (D > 0 ? D : 1); ++k) yc[k] = 0.0f;
    write_record<D, MODE>(a.rec, t, yc, 0.0, 0.0f, 0.0f, a.sc);
  }
  if (a.bparts) {
    block_reduce_part(mm, ms, dmx, dmn);
    if (threadIdx.x == 0) a.bparts[blockIdx.x] = BlockPart{mm, ms, dmx, dmn};
  }
}

__global__ __launch_bounds__(kBlock) void k_reduce(ReduceArgs a) {
  if (a.kind != kReduceInit && get_done(&a.st->done)) return;
  reduce_scalars(a);
}

// G-Sinkhorn with the Berg entropy: lambda*(stored f, stored g) into st->lam_step, by one
// block of kBergThreads (Newton over all potentials), between the f-step's combine and its
// reduction. The previous step (tau_f) is the start.
constexpr int kBergThreads = 1024;
__global__ __launch_bounds__(kBergThreads) void k_berg_lambda(ReduceArgs a) {
  if (get_done(&a.st->done)) return;
  const double l = berg_lambda<kBergThreads>(a, a.st->tau_f);
  if (threadIdx.x == 0) a.st->lam_step = l;
}

// Threads per target in the combine kernel.
constexpr int kCombLanes = 2;
constexpr int kCombTargets = kBlock / kCombLanes;

template <int D, int MODE>
__global__ __launch_bounds__(kBlock) void k_combine(CombineArgs a) {
  combine_block<D, MODE, kCombLanes>(a, blockIdx.x * kCombTargets, blockIdx.x);
}

// Zeroes the flags of the state and computes the common mean of x and y (points costs).
// Centring, stage 1: block b sums the coordinates of its slice of the points of x | y into
// part[b][k] (one double accumulator per dimension and thread, then one block sum per
// dimension); stage 2 adds the block partials in a fixed order, so mu is reproducible.
template <int D>
__global__ __launch_bounds__(kBlock) void k_center_part(const float *x, int n, const float *y,
                                                        int m, int d, double *part) {
  const int tot = n + m;
  const int chunk = (tot + (int)gridDim.x - 1) / (int)gridDim.x;
  const int p0 = blockIdx.x * chunk, p1 = min(tot, p0 + chunk);
  double acc[D];
#pragma unroll
  for (int k = 0; k < D; ++k) acc[k] = 0.0;
  for (int q = p0 + threadIdx.x; q < p1; q += kBlock) {
    const float *src = q < n ? x + (size_t)q * d : y + (size_t)(q - n) * d;
#pragma unroll
    for (int k = 0; k < D; ++k)
      if (k < d) acc[k] += (double)src[k];
  }
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const double v = block_sum(acc[k]);
    if (threadIdx.x == 0) part[(size_t)blockIdx.x * kMaxDim + k] = v;
  }
}

__global__ __launch_bounds__(kBlock) void k_center(const double *part, int nb, int tot, int d,
                                                   SolveState *st) {
  const int k = threadIdx.x;
  if (k < kMaxDim) {
    double v = 0.0;
    if (k < d)
      for (int b = 0; b < nb; ++b) v += part[(size_t)b * kMaxDim + k];
    st->mu[k] = k < d ? v / (double)tot : 0.0;
  }
  if (k == 0) {
    st->error = 0;
    st->done = 0;
    st->pos_a = 0;
    st->pos_b = 0;
    st->iter = 0;
    st->fresh = 0;
  }
}

// Spread of the centred clouds, stage 1: block b writes the largest |x - mu|^2 and
// |y - mu|^2 of its slice of x | y to part[2b], part[2b + 1]; stage 2 (one block) takes the
// maxima.
template <int D>
__global__ __launch_bounds__(kBlock) void k_span_part(const float *x, int n, const float *y,
                                                      int m, int d, const SolveState *st,
                                                      double *part) {
  __shared__ double sx[kBlock], sy[kBlock];
  const int tot = n + m;
  const int chunk = (tot + (int)gridDim.x - 1) / (int)gridDim.x;
  const int p0 = blockIdx.x * chunk, p1 = min(tot, p0 + chunk);
  double mx = 0.0, my = 0.0;
  for (int q = p0 + threadIdx.x; q < p1; q += kBlock) {
    const float *src = q < n ? x + (size_t)q * d : y + (size_t)(q - n) * d;
    double r2 = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k)
      if (k < d) {
        const double v = (double)src[k] - st->mu[k];
        r2 = fma(v, v, r2);
      }
    if (q < n) mx = fmax(mx, r2); else my = fmax(my, r2);
  }
  sx[threadIdx.x] = mx;
  sy[threadIdx.x] = my;
  __syncthreads();
  for (int off = kBlock / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      sx[threadIdx.x] = fmax(sx[threadIdx.x], sx[threadIdx.x + off]);
      sy[threadIdx.x] = fmax(sy[threadIdx.x], sy[threadIdx.x + off]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = sx[0];
    part[2 * blockIdx.x + 1] = sy[0];
  }
}

__global__ __launch_bounds__(kBlock) void k_span(const double *part, int nb, SolveState *st) {
  if (threadIdx.x != 0) return;
  double mx = 0.0, my = 0.0;
  for (int b = 0; b < nb; ++b) {
    mx = fmax(mx, part[2 * b]);
    my = fmax(my, part[2 * b + 1]);
  }
  st->span_x2 = mx;
  st->span_y2 = my;
}

// max |stored + offset| over each side's potentials (one block; runs once per solve).
__global__ __launch_bounds__(1024) void k_pot_absmax(const float *pf, int n, const float *pg, int m,
                                                     SolveState *st) {
  __shared__ double sf[1024], sg[1024];
  const double of = st->off_f_prev, og = st->off_g_prev;
  double af = 0.0, ag = 0.0;
  for (int i = threadIdx.x; i < n; i += 1024) af = fmax(af, fabs((double)pf[i] + of));
  for (int j = threadIdx.x; j < m; j += 1024) ag = fmax(ag, fabs((double)pg[j] + og));
  sf[threadIdx.x] = af;
  sg[threadIdx.x] = ag;
  __syncthreads();
  for (int off = 512; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      sf[threadIdx.x] = fmax(sf[threadIdx.x], sf[threadIdx.x + off]);
      sg[threadIdx.x] = fmax(sg[threadIdx.x], sg[threadIdx.x + off]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    st->fabs_max = sf[0];
    st->gabs_max = sg[0];
  }
}

template <int D>
hipError_t span_part_for(const float *x, int n, const float *y, int m, int d, int nb,
                         const SolveState *st, double *part, hipStream_t s) {
  hipLaunchKernelGGL((k_span_part<D>), dim3(nb), dim3(kBlock), 0, s, x, n, y, m, d, st, part);
  return hipGetLastError();
}

template <int D>
hipError_t center_part_for(const float *x, int n, const float *y, int m, int d, int nb,
                           double *part, hipStream_t s) {
  hipLaunchKernelGGL((k_center_part<D>), dim3(nb), dim3(kBlock), 0, s, x, n, y, m, d, part);
  return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void k_validate(const float *a, int n, const float *b, int m,
                                                     SolveState *st) {
  const int stride = gridDim.x * kBlock;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n + m; i += stride) {
    const float w = i < n ? a[i] : b[i - n];
    if (!(w >= 0.0f) || isinf(w)) atomicOr(&st->error, kErrWeights);
    if (w > 0.0f) {
      if (i < n) st->pos_a = 1; else st->pos_b = 1;
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_finalize(const float *pot, int n, int which,
                                                     const SolveState *st, float *out) {
  // the offsets of the reported potentials recorded by the last f-step reduction: TI
  // tau_f + lambda and tau_g - lambda, G-Sinkhorn lambda and -lambda, plain Sinkhorn 0
  const double off = which == 0 ? st->off_f_prev : st->off_g_prev;
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t < n) out[t] = (float)((double)pot[t] + off);
}

// Dual value terms. Threads i < n (targets of the row softmin over beta with g):
//   m(pi) partial: log alpha_i + (f_i - S_i)/eps,  S_i = Smin_beta^eps(C_{i,:} - g);
//   rho1 alpha_i (1 - e^{-f_i/rho1}) and alpha_i. Threads j < m: rho2 beta_j (1 - e^{-g_j/rho2}), beta_j.
template <int D, int MODE>
__global__ __launch_bounds__(kBlock) void k_dual_terms(DualArgs a) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  double mm = -INFINITY, ms = 0.0, A = 0.0, B = 0.0, ma = 0.0, mb = 0.0;
  if (t < a.n) {
    double lse2 = combine_lse2(a.part, a.nsplit, a.n, t);
    float yc[D > 0 ? D : 1];
    if constexpr (is_sq(MODE)) lse2 -= a.sc * centred<D>(a.x, a.d, t, a.st->mu, yc);
    const double S = -lse2 / a.sc;
    const double w = a.alpha[t], f = a.f[t];
    if (w > 0.0) { mm = log(w) + (f - S) / a.eps; ms = 1.0; }
    A = w * (-expm1(-f / a.rho1));
    ma = w;
  }
  if (t < a.m) {
    const double w = a.beta[t], g = a.g[t];
    B = w * (-expm1(-g / a.rho2));
    mb = w;
  }
  double dummy0 = 0.0, dummy1 = 0.0;
  block_reduce_part(mm, ms, dummy0, dummy1);
  A = block_sum(A);
  B = block_sum(B);
  ma = block_sum(ma);
  mb = block_sum(mb);
  if (threadIdx.x == 0) {
    double *o = a.acc + (size_t)blockIdx.x * 6;
    o[0] = mm; o[1] = ms; o[2] = A; o[3] = B; o[4] = ma; o[5] = mb;
  }
}

__global__ __launch_bounds__(kBlock) void k_dual_reduce(DualArgs a, int nb) {
  double mm = -INFINITY, ms = 0.0, A = 0.0, B = 0.0, ma = 0.0, mb = 0.0;
  for (int b = threadIdx.x; b < nb; b += kBlock) {
    const double *o = a.acc + (size_t)b * 6;
    lse_merge(mm, ms, o[0], o[1]);
    A += o[2]; B += o[3]; ma += o[4]; mb += o[5];
  }
  double dummy0 = 0.0, dummy1 = 0.0;
  block_reduce_part(mm, ms, dummy0, dummy1);
  A = block_sum(A);
  B = block_sum(B);
  ma = block_sum(ma);
  mb = block_sum(mb);
  if (threadIdx.x == 0) {
    const double mpi = (mm == -INFINITY) ? 0.0 : exp(mm) * ms;
    const double v = a.rho1 * A + a.rho2 * B - a.eps * (mpi - ma * mb);
    a.st->value = v;
    if (!isfinite(v)) a.st->error |= kErrNumeric;
  }
}

template <int D, int MODE>
hipError_t combine_for(const CombineArgs &a, hipStream_t s) {
  const int nb = (a.nt + kCombTargets - 1) / kCombTargets;
  hipLaunchKernelGGL((k_combine<D, MODE>), dim3(nb), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

template <int D, int MODE>
hipError_t records_for(const RecordArgs &a, hipStream_t s) {
  const int nb = (rec_count(a.n) + kBlock - 1) / kBlock;
  hipLaunchKernelGGL((k_build_records<D, MODE>), dim3(nb), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

template <int D, int MODE>
hipError_t dual_for(const DualArgs &a, int nb, hipStream_t s) {
  hipLaunchKernelGGL((k_dual_terms<D, MODE>), dim3(nb), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

// Dispatch on (mode, bucketed dimension).
#define UOT_DISPATCH(FN, MODE_, D_, ...)                                         \
  do {                                                                           \
    if ((MODE_) == kDense) return FN<0, kDense>(__VA_ARGS__);                    \
    const int b_ = dim_bucket(D_);                                               \
    if ((MODE_) == kSqEuc) {                                                     \
      switch (b_) {                                                              \
        case 1: return FN<1, kSqEuc>(__VA_ARGS__);                               \
        case 2: return FN<2, kSqEuc>(__VA_ARGS__);                               \
        case 3: return FN<3, kSqEuc>(__VA_ARGS__);                               \
        case 4: return FN<4, kSqEuc>(__VA_ARGS__);                               \
        case 5: return FN<5, kSqEuc>(__VA_ARGS__);                               \
        case 6: return FN<6, kSqEuc>(__VA_ARGS__);                               \
        case 7: return FN<7, kSqEuc>(__VA_ARGS__);                               \
        case 8: return FN<8, kSqEuc>(__VA_ARGS__);                               \
        case 12: return FN<12, kSqEuc>(__VA_ARGS__);                             \
        case 16: return FN<16, kSqEuc>(__VA_ARGS__);                             \
        case 24: return FN<24, kSqEuc>(__VA_ARGS__);                             \
        case 32: return FN<32, kSqEuc>(__VA_ARGS__);                             \
        case 48: return FN<48, kSqEuc>(__VA_ARGS__);                             \
        case 64: return FN<64, kSqEuc>(__VA_ARGS__);                             \
      }                                                                          \
    } else if ((MODE_) == kPower) {                                              \
      switch (b_) {                                                              \
        case 1: return FN<1, kPower>(__VA_ARGS__);                               \
        case 2: return FN<2, kPower>(__VA_ARGS__);                               \
        case 3: return FN<3, kPower>(__VA_ARGS__);                               \
        case 4: return FN<4, kPower>(__VA_ARGS__);                               \
        case 5: return FN<5, kPower>(__VA_ARGS__);                               \
        case 6: return FN<6, kPower>(__VA_ARGS__);                               \
        case 7: return FN<7, kPower>(__VA_ARGS__);                               \
        case 8: return FN<8, kPower>(__VA_ARGS__);                               \
        case 12: return FN<12, kPower>(__VA_ARGS__);                             \
        case 16: return FN<16, kPower>(__VA_ARGS__);                             \
        case 24: return FN<24, kPower>(__VA_ARGS__);                             \
        case 32: return FN<32, kPower>(__VA_ARGS__);                             \
        case 48: return FN<48, kPower>(__VA_ARGS__);                             \
        case 64: return FN<64, kPower>(__VA_ARGS__);                             \
      }                                                                          \
    } else if ((MODE_) == kSqEucMx) {                                            \
      switch (b_) {                                                              \
        case 1: return FN<1, kSqEucMx>(__VA_ARGS__);                             \
        case 2: return FN<2, kSqEucMx>(__VA_ARGS__);                             \
        case 3: return FN<3, kSqEucMx>(__VA_ARGS__);                             \
        case 4: return FN<4, kSqEucMx>(__VA_ARGS__);                             \
        case 5: return FN<5, kSqEucMx>(__VA_ARGS__);                             \
        case 6: return FN<6, kSqEucMx>(__VA_ARGS__);                             \
        case 7: return FN<7, kSqEucMx>(__VA_ARGS__);                             \
        case 8: return FN<8, kSqEucMx>(__VA_ARGS__);                             \
        case 12: return FN<12, kSqEucMx>(__VA_ARGS__);                           \
        case 16: return FN<16, kSqEucMx>(__VA_ARGS__);                           \
      }                                                                          \
    }                                                                            \
    return hipErrorInvalidValue;                                                 \
  } while (0)

}  // namespace

int combine_blocks(int nt) { return (nt + kCombTargets - 1) / kCombTargets; }

hipError_t launch_combine(const CombineArgs &a, hipStream_t s) {
  UOT_DISPATCH(combine_for, a.mode, a.d, a, s);
}

hipError_t launch_build_records(const RecordArgs &a, hipStream_t s) {
  UOT_DISPATCH(records_for, a.mode, a.d, a, s);
}

hipError_t launch_berg_lambda(const ReduceArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_berg_lambda, dim3(1), dim3(kBergThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_reduce(const ReduceArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_center(const float *x, int n, const float *y, int m, int d, SolveState *st,
                         double *part, hipStream_t s) {
  int nb = 0;
  if (d > 0) {
    nb = (n + m + kBlock - 1) / kBlock;
    if (nb > kCenterBlocks) nb = kCenterBlocks;
    hipError_t e = hipErrorInvalidValue;
    switch (dim_bucket(d)) {
      case 1: e = center_part_for<1>(x, n, y, m, d, nb, part, s); break;
      case 2: e = center_part_for<2>(x, n, y, m, d, nb, part, s); break;
      case 3: e = center_part_for<3>(x, n, y, m, d, nb, part, s); break;
      case 4: e = center_part_for<4>(x, n, y, m, d, nb, part, s); break;
      case 5: e = center_part_for<5>(x, n, y, m, d, nb, part, s); break;
      case 6: e = center_part_for<6>(x, n, y, m, d, nb, part, s); break;
      case 7: e = center_part_for<7>(x, n, y, m, d, nb, part, s); break;
      case 8: e = center_part_for<8>(x, n, y, m, d, nb, part, s); break;
      case 12: e = center_part_for<12>(x, n, y, m, d, nb, part, s); break;
      case 16: e = center_part_for<16>(x, n, y, m, d, nb, part, s); break;
      case 24: e = center_part_for<24>(x, n, y, m, d, nb, part, s); break;
      case 32: e = center_part_for<32>(x, n, y, m, d, nb, part, s); break;
      case 48: e = center_part_for<48>(x, n, y, m, d, nb, part, s); break;
      case 64: e = center_part_for<64>(x, n, y, m, d, nb, part, s); break;
      default: break;
    }
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_center, dim3(1), dim3(kBlock), 0, s, part, nb, n + m, d, st);
  return hipGetLastError();
}

hipError_t launch_span(const float *x, int n, const float *y, int m, int d, SolveState *st,
                       double *part, hipStream_t s) {
  int nb = (n + m + kBlock - 1) / kBlock;
  if (nb > kCenterBlocks) nb = kCenterBlocks;
  hipError_t e = hipErrorInvalidValue;
  switch (dim_bucket(d)) {
    case 1: e = span_part_for<1>(x, n, y, m, d, nb, st, part, s); break;
    case 2: e = span_part_for<2>(x, n, y, m, d, nb, st, part, s); break;
    case 3: e = span_part_for<3>(x, n, y, m, d, nb, st, part, s); break;
    case 4: e = span_part_for<4>(x, n, y, m, d, nb, st, part, s); break;
    case 5: e = span_part_for<5>(x, n, y, m, d, nb, st, part, s); break;
    case 6: e = span_part_for<6>(x, n, y, m, d, nb, st, part, s); break;
    case 7: e = span_part_for<7>(x, n, y, m, d, nb, st, part, s); break;
    case 8: e = span_part_for<8>(x, n, y, m, d, nb, st, part, s); break;
    case 12: e = span_part_for<12>(x, n, y, m, d, nb, st, part, s); break;
    case 16: e = span_part_for<16>(x, n, y, m, d, nb, st, part, s); break;
    case 24: e = span_part_for<24>(x, n, y, m, d, nb, st, part, s); break;
    case 32: e = span_part_for<32>(x, n, y, m, d, nb, st, part, s); break;
    case 48: e = span_part_for<48>(x, n, y, m, d, nb, st, part, s); break;
    case 64: e = span_part_for<64>(x, n, y, m, d, nb, st, part, s); break;
    default: break;
  }
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_span, dim3(1), dim3(kBlock), 0, s, part, nb, st);
  return hipGetLastError();
}

hipError_t launch_pot_absmax(const float *pf, int n, const float *pg, int m, SolveState *st,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_pot_absmax, dim3(1), dim3(1024), 0, s, pf, n, pg, m, st);
  return hipGetLastError();
}

hipError_t launch_validate(const float *a, int n, const float *b, int m, SolveState *st,
                           hipStream_t s) {
  int nb = (n + m + kBlock - 1) / kBlock;
  if (nb > 1024) nb = 1024;
  hipLaunchKernelGGL(k_validate, dim3(nb), dim3(kBlock), 0, s, a, n, b, m, st);
  return hipGetLastError();
}

hipError_t launch_finalize(const float *pot, int n, double off_sel, int which, SolveState *st,
                           float *out, hipStream_t s) {
  (void)off_sel;
  hipLaunchKernelGGL(k_finalize, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, pot, n,
                     which, st, out);
  return hipGetLastError();
}

hipError_t launch_dual_terms(const DualArgs &a, int *nblocks, hipStream_t s) {
  const int nb = ((a.n > a.m ? a.n : a.m) + kBlock - 1) / kBlock;
  *nblocks = nb;
  UOT_DISPATCH(dual_for, a.mode, a.d, a, nb, s);
}

hipError_t launch_dual_reduce(const DualArgs &a, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL(k_dual_reduce, dim3(1), dim3(kBlock), 0, s, a, nblocks);
  return hipGetLastError();
}

}  // namespace uot
