// Internal definitions shared by the HIP kernels and the host orchestration of libuot.so.
// Not part of the public ABI (that is include/uot.h).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace uot {

constexpr double kLog2e = 1.4426950408889634074;
constexpr double kLn2 = 0.6931471805599453094;
constexpr int kMaxDim = 64;
constexpr int kBlock = 256;  // threads per block of the O(N) kernels

// How C is formed inside a kernel.
enum CostMode : int {
  kDense = 0,    // stored C (row-major, leading dimension ldc)
  kSqEuc = 1,    // points, p = 2: expanded form |x|^2 + |y|^2 - 2<x,y> on centred points
  kPower = 2,    // points, general p: direct differences, ||x - y||^p
  kSqEucMx = 3,  // as kSqEuc, source records split into bf16 pieces for the matrix cores
};
__host__ __device__ constexpr bool is_sq(int mode) { return mode == kSqEuc || mode == kSqEucMx; }

// bf16-split form of the squared-Euclidean exponent. Each float32 value v is carried by three
// bf16 pieces v = v0 + v1 + v2 (split3); the product u*y of a coordinate is carried by the six
// piece products (0,0) (0,1) (1,0) (0,2) (2,0) (1,1), which leave out only terms of relative
// size 2^-24 and below; b takes three slots against the constant 1, and the running reference
// -sigma of a target two slots (two pieces; sigma is kept exactly representable by them)
// against the constant 1 of the source side. Slot 6k + r holds piece mx_piece_u(r) of u_k
// (source side) and piece mx_piece_y(r) of y_k (target side); slots 6D .. 6D + 2 hold
// b0, b1, b2 (target side: 1); slots 6D + 3, 6D + 4 hold 1 (target side: the pieces of
// -sigma); the rest, up to a multiple of 16 (the depth of one instruction), are 0.
__host__ __device__ constexpr int mx_slots(int D) { return (6 * D + 5 + 15) / 16 * 16; }
__host__ __device__ constexpr int mx_piece_u(int r) {
  return r == 2 ? 1 : r == 4 ? 2 : r == 5 ? 1 : 0;
}
__host__ __device__ constexpr int mx_piece_y(int r) {
  return r == 1 ? 1 : r == 3 ? 2 : r == 5 ? 1 : 0;
}
constexpr int kMxMaxDim = 16;  // largest dimension bucket with bf16-split records

// Splits v into bf16 pieces (round to nearest even) with v0 + v1 + v2 = v up to less than
// 2^-24 |v|; each residual is exact in float32. A non-finite v gives (v, 0, 0).
static __device__ inline void split3(float v, __bf16 &v0, __bf16 &v1, __bf16 &v2) {
  v0 = (__bf16)v;
  if (!__builtin_isfinite(v)) {
    v1 = v2 = (__bf16)0.0f;
    return;
  }
  const float r1 = v - (float)v0;
  v1 = (__bf16)r1;
  v2 = (__bf16)(r1 - (float)v1);
}

// Point dimensions are padded (with zero coordinates) up to one of the compiled buckets.
__host__ __device__ constexpr int dim_bucket(int d) {
  return d <= 8 ? d : d <= 12 ? 12 : d <= 16 ? 16 : d <= 24 ? 24 : d <= 32 ? 32 : d <= 48 ? 48 : 64;
}

// Source-record stride in floats for a cost mode and a (bucketed) dimension D. A source
// record holds what a softmin needs of one source point: D coordinates (scaled for kSqEuc,
// zero beyond the true dimension) then the log2-domain offset b, zero-padded to a multiple
// of 4 floats (16-byte aligned records; the matrix-core contraction reads the zeros);
// kSqEucMx records hold the mx_slots(D) bf16 source-side slots instead (two per float);
// dense records hold b only.
__host__ __device__ constexpr int rec_stride(int mode, int D) {
  return mode == kDense ? 1 : mode == kSqEucMx ? mx_slots(D) / 2 : ((D + 1 + 3) / 4) * 4;
}
__host__ __device__ constexpr int rec_stride_for(int mode, int d) {
  return rec_stride(mode, dim_bucket(d));
}
// Record arrays hold this many records: whole tiles of 32, the tail filled with weight-0
// records (b = -inf) that the matrix-core kernel reads without masking.
__host__ __device__ constexpr int rec_count(int n) { return (n + 31) / 32 * 32; }

// Device-resident scalar state of one solve, all double precision.
// Potentials are stored untranslated ("hat" values); the reported TI potentials are
//   f = fhat + off_f,  g = ghat + off_g,  off_f = tau_f + lambda,  off_g = tau_g - lambda.
struct SolveState {
  double sA;          // Smin_alpha^rho1(fb) of the current fb = fhat + tau_f
  double sB;          // Smin_beta^rho2(gb) of the current gb = ghat + tau_g
  double tau_f;       // pending scalar translation of the stored f
  double tau_g;       // pending scalar translation of the stored g
  double lambda;      // lambda*(fb, gb)
  double off_f_prev;  // off_f after the previous iteration
  double off_g_prev;  // off_g after the previous iteration
  double gdiff_max;   // max_j (ghat_new - ghat_old) of the latest g-step
  double gdiff_min;   // min_j (ghat_new - ghat_old)
  double delta;       // change of the reported potentials at the last iteration
  double value;       // scratch for single-value reductions (dual value)
  int32_t iter;       // completed iterations
  int32_t done;       // 1 once converged or failed: solver kernels return at once
  int32_t error;      // bit 1: invalid weights, bit 2: non-finite result
  int32_t pos_a;      // some alpha_i > 0
  int32_t pos_b;      // some beta_j > 0
  int32_t fresh;      // 1 after an Anderson extrapolation: the next change is +inf
  double lam_step;    // G-Sinkhorn, Berg entropy: lambda*(stored f, stored g) of this step
  double span_x2;     // max_i |x_i - mu|^2 and max_j |y_j - mu|^2 (p = 2 form check)
  double span_y2;
  double fabs_max;    // max |f| and max |g| of the reported potentials (p = 2 form check)
  double gabs_max;
  double mu[kMaxDim]; // common centring of x and y (points costs)
};

enum : int32_t { kErrWeights = 1, kErrNumeric = 2 };

// One block's partial reductions in a combine kernel.
struct BlockPart {
  double mass_max;  // log-sum-exp of the tilted mass: running max
  double mass_sum;  //   and sum of exp(v - max)
  double dmax;      // max of (new - old) potential differences
  double dmin;      // min of the same
};

// Epilogue of a half-step (all double): given the softmin S_t over the current sources,
//   hnew_t = k_t * (S_t - tau_src) - c_t * s_src
// (KL prox, and for TI the translation term of App. B; c_t = 0 for plain Sinkhorn).
// Entropy of the marginal penalties (Sec. 3): rho KL, or the Berg entropy
// phi(x) = rho (x - 1 - log x), phi*(x) = -rho log(1 - x/rho).
enum Entropy : int32_t { kEntropyKL = 0, kEntropyBerg = 1 };

struct Epilogue {
  double k_t;       // rho_t / (eps + rho_t)
  double c_t;       // TI: eps rho_t / ((eps + rho_t)(rho1 + rho2)); plain: 0
  double rho_t;     // penalty of the target side (for its tilted mass)
  double kappa_t;   // TI: kappa of the target side; plain: 0 (used by the reduction)
  int32_t src_is_x; // 1: sources are the x/alpha side (g-step)
  int32_t ti;
  int32_t entropy = kEntropyKL;  // kEntropyBerg: hnew solves e^{(h - S')/eps} = rho/(rho + h)
};

// Start/stop events attached to one kernel dispatch (timestamps of the dispatch itself, no
// separate event commands in the stream).
struct LaunchTiming {
  hipEvent_t start, stop;
};

// Launches kern, through hipExtLaunchKernelGGL with the events of t when t is non-null.
template <typename F, typename... Args>
hipError_t launch_timed(F kern, dim3 grid, dim3 block, hipStream_t st, const LaunchTiming *t,
                        Args... args) {
  if (t)
    hipExtLaunchKernelGGL(kern, grid, block, 0, st, t->start, t->stop, 0, args...);
  else
    hipLaunchKernelGGL(kern, grid, block, 0, st, args...);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Launch wrappers (defined in the .hip files). All return hipError_t of the launch.
// ---------------------------------------------------------------------------------------
// Scalar reduction of a half-step (tilted masses, TI translations, lambda*, change,
// convergence test) from its per-block partials.
struct ReduceArgs {
  const BlockPart *bparts;
  int nb;
  SolveState *st;
  int kind;
  int ti;
  double rho1, rho2, kappa_t, tau1, tau2;
  double tol;
  int check_every;
  double *tau_out = nullptr;  // kReduceF with Anderson: receives tau_f
  // G-Sinkhorn (gvar): kReduceF sets lambda = lambda*(stored f, stored g) and carries it as
  // the translation of the stored f; with the Berg entropy lambda* is found by a bracketed
  // Newton iteration over the stored potentials (pot_f [nf], pot_g [ng], weights w_f, w_g).
  int gvar = 0;
  int entropy = kEntropyKL;
  const float *pot_f = nullptr, *pot_g = nullptr, *w_f = nullptr, *w_g = nullptr;
  int nf = 0, ng = 0;
};

struct PointsArgs {
  const float *rec;    // source records [ns, rec_stride]
  int ns;
  int split_len;       // sources per split (multiple of 8)
  int nsplit;
  const float *tgt;    // raw target coordinates [nt, d]
  int nt;
  int d;
  const double *mu;    // centring (device, inside SolveState)
  float sc;            // log2(e)/eps
  float half_p;        // p/2 (kPower)
  float2 *part;        // [nsplit, nt] (running max, sum) in log2 domain
  const int32_t *done; // early-exit flag (may be NULL)
  // Matrix-core kernels only: when red_on is set, one extra block of the launch reduces the
  // previous half-step's block partials (red) beside the softmin blocks, which read none of
  // the scalars it writes.
  ReduceArgs red;
  int red_on;
};

hipError_t launch_points_partial(int mode, const PointsArgs &a, hipStream_t st,
                                 const LaunchTiming *t = nullptr);
int points_targets_per_block(int mode, int d);
int points_split_align(int mode, int d);   // split lengths are multiples of this
// Resident 256-thread blocks per CU of the selected points kernel (0 if unknown).
int points_blocks_per_cu(int mode, int d);
bool points_uses_mfma(int mode, int d);
// Points-softmin kernel selection (process-wide): matrix cores for p = 2 unless forced.
// Auto: bf16-split matrix-core form up to dimension bucket kMxMaxDim, float32 matrix-core
// form above it. Direct: p = 2 on the vector ALU through the differences x - y (kPower
// records and kernels with p = 2), free of the rounding of the expanded form.
enum PointsVariant : int {
  kPointsAuto = 0, kPointsValu = 1, kPointsMfmaF32 = 2, kPointsMfmaBf16 = 3, kPointsDirect = 4
};
extern int g_points_variant;
// Record mode of a points cost of mode kSqEuc / kPower and dimension d under the current
// points-kernel setting (kSqEucMx when the bf16-split matrix-core kernel runs).
int points_record_mode(int mode, int d);

struct DenseArgs {
  const float *C;
  int64_t ldc;
  int n, m;            // C is n x m
  const float *rec;    // source records (1 float each): rows (cols kernel) or columns (rows kernel)
  int split_len;       // rows per split (cols kernel)
  int nsplit;
  float sc;
  float2 *part;        // cols: [nsplit, m]; rows: [1, n]
  const int32_t *done;
};

hipError_t launch_dense_cols_partial(const DenseArgs &a, hipStream_t st,
                                     const LaunchTiming *t = nullptr);
hipError_t launch_dense_rows(const DenseArgs &a, hipStream_t st, const LaunchTiming *t = nullptr);
int dense_cols_per_block();
int dense_rows_per_block();

// kReduceRestart: the x side was replaced by an Anderson extrapolation written without
// translation: Smin_alpha^rho1 of it from the block partials, tau_f = 0.
enum ReduceKind : int { kReduceInit = 0, kReduceG = 1, kReduceF = 2, kReduceRestart = 3 };

// Epilogue kernels (kernels_epilogue.hip).
struct CombineArgs {
  const float2 *part;  // [nsplit, nt]
  int nsplit;
  int nt;
  int mode, d;
  const float *tgt;    // raw target coordinates (points) or NULL
  const float *w;      // target weights [nt]
  float *pot;          // stored target potential [nt] (in: old, out: new)
  float *rec_out;      // target records for the next half-step [nt, stride]
  BlockPart *bparts;   // [gridDim]
  SolveState *st;
  Epilogue ep;
  double sc;           // log2(e)/eps (double)
  double eps;
  float *snap = nullptr;  // Anderson: receives a copy of the new stored potential
};

// Combine + epilogue; each block writes its (tilted mass, change range) partial to bparts,
// which launch_reduce then reduces into the scalar state (a one-block launch: cheaper than
// an atomic ticket and a last-block reduction inside the combine), or runs as a spare
// block of the next matrix-core softmin launch.
hipError_t launch_combine(const CombineArgs &a, hipStream_t st);
int combine_blocks(int nt);

hipError_t launch_reduce(const ReduceArgs &a, hipStream_t st);
hipError_t launch_berg_lambda(const ReduceArgs &a, hipStream_t st);

// Build source records from a potential (solve start, dual value, plan, backward).
struct RecordArgs {
  const float *pts;    // raw coordinates [n, d] (points) or NULL
  const float *w;      // weights [n]
  const float *pot;    // potential [n] or NULL (zeros)
  float *pot_copy;     // if non-NULL, receives the potential (stored copy)
  double pot_off;      // constant added to the potential
  int n, mode, d;
  float *rec;          // [n, stride]
  BlockPart *bparts;   // tilted mass partials for rho (or NULL)
  double rho;
  double sc;
  SolveState *st;
};
hipError_t launch_build_records(const RecordArgs &a, hipStream_t st);

// Centring mu of the points (mean of x | y) and the per-call flags of SolveState; part:
// kCenterBlocks * kMaxDim doubles of device scratch.
constexpr int kCenterBlocks = 64;
hipError_t launch_center(const float *x, int n, const float *y, int m, int d, SolveState *st,
                         double *part, hipStream_t s);
// max |x - mu|^2 and max |y - mu|^2 into st->span_x2, st->span_y2 (after launch_center; part
// as there), and max |f| and max |g| of the reported potentials (stored value plus the
// offsets of the last F-reduction) into st->fabs_max, st->gabs_max.
hipError_t launch_span(const float *x, int n, const float *y, int m, int d, SolveState *st,
                       double *part, hipStream_t s);
hipError_t launch_pot_absmax(const float *pf, int n, const float *pg, int m, SolveState *st,
                             hipStream_t s);
hipError_t launch_validate(const float *a, int n, const float *b, int m, SolveState *st,
                           hipStream_t s);
hipError_t launch_finalize(const float *pot, int n, double off_sel, int which, SolveState *st,
                           float *out, hipStream_t s);

// Dual value pieces.
struct DualArgs {
  const float2 *part;  // row softmin partials over the m sources [nsplit, n]
  int nsplit;
  int n, m, mode, d;
  const float *x;      // raw x for the kSqEuc target constant
  const float *alpha, *beta, *f, *g;
  SolveState *st;
  double sc, eps, rho1, rho2;
  double *acc;         // [gridDim, 4] block partials
};
hipError_t launch_dual_terms(const DualArgs &a, int *nblocks, hipStream_t s);
hipError_t launch_dual_reduce(const DualArgs &a, int nblocks, hipStream_t s);

// Plan application / gradient accumulation over sources (kernels_apply.hip).
struct ApplyArgs {
  int mode, d;
  // dense: C, ldc; transpose = 0 means targets are rows of C, 1 means columns
  const float *C;
  int64_t ldc;
  int transpose;
  // points
  const float *tgt;    // raw target coords [nt, d]
  const float *src;    // raw source coords [ns, d]
  const double *mu;    // centring (SolveState::mu)
  double p;
  int nt, ns;
  const float *w_t, *w_s;    // target / source weights
  const float *h_t, *h_s;    // target / source potentials
  float sc;
  // V: [ns, k] with leading dim ldv (the marginals, V = ones, take kernels_grad.hip)
  const float *V;
  int k;
  int64_t ldv;
  float *out;
  int64_t ldout;
};
size_t apply_partial_bytes(int nt, int ns);
hipError_t launch_apply_with_scratch(const ApplyArgs &a, void *scratch, hipStream_t s);

// Envelope gradients and plan marginals of one side (kernels_grad.hip).
//
// Source records, in doubles: the centred coordinates s' = s - mu (D), |s'|^2, and
// b_s = sc h_s + log2 w_s; then the centred coordinates again as D floats (for the
// accumulators), padded to a whole double.
__host__ __device__ constexpr int grad_rec_stride(int D) { return D + 2 + (D + 1) / 2; }
// Partials per (split, target): reference, sum of 2^{e - ref}, and in grad mode the weighted
// sum lw = sum q w and the d accumulators sum q w s'_k, i.e. grad_part_stride(bucket) floats;
// the stored-cost softmin partials (max, sum) have the layout of grad_part_stride(0).
__host__ __device__ constexpr int grad_part_stride(int D) { return D > 0 ? D + 3 : 2; }
constexpr int kGradMaxSplits = 16;
// Source records of the backward pass are followed by kGradPadRows padding records (zero
// coordinates and norms, b = -inf) so a 16-source step may run past the last source.
constexpr int kGradPadRows = 16;
struct GradRecordArgs {
  const float *pts;    // raw source coordinates [n, d]
  const float *w;      // source weights [n]
  const float *pot;    // source potential [n]
  const double *mu;    // centring (SolveState::mu)
  int n, d;
  double sc;
  double *rec;         // [n + kGradPadRows, grad_rec_stride(bucket)]
};
struct GradArgs {
  const float *tgt;    // raw target coordinates [nt, d]
  int nt, d;
  const double *mu;    // centring (SolveState::mu)
  const float *h_t;    // target potential
  const double *rec;   // source records [ns, grad_rec_stride(bucket)]
  int ns, split_len, nsplit;
  double sc, half_p;
  float p;
  int grad;            // 1: accumulate the point gradient (else sums only)
  float *part;         // [nsplit, nt, grad_part_stride(grad ? bucket : 0)], or
                       // [nsplit, nt, grad_part_stride(16)] for a payload pass
  // Payload pass (plan application, matrix-core pass only): V != nullptr accumulates
  // sum_s q_ts V[s, c] for c < vcols <= 16 (V offset to its first column, row stride ldv)
  // in place of the gradient sums.
  const float *V = nullptr;
  int64_t ldv = 0;
  int vcols = 0;
};
struct GradCombineArgs {
  const float *part;   // partials as GradArgs::part (or stored-cost softmin partials)
  int nsplit, nt, d;
  const float *tgt;    // raw target coordinates [nt, d] (point gradient only)
  const double *mu;    // centring (point gradient only)
  const float *h_t, *w_t;  // target potential and weights
  double sc, eps, rho, gout;
  double pfac;         // 2 for p = 2, else 1
  const double *mass_other;  // total mass of the source side (device)
  float *marg;         // optional: plan marginal w_t rowsum_t, element t at marg[t * marg_stride]
  int64_t marg_stride;
  float *dw;           // optional: weight gradient
  float *dpts;         // optional: point gradient [nt, d] (needs grad partials)
  float *apply_out = nullptr;  // optional: plan applied to a payload, out[t * ldout + c]
  int64_t ldout = 0;           //   for c < d (partials of a payload pass; d = its columns)
};
// Plan application to a payload on a stored cost (kernels_grad.hip): per 16-source step and
// 16-target group the exponents e_ts = b_s - sc C_ts (float32, as the stored-cost softmins),
// one exp2 per entry, and sum_s q_ts V[s, c] on the float32 matrix cores; partials in the
// layout of a payload pass, merged by launch_grad_combine.
struct DensePayloadArgs {
  const float *C;
  int64_t ldc;
  int trans;           // 1: the targets are the columns of C (the sources its rows)
  int vec4;            // rows of C 16-byte aligned (C and ldc): 16-byte loads when !trans
  int nt, ns;
  const float *rec;    // source records b_s = sc h_s + log2 w_s [ns]
  float sc;
  int split_len, nsplit;  // split lengths are multiples of 16
  const float *V;      // payload, offset to its first column, row stride ldv
  int64_t ldv;
  int vcols;           // <= 16
  float *part;         // [nsplit, nt, grad_part_stride(16)]
};
hipError_t launch_dense_payload(const DensePayloadArgs &a, hipStream_t s);

int grad_targets_per_block(int d);
int grad_source_align(int d);  // split lengths of the backward pass are multiples of this
bool grad_payload_supported(int d);  // the matrix-core pass runs payload passes for this d
hipError_t launch_grad_records(const GradRecordArgs &a, hipStream_t s);
hipError_t launch_grad_partial(const GradArgs &a, hipStream_t s, const LaunchTiming *t = nullptr);
hipError_t launch_grad_combine(const GradCombineArgs &a, hipStream_t s);

hipError_t launch_sum(const float *w, int n, double *out, hipStream_t s);

// Anderson extrapolation (kernels_anderson.hip): from the stored iterates of one cycle,
// x_k = H[k] + taus[k] (k = 0..K), computes c and writes x = sum_k c_k x_{k+1} to pot and
// H[0], taus[0] = 0, fresh = 1. gram: anderson_gram_bytes(n); c: kAndersonMaxK doubles.
constexpr int kAndersonMaxK = 8;
struct AndersonArgs {
  const float *H;      // [K + 1, ldh]
  int64_t ldh;
  double *taus;        // [K + 1]
  int n, K;
  double r;
  int normalize;       // 1: Gram matrix divided by its Frobenius norm before adding r
  double *gram;
  double *c;
  float *pot;          // stored potential of the x side (out)
  float *H0;           // H[0] (out)
  double *tau0;        // taus[0] (out)
  SolveState *st;
};
hipError_t launch_anderson(const AndersonArgs &a, hipStream_t s);
size_t anderson_gram_bytes(int n);

// 1-D Frank-Wolfe (kernels_fw.hip): problem b owns [offN[b], offN[b+1]) of x, alpha, f and
// the double scratch fb, Ac, r, and [offM[b], offM[b+1]) of y, beta, g, gb, Bc, s.
struct FwLaunch {
  int B;
  const int64_t *offN, *offM;  // device [B + 1]
  const float *x, *y, *alpha, *beta;
  const double *rho1, *rho2;
  double p;
  int line_search, max_iter;
  double tol;
  double *fb, *gb, *Ac, *Bc, *r, *s;
  float *f, *g;
  int32_t *iters;
  double *gap;
  int32_t *status;
  int max_blocks;
};
hipError_t launch_fw1d(const FwLaunch &l, hipStream_t s);

// 1-D barycenters (kernels_fw.hip): problem b has K measures m = b*K + k on
// [off[m], off[m+1]); per-point double scratch fb, Ac, r; barycenter outputs at offset
// off[b*K] - b*K + b, off[(b+1)K] - off[bK] - K + 1 entries.
constexpr int kBaryMaxMeasures = 16;
struct BaryLaunch {
  int B, K;
  const int64_t *off;
  const float *x, *alpha;
  const double *w, *rho;
  int max_iter;
  double tol;
  double *fb, *Ac, *r;
  float *f, *bx, *bw;
  int32_t *iters;
  double *gap;
  int32_t *status;
  int max_blocks;
};
hipError_t launch_fw_bary(const BaryLaunch &l, hipStream_t s);

}  // namespace uot
