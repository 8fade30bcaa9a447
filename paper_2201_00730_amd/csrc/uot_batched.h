// Internal definitions of the batched solver (kernels_batched.hip, batched_api.hip).
#pragma once

#include "uot_internal.h"

namespace uot {

constexpr int kBatchMaxDim = 8;  // point dimension limit of the batched solver

// Per-problem status (the public codes are the non-negative ones, see uot.h).
enum : int32_t {
  kBatchRunning = -1,
  kBatchConverged = 0,
  kBatchMaxIter = 1,
  kBatchInvalid = 2,
  kBatchNumeric = 3,
};

// Sources per work item of the split item level (a multiple of the kernel's 8-source tile).
constexpr int kBatchSplitLen = 512;

// Largest share of eps, E log2(e) / eps, that the expanded form's rounding E may take for a
// problem to use it (the single-problem solvers' threshold on the same quantity).
constexpr double kBatchFormDelta = 3e-4;

// Record stride of the batched kernels (D coordinates, b, padding to a multiple of 4).
__host__ __device__ constexpr int batched_rec_stride(int D) { return (D + 1 + 3) / 4 * 4; }

// Scalar state of one problem (same meaning as SolveState).
struct BatchState {
  double sA, sB, tau_f, tau_g, lambda;
  double off_f_prev, off_g_prev, gdiff_max, gdiff_min, delta;
  int32_t iter;
  int32_t done;
  int32_t status;
  int32_t expanded;  // p = 2: exponents in the expanded form (set once, by the rounding rule)
};

// Records of the batched kernels: D coordinates, the offset b, and where the stride leaves a
// slot (p = 2), b - ||u'||^2 for the expanded form of the exponent.
__host__ __device__ constexpr bool batched_has_expanded_slot(int D) {
  return batched_rec_stride(D) >= D + 2;
}

// Counters of the batched solver, copied to the host after every chunk of iterations.
struct BatchCounters {
  int nact_g, nact_f;              // active work items of each side (after the compaction)
  int ctr_g, ctr_f;                // dynamic work counters
  int running;                     // problems not done
  int pad_[3];
  unsigned long long busy;         // wave time on work items (s_memrealtime ticks), cumulative
  unsigned long long t_compact;    // s_memrealtime at the latest compaction
  double work;                     // sum of N_p M_p over the running problems
};

struct BatchedArgs {
  int B;
  int d, mode;
  float half_p;
  const int64_t *offN, *offM;      // device [B+1]
  const float *x, *y, *alpha, *beta;
  const double *eps, *rho1, *rho2;  // device [B]
  int max_iter;
  double tol;
  int check_every;
  BatchState *state;               // [B]
  double *mu;                      // [B, kBatchMaxDim]
  float *pot_x, *pot_y;            // stored (untranslated) potentials
  float *rec_x, *rec_y;            // source records
  // Per target, the base-2 log-sum-exp of its softmin at its side's last half-step (NaN
  // before the first): the next half-step's exponent reference for that target.
  float *lref_x, *lref_y;
  const int4 *items_g, *items_f;   // (problem, first target, count, slot)
  // Split item level only (else NULL): (first source, source count, first slot of the
  // item's group, group size) per item. A group is one chunk of <= 64 targets whose sources
  // are split over consecutive slots; the last item of a group to finish merges the group's
  // per-target (max, sum) partials and runs the epilogue.
  const int4 *items2_g, *items2_f;
  float2 *spart_g, *spart_f;       // [slots, 64] per-target (max, sum) of a split item
  int *gtick_g, *gtick_f;          // [slots] group arrival counters (at a group's first slot)
  const int *pitem_g, *pitem_f;    // [B+1] item ranges per problem
  int n_items_g, n_items_f;
  int *act_g, *act_f;              // active item lists
  int *nact_g, *nact_f;            // their lengths
  int *ctr_g, *ctr_f;              // dynamic work counters
  int *running;                    // problems not done (after the last compaction)
  BlockPart *part_g, *part_f;      // per-item partials
  int *ticket_g, *ticket_f;        // [B] arrival counters
  // Load statistics (NULL = off): the busy, t_compact and work fields of BatchCounters.
  BatchCounters *stats;
};

hipError_t launch_batched_init(const BatchedArgs &a, hipStream_t s);
hipError_t launch_batched_half(const BatchedArgs &a, int g_step, int blocks, hipStream_t s);
hipError_t launch_batched_compact(const BatchedArgs &a, hipStream_t s);
hipError_t launch_batched_finalize(const BatchedArgs &a, float *f, float *g, int32_t *iters,
                                   int32_t *status, hipStream_t s);
int batched_half_blocks_per_cu(const BatchedArgs &a);

}  // namespace uot
