// Batched MPPI: many independent instances (each with its own K, T, lambda,
// sigma, noise stream and cost data) advanced by one launch per phase.
//
// The work lists are host-built tile tables over a device instance table
// (BatchInst): a workgroup picks its tile, reads the instance descriptor with
// wave-uniform scalar loads and runs the same device bodies as the
// single-instance kernels (noise.h, rollout.h, softmin.h).  Sample tiles are
// ordered longest horizon first, so the hardware dispatcher starts the long
// rollouts early and fills the tail with short ones.  The per-iteration launch
// sequence of a batch is captured once in a hipGraph by the host code.
#include "noise.h"
#include "rollout.h"
#include "softmin.h"
#include "worklist.h"

namespace mppi {

static_assert(sizeof(WorkItem) == sizeof(int2) && alignof(WorkItem) <= alignof(int2),
              "work lists are uploaded as int2 tables");

// (a1) every normal of a tile's samples; one thread per sample loops
// over the Philox calls of its sample, each call storing four coalesced rows.
__global__ __launch_bounds__(kBatchMaxTile) void batch_noise_kernel(
    const BatchInst* __restrict__ insts, const int2* __restrict__ tiles) {
  const int2 tl = tiles[blockIdx.x];
  const BatchInst& b = insts[tl.x];
  const int k = tl.y * static_cast<int>(blockDim.x) + threadIdx.x;
  if (k >= b.K) return;
  const uint32_t it = b.st->iteration;
  const int ncall = (b.TM + 3) / 4;
  const int m = b.TM / b.T;
  for (int c = 0; c < ncall; ++c)
    noise::emit_call(b.key0, b.key1, it, b.instance, k, c, b.TM, m, b.sigma.v, b.eps, b.ldk,
                     b.p.sigma_t, b.p.mean_sample && k == 0);
}

// (a2) one lane per sample over a tile of samples of one instance;
// the instance's cost data and controls are staged in LDS per workgroup.
template <class Model, int INTEG, class Cost, bool COUNT>
__global__ __launch_bounds__(kBatchMaxTile) void batch_rollout_kernel(
    const BatchInst* __restrict__ insts, const int2* __restrict__ tiles) {
  extern __shared__ float4 lds[];
  const int2 tl = tiles[blockIdx.x];
  const BatchInst& b = insts[tl.x];
  const DevParams& p = b.p;
  const float* lds_u = stage_rollout_lds<Cost>(p, b.u, b.TM, lds);
  const int k = tl.y * static_cast<int>(blockDim.x) + threadIdx.x;
  if (k >= b.K) return;  // no barrier follows
  const RolloutResult r =
      rollout_lane<Model, INTEG, Cost, COUNT>(p, b.x0, lds_u, b.eps + k, b.ldk, b.T, lds,
                                              k < p.n_plain);
  b.S[k] = r.cost;
  if constexpr (COUNT) b.crashes[k] = r.crashes;
}

// (a3)-(a5) one workgroup per instance; (a6) one workgroup per row of the update.
__global__ __launch_bounds__(kWeightsBlock) void batch_weights_kernel(
    const BatchInst* __restrict__ insts) {
  const BatchInst& b = insts[blockIdx.x];
  weights_body(b.S, b.K, b.lambda, b.inv_lambda, b.e, b.st, b.p.n_plain);
}

__global__ __launch_bounds__(kGemvBlock) void batch_gemv_kernel(const BatchInst* __restrict__ insts,
                                                                const int2* __restrict__ tiles) {
  const int2 tl = tiles[blockIdx.x];
  const BatchInst& b = insts[tl.x];
  // the host checks every row tile against T*m before the upload; a row past
  // the instance's would read and write another instance's buffers
  if (tl.y >= b.TM) return;  // uniform over the workgroup: no barrier is skipped by part of it
  gemv_row(b.eps, b.ldk, b.K, b.e, b.st, b.u, b.step, tl.y, false);
}

__global__ void batch_set_iteration_kernel(const BatchInst* __restrict__ insts, int n,
                                           uint32_t iteration) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) insts[i].st->iteration = iteration;
}

namespace {

using BatchFn = void (*)(const BatchInst*, const int2*);

template <class Model, int INTEG, class Cost>
BatchFn pick(bool count) {
  if (count) return batch_rollout_kernel<Model, INTEG, Cost, true>;
  return batch_rollout_kernel<Model, INTEG, Cost, false>;
}

template <class Model, int INTEG>
BatchFn pick_generic(uint32_t cost, bool count) {
  if (cost == MPPI_COST_QUADRATIC) return pick<Model, INTEG, CostQuadratic>(count);
  if (cost == MPPI_COST_TRACK) return pick<Model, INTEG, CostTrack>(count);
  return nullptr;
}

template <class Model, int INTEG>
BatchFn pick_wheeled(uint32_t cost, bool count) {
  switch (cost) {
    case MPPI_COST_PATH_CIRCLES: return pick<Model, INTEG, CostPath<true>>(count);
    case MPPI_COST_PATH_COSTMAP: return pick<Model, INTEG, CostPath<false>>(count);
    case MPPI_COST_GOAL_CIRCLES: return pick<Model, INTEG, CostGoalCircles>(count);
    default: return pick_generic<Model, INTEG>(cost, count);
  }
}

template <int INTEG>
BatchFn pick_model(uint32_t dynamics, uint32_t cost, bool accurate, bool count) {
  switch (dynamics) {
    case MPPI_DYN_DOUBLE_INTEGRATOR: return pick_generic<DoubleIntegrator, INTEG>(cost, count);
    case MPPI_DYN_BICYCLE:
      return accurate ? pick_wheeled<Bicycle<false>, INTEG>(cost, count)
                      : pick_wheeled<Bicycle<true>, INTEG>(cost, count);
    case MPPI_DYN_QUADROTOR:
      if (cost == MPPI_COST_HOVER) return pick<Quadrotor, INTEG, CostHover>(count);
      return pick_generic<Quadrotor, INTEG>(cost, count);
    default: return nullptr;
  }
}

}  // namespace

hipError_t launch_batch_noise(const BatchPlan& b, hipStream_t stream) {
  hipLaunchKernelGGL(batch_noise_kernel, dim3(b.n_sample_tiles), dim3(b.tile), 0, stream,
                     b.insts, b.sample_tiles);
  return hipGetLastError();
}

hipError_t launch_batch_rollout(uint32_t dynamics, uint32_t integrator, uint32_t cost,
                                bool accurate_trig, bool count, const BatchPlan& b,
                                hipStream_t stream) {
  BatchFn fn = integrator == MPPI_INT_EULER ? pick_model<kEuler>(dynamics, cost, accurate_trig, count)
                                            : pick_model<kRK4>(dynamics, cost, accurate_trig, count);
  if (!fn) return hipErrorInvalidValue;
  if (b.rollout_lds > 48 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       static_cast<int>(b.rollout_lds));
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(fn, dim3(b.n_sample_tiles), dim3(b.tile), b.rollout_lds, stream, b.insts,
                     b.sample_tiles);
  return hipGetLastError();
}

hipError_t launch_batch_update(const BatchPlan& b, hipStream_t stream) {
  hipLaunchKernelGGL(batch_weights_kernel, dim3(b.n_inst), dim3(kWeightsBlock), 0, stream, b.insts);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(batch_gemv_kernel, dim3(b.n_row_tiles), dim3(kGemvBlock), 0, stream, b.insts,
                     b.row_tiles);
  return hipGetLastError();
}

hipError_t launch_batch_set_iteration(const BatchPlan& b, uint32_t iteration, hipStream_t stream) {
  hipLaunchKernelGGL(batch_set_iteration_kernel, dim3((b.n_inst + 255) / 256), dim3(256), 0, stream,
                     b.insts, b.n_inst, iteration);
  return hipGetLastError();
}

}  // namespace mppi
