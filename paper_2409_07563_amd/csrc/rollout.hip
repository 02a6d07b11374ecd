// Step (a2): fused rollout + cost.  One lane per sample keeps the state in
// registers for the whole horizon; per step it reads its noise (coalesced:
// lanes are consecutive samples of one [T*m][ldk] row), forms v = u_t + eps,
// advances the dynamics and adds the running cost with compensated (Kahan)
// summation; the terminal cost closes the sum.  u_t, the spline and every
// cost weight are wave-uniform; u (all T steps), the obstacle grid and the
// spline are staged once per workgroup into LDS, so no step waits on a scalar
// or global load of them.  The noise of step t+1 is requested before step t
// is computed so that its memory latency overlaps the arithmetic.
#include "common.h"
#include "costs.h"
#include "dynamics.h"

namespace mppi {

constexpr int kRolloutBlock = 64;

template <class Model, int INTEG, class Cost, bool COUNT>
__global__ __launch_bounds__(kRolloutBlock) void rollout_kernel(
    DevParams p, const float* __restrict__ x0, const float* __restrict__ u,
    const float* __restrict__ eps, int64_t ldk, int K, int T, float* __restrict__ S,
    int32_t* __restrict__ crashes) {
  constexpr int N = Model::N, M = Model::M;
  extern __shared__ float4 lds[];
  constexpr bool kStage = Cost::kStage;
  const int u_off4 = kStage ? p.stage_words4 : 0;
  float* lds_u = reinterpret_cast<float*>(lds + u_off4);
  if constexpr (kStage)
    for (int i = threadIdx.x; i < p.stage_words4; i += blockDim.x) lds[i] = p.stage[i];
  for (int i = threadIdx.x; i < T * M; i += blockDim.x) lds_u[i] = u[i];
  __syncthreads();
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;  // no barrier follows
  float x[N], comp[N > 0 ? N : 1];
#pragma unroll
  for (int i = 0; i < N; ++i) { x[i] = x0[i]; comp[i] = 0.0f; }
  const float* e = eps + k;
  float nxt[M];
#pragma unroll
  for (int j = 0; j < M; ++j) nxt[j] = e[j * ldk];
  typename Cost::State cs;
  Cost::init(cs, x, p, lds);
  float sum = 0.0f, sum_c = 0.0f;
  int ncrash = 0;
  for (int t = 0; t < T; ++t) {
    float v[M];
#pragma unroll
    for (int j = 0; j < M; ++j) v[j] = lds_u[t * M + j] + nxt[j];
    if (t + 1 < T) {
      const float* en = e + static_cast<int64_t>(t + 1) * M * ldk;
#pragma unroll
      for (int j = 0; j < M; ++j) nxt[j] = en[j * ldk];
    }
    step<Model, INTEG>(x, v, comp, p);
    bool hit;
    const float l = Cost::template running<N, M>(x, comp, v, t, p, lds, cs, hit);
    if constexpr (COUNT) ncrash += hit ? 1 : 0;
    const float y = l - sum_c;
    const float s = sum + y;
    sum_c = (s - sum) - y;
    sum = s;
  }
  sum = sum + (terminal_cost<Cost, N>(x, T, p, lds, cs) - sum_c);
  S[k] = __builtin_isfinite(sum) ? sum : __builtin_inff();
  if constexpr (COUNT) crashes[k] = ncrash;
}

namespace {

using RolloutFn = void (*)(DevParams, const float*, const float*, const float*, int64_t, int,
                           int, float*, int32_t*);

template <class Model, int INTEG, class Cost>
RolloutFn pick(bool count) {
  if (count) return rollout_kernel<Model, INTEG, Cost, true>;
  return rollout_kernel<Model, INTEG, Cost, false>;
}

// costs defined for every model, and those that need the bicycle's layout
// (px, py, yaw, speed, ...) or the quadrotor's
template <class Model, int INTEG>
RolloutFn pick_generic(uint32_t cost, bool count) {
  if (cost == MPPI_COST_QUADRATIC) return pick<Model, INTEG, CostQuadratic>(count);
  if (cost == MPPI_COST_TRACK) return pick<Model, INTEG, CostTrack>(count);
  return nullptr;
}

template <class Model, int INTEG>
RolloutFn pick_wheeled(uint32_t cost, bool count) {
  switch (cost) {
    case MPPI_COST_PATH_CIRCLES: return pick<Model, INTEG, CostPath<true>>(count);
    case MPPI_COST_PATH_COSTMAP: return pick<Model, INTEG, CostPath<false>>(count);
    case MPPI_COST_GOAL_CIRCLES: return pick<Model, INTEG, CostGoalCircles>(count);
    default: return pick_generic<Model, INTEG>(cost, count);
  }
}

template <int INTEG>
RolloutFn pick_model(uint32_t dynamics, uint32_t cost, bool accurate, bool count) {
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

RolloutFn select(uint32_t dynamics, uint32_t integ, uint32_t cost, bool accurate, bool count) {
  if (integ == MPPI_INT_EULER) return pick_model<kEuler>(dynamics, cost, accurate, count);
  if (integ == MPPI_INT_RK4) return pick_model<kRK4>(dynamics, cost, accurate, count);
  return nullptr;
}

bool uses_stage(uint32_t cost) {
  return cost == MPPI_COST_PATH_CIRCLES || cost == MPPI_COST_PATH_COSTMAP ||
         cost == MPPI_COST_GOAL_CIRCLES;
}

int Model_m(uint32_t dynamics) { return dynamics == MPPI_DYN_QUADROTOR ? 4 : 2; }

}  // namespace

size_t rollout_lds_bytes(uint32_t dynamics, uint32_t cost, int stage_words4, int T) {
  return (uses_stage(cost) ? sizeof(float4) * static_cast<size_t>(stage_words4) : 0) +
         sizeof(float) * static_cast<size_t>(T) * Model_m(dynamics);
}

bool rollout_supported(uint32_t dynamics, uint32_t integrator, uint32_t cost) {
  return select(dynamics, integrator, cost, false, false) != nullptr;
}

hipError_t launch_rollout(uint32_t dynamics, uint32_t integrator, uint32_t cost,
                          bool accurate_trig, const DevParams& p, const float* d_x0,
                          const float* d_u, const float* d_eps, int64_t ldk, int K, int T,
                          float* d_S, int32_t* d_crashes, hipStream_t stream) {
  RolloutFn fn = select(dynamics, integrator, cost, accurate_trig, d_crashes != nullptr);
  if (!fn) return hipErrorInvalidValue;
  const size_t lds = (uses_stage(cost) ? sizeof(float4) * static_cast<size_t>(p.stage_words4) : 0) +
                     sizeof(float) * static_cast<size_t>(T) * Model_m(dynamics);
  if (lds > 48 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       static_cast<int>(lds));
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(fn, dim3((K + kRolloutBlock - 1) / kRolloutBlock), dim3(kRolloutBlock), lds,
                     stream, p, d_x0, d_u, d_eps, ldk, K, T, d_S, d_crashes);
  return hipGetLastError();
}

}  // namespace mppi
