// Step (a2): fused rollout + cost.  One lane per sample keeps the state in
// registers for the whole horizon; per step it reads its noise (coalesced:
// lanes are consecutive samples of one [T*m][ldk] row), forms v = u_t + eps,
// advances the dynamics and adds the running cost with compensated (Kahan)
// summation; the terminal cost closes the sum.  u_t and every cost constant
// are wave-uniform and arrive through scalar loads.  The noise of step t+1 is
// requested before step t is computed so that its HBM latency overlaps the
// arithmetic.
#include "common.h"
#include "costs.h"
#include "dynamics.h"

namespace mppi {

template <class Model, int INTEG, class Cost, bool COUNT>
__global__ __launch_bounds__(64) void rollout_kernel(DevParams p, const float* __restrict__ x0,
                                                     const float* __restrict__ u,
                                                     const float* __restrict__ eps, int64_t ldk,
                                                     int K, int T, float* __restrict__ S,
                                                     int32_t* __restrict__ crashes) {
  constexpr int N = Model::N, M = Model::M;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  float x[N];
#pragma unroll
  for (int i = 0; i < N; ++i) x[i] = x0[i];
  const float* e = eps + k;
  float nxt[M];
#pragma unroll
  for (int j = 0; j < M; ++j) nxt[j] = e[j * ldk];
  float sum = 0.0f, comp = 0.0f;
  int ncrash = 0;
  for (int t = 0; t < T; ++t) {
    float v[M];
#pragma unroll
    for (int j = 0; j < M; ++j) v[j] = u[t * M + j] + nxt[j];
    if (t + 1 < T) {
      const float* en = e + static_cast<int64_t>(t + 1) * M * ldk;
#pragma unroll
      for (int j = 0; j < M; ++j) nxt[j] = en[j * ldk];
    }
    step<Model, INTEG>(x, v, p);
    bool hit;
    const float l = Cost::template running<N, M>(x, v, t, p, hit);
    if constexpr (COUNT) ncrash += hit ? 1 : 0;
    const float y = l - comp;
    const float s = sum + y;
    comp = (s - sum) - y;
    sum = s;
  }
  {
    const float y = terminal_cost<Cost, N>(x, T, p) - comp;
    sum = sum + y;
  }
  S[k] = __builtin_isfinite(sum) ? sum : __builtin_inff();
  if constexpr (COUNT) crashes[k] = ncrash;
}

namespace {

using RolloutFn = void (*)(DevParams, const float*, const float*, const float*, int64_t, int,
                           int, float*, int32_t*);

template <class Model, int INTEG, class Cost>
RolloutFn pick(bool count) {
  return count ? rollout_kernel<Model, INTEG, Cost, true> : rollout_kernel<Model, INTEG, Cost, false>;
}

template <class Model, int INTEG>
RolloutFn pick_cost(uint32_t cost, bool count, bool wheeled, bool quad) {
  switch (cost) {
    case MPPI_COST_QUADRATIC: return pick<Model, INTEG, CostQuadratic>(count);
    case MPPI_COST_TRACK: return pick<Model, INTEG, CostTrack>(count);
    case MPPI_COST_PATH_CIRCLES:
      return wheeled ? pick<Model, INTEG, CostPath<true>>(count) : nullptr;
    case MPPI_COST_PATH_COSTMAP:
      return wheeled ? pick<Model, INTEG, CostPath<false>>(count) : nullptr;
    case MPPI_COST_GOAL_CIRCLES:
      return wheeled ? pick<Model, INTEG, CostGoalCircles>(count) : nullptr;
    case MPPI_COST_HOVER: return quad ? pick<Model, INTEG, CostHover>(count) : nullptr;
    default: return nullptr;
  }
}

template <class Model>
RolloutFn pick_integrator(uint32_t integ, uint32_t cost, bool count, bool wheeled, bool quad) {
  if (integ == MPPI_INT_EULER) return pick_cost<Model, kEuler>(cost, count, wheeled, quad);
  if (integ == MPPI_INT_RK4) return pick_cost<Model, kRK4>(cost, count, wheeled, quad);
  return nullptr;
}

RolloutFn select(uint32_t dynamics, uint32_t integ, uint32_t cost, bool count) {
  switch (dynamics) {
    case MPPI_DYN_DOUBLE_INTEGRATOR:
      return pick_integrator<DoubleIntegrator>(integ, cost, count, false, false);
    case MPPI_DYN_BICYCLE:
      return pick_integrator<Bicycle>(integ, cost, count, true, false);
    case MPPI_DYN_QUADROTOR:
      return pick_integrator<Quadrotor>(integ, cost, count, false, true);
    default:
      return nullptr;
  }
}

}  // namespace

bool rollout_supported(uint32_t dynamics, uint32_t integrator, uint32_t cost) {
  return select(dynamics, integrator, cost, false) != nullptr;
}

hipError_t launch_rollout(uint32_t dynamics, uint32_t integrator, uint32_t cost,
                          const DevParams& p, const float* d_x0, const float* d_u,
                          const float* d_eps, int64_t ldk, int K, int T, float* d_S,
                          int32_t* d_crashes, hipStream_t stream) {
  RolloutFn fn = select(dynamics, integrator, cost, d_crashes != nullptr);
  if (!fn) return hipErrorInvalidValue;
  constexpr int kBlock = 64;
  hipLaunchKernelGGL(fn, dim3((K + kBlock - 1) / kBlock), dim3(kBlock), 0, stream, p, d_x0, d_u,
                     d_eps, ldk, K, T, d_S, d_crashes);
  return hipGetLastError();
}

}  // namespace mppi
