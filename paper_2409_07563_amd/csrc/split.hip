// Step (a2) in the split form (arXiv 2409.07563, section "Split Kernel
// Description"): the dynamics run in one kernel, which writes every sample's
// states to a trajectory buffer, and the running costs in a second kernel
// that is parallel over time, because the cost of a step needs only that
// step's state and control.  The fused kernels (rollout.hip) keep the states
// in registers but evaluate the costs sequentially in time; the split form
// pays two passes over the trajectory buffer (it stays in the last-level
// cache at the sizes of interest) to evaluate the costs with T times the
// parallelism, which wins when the cost is expensive (the cost-complexity
// load of the Results section).  The autotuner times both forms.
//
// Trajectory layout: traj[t][c][ldk] (k fastest, coalesced for both kernels),
// c < NY: the post-step state x_{t+1} (N components) and, for the costmap
// cost (NY = N + 2), the compensation terms of the position, which that
// cost's interpolation reads.
#include "quad.h"
#include "rollout.h"

namespace mppi {

constexpr int kSplitMaxBlock = 256;

// ---- dynamics: one lane per sample -----------------------------------------
template <class Model, int INTEG, int NY>
__global__ __launch_bounds__(kSplitMaxBlock) void split_dynamics_kernel(
    DevParams p, const float* __restrict__ x0, const float* __restrict__ u,
    const float* __restrict__ eps, int64_t ldk, int K, int T, float* __restrict__ traj) {
  constexpr int N = Model::N, M = Model::M;
  static_assert(NY == N || NY == N + 2, "trajectory words");
  extern __shared__ float4 lds[];
  const float* lds_u = stage_rollout_lds<CostQuadratic>(p, u, T * M, lds);  // u only
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;  // no barrier follows
  const float mean = k < p.n_plain ? 1.0f : 0.0f;  // drawn around u, or around zero
  float x[N], comp[N];
#pragma unroll
  for (int i = 0; i < N; ++i) { x[i] = x0[i]; comp[i] = 0.0f; }
  float* y = traj + k;
  noise_steps<M, 8>(eps + k, ldk, T, [&](int t, const float* n, int) {
    float v[M];
#pragma unroll
    for (int j = 0; j < M; ++j) v[j] = mean * lds_u[t * M + j] + n[j];
    step<Model, INTEG>(x, v, comp, p);
    float* yt = y + static_cast<int64_t>(t) * NY * ldk;
#pragma unroll
    for (int i = 0; i < N; ++i) yt[i * ldk] = x[i];
    if constexpr (NY > N) {
      yt[N * ldk] = comp[0];
      yt[(N + 1) * ldk] = comp[1];
    }
  });
}

// ---- dynamics: the bicycle with RK4, four lanes per sample -------------------
// The quad's lanes hold the same state after each step; lane j stores
// component j, and a second value: lane 0 the steer, lanes 1 and 2 the
// compensation terms (costmap), the others their component again (the same
// value to the same address), so both stores are unconditional.
template <bool FAST, int NY>
__global__ __launch_bounds__(kSplitMaxBlock) void split_bicycle_quad_kernel(
    DevParams p, const float* __restrict__ x0, const float* __restrict__ u,
    const float* __restrict__ eps, int64_t ldk, int K, int T, float* __restrict__ traj) {
  constexpr int N = 5, M = 2;
  extern __shared__ float4 lds[];
  const float* lds_u = stage_rollout_lds<CostQuadratic>(p, u, T * M, lds);
  const int gl = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = gl & 3;
  const int k = gl >> 2;
  if (k >= K) return;  // whole quads leave together; no barrier follows
  const float mean = k < p.n_plain ? 1.0f : 0.0f;  // drawn around u, or around zero
  const float cdt = j == 0 ? 0.0f : (j == 3 ? p.dt : p.half_dt);
  const float wj = (j == 1 || j == 2) ? 2.0f : 1.0f;
  float x[N], comp[N];
#pragma unroll
  for (int i = 0; i < N; ++i) { x[i] = x0[i]; comp[i] = 0.0f; }
  const int row2 = j == 0 ? 4 : (NY > N && j == 1 ? 5 : (NY > N && j == 2 ? 6 : j));
  float* y = traj + k;
  noise_steps<M, 8>(eps + k, ldk, T, [&](int t, const float* n, int) {
    float v[M];
#pragma unroll
    for (int c = 0; c < M; ++c) v[c] = mean * lds_u[t * M + c] + n[c];
    bicycle_quad_step<FAST>(x, comp, v, j, cdt, wj, p);
    // selects, not branches
    float own = x[0];
    own = j == 1 ? x[1] : own;
    own = j == 2 ? x[2] : own;
    own = j == 3 ? x[3] : own;
    float second = j == 0 ? x[4] : own;
    if constexpr (NY > N) {
      second = j == 1 ? comp[0] : second;
      second = j == 2 ? comp[1] : second;
    }
    float* yt = y + static_cast<int64_t>(t) * NY * ldk;
    yt[j * ldk] = own;
    yt[row2 * ldk] = second;
  });
}

// ---- costs: parallel over time -----------------------------------------------
// The steps of 64 consecutive samples (lane = sample) are shared by G waves:
// W waves per workgroup (blockDim.x = 64 W) times C workgroups (gridDim.y).
// Wave g = c W + w evaluates the steps t = g, g + G, ... of its lane's
// sample, with the next step's loads issued before the current step's cost,
// and keeps a compensated partial sum.  Wave 0 of a workgroup adds the W
// partials in wave order (chunk 0 also the terminal cost); with C = 1 that is
// the cost, otherwise it goes to part[c][ldk] and split_sum_kernel adds the C
// chunks in chunk order.  The cost data and u are staged in LDS as in the
// fused kernels.
template <int N, int M, int NY, class Cost, bool COUNT>
__global__ __launch_bounds__(kWave * kSplitMaxWaves) void split_cost_kernel(
    DevParams p, const float* __restrict__ u, const float* __restrict__ eps, int64_t ldk, int K,
    int T, const float* __restrict__ traj, float* __restrict__ S, int32_t* __restrict__ crashes,
    float* __restrict__ part_sum, int32_t* __restrict__ part_hits) {
  extern __shared__ float4 lds[];
  __shared__ float part[kSplitMaxWaves][kWave];
  __shared__ int hits[kSplitMaxWaves][kWave];
  const float* lds_u = stage_rollout_lds<Cost>(p, u, T * M, lds);
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  const int W = blockDim.x / kWave;
  const int C = gridDim.y, c = blockIdx.y;
  const int G = C * W, g = c * W + w;
  const int k = blockIdx.x * kWave + lane;
  const bool live = k < K;
  const bool plain = k < p.n_plain;  // drawn around u (else around zero)
  const float mean = plain ? 1.0f : 0.0f;
  typename Cost::State cs;
  {
    const float xz[N] = {};
    Cost::init(cs, xz, p, lds);
  }
  float sum = 0.0f, sum_c = 0.0f;
  int nh = 0;
  if (live && g < T) {
    float yn[NY], en[M];
    auto fetch = [&](int t) {
      const float* y = traj + static_cast<int64_t>(t) * NY * ldk + k;
#pragma unroll
      for (int q = 0; q < NY; ++q) yn[q] = y[q * ldk];
      const float* e = eps + static_cast<int64_t>(t) * M * ldk + k;
#pragma unroll
      for (int j = 0; j < M; ++j) en[j] = e[j * ldk];
    };
    fetch(g);
    for (int t = g; t < T; t += G) {
      float x[N], comp[N], v[M];
#pragma unroll
      for (int i = 0; i < N; ++i) { x[i] = yn[i]; comp[i] = 0.0f; }
      if constexpr (NY > N) {
        comp[0] = yn[N];
        comp[1] = yn[N + 1];
      }
#pragma unroll
      for (int j = 0; j < M; ++j) v[j] = mean * lds_u[t * M + j] + en[j];
      if (t + G < T) fetch(t + G);
      bool hit;
      float l = Cost::template running<N, M>(x, comp, v, t, p, lds, cs, hit);
      if (p.importance && plain) l += is_term<M>(p, t, v, lds_u + t * M);
      if (p.cosines) l += inflation(p);
      if constexpr (COUNT) nh += hit ? 1 : 0;
      const float yk = l - sum_c;
      const float s = sum + yk;
      sum_c = (s - sum) - yk;
      sum = s;
    }
  }
  part[w][lane] = sum - sum_c;
  if constexpr (COUNT) hits[w][lane] = nh;
  __syncthreads();
  if (w != 0 || !live) return;  // no barrier follows
  float tot = 0.0f, tc = 0.0f;
  for (int i = 0; i < W; ++i) {
    const float yk = part[i][lane] - tc;
    const float s = tot + yk;
    tc = (s - tot) - yk;
    tot = s;
  }
  if (c == 0) {
    float xT[N];
    const float* y = traj + static_cast<int64_t>(T - 1) * NY * ldk + k;
#pragma unroll
    for (int i = 0; i < N; ++i) xT[i] = y[i * ldk];
    tot = tot + (terminal_cost<Cost, N>(xT, T, p, lds, cs) - tc);
  } else {
    tot = tot - tc;
  }
  int n = 0;
  if constexpr (COUNT)
    for (int i = 0; i < W; ++i) n += hits[i][lane];
  if (C == 1) {
    S[k] = __builtin_isfinite(tot) ? tot : __builtin_inff();
    if constexpr (COUNT) crashes[k] = n;
  } else {
    part_sum[static_cast<int64_t>(c) * ldk + k] = tot;
    if constexpr (COUNT) part_hits[static_cast<int64_t>(c) * ldk + k] = n;
  }
}

// S[k] = sum of the C chunk partials in chunk order (compensated).
__global__ __launch_bounds__(256) void split_sum_kernel(const float* __restrict__ part_sum,
                                                        const int32_t* __restrict__ part_hits,
                                                        int C, int64_t ldk, int K,
                                                        float* __restrict__ S,
                                                        int32_t* __restrict__ crashes) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  float tot = 0.0f, tc = 0.0f;
  int n = 0;
  for (int c = 0; c < C; ++c) {
    const float yk = part_sum[static_cast<int64_t>(c) * ldk + k] - tc;
    const float s = tot + yk;
    tc = (s - tot) - yk;
    tot = s;
    if (crashes) n += part_hits[static_cast<int64_t>(c) * ldk + k];
  }
  tot = tot - tc;
  S[k] = __builtin_isfinite(tot) ? tot : __builtin_inff();
  if (crashes) crashes[k] = n;
}

namespace {

using DynFn = void (*)(DevParams, const float*, const float*, const float*, int64_t, int, int,
                       float*);
using CostFn = void (*)(DevParams, const float*, const float*, int64_t, int, int, const float*,
                        float*, int32_t*, float*, int32_t*);

bool is_costmap(uint32_t cost) { return cost == MPPI_COST_PATH_COSTMAP; }

template <class Model, int INTEG>
DynFn dyn_words(bool costmap) {
  if (costmap) return split_dynamics_kernel<Model, INTEG, Model::N + 2>;
  return split_dynamics_kernel<Model, INTEG, Model::N>;
}

template <int INTEG>
DynFn dyn_model(uint32_t dynamics, bool accurate, bool costmap) {
  switch (dynamics) {
    case MPPI_DYN_DOUBLE_INTEGRATOR: return dyn_words<DoubleIntegrator, INTEG>(false);
    case MPPI_DYN_BICYCLE:
      return accurate ? dyn_words<Bicycle<false>, INTEG>(costmap)
                      : dyn_words<Bicycle<true>, INTEG>(costmap);
    case MPPI_DYN_QUADROTOR: return dyn_words<Quadrotor, INTEG>(false);
    default: return nullptr;
  }
}

DynFn select_dyn(uint32_t dynamics, uint32_t integ, uint32_t cost, bool accurate, int lanes) {
  const bool costmap = is_costmap(cost);
  if (lanes == 4) {
    if (dynamics != MPPI_DYN_BICYCLE || integ != MPPI_INT_RK4) return nullptr;
    if (accurate)
      return costmap ? split_bicycle_quad_kernel<false, 7> : split_bicycle_quad_kernel<false, 5>;
    return costmap ? split_bicycle_quad_kernel<true, 7> : split_bicycle_quad_kernel<true, 5>;
  }
  if (lanes != 1) return nullptr;
  if (integ == MPPI_INT_EULER) return dyn_model<kEuler>(dynamics, accurate, costmap);
  if (integ == MPPI_INT_RK4) return dyn_model<kRK4>(dynamics, accurate, costmap);
  return nullptr;
}

template <int N, int M, int NY, class Cost>
CostFn cost_fn(bool count) {
  if (count) return split_cost_kernel<N, M, NY, Cost, true>;
  return split_cost_kernel<N, M, NY, Cost, false>;
}

template <int N, int M>
CostFn cost_generic(uint32_t cost, bool count) {
  if (cost == MPPI_COST_QUADRATIC) return cost_fn<N, M, N, CostQuadratic>(count);
  if (cost == MPPI_COST_TRACK) return cost_fn<N, M, N, CostTrack>(count);
  return nullptr;
}

CostFn select_cost(uint32_t dynamics, uint32_t cost, bool count) {
  switch (dynamics) {
    case MPPI_DYN_DOUBLE_INTEGRATOR: return cost_generic<4, 2>(cost, count);
    case MPPI_DYN_BICYCLE:
      switch (cost) {
        case MPPI_COST_PATH_CIRCLES: return cost_fn<5, 2, 5, CostPath<true>>(count);
        case MPPI_COST_PATH_COSTMAP: return cost_fn<5, 2, 7, CostPath<false>>(count);
        case MPPI_COST_GOAL_CIRCLES: return cost_fn<5, 2, 5, CostGoalCircles>(count);
        default: return cost_generic<5, 2>(cost, count);
      }
    case MPPI_DYN_QUADROTOR:
      if (cost == MPPI_COST_HOVER) return cost_fn<13, 4, 13, CostHover>(count);
      return cost_generic<13, 4>(cost, count);
    default: return nullptr;
  }
}

hipError_t allow_lds(const void* fn, size_t lds) {
  if (lds <= 48 * 1024) return hipSuccess;
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                             static_cast<int>(lds));
}

}  // namespace

bool rollout_split_supported(uint32_t dynamics, uint32_t integrator, uint32_t cost) {
  return select_dyn(dynamics, integrator, cost, false, 1) != nullptr &&
         select_cost(dynamics, cost, false) != nullptr;
}

int split_traj_words(uint32_t dynamics, uint32_t cost) {
  const int n = dynamics == MPPI_DYN_QUADROTOR ? 13 : (dynamics == MPPI_DYN_DOUBLE_INTEGRATOR ? 4 : 5);
  return n + (is_costmap(cost) ? 2 : 0);
}

hipError_t launch_rollout_split(uint32_t dynamics, uint32_t integrator, uint32_t cost,
                                bool accurate_trig, int lanes, const DevParams& p,
                                const float* d_x0, const float* d_u, const float* d_eps,
                                int64_t ldk, int K, int T, float* d_traj, float* d_part,
                                float* d_S, int32_t* d_crashes, hipStream_t stream, int block,
                                int waves) {
  if (block != 64 && block != 128 && block != 256) return hipErrorInvalidValue;
  if (waves < 1 || waves > kSplitMaxWaves * kSplitMaxChunks || (waves & (waves - 1)))
    return hipErrorInvalidValue;
  const int W = waves < kSplitMaxWaves ? waves : kSplitMaxWaves;
  const int C = waves / W;
  const bool count = d_crashes != nullptr;
  DynFn dyn = select_dyn(dynamics, integrator, cost, accurate_trig, lanes);
  CostFn cfn = select_cost(dynamics, cost, count);
  if (!dyn || !cfn) return hipErrorInvalidValue;
  const int M = dynamics == MPPI_DYN_QUADROTOR ? 4 : 2;
  const size_t u_bytes = sizeof(float) * static_cast<size_t>(T) * M;
  hipError_t e = allow_lds(reinterpret_cast<const void*>(dyn), u_bytes);
  if (e != hipSuccess) return e;
  const int64_t threads = static_cast<int64_t>(K) * lanes;
  hipLaunchKernelGGL(dyn, dim3(static_cast<unsigned>((threads + block - 1) / block)), dim3(block),
                     u_bytes, stream, p, d_x0, d_u, d_eps, ldk, K, T, d_traj);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t lds = rollout_lds_bytes(dynamics, cost, p.stage_words4, T);
  e = allow_lds(reinterpret_cast<const void*>(cfn), lds);
  if (e != hipSuccess) return e;
  float* part_sum = d_part;
  int32_t* part_hits = reinterpret_cast<int32_t*>(d_part + kSplitMaxChunks * ldk);
  hipLaunchKernelGGL(cfn, dim3(static_cast<unsigned>((K + kWave - 1) / kWave), C),
                     dim3(kWave * W), lds, stream, p, d_u, d_eps, ldk, K, T, d_traj, d_S,
                     d_crashes, part_sum, part_hits);
  e = hipGetLastError();
  if (e != hipSuccess || C == 1) return e;
  hipLaunchKernelGGL(split_sum_kernel, dim3(static_cast<unsigned>((K + 255) / 256)), dim3(256), 0,
                     stream, part_sum, part_hits, C, ldk, K, d_S, d_crashes);
  return hipGetLastError();
}

}  // namespace mppi
