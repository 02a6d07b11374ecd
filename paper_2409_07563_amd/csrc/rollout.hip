// Step (a2) for one instance: the fused rollout + cost kernels (one lane per
// sample, or 4 / 8 / 16 lanes per sample for the bicycle with RK4) and the
// choice between them.  The per-lane body lives in rollout.h.  u, the obstacle grid
// and the spline are staged once per workgroup into LDS, so no step waits on
// a scalar or global load of them; the noise is requested a few steps ahead
// of its use (NoiseAhead) so that its memory latency overlaps the arithmetic.
#include "noise.h"
#include "quad.h"
#include "rollout.h"

namespace mppi {

// Workgroup size: a launch parameter (64, 128 or 256 threads; the autotuner
// picks it), so the kernels are compiled for the largest.
constexpr int kRolloutMaxBlock = 256;

template <class Model, int INTEG, class Cost, bool COUNT>
__global__ __launch_bounds__(kRolloutMaxBlock) void rollout_kernel(
    DevParams p, const float* __restrict__ x0, const float* __restrict__ u,
    const float* __restrict__ eps, int64_t ldk, int K, int T, float* __restrict__ S,
    int32_t* __restrict__ crashes, int rblocks, NoiseJob job) {
  if (static_cast<int>(blockIdx.x) >= rblocks) {  // the next iteration's noise
    next_noise(job, blockIdx.x - rblocks);
    return;
  }
  extern __shared__ float4 lds[];
  const float* lds_u = stage_rollout_lds<Cost>(p, u, T * Model::M, lds);
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;  // no barrier follows
  const RolloutResult r =
      rollout_lane<Model, INTEG, Cost, COUNT>(p, x0, lds_u, eps + k, ldk, T, lds, k < p.n_plain);
  S[k] = r.cost;
  if constexpr (COUNT) crashes[k] = r.crashes;
}

// ---------------------------------------------------------------------------
// Bicycle + RK4 with L = 4, 8 or 16 lanes per sample, the MI355X form of the
// paper's intra-sample thread axis (Sec. III-C).  Within each DPP quad, lane
// j = lane mod 4 evaluates RK4 stage j (bicycle_quad_step, quad.h); every
// lane ends with bitwise the same state.  With L > 4 the quads of a sample repeat the
// same dynamics and exist to share the running cost: lane s = lane mod L
// latches the steps t = s (mod L), and every L steps all L lanes evaluate
// their latched step at once, so the cost (the LDS-latency-bound spline and
// obstacle lookups) is amortised L ways and the sample count K fills L times
// as many waves.  Each lane keeps a compensated partial sum, summed over the
// L lanes in a fixed butterfly order at the end.
//
// The step loop runs through noise_steps (the noise of step t + 8 requested
// into the register slot step t has just used), and the latch is a select, so
// the steps between two cost evaluations are straight-line code.
// ---------------------------------------------------------------------------
// sum over the L lanes of a sample (every lane gets the same value)
template <int L>
__device__ __forceinline__ float group_sum(float v) {
  v = quad_sum(v);
  if constexpr (L >= 8) v += __shfl_xor(v, 4, kWave);
  if constexpr (L >= 16) v += __shfl_xor(v, 8, kWave);
  return v;
}
template <int L>
__device__ __forceinline__ int group_sum_int(int c) {
  c += __builtin_amdgcn_update_dpp(0, c, kQuadSwap1, 0xF, 0xF, false);
  c += __builtin_amdgcn_update_dpp(0, c, kQuadSwap2, 0xF, 0xF, false);
  if constexpr (L >= 8) c += __shfl_xor(c, 4, kWave);
  if constexpr (L >= 16) c += __shfl_xor(c, 8, kWave);
  return c;
}

template <class Cost, bool FAST, bool COUNT, int L>
__global__ __launch_bounds__(kRolloutMaxBlock) void rollout_bicycle_group_kernel(
    DevParams p, const float* __restrict__ x0, const float* __restrict__ u,
    const float* __restrict__ eps, int64_t ldk, int K, int T, float* __restrict__ S,
    int32_t* __restrict__ crashes, int rblocks, NoiseJob job) {
  static_assert(L == 4 || L == 8 || L == 16, "lanes per sample");
  if (static_cast<int>(blockIdx.x) >= rblocks) {  // the next iteration's noise
    next_noise(job, blockIdx.x - rblocks);
    return;
  }
  constexpr int N = 5, M = 2;
  extern __shared__ float4 lds[];
  const float* lds_u = stage_rollout_lds<Cost>(p, u, T * M, lds);
  const int gl = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = gl & 3;           // RK4 stage
  const int slot = gl & (L - 1);  // latches the steps t = slot (mod L)
  const int k = gl / L;
  if (k >= K) return;  // whole groups leave together; no barrier follows
  const float mean = k < p.n_plain ? 1.0f : 0.0f;  // drawn around u, or around zero
  // stage coefficient c_j dt (0, dt/2, dt/2, dt) and RK4 weight (1, 2, 2, 1)
  const float cdt = j == 0 ? 0.0f : (j == 3 ? p.dt : p.half_dt);
  const float wj = (j == 1 || j == 2) ? 2.0f : 1.0f;
  float x[N], comp[N];
#pragma unroll
  for (int i = 0; i < N; ++i) { x[i] = x0[i]; comp[i] = 0.0f; }
  // the step this lane evaluates the running cost of
  float lx[N] = {}, lc[N] = {}, lv[M] = {};
  int lt = -1;
  typename Cost::State cs;
  Cost::init(cs, x, p, lds);
  float sum = 0.0f, sum_c = 0.0f;
  int ncrash = 0;
  auto evaluate = [&]() {
    bool hit;
    float l = Cost::template running<N, M>(lx, lc, lv, lt, p, lds, cs, hit);
    if (p.importance && mean != 0.0f) l += is_term<M>(p, lt, lv, lds_u + lt * M);
    if (p.cosines) l += inflation(p);
    if constexpr (COUNT) ncrash += hit ? 1 : 0;
    const float y = l - sum_c;
    const float s = sum + y;
    sum_c = (s - sum) - y;
    sum = s;
  };
  noise_steps<M, 8>(eps + k, ldk, T, [&](int t, const float* nz, int d) {
    float v[M];
#pragma unroll
    for (int c = 0; c < M; ++c) v[c] = mean * lds_u[t * M + c] + nz[c];
    bicycle_quad_step<FAST>(x, comp, v, j, cdt, wj, p);
    // latch this step for lane t mod L (selects, no branch) ...
    const bool mine = (t & (L - 1)) == slot;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      lx[i] = mine ? x[i] : lx[i];
      lc[i] = mine ? comp[i] : lc[i];
    }
#pragma unroll
    for (int c = 0; c < M; ++c) lv[c] = mine ? v[c] : lv[c];
    lt = mine ? t : lt;
    // ... and evaluate a full group every L steps (the step blocks start at
    // multiples of 8, so for L <= 8 the positions are fixed by d)
    const bool full = L <= 8 ? (d & (L - 1)) == L - 1 : (t & (L - 1)) == L - 1;
    if (full) {
      evaluate();
      lt = -1;
    }
  });
  if (lt >= 0) evaluate();  // the last, incomplete group of steps
  // terminal cost once per sample (slot 0), then the group's partial sums
  const float phi = terminal_cost<Cost, N>(x, T, p, lds, cs);
  if (slot == 0) {
    const float y = phi - sum_c;
    const float s = sum + y;
    sum_c = (s - sum) - y;
    sum = s;
  }
  const float total = group_sum<L>(sum - sum_c);
  if (slot == 0) S[k] = __builtin_isfinite(total) ? total : __builtin_inff();
  if constexpr (COUNT) {
    const int c = group_sum_int<L>(ncrash);
    if (slot == 0) crashes[k] = c;
  }
}

namespace {

using RolloutFn = void (*)(DevParams, const float*, const float*, const float*, int64_t, int,
                           int, float*, int32_t*, int, NoiseJob);

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

template <class Cost, bool FAST, int L>
RolloutFn pick_group(bool count) {
  if (count) return rollout_bicycle_group_kernel<Cost, FAST, true, L>;
  return rollout_bicycle_group_kernel<Cost, FAST, false, L>;
}

template <class Cost, bool FAST>
RolloutFn pick_group_lanes(int lanes, bool count) {
  switch (lanes) {
    case 4: return pick_group<Cost, FAST, 4>(count);
    case 8: return pick_group<Cost, FAST, 8>(count);
    case 16: return pick_group<Cost, FAST, 16>(count);
    default: return nullptr;
  }
}

template <bool FAST>
RolloutFn pick_group_cost(uint32_t cost, int lanes, bool count) {
  switch (cost) {
    case MPPI_COST_PATH_CIRCLES: return pick_group_lanes<CostPath<true>, FAST>(lanes, count);
    case MPPI_COST_PATH_COSTMAP: return pick_group_lanes<CostPath<false>, FAST>(lanes, count);
    case MPPI_COST_GOAL_CIRCLES: return pick_group_lanes<CostGoalCircles, FAST>(lanes, count);
    case MPPI_COST_QUADRATIC: return pick_group_lanes<CostQuadratic, FAST>(lanes, count);
    case MPPI_COST_TRACK: return pick_group_lanes<CostTrack, FAST>(lanes, count);
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

bool rollout_quad_available(uint32_t dynamics, uint32_t integrator) {
  return dynamics == MPPI_DYN_BICYCLE && integrator == MPPI_INT_RK4;
}

hipError_t launch_rollout(uint32_t dynamics, uint32_t integrator, uint32_t cost,
                          bool accurate_trig, int lanes, const DevParams& p, const float* d_x0,
                          const float* d_u, const float* d_eps, int64_t ldk, int K, int T,
                          float* d_S, int32_t* d_crashes, hipStream_t stream, int block,
                          const NoiseJob* next) {
  if (block != 64 && block != 128 && block != 256) return hipErrorInvalidValue;
  const bool count = d_crashes != nullptr;
  const bool group = lanes > 1;
  if (group && !rollout_quad_available(dynamics, integrator)) return hipErrorInvalidValue;
  RolloutFn fn = group ? (accurate_trig ? pick_group_cost<false>(cost, lanes, count)
                                        : pick_group_cost<true>(cost, lanes, count))
                       : select(dynamics, integrator, cost, accurate_trig, count);
  if (!fn) return hipErrorInvalidValue;
  const int lanes_per_sample = group ? lanes : 1;
  const size_t lds = (uses_stage(cost) ? sizeof(float4) * static_cast<size_t>(p.stage_words4) : 0) +
                     sizeof(float) * static_cast<size_t>(T) * Model_m(dynamics);
  if (lds > 48 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       static_cast<int>(lds));
    if (e != hipSuccess) return e;
  }
  const int64_t threads = static_cast<int64_t>(K) * lanes_per_sample;
  const int rblocks = static_cast<int>((threads + block - 1) / block);
  NoiseJob job{};
  int blocks = rblocks;
  if (next) {
    job = *next;
    blocks += noise_job_blocks(&job, block);
  }
  hipLaunchKernelGGL(fn, dim3(static_cast<unsigned>(blocks)), dim3(block), lds, stream, p, d_x0,
                     d_u, d_eps, ldk, K, T, d_S, d_crashes, rblocks, job);
  return hipGetLastError();
}

}  // namespace mppi
