// Device bodies of the fused rollout + cost (step a2), shared by the
// single-instance kernels (rollout.hip) and the batched kernels (batch.hip).
//
// One lane per sample keeps the state in registers for the whole horizon;
// per step it takes its noise (coalesced: lanes are consecutive samples of one
// [T*m][ldk] row; requested a few steps ahead), forms v = u_t + eps, advances
// the dynamics and adds the
// running cost with compensated (Kahan) summation; the terminal cost closes
// the sum.  u (all T steps) and the read-only cost data (obstacle grid,
// spline) are staged once per workgroup into LDS by stage_rollout_lds.
#pragma once

#include "common.h"
#include "costs.h"
#include "dynamics.h"

namespace mppi {

// LDS layout: [cost stage (float4 words, if the cost stages any)][u: T*M floats]
template <class Cost>
__device__ __forceinline__ float* stage_rollout_lds(const DevParams& p, const float* __restrict__ u,
                                                    int TM, float4* lds) {
  const int u_off4 = Cost::kStage ? p.stage_words4 : 0;
  float* lds_u = reinterpret_cast<float*>(lds + u_off4);
  if constexpr (Cost::kStage)
    for (int i = threadIdx.x; i < p.stage_words4; i += blockDim.x) lds[i] = p.stage[i];
  for (int i = threadIdx.x; i < TM; i += blockDim.x) lds_u[i] = u[i];
  __syncthreads();
  return lds_u;
}

// The noise of the next D steps of one sample, requested D steps before its
// use so that the L2 / HBM latency of a load (about a microsecond) overlaps
// several steps of arithmetic rather than one.  e points at eps[0][0][k];
// steps at or past T are never read.
template <int M, int D = 4>
struct NoiseAhead {
  float q[D][M];
  const float* e;
  int64_t ldk;
  int T;
  __device__ __forceinline__ void init(const float* e_, int64_t ldk_, int T_) {
    e = e_;
    ldk = ldk_;
    T = T_;
#pragma unroll
    for (int d = 0; d < D; ++d)
#pragma unroll
      for (int j = 0; j < M; ++j)
        q[d][j] = d < T ? e[static_cast<int64_t>(d * M + j) * ldk] : 0.0f;
  }
  // the noise of step t (the front of the ring), then the request of step t + D
  __device__ __forceinline__ void pop(int t, float* out) {
#pragma unroll
    for (int j = 0; j < M; ++j) out[j] = q[0][j];
#pragma unroll
    for (int d = 0; d + 1 < D; ++d)
#pragma unroll
      for (int j = 0; j < M; ++j) q[d][j] = q[d + 1][j];
    if (t + D < T) {
      const float* en = e + static_cast<int64_t>(t + D) * M * ldk;
#pragma unroll
      for (int j = 0; j < M; ++j) q[D - 1][j] = en[j * ldk];
    }
  }
};

// The importance-sampling term of step t (section "MPPI-Generic's MPPI
// Implementation", Eq. information_theoretic_weighting, beta = 1):
// lambda (v - u/2)' Sigma_t^-1 u with the coefficients lambda / sigma^2 of the
// step (per step with a sigma table).  Only for samples drawn around u: the
// term of a zero-mean sample is zero.
template <int M>
__device__ __forceinline__ float is_term(const DevParams& p, int t, const float* v,
                                         const float* u) {
  const float* cf = p.is_coef_t ? p.is_coef_t + t * M : p.is_coef;
  float s = 0.0f;
#pragma unroll
  for (int j = 0; j < M; ++j) s += (cf[j] * u[j]) * (v[j] - 0.5f * u[j]);
  return s;
}

// The cost-complexity load of the paper's Results section: p.cosines nested
// cosines of 1, scaled by zero, so it adds exactly +0 to a cost (the chain
// stays positive) and costs only time.
__device__ __forceinline__ float inflation(const DevParams& p) {
  float z = 1.0f;
  for (int i = 0; i < p.cosines; ++i) z = cosf(z);
  return 0.0f * z;
}

// Runs body(t, n, d) for t = 0 .. T-1, n the noise of step t (M floats) and
// d = t mod D.  The noise of step t + D is requested at step t into the
// register slot step t has just used: the slots are fixed (the step loop is
// unrolled by D) and rows past the horizon are clamped to row T - 1, so the
// unrolled body has no branch of its own and the wait for a step's noise
// comes D steps after its request (a rotating queue, by contrast, makes the
// compiler wait for the newest request at every step).  e points at
// eps[0][0][k].
template <int M, int D, class Body>
__device__ __forceinline__ void noise_steps(const float* __restrict__ e, int64_t ldk, int T,
                                            Body&& body) {
  float q[D][M];
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const int r = d < T ? d : T - 1;
#pragma unroll
    for (int c = 0; c < M; ++c) q[d][c] = e[static_cast<int64_t>(r * M + c) * ldk];
  }
  int t0 = 0;
  for (; t0 + D <= T; t0 += D) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      float n[M];
#pragma unroll
      for (int c = 0; c < M; ++c) n[c] = q[d][c];
      const int t = t0 + d;
      const int r = t + D < T ? t + D : T - 1;
#pragma unroll
      for (int c = 0; c < M; ++c) q[d][c] = e[static_cast<int64_t>(r * M + c) * ldk];
      body(t, n, d);
    }
  }
#pragma unroll
  for (int d = 0; d < D; ++d)
    if (t0 + d < T) body(t0 + d, q[d], d);
}

struct RolloutResult {
  float cost;
  int crashes;
};

// The state of one sample's rollout in one lane: the model state and its
// compensation, the cost's state and the compensated running-cost sum.
// step(t, n) takes the noise n of step t (M floats): v = mean u_t + n (an
// unconditional load of u and one FMA, exactly u + n for mean = 1, so no
// branch guards the load), one dynamics step, the running cost on the new
// state; finish(T) adds the terminal cost.
template <class Model, int INTEG, class Cost, bool COUNT>
struct LaneRollout {
  static constexpr int N = Model::N, M = Model::M;
  float x[N], comp[N];
  typename Cost::State cs;
  float sum, sum_c;
  int ncrash;
  float mean;
  bool plain;

  __device__ __forceinline__ LaneRollout(const DevParams& p, const float* __restrict__ x0,
                                         const float4* lds, bool plain_) {
#pragma unroll
    for (int i = 0; i < N; ++i) { x[i] = x0[i]; comp[i] = 0.0f; }
    Cost::init(cs, x, p, lds);
    sum = 0.0f;
    sum_c = 0.0f;
    ncrash = 0;
    plain = plain_;
    mean = plain ? 1.0f : 0.0f;
  }
  __device__ __forceinline__ void step(const DevParams& p, const float* lds_u, const float4* lds,
                                       int t, const float* n) {
    float v[M];
#pragma unroll
    for (int j = 0; j < M; ++j) v[j] = mean * lds_u[t * M + j] + n[j];
    mppi::step<Model, INTEG>(x, v, comp, p);
    bool hit;
    float l = Cost::template running<N, M>(x, comp, v, t, p, lds, cs, hit);
    if (p.importance && plain) l += is_term<M>(p, t, v, lds_u + t * M);
    if (p.cosines) l += inflation(p);
    if constexpr (COUNT) ncrash += hit ? 1 : 0;
    const float y = l - sum_c;
    const float s = sum + y;
    sum_c = (s - sum) - y;
    sum = s;
  }
  __device__ __forceinline__ RolloutResult finish(const DevParams& p, int T, const float4* lds) {
    const float tot = sum + (terminal_cost<Cost, N>(x, T, p, lds, cs) - sum_c);
    return RolloutResult{__builtin_isfinite(tot) ? tot : __builtin_inff(), ncrash};
  }
};

// One lane per sample: e points at eps[0][0][k] of this lane's sample;
// plain: the sample is drawn around u (else around zero, v = eps).
template <class Model, int INTEG, class Cost, bool COUNT>
__device__ __forceinline__ RolloutResult rollout_lane(const DevParams& p,
                                                      const float* __restrict__ x0,
                                                      const float* lds_u,
                                                      const float* __restrict__ e, int64_t ldk,
                                                      int T, const float4* lds, bool plain) {
  constexpr int M = Model::M;
  LaneRollout<Model, INTEG, Cost, COUNT> lane(p, x0, lds, plain);
  auto body = [&](int t, const float* n, int) { lane.step(p, lds_u, lds, t, n); };
  if constexpr (M <= 2) {
    noise_steps<M, 8>(e, ldk, T, body);  // noise requested 8 steps ahead
  } else {
    // the four-control quadrotor: its long step covers the latency of a
    // request made one step ahead, and a rolled loop keeps its large body small
    NoiseAhead<M> ahead;
    ahead.init(e, ldk, T);
    for (int t = 0; t < T; ++t) {
      float n[M];
      ahead.pop(t, n);
      body(t, n, 0);
    }
  }
  return lane.finish(p, T, lds);
}

}  // namespace mppi
