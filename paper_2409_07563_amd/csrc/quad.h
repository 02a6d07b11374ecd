// The kinematic bicycle's RK4 step with its four stages on the four lanes of
// a DPP quad (lane j = stage j), shared by the grouped fused rollout and the
// split form's dynamics kernel.  For the kinematic bicycle the stage yaw
// rates k_psi = s_j tan(steer_j) / L depend only on speed and steer, which
// are linear in time over a step, so all four tan / sin / cos evaluations run
// at once and one in-quad shift delivers k_psi of the previous stage for
// yaw_j = yaw + c_j dt k_psi(j-1).  Three quad sums assemble the increment;
// every lane of the quad ends with bitwise the same state (binary32 addition
// commutes).
#pragma once

#include "dynamics.h"

namespace mppi {

// quad_perm selectors: [1,0,3,2], [2,3,0,1] and the shift [0,0,1,2]
constexpr int kQuadSwap1 = 0xB1, kQuadSwap2 = 0x4E, kQuadShift = 0x90;
// Every lane of a quad reads a valid source under these permutations, so the
// move needs no initialised destination (no extra register move per use).
template <int CTRL>
__device__ __forceinline__ float quad_dpp(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}
__device__ __forceinline__ float quad_sum(float v) {
  const float a = v + quad_dpp<kQuadSwap1>(v);
  return a + quad_dpp<kQuadSwap2>(a);
}

// x, comp: the state and its compensation (identical on the quad's lanes);
// v: the step's control; j = lane mod 4; cdt = c_j dt (0, dt/2, dt/2, dt);
// wj = the RK4 weight of stage j (1, 2, 2, 1).
template <bool FAST>
__device__ __forceinline__ void bicycle_quad_step(float* x, float* comp, const float* v, int j,
                                                  float cdt, float wj, const DevParams& p) {
  constexpr int N = 5;
  const float sj = x[3] + cdt * v[0];
  const float dj = x[4] + cdt * v[1];
  float tn;
  if constexpr (FAST) {
    tn = __sinf(dj) * __builtin_amdgcn_rcpf(__cosf(dj));
  } else {
    tn = tanf(dj);
  }
  const float kpsi = sj * tn * p.inv_wheelbase;
  const float kprev = quad_dpp<kQuadShift>(kpsi);
  const float yj = j == 0 ? x[2] : x[2] + cdt * kprev;
  float sn, co;
  if constexpr (FAST) {
    sn = __sinf(yj);
    co = __cosf(yj);
  } else {
    sincosf(yj, &sn, &co);
  }
  const float gx = quad_sum(wj * (sj * co));
  const float gy = quad_sum(wj * (sj * sn));
  const float gp = quad_sum(wj * kpsi);
  const float x0s[N] = {x[0], x[1], x[2], x[3], x[4]};
  // speed and steer have the constant derivatives (a, steer rate) over the
  // step: their RK4 increment is dt v
  const float inc[N] = {p.sixth_dt * gx, p.sixth_dt * gy, p.sixth_dt * gp, p.dt * v[0],
                        p.dt * v[1]};
  advance<Bicycle<FAST>>(x, x0s, inc, comp);
}

}  // namespace mppi
