// Discrete dynamics x_{t+1} = F(x_t, v_t) (arXiv 2409.07563, Eq. dynamics),
// evaluated per sample in registers: forward Euler (the paper's default) or
// classic RK4 with the control held over the step.
//
// Precision: the first Model::kComp state components (positions that grow to
// tens of metres while a step moves them by centimetres) are advanced with
// compensated (Kahan) summation; the running compensation term is kept in
// registers and also handed to the cost, which uses it where a cost is steep
// in position (the costmap).  Without it binary32 rounding of p + dp
// accumulates over the horizon.
#pragma once

#include "common.h"

namespace mppi {

// (px, py, vx, vy), control (ax, ay)
struct DoubleIntegrator {
  static constexpr int N = 4, M = 2, kComp = 0;
  __device__ __forceinline__ static void deriv(const float* x, const float* v, float* d,
                                               const DevParams&) {
    d[0] = x[2]; d[1] = x[3]; d[2] = v[0]; d[3] = v[1];
  }
  __device__ __forceinline__ static void post_step(float*, const DevParams&) {}
};

// Kinematic bicycle (px, py, yaw, speed, steer), control (accel, steer rate).
// FAST: the hardware sine/cosine units (v_sin_f32 / v_cos_f32), as the paper
// does with CUDA's trigonometric intrinsics (Sec. III-B); otherwise the
// correctly range-reduced library functions.
template <bool FAST>
struct Bicycle {
  static constexpr int N = 5, M = 2, kComp = 2;
  __device__ __forceinline__ static void deriv(const float* x, const float* v, float* d,
                                               const DevParams& p) {
    float sn, cs, tn;
    if constexpr (FAST) {
      sn = __sinf(x[2]);
      cs = __cosf(x[2]);
      tn = __sinf(x[4]) * __builtin_amdgcn_rcpf(__cosf(x[4]));
    } else {
      sincosf(x[2], &sn, &cs);
      tn = tanf(x[4]);
    }
    d[0] = x[3] * cs;
    d[1] = x[3] * sn;
    d[2] = x[3] * tn * p.inv_wheelbase;
    d[3] = v[0];
    d[4] = v[1];
  }
  __device__ __forceinline__ static void post_step(float*, const DevParams&) {}
};

// Rigid-body quadrotor: p(3), q = (w, x, y, z), v(3) world frame, omega(3) body
// frame; control (thrust, tau_x, tau_y, tau_z).  q is renormalised after each
// step.
struct Quadrotor {
  static constexpr int N = 13, M = 4, kComp = 0;
  __device__ __forceinline__ static void deriv(const float* x, const float* v, float* d,
                                               const DevParams& p) {
    const float qw = x[3], qx = x[4], qy = x[5], qz = x[6];
    const float wx = x[10], wy = x[11], wz = x[12];
    d[0] = x[7]; d[1] = x[8]; d[2] = x[9];
    d[3] = 0.5f * (-qx * wx - qy * wy - qz * wz);
    d[4] = 0.5f * (qw * wx + qy * wz - qz * wy);
    d[5] = 0.5f * (qw * wy + qz * wx - qx * wz);
    d[6] = 0.5f * (qw * wz + qx * wy - qy * wx);
    const float a = v[0] * p.inv_mass;
    d[7] = 2.0f * (qx * qz + qw * qy) * a;
    d[8] = 2.0f * (qy * qz - qw * qx) * a;
    d[9] = (1.0f - 2.0f * (qx * qx + qy * qy)) * a - p.gravity;
    const float h0 = p.inertia[0] * wx, h1 = p.inertia[1] * wy, h2 = p.inertia[2] * wz;
    d[10] = (v[1] - (wy * h2 - wz * h1)) * p.inv_inertia[0];
    d[11] = (v[2] - (wz * h0 - wx * h2)) * p.inv_inertia[1];
    d[12] = (v[3] - (wx * h1 - wy * h0)) * p.inv_inertia[2];
  }
  __device__ __forceinline__ static void post_step(float* x, const DevParams&) {
    const float inv = rsqrtf(x[3] * x[3] + x[4] * x[4] + x[5] * x[5] + x[6] * x[6]);
    x[3] *= inv; x[4] *= inv; x[5] *= inv; x[6] *= inv;
  }
};

enum { kEuler = MPPI_INT_EULER, kRK4 = MPPI_INT_RK4 };

// x <- x + inc, compensated for the first kComp components (comp[] carries the
// rounding error of the previous additions with its sign flipped).
template <class Model>
__device__ __forceinline__ void advance(float* x, const float* x0, const float* inc,
                                        float* comp) {
#pragma unroll
  for (int i = 0; i < Model::N; ++i) {
    if (i < Model::kComp) {
      const float y = inc[i] - comp[i];
      const float t = x0[i] + y;
      comp[i] = (t - x0[i]) - y;
      x[i] = t;
    } else {
      x[i] = x0[i] + inc[i];
    }
  }
}

// One step.  res (optional): a residual r added as dt * r to the increment
// (the MLP residual dynamics evaluate it on the pre-step state).
template <class Model, int INTEG>
__device__ __forceinline__ void step(float* x, const float* v, float* comp, const DevParams& p,
                                     const float* res = nullptr) {
  constexpr int N = Model::N;
  float x0[N], inc[N];
#pragma unroll
  for (int i = 0; i < N; ++i) x0[i] = x[i];
  if constexpr (INTEG == kEuler) {
    float d[N];
    Model::deriv(x0, v, d, p);
#pragma unroll
    for (int i = 0; i < N; ++i) inc[i] = p.dt * d[i];
  } else {
    float k[N], acc[N], xs[N];
    Model::deriv(x0, v, k, p);
#pragma unroll
    for (int i = 0; i < N; ++i) { acc[i] = k[i]; xs[i] = x0[i] + p.half_dt * k[i]; }
    Model::deriv(xs, v, k, p);
#pragma unroll
    for (int i = 0; i < N; ++i) { acc[i] += 2.0f * k[i]; xs[i] = x0[i] + p.half_dt * k[i]; }
    Model::deriv(xs, v, k, p);
#pragma unroll
    for (int i = 0; i < N; ++i) { acc[i] += 2.0f * k[i]; xs[i] = x0[i] + p.dt * k[i]; }
    Model::deriv(xs, v, k, p);
#pragma unroll
    for (int i = 0; i < N; ++i) inc[i] = p.sixth_dt * (acc[i] + k[i]);
  }
  if (res) {
#pragma unroll
    for (int i = 0; i < N; ++i) inc[i] += p.dt * res[i];
  }
  advance<Model>(x, x0, inc, comp);
  Model::post_step(x, p);
}

}  // namespace mppi
