// Running cost l(x_{t+1}, v_t) and terminal cost phi(x_T) of the MPPI rollout
// (arXiv 2409.07563, Algorithm 1: the cost is charged after each dynamics step
// on the new state and the sampled control, then phi on the final state).
// The meaning of DevParams::w per cost kind is documented with mppi_cost in
// include/mppi.h.
#pragma once

#include "common.h"

namespace mppi {

// l = sum_i Q_i (x_i - g_i)^2 + sum_j R_j v_j^2;  phi = sum_i Qf_i (x_i - g_i)^2
// Every cost has a per-lane State (carried in registers across the horizon)
// and reads staged data from `lds`; kStage says whether the kernel must stage
// the read-only cost data.
struct NoState {};

struct CostQuadratic {
  static constexpr bool kStage = false;
  using State = NoState;
  __device__ __forceinline__ static void init(State&, const float*, const DevParams&,
                                              const float4*) {}
  template <int N, int M>
  __device__ __forceinline__ static float running(const float* x, const float* comp, const float* v, int,
                                                  const DevParams& p, const float4* lds, State&,
                                                  bool& hit) {
    float c = 0.0f;
#pragma unroll
    for (int i = 0; i < N; ++i) { const float e = x[i] - p.ref[i]; c += p.w[i] * e * e; }
#pragma unroll
    for (int j = 0; j < M; ++j) c += p.w[8 + j] * v[j] * v[j];
    hit = false;
    return c;
  }
  template <int N>
  __device__ __forceinline__ static float terminal(const float* x, const DevParams& p) {
    float c = 0.0f;
#pragma unroll
    for (int i = 0; i < N; ++i) { const float e = x[i] - p.ref[i]; c += p.w[16 + i] * e * e; }
    return c;
  }
};

// The spline segment of a lane's current position, cached in registers: a
// trajectory moves a few centimetres per step, so the segment rarely changes
// and re-selecting it costs two compares; a change reloads the segment's
// knots and coefficients from LDS.  Segment s covers [knot_s, knot_{s+1})
// (the last one also its right end), matching a search over all segments.
struct SplineCursor {
  int seg;
  float lo, hi;  // knots of seg and seg+1
  float4 c;
};

__device__ __forceinline__ void spline_load(SplineCursor& sc, int seg, const DevParams& p,
                                            const float4* lds) {
  const float* knots = reinterpret_cast<const float*>(lds + p.spline_knot4);
  sc.seg = seg;
  sc.lo = knots[seg];
  sc.hi = knots[seg + 1];
  sc.c = lds[p.spline_coef4 + seg];
}

// Moves the cursor to the segment of px (already clamped to the knot range).
__device__ __forceinline__ void spline_seek(SplineCursor& sc, float px, const DevParams& p,
                                            const float4* lds) {
  const float* knots = reinterpret_cast<const float*>(lds + p.spline_knot4);
  int seg = sc.seg;
  if (px >= sc.hi || px < sc.lo) {
    while (seg + 1 < p.nseg && px >= knots[seg + 1]) ++seg;
    while (seg > 0 && px < knots[seg]) --seg;
    spline_load(sc, seg, p, lds);
  }
}

__device__ __forceinline__ float path_terms(const float* x, SplineCursor& sc,
                                            const DevParams& p, const float4* lds) {
  const float* knots = reinterpret_cast<const float*>(lds + p.spline_knot4);
  const float px = fminf(fmaxf(x[0], knots[0]), knots[p.nseg]);
  spline_seek(sc, px, p, lds);
  const float4 c = sc.c;
  const float k0 = sc.lo;
  const float d = px - k0;
  const float y = c.x + d * (c.y + d * (c.z + d * c.w));
  const float dy = c.y + d * (2.0f * c.z + 3.0f * d * c.w);
  const float e = x[1] - y;
  const float eh = x[2] - atanf(dy);
  const float es = x[3] - p.w[3];
  return p.w[0] * e * e + p.w[1] * eh * eh + p.w[2] * es * es;
}

// Point-in-any-circle test (inclusive boundary) through the uniform grid
// staged in LDS: only the circles listed in the point's cell are tested.  A
// circle is listed in every cell its bounding box, inflated by far more than
// the binary32 error of the cell computation, touches, so every circle that
// contains the point is in the list (points off the grid clamp to an edge
// cell, whose circles cannot contain them).
__device__ __forceinline__ bool in_any_circle(float px, float py, const DevParams& p,
                                              const float4* lds) {
  const float gx = fminf(fmaxf((px - p.grid_x0) * p.grid_inv_cell, 0.0f),
                         static_cast<float>(p.grid_nx - 1));
  const float gy = fminf(fmaxf((py - p.grid_y0) * p.grid_inv_cell, 0.0f),
                         static_cast<float>(p.grid_ny - 1));
  const int cell = static_cast<int>(gy) * p.grid_nx + static_cast<int>(gx);
  const uint32_t* off = reinterpret_cast<const uint32_t*>(lds);
  const float4* ent = lds + p.grid_off4;  // grid at the start of the stage
  const uint32_t b = off[cell], e = off[cell + 1];
  bool hit = false;
  for (uint32_t j = b; j < e; ++j) {
    const float4 c = ent[j];
    const float dx = px - c.x, dy = py - c.y;
    hit |= (dx * dx + dy * dy) <= c.z;
  }
  return hit;
}

// One cell of a two-valued costmap from the LDS bitmap (see DevParams).
__device__ __forceinline__ float map_cell_bit(const uint32_t* bits, int idx, const DevParams& p) {
  return (bits[idx >> 5] >> (idx & 31)) & 1u ? p.map_v1 : p.map_v0;
}

// Bilinear costmap between cell centres, clamped to the edge cells.  The
// cell comes from the rounded cell coordinate; the interpolation fractions are
// measured from that cell's centre (exact in binary32 for the usual
// power-of-two-friendly resolutions) and include the position's compensation
// term, so they do not inherit the rounding of a coordinate near 256 cells.
// The four corner values come from the LDS bitmap when the map is staged as
// one (the same binary32 values as the map's, so the result is identical),
// else from the map in memory (L2).
__device__ __forceinline__ float costmap_value(float px, float py, float cpx, float cpy,
                                               const DevParams& p, const float4* lds) {
  const float gx = fminf(fmaxf((px - p.map_x0) * p.map_inv_res - 0.5f, 0.0f),
                         static_cast<float>(p.map_w - 1));
  const float gy = fminf(fmaxf((py - p.map_y0) * p.map_inv_res - 0.5f, 0.0f),
                         static_cast<float>(p.map_h - 1));
  const int ix = min(static_cast<int>(gx), p.map_w - 2);
  const int iy = min(static_cast<int>(gy), p.map_h - 2);
  const float res = p.map_res;
  const float cx = p.map_x0 + (static_cast<float>(ix) + 0.5f) * res;
  const float cy = p.map_y0 + (static_cast<float>(iy) + 0.5f) * res;
  const float fx = fminf(fmaxf(((px - cx) - cpx) * p.map_inv_res, 0.0f), 1.0f);
  const float fy = fminf(fmaxf(((py - cy) - cpy) * p.map_inv_res, 0.0f), 1.0f);
  float m00, m01, m10, m11;
  if (p.map_bits4 >= 0) {
    const uint32_t* bits = reinterpret_cast<const uint32_t*>(lds + p.map_bits4);
    const int idx = iy * p.map_w + ix;
    m00 = map_cell_bit(bits, idx, p);
    m01 = map_cell_bit(bits, idx + 1, p);
    m10 = map_cell_bit(bits, idx + p.map_w, p);
    m11 = map_cell_bit(bits, idx + p.map_w + 1, p);
  } else {
    const float* row = p.costmap + static_cast<int64_t>(iy) * p.map_w + ix;
    m00 = row[0];
    m01 = row[1];
    m10 = row[p.map_w];
    m11 = row[p.map_w + 1];
  }
  return (1.0f - fx) * (1.0f - fy) * m00 + fx * (1.0f - fy) * m01 + (1.0f - fx) * fy * m10 +
         fx * fy * m11;
}

template <bool CIRCLES>
struct CostPath {
  static constexpr bool kStage = true;
  using State = SplineCursor;
  __device__ __forceinline__ static void init(State& st, const float*, const DevParams& p,
                                              const float4* lds) {
    spline_load(st, 0, p, lds);
  }
  template <int N, int M>
  __device__ __forceinline__ static float running(const float* x, const float* comp, const float* v, int,
                                                  const DevParams& p, const float4* lds, State& st,
                                                  bool& hit) {
    float c = path_terms(x, st, p, lds) + p.w[4] * v[0] * v[0] + p.w[5] * v[1] * v[1];
    if constexpr (CIRCLES) {
      hit = in_any_circle(x[0], x[1], p, lds);
      c += hit ? p.w[6] : 0.0f;
    } else {
      hit = false;
      c += costmap_value(x[0], x[1], comp[0], comp[1], p, lds);
    }
    return c;
  }
  template <int N>
  __device__ __forceinline__ static float terminal(const float* x, const DevParams& p,
                                                   const float4* lds, State& st) {
    return p.w[7] * path_terms(x, st, p, lds);
  }
};

// Quadrotor hover at a waypoint (ref = waypoint 3, q_ref 4, u_hover 4).
struct CostHover {
  static constexpr bool kStage = false;
  using State = NoState;
  __device__ __forceinline__ static void init(State&, const float*, const DevParams&,
                                              const float4*) {}
  __device__ __forceinline__ static float state_terms(const float* x, const DevParams& p) {
    float cp = 0.0f, cv = 0.0f, cw = 0.0f;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const float e = x[i] - p.ref[i];
      cp += e * e;
      cv += x[7 + i] * x[7 + i];
      cw += x[10 + i] * x[10 + i];
    }
    const float dq = x[3] * p.ref[3] + x[4] * p.ref[4] + x[5] * p.ref[5] + x[6] * p.ref[6];
    return p.w[0] * cp + p.w[1] * cv + p.w[2] * cw + p.w[3] * (1.0f - dq * dq);
  }
  template <int N, int M>
  __device__ __forceinline__ static float running(const float* x, const float* comp, const float* v, int,
                                                  const DevParams& p, const float4* lds, State&,
                                                  bool& hit) {
    float c = state_terms(x, p);
    float cu = 0.0f;
#pragma unroll
    for (int j = 0; j < 4; ++j) { const float e = v[j] - p.ref[7 + j]; cu += e * e; }
    float cb = 0.0f;
#pragma unroll
    for (int i = 0; i < 3; ++i) { const float o = fmaxf(fabsf(x[i]) - p.w[6], 0.0f); cb += o * o; }
    hit = false;
    return c + p.w[4] * cu + p.w[5] * cb;
  }
  template <int N>
  __device__ __forceinline__ static float terminal(const float* x, const DevParams& p) {
    return p.w[7] * state_terms(x, p);
  }
};

// Time-indexed tracking: l_t = (x - ref_{t+1})' Q (x - ref_{t+1}) + v' R v.
struct CostTrack {
  static constexpr bool kStage = false;
  using State = NoState;
  __device__ __forceinline__ static void init(State&, const float*, const DevParams&,
                                              const float4*) {}
  template <int N, int M>
  __device__ __forceinline__ static float running(const float* x, const float* comp, const float* v, int t,
                                                  const DevParams& p, const float4* lds, State&,
                                                  bool& hit) {
    const float* r = p.ref + static_cast<int64_t>(t + 1) * N;
    float c = 0.0f;
#pragma unroll
    for (int i = 0; i < N; ++i) { const float e = x[i] - r[i]; c += p.w[i] * e * e; }
#pragma unroll
    for (int j = 0; j < M; ++j) c += p.w[8 + j] * v[j] * v[j];
    hit = false;
    return c;
  }
  // the terminal reference row is read by the kernel through t = T - 1
  template <int N>
  __device__ __forceinline__ static float terminal_at(const float* x, int T, const DevParams& p) {
    const float* r = p.ref + static_cast<int64_t>(T) * N;
    float c = 0.0f;
#pragma unroll
    for (int i = 0; i < N; ++i) { const float e = x[i] - r[i]; c += p.w[i] * e * e; }
    return p.w[16] * c;
  }
};

// Goal distance with circular obstacles (bicycle).
struct CostGoalCircles {
  static constexpr bool kStage = true;
  using State = NoState;
  __device__ __forceinline__ static void init(State&, const float*, const DevParams&,
                                              const float4*) {}
  template <int N, int M>
  __device__ __forceinline__ static float running(const float* x, const float* comp, const float* v, int,
                                                  const DevParams& p, const float4* lds, State&,
                                                  bool& hit) {
    const float dx = x[0] - p.ref[0], dy = x[1] - p.ref[1];
    float c = p.w[0] * (dx * dx + dy * dy) + p.w[1] * v[0] * v[0] + p.w[2] * v[1] * v[1];
    hit = in_any_circle(x[0], x[1], p, lds);
    return c + (hit ? p.w[3] : 0.0f);
  }
  template <int N>
  __device__ __forceinline__ static float terminal(const float* x, const DevParams& p) {
    const float dx = x[0] - p.ref[0], dy = x[1] - p.ref[1];
    return p.w[4] * p.w[0] * (dx * dx + dy * dy);
  }
};

// Uniform access to the terminal cost (TRACK needs the horizon, the path cost
// its staged spline and cursor).
template <class Cost, int N>
__device__ __forceinline__ float terminal_cost(const float* x, int T, const DevParams& p,
                                               const float4* lds, typename Cost::State& st) {
  if constexpr (__is_same(Cost, CostTrack)) {
    return CostTrack::terminal_at<N>(x, T, p);
  } else if constexpr (__is_same(Cost, CostPath<true>) || __is_same(Cost, CostPath<false>)) {
    return Cost::template terminal<N>(x, p, lds, st);
  } else {
    return Cost::template terminal<N>(x, p);
  }
}

}  // namespace mppi
