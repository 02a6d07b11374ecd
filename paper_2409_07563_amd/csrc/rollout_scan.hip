// Step (a2) for one instance, time-parallel form: the kinematic bicycle with
// RK4, its horizon spread over the 16 lanes of one DPP row per sample.
//
// With the control held over a step, the bicycle's RK4 step separates:
//   - speed and steer have constant derivatives (a, steer rate), so
//     s_{t+1} = s_t + dt a_t and steer_{t+1} = steer_t + dt r_t: prefix sums
//     of the controls;
//   - the stage yaw rates k_j = s_j tan(steer_j) / L depend only on
//     (s_t, steer_t, a_t, r_t), with k_3 = k_2: the yaw increment
//     dt/6 (k_1 + 4 k_2 + k_4) is known once s_t and steer_t are, and the yaw
//     is their prefix sum;
//   - the position increments dt/6 sum_j w_j s_j (cos, sin)(yaw_t + c_j dt
//     k_{j-1}) depend only on yaw_t and the same stage values: with the yaw
//     known they are independent, and the position is their prefix sum.
// So one rollout is three rounds of (independent per-step arithmetic, then a
// prefix sum over time), after which every step's state is known and the
// running costs are evaluated in parallel (the time-parallel cost of the
// paper's split kernel, section "Split Kernel Description", here inside one
// kernel and without the trajectory ever leaving registers).
//
// Lane c of a sample's row owns the contiguous steps [c C, c C + C), C =
// ceil(T / 16): each round runs its C steps sequentially, and the row's 16
// chunk totals are combined by a 4-step DPP scan (row_shr 1, 2, 4, 8).
// Positions are summed with compensation: Kahan within the chunk and a
// double-binary32 (TwoSum) scan across the row, so the position keeps the
// accuracy of the sequential kernels' compensated sum.  The running costs are
// summed per lane (Kahan) and over the row in a fixed order.
#include "noise.h"
#include "rollout.h"
#include "rowscan.h"

namespace mppi {

namespace {

constexpr int kScanMaxBlock = 256;

// Sums over a sample's group of L lanes: one DPP row (L = 16) or two
// adjacent rows (L = 32: rows 0-1 and 2-3 of a wave).  Lane 15 of rows 0
// and 2 is broadcast into rows 1 and 3 (0 in rows 0 and 2).
__device__ __forceinline__ float row_bcast15(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x142, 0xA, 0xF, false));
}
__device__ __forceinline__ int row_bcast15_int(int v) {
  return __builtin_amdgcn_update_dpp(0, v, 0x142, 0xA, 0xF, false);
}
// inclusive prefix sum over the group
template <int L>
__device__ __forceinline__ float group_scan(float v) {
  v = row_scan(v);
  if constexpr (L == 32) v += row_bcast15(v);
  return v;
}
template <int L>
__device__ __forceinline__ int group_scan_int(int v) {
  v = row_scan_int(v);
  if constexpr (L == 32) v += row_bcast15_int(v);
  return v;
}
// the value of the group's previous lane (0 in its first lane)
template <int L>
__device__ __forceinline__ float group_shift(float v) {
  if constexpr (L == 16) {
    return row_dpp<kRowShr1>(v);
  } else {
    const int lw = static_cast<int>(threadIdx.x) & (kWave - 1);
    const float prev = __shfl(v, (lw + kWave - 1) & (kWave - 1), kWave);
    return (lw & (L - 1)) == 0 ? 0.0f : prev;
  }
}
// exclusive prefix sum over the group
template <int L>
__device__ __forceinline__ float group_exclusive(float v) {
  if constexpr (L == 16) return row_exclusive(v);
  return group_shift<L>(group_scan<L>(v));
}

// (h, l) += (bh, bl) in double-binary32 arithmetic (Knuth's TwoSum of the
// high parts, the low parts added to its error, renormalised).
__device__ __forceinline__ void dd_add(float& h, float& l, float bh, float bl) {
  const float s = h + bh;
  const float z = s - h;
  float e = (h - (s - z)) + (bh - z);
  e += l + bl;
  const float hs = s + e;
  l = e - (hs - s);
  h = hs;
}
template <int CTRL>
__device__ __forceinline__ void dd_scan_step(float& h, float& l) {
  const float oh = row_dpp<CTRL>(h), ol = row_dpp<CTRL>(l);
  dd_add(h, l, oh, ol);
}
// exclusive double-binary32 prefix sum over the group
template <int L>
__device__ __forceinline__ void dd_group_exclusive(float& h, float& l) {
  dd_scan_step<kRowShr1>(h, l);
  dd_scan_step<kRowShr2>(h, l);
  dd_scan_step<kRowShr4>(h, l);
  dd_scan_step<kRowShr8>(h, l);
  if constexpr (L == 32) {
    const float oh = row_bcast15(h), ol = row_bcast15(l);
    if ((threadIdx.x >> 4) & 1) dd_add(h, l, oh, ol);  // rows 1 and 3
  }
  h = group_shift<L>(h);
  l = group_shift<L>(l);
}

template <bool FAST>
__device__ __forceinline__ float tan_of(float x) {
  if constexpr (FAST) {
    return __sinf(x) * __builtin_amdgcn_rcpf(__cosf(x));
  } else {
    return tanf(x);
  }
}
template <bool FAST>
__device__ __forceinline__ void sincos_of(float x, float* s, float* c) {
  if constexpr (FAST) {
    *s = __sinf(x);
    *c = __cosf(x);
  } else {
    sincosf(x, s, c);
  }
}

}  // namespace

// L: lanes per sample (16: one DPP row, or 32: two); CMAX: the chunk length
// the kernel is compiled for (C <= CMAX, T <= L CMAX); steps j >= C of a
// chunk are zero.
template <class Cost, bool FAST, bool COUNT, int CMAX, int L>
__global__ __launch_bounds__(kScanMaxBlock) void rollout_bicycle_scan_kernel(
    DevParams p, const float* __restrict__ x0, const float* __restrict__ u,
    const float* __restrict__ eps, int64_t ldk, int K, int T, int C, float* __restrict__ S,
    int32_t* __restrict__ crashes, int rblocks, NoiseJob job) {
  if (static_cast<int>(blockIdx.x) >= rblocks) {  // the next iteration's noise
    next_noise(job, blockIdx.x - rblocks);
    return;
  }
  constexpr int N = 5, M = 2;
  extern __shared__ float4 lds[];
  const float* lds_u = stage_rollout_lds<Cost>(p, u, T * M, lds);
  const int gl = blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = gl & (L - 1);  // chunk of the horizon
  const int k = gl / L;
  if (k >= K) return;  // whole groups leave together; no barrier follows
  const int t0 = lane * C;
  const int nloc = max(0, min(C, T - t0));  // steps of this lane
  const float mean = k < p.n_plain ? 1.0f : 0.0f;  // drawn around u, or around zero

  // every noise value of the chunk is requested before any arithmetic
  float va[CMAX], vr[CMAX];
  const float* e = eps + k;
#pragma unroll
  for (int j = 0; j < CMAX; ++j) {
    const int t = min(t0 + j, T - 1);
    va[j] = j < C ? e[static_cast<int64_t>(t * M) * ldk] : 0.0f;
    vr[j] = j < C ? e[static_cast<int64_t>(t * M + 1) * ldk] : 0.0f;
  }
  // v = mean u + eps (exactly u + eps for mean = 1); zero past the horizon
  float tot_a = 0.0f, tot_r = 0.0f;
#pragma unroll
  for (int j = 0; j < CMAX; ++j) {
    const bool in = j < nloc;
    const int t = min(t0 + j, T - 1);
    va[j] = in ? mean * lds_u[t * M] + va[j] : 0.0f;
    vr[j] = in ? mean * lds_u[t * M + 1] + vr[j] : 0.0f;
    tot_a = fmaf(p.dt, va[j], tot_a);
    tot_r = fmaf(p.dt, vr[j], tot_r);
  }
  // round 1: speed and steer at the chunk's first step
  const float s_c = x0[3] + group_exclusive<L>(tot_a);
  const float d_c = x0[4] + group_exclusive<L>(tot_r);

  // round 2: stage yaw rates and yaw increments
  float k1[CMAX], k2[CMAX], dpsi[CMAX];
  float tot_psi = 0.0f;
  {
    float s = s_c, d = d_c;
    float tn = tan_of<FAST>(d);
#pragma unroll
    for (int j = 0; j < CMAX; ++j) {
      const float sh = fmaf(p.half_dt, va[j], s), dh = fmaf(p.half_dt, vr[j], d);
      const float sf = fmaf(p.dt, va[j], s), df = fmaf(p.dt, vr[j], d);
      const float tf = tan_of<FAST>(df);
      const float a1 = s * tn * p.inv_wheelbase;
      const float a2 = sh * tan_of<FAST>(dh) * p.inv_wheelbase;
      const float a4 = sf * tf * p.inv_wheelbase;
      // the RK4 combination in the sequential kernels' order (k3 = k2)
      float acc = a1;
      acc += 2.0f * a2;
      acc += 2.0f * a2;
      const float inc = p.sixth_dt * (acc + a4);
      const bool in = j < nloc;
      k1[j] = a1;
      k2[j] = a2;
      dpsi[j] = in ? inc : 0.0f;
      tot_psi += dpsi[j];
      s = sf;
      d = df;
      tn = tf;
    }
  }
  const float psi_c = x0[2] + group_exclusive<L>(tot_psi);

  // round 3: position increments (four sin / cos pairs per step)
  float dpx[CMAX], dpy[CMAX];
  float hx = 0.0f, lx = 0.0f, hy = 0.0f, ly = 0.0f;  // compensated chunk totals
  {
    float s = s_c, psi = psi_c;
#pragma unroll
    for (int j = 0; j < CMAX; ++j) {
      const float sh = fmaf(p.half_dt, va[j], s);
      const float sf = fmaf(p.dt, va[j], s);
      float sn1, cs1, sn2, cs2, sn3, cs3, sn4, cs4;
      sincos_of<FAST>(psi, &sn1, &cs1);
      sincos_of<FAST>(psi + p.half_dt * k1[j], &sn2, &cs2);
      sincos_of<FAST>(psi + p.half_dt * k2[j], &sn3, &cs3);
      sincos_of<FAST>(psi + p.dt * k2[j], &sn4, &cs4);
      float ax = s * cs1, ay = s * sn1;
      ax += 2.0f * (sh * cs2);
      ay += 2.0f * (sh * sn2);
      ax += 2.0f * (sh * cs3);
      ay += 2.0f * (sh * sn3);
      const bool in = j < nloc;
      dpx[j] = in ? p.sixth_dt * (ax + sf * cs4) : 0.0f;
      dpy[j] = in ? p.sixth_dt * (ay + sf * sn4) : 0.0f;
      // Kahan: (h, -l) carries the sum and its rounding error
      {
        const float y = dpx[j] + lx;
        const float t = hx + y;
        lx = y - (t - hx);
        hx = t;
      }
      {
        const float y = dpy[j] + ly;
        const float t = hy + y;
        ly = y - (t - hy);
        hy = t;
      }
      psi += dpsi[j];
      s = sf;
    }
  }
  dd_group_exclusive<L>(hx, lx);
  dd_group_exclusive<L>(hy, ly);

  // round 4: every step's post-step state and its running cost
  typename Cost::State cs;
  float x[N], comp[N] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
  x[0] = x0[0]; x[1] = x0[1]; x[2] = psi_c; x[3] = s_c; x[4] = d_c;
  Cost::init(cs, x, p, lds);
  float sum = 0.0f, sum_c = 0.0f;
  int ncrash = 0;
  auto add = [&](float l) {
    const float y = l - sum_c;
    const float s = sum + y;
    sum_c = (s - sum) - y;
    sum = s;
  };
  {
    float psi = psi_c, s = s_c, d = d_c;
#pragma unroll
    for (int j = 0; j < CMAX; ++j) {
      if (j >= nloc) continue;  // past this lane's steps
      const int t = t0 + j;
      // position relative to x0 after this step, compensated
      {
        const float y = dpx[j] + lx;
        const float tt = hx + y;
        lx = y - (tt - hx);
        hx = tt;
      }
      {
        const float y = dpy[j] + ly;
        const float tt = hy + y;
        ly = y - (tt - hy);
        hy = tt;
      }
      psi += dpsi[j];
      s = fmaf(p.dt, va[j], s);
      d = fmaf(p.dt, vr[j], d);
      // absolute position: x0 + (h + l) rounded once, its rounding error kept
      // as the compensation (true value = x - comp)
      const float X = x0[0] + hx, Y = x0[1] + hy;
      const float zx = X - x0[0], zy = Y - x0[1];
      const float ex = ((x0[0] - (X - zx)) + (hx - zx)) + lx;
      const float ey = ((x0[1] - (Y - zy)) + (hy - zy)) + ly;
      x[0] = X; x[1] = Y; x[2] = psi; x[3] = s; x[4] = d;
      comp[0] = -ex;
      comp[1] = -ey;
      const float v[M] = {va[j], vr[j]};
      bool hit;
      float l = Cost::template running<N, M>(x, comp, v, t, p, lds, cs, hit);
      if (p.importance && mean != 0.0f) l += is_term<M>(p, t, v, lds_u + t * M);
      if (p.cosines) l += inflation(p);
      if constexpr (COUNT) ncrash += hit ? 1 : 0;
      add(l);
    }
  }
  // the lane holding step T - 1 adds the terminal cost on x_T
  if (nloc > 0 && t0 + nloc == T) add(terminal_cost<Cost, N>(x, T, p, lds, cs));
  // the group's sum in a fixed order; its last lane holds it
  const float total = group_scan<L>(sum - sum_c);
  if (lane == L - 1) S[k] = __builtin_isfinite(total) ? total : __builtin_inff();
  if constexpr (COUNT) {
    const int n = group_scan_int<L>(ncrash);
    if (lane == L - 1) crashes[k] = n;
  }
}

namespace {

using ScanFn = void (*)(DevParams, const float*, const float*, const float*, int64_t, int, int,
                        int, float*, int32_t*, int, NoiseJob);

template <class Cost, bool FAST, int CMAX, int L>
ScanFn pick_scan(bool count) {
  if (count) return rollout_bicycle_scan_kernel<Cost, FAST, true, CMAX, L>;
  return rollout_bicycle_scan_kernel<Cost, FAST, false, CMAX, L>;
}

template <class Cost, bool FAST>
ScanFn pick_scan_chunk(int C, int L, bool count) {
  // the chunk loops run CMAX steps.  16 lanes: compiled for the chunks of
  // T = 64, 112, 160, 208 and 256 (C = 4, 7, 10, 13, 16; T = 100 and 200
  // take C = 7, 13); 32 lanes: T = 128 and 256 (C = 4, 8)
  if (L == 32) {
    if (C <= 4) return pick_scan<Cost, FAST, 4, 32>(count);
    if (C <= 8) return pick_scan<Cost, FAST, 8, 32>(count);
    return nullptr;
  }
  if (L != 16) return nullptr;
  if (C <= 4) return pick_scan<Cost, FAST, 4, 16>(count);
  if (C <= 7) return pick_scan<Cost, FAST, 7, 16>(count);
  if (C <= 10) return pick_scan<Cost, FAST, 10, 16>(count);
  if (C <= 13) return pick_scan<Cost, FAST, 13, 16>(count);
  if (C <= 16) return pick_scan<Cost, FAST, 16, 16>(count);
  return nullptr;
}

template <bool FAST>
ScanFn pick_scan_cost(uint32_t cost, int C, int L, bool count) {
  switch (cost) {
    case MPPI_COST_PATH_CIRCLES: return pick_scan_chunk<CostPath<true>, FAST>(C, L, count);
    case MPPI_COST_PATH_COSTMAP: return pick_scan_chunk<CostPath<false>, FAST>(C, L, count);
    case MPPI_COST_GOAL_CIRCLES: return pick_scan_chunk<CostGoalCircles, FAST>(C, L, count);
    case MPPI_COST_QUADRATIC: return pick_scan_chunk<CostQuadratic, FAST>(C, L, count);
    case MPPI_COST_TRACK: return pick_scan_chunk<CostTrack, FAST>(C, L, count);
    default: return nullptr;
  }
}

}  // namespace

bool rollout_scan_supported(uint32_t dynamics, uint32_t integrator, uint32_t cost, int T,
                            int lanes) {
  if (lanes != 16 && lanes != 32) return false;
  const int C = (T + lanes - 1) / lanes;
  return dynamics == MPPI_DYN_BICYCLE && integrator == MPPI_INT_RK4 && T >= 1 &&
         pick_scan_cost<true>(cost, C, lanes, false) != nullptr;
}

hipError_t launch_rollout_scan(uint32_t dynamics, uint32_t integrator, uint32_t cost,
                               bool accurate_trig, const DevParams& p, const float* d_x0,
                               const float* d_u, const float* d_eps, int64_t ldk, int K, int T,
                               float* d_S, int32_t* d_crashes, hipStream_t stream, int block,
                               const NoiseJob* next, int lanes) {
  if (block != 64 && block != 128 && block != 256) return hipErrorInvalidValue;
  if (!rollout_scan_supported(dynamics, integrator, cost, T, lanes) || K < 1)
    return hipErrorInvalidValue;
  const int C = (T + lanes - 1) / lanes;
  const bool count = d_crashes != nullptr;
  ScanFn fn = accurate_trig ? pick_scan_cost<false>(cost, C, lanes, count)
                            : pick_scan_cost<true>(cost, C, lanes, count);
  if (!fn) return hipErrorInvalidValue;
  const size_t lds = rollout_lds_bytes(dynamics, cost, p.stage_words4, T);
  if (lds > 48 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       static_cast<int>(lds));
    if (e != hipSuccess) return e;
  }
  const int64_t threads = static_cast<int64_t>(K) * lanes;
  const int rblocks = static_cast<int>((threads + block - 1) / block);
  NoiseJob job{};
  int blocks = rblocks;
  if (next) {
    job = *next;
    blocks += noise_job_blocks(&job, block);
  }
  hipLaunchKernelGGL(fn, dim3(static_cast<unsigned>(blocks)), dim3(block), lds, stream, p, d_x0,
                     d_u, d_eps, ldk, K, T, C, d_S, d_crashes, rblocks, job);
  return hipGetLastError();
}

}  // namespace mppi
