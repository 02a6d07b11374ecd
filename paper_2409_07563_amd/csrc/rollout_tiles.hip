// Step (a2) for the bicycle with an MLP residual (x_{t+1} = RK4 / Euler step
// + dt g([x_t; v_t])), and the checkpointing forward of the adjoint.
//
// A wave owns a tile of 16 samples.  The MLP runs on the matrix cores over
// the tile (mlp.h); every lane group g = lane / 16 carries a full copy of its
// sample's state, so the bicycle step and the cost run lane-locally, and the
// MLP input and output need only register selects and four-lane gathers.
// The nominal controls are staged in LDS.
//
// Checkpoints (optional): the state and the compensation terms of the
// positions at t = 0, c, 2c, ... are stored as ckpt[s][7][ldk], so the
// adjoint can rebuild each segment bit for bit.
#include <type_traits>

#include "mlp.h"
#include "rollout.h"

namespace mppi {

constexpr int kTile = 16;
constexpr int kCkptWords = 7;

// BF: the MLP's products on bfloat16 operands (mlp::WeightsBf)
template <int MT, int INTEG, class Cost, bool FAST, bool BF>
__global__ __launch_bounds__(kWave) void rollout_tile_kernel(
    DevParams p, const float* __restrict__ x0, const float* __restrict__ u,
    const float* __restrict__ eps, int64_t ldk, int K, int T, float* __restrict__ S,
    float* __restrict__ ckpt, int ckpt_every) {
  using Model = Bicycle<FAST>;
  constexpr int N = Model::N, M = Model::M;
  extern __shared__ float4 lds[];
  const float* lds_u = stage_rollout_lds<Cost>(p, u, T * M, lds);
  const int lane = threadIdx.x, n = lane % kTile, g = lane / kTile;
  const int k = blockIdx.x * kTile + n;
  const bool live = k < K;
  const bool plain = k < p.n_plain;  // drawn around u (else around zero)
  // v = mean u + eps: an unconditional load and one FMA (mean u + eps is
  // exactly u + eps for mean = 1), no branch around the load of u
  const float mean = plain ? 1.0f : 0.0f;
  // lanes past K recompute sample K-1 (they take part in the MFMAs) and store nothing
  const float* e = eps + (live ? k : K - 1);
  std::conditional_t<BF, mlp::WeightsBf<MT ? MT : 1>, mlp::Weights<MT ? MT : 1>> W;
  if constexpr (MT > 0) {
    if constexpr (BF) W.load(p.mlp_bf, p.mlp, lane);
    else W.load(p.mlp, lane);
  }
  float x[N], comp[N];
#pragma unroll
  for (int i = 0; i < N; ++i) { x[i] = x0[i]; comp[i] = 0.0f; }
  typename Cost::State cs;
  Cost::init(cs, x, p, lds);
  float sum = 0.0f, sum_c = 0.0f;
  int next_ckpt = 0;
  float* ck = ckpt ? ckpt + k : nullptr;
  noise_steps<M, 8>(e, ldk, T, [&](int t, const float* nz, int) {
    float v[M];
#pragma unroll
    for (int j = 0; j < M; ++j) v[j] = mean * lds_u[t * M + j] + nz[j];
    if (ck && t == next_ckpt) {
      if (g == 0 && live) {
#pragma unroll
        for (int i = 0; i < N; ++i) ck[i * ldk] = x[i];
        ck[5 * ldk] = comp[0];
        ck[6 * ldk] = comp[1];
      }
      ck += kCkptWords * ldk;
      next_ckpt += ckpt_every;
    }
    if constexpr (MT > 0) {
      float res[N];
      mlp::residual<MT>(W, x, v, g, n, res);
      step<Model, INTEG>(x, v, comp, p, res);
    } else {
      step<Model, INTEG>(x, v, comp, p);
    }
    bool hit;
    float l = Cost::template running<N, M>(x, comp, v, t, p, lds, cs, hit);
    if (p.importance && plain) l += is_term<M>(p, t, v, lds_u + t * M);
    if (p.cosines) l += inflation(p);
    const float y = l - sum_c;
    const float s = sum + y;
    sum_c = (s - sum) - y;
    sum = s;
  });
  sum = sum + (terminal_cost<Cost, N>(x, T, p, lds, cs) - sum_c);
  if (g == 0 && live) S[k] = __builtin_isfinite(sum) ? sum : __builtin_inff();
}

// The same rollout with the MLP split over SW waves of one workgroup (SW = 2
// or 4, H = 16 MT hidden units): wave w owns the MT / SW M-tiles q = w MT/SW
// ... of both hidden layers and the same K-tiles of the output layer.  Per
// step the waves exchange their h1 tiles and their per-K-tile output partials
// through LDS (double-buffered by step parity, two barriers).  Every
// per-element accumulation runs in the same order as in the one-wave kernel
// (layer 2: K-steps (tt, i) in order; output: the K-tile partials summed 0,
// 1, ..., MT-1), so the results are bitwise the same.  One leader wave per
// tile (wave blockIdx mod SW, so that the leaders of the tiles spread over
// the SIMDs) takes the bicycle step and the running cost and hands the new
// state to the other waves through LDS at a third barrier: the step's VALU
// work is done once per tile instead of SW times.  More waves keep more
// SIMDs busy, and a wave's matrix-core work overlaps another wave's VALU
// work.
// BF (the bfloat16 products of mlp::hidden_bf / output_bf): the waves
// exchange their h2 tiles instead of output partials, and the leader forms
// the output over every K-block in order, so each product is the one-wave
// kernel's and the results are bitwise the same as there too.
template <int MT, int SW, int INTEG, class Cost, bool FAST, bool BF = false>
__global__ __launch_bounds__(kWave * SW) void rollout_tile_split_kernel(
    DevParams p, const float* __restrict__ x0, const float* __restrict__ u,
    const float* __restrict__ eps, int64_t ldk, int K, int T, float* __restrict__ S,
    float* __restrict__ ckpt, int ckpt_every) {
  static_assert(MT % SW == 0, "tiles per wave");
  constexpr int TW = MT / SW;  // M-tiles per wave
  using Model = Bicycle<FAST>;
  using f4 = mlp::f4;
  using P = mlp::Pack<MT>;
  constexpr int N = Model::N, M = Model::M;
  __shared__ f4 xh[2][MT][kWave];  // h1 tiles
  __shared__ f4 xg[2][MT][kWave];  // output partials per K-tile (BF: h2 tiles)
  __shared__ float xs[kTile][8];   // the leader's new state of the tile's samples
  extern __shared__ float4 lds[];
  const float* lds_u = stage_rollout_lds<Cost>(p, u, T * M, lds);
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  const int n = lane % kTile, g = lane / kTile;
  const bool leader = w == static_cast<int>(blockIdx.x % SW);
  const int k = blockIdx.x * kTile + n;
  const bool live = k < K;
  const bool plain = k < p.n_plain;  // drawn around u (else around zero)
  // v = mean u + eps: an unconditional load and one FMA (mean u + eps is
  // exactly u + eps for mean = 1), no branch around the load of u
  const float mean = plain ? 1.0f : 0.0f;
  const float* e = eps + (live ? k : K - 1);
  // this wave's operands (tiles q0 .. q0 + TW - 1)
  const int q0 = w * TW;
  const float* pk = p.mlp + lane;
  auto at = [&](int row) { return pk[row * kWave]; };
  // binary32 operands (unused in BF), and the bfloat16 ones (unused otherwise)
  constexpr int KB = mlp::PackBf<MT>::KB;
  constexpr int TWF = BF ? 1 : TW, MTF = BF ? 1 : MT;
  constexpr int TWB = BF ? TW : 1, KBB = BF ? KB : 1;
  float w1[TWF][2], w2[TWF][MTF][4], w3[TWF][4];
  mlp::bf8 v1[TWB], v2[TWB][KBB], v3[KBB];
  f4 b1[TW], b2[TW], b3[TW];
#pragma unroll
  for (int q = 0; q < TW; ++q) {
    const int t = q0 + q;
    if constexpr (BF) {
      using PB = mlp::PackBf<MT>;
      const uint4* bp = p.mlp_bf + lane;
      v1[q] = __builtin_bit_cast(mlp::bf8, bp[(PB::kW1 + t) * kWave]);
#pragma unroll
      for (int kb = 0; kb < KB; ++kb)
        v2[q][kb] = __builtin_bit_cast(mlp::bf8, bp[(PB::kW2 + t * KB + kb) * kWave]);
    } else {
      w1[q][0] = at(P::kW1 + 2 * t);
      w1[q][1] = at(P::kW1 + 2 * t + 1);
#pragma unroll
      for (int tt = 0; tt < MT; ++tt)
#pragma unroll
        for (int i = 0; i < 4; ++i) w2[q][tt][i] = at(P::kW2 + (t * MT + tt) * 4 + i);
#pragma unroll
      for (int i = 0; i < 4; ++i) w3[q][i] = at(P::kW3 + 4 * t + i);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      b1[q][i] = at(P::kB1 + 4 * t + i);
      b2[q][i] = at(P::kB2 + 4 * t + i);
      b3[q][i] = (BF || t == 0) ? at(P::kB3 + i) : 0.0f;
    }
  }
  if constexpr (BF) {
    using PB = mlp::PackBf<MT>;
#pragma unroll
    for (int kb = 0; kb < KB; ++kb)
      v3[kb] = __builtin_bit_cast(mlp::bf8, p.mlp_bf[(PB::kW3 + kb) * kWave + lane]);
  }
  float x[N], comp[N];
#pragma unroll
  for (int i = 0; i < N; ++i) { x[i] = x0[i]; comp[i] = 0.0f; }
  typename Cost::State cs;
  Cost::init(cs, x, p, lds);
  float sum = 0.0f, sum_c = 0.0f;
  int next_ckpt = 0;
  float* ck = ckpt ? ckpt + k : nullptr;
  noise_steps<M, 8>(e, ldk, T, [&](int t, const float* nz, int) {
    const int par = t & 1;
    float v[M];
#pragma unroll
    for (int j = 0; j < M; ++j) v[j] = mean * lds_u[t * M + j] + nz[j];
    if (ck && t == next_ckpt) {
      if (leader && g == 0 && live) {  // the leader's compensation is current
#pragma unroll
        for (int i = 0; i < N; ++i) ck[i * ldk] = x[i];
        ck[5 * ldk] = comp[0];
        ck[6 * ldk] = comp[1];
      }
      ck += kCkptWords * ldk;
      next_ckpt += ckpt_every;
    }
    // layer 1, own tiles
    if constexpr (BF) {
      const mlp::bf8 zb = mlp::input_operand_bf(x, v, g);
#pragma unroll
      for (int q = 0; q < TW; ++q) xh[par][q0 + q][lane] = mlp::tanh4(mlp::mfma_bf(v1[q], zb, b1[q]));
    } else {
      const float z0 = mlp::input_operand(x, v, g, 0), z1 = mlp::input_operand(x, v, g, 1);
#pragma unroll
      for (int q = 0; q < TW; ++q)
        xh[par][q0 + q][lane] =
            mlp::tanh4(mlp::mfma(w1[q][1], z1, mlp::mfma(w1[q][0], z0, b1[q])));
    }
    __syncthreads();
    f4 h1[MT];  // every tile, the own ones included, read back from LDS
#pragma unroll
    for (int tt = 0; tt < MT; ++tt) h1[tt] = xh[par][tt][lane];
    // layer 2, own tiles, over all of h1
    f4 acc[TW];
#pragma unroll
    for (int q = 0; q < TW; ++q) acc[q] = b2[q];
    if constexpr (BF) {
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) {
        const mlp::bf8 hb = mlp::kblock_operand<MT>(h1, kb);
#pragma unroll
        for (int q = 0; q < TW; ++q) acc[q] = mlp::mfma_bf(v2[q][kb], hb, acc[q]);
      }
      // the own h2 tiles to the leader
#pragma unroll
      for (int q = 0; q < TW; ++q) xg[par][q0 + q][lane] = mlp::tanh4(acc[q]);
    } else {
#pragma unroll
      for (int tt = 0; tt < MT; ++tt)
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int q = 0; q < TW; ++q) acc[q] = mlp::mfma(w2[q][tt][i], h1[tt][i], acc[q]);
      // output partials of the own K-tiles
#pragma unroll
      for (int q = 0; q < TW; ++q) {
        const f4 h2 = mlp::tanh4(acc[q]);
        f4 part = b3[q];
#pragma unroll
        for (int i = 0; i < 4; ++i) part = mlp::mfma(w3[q][i], h2[i], part);
        xg[par][q0 + q][lane] = part;
      }
    }
    __syncthreads();
    if (leader) {  // a wave-uniform branch
      f4 out;
      if constexpr (BF) {
        f4 h2[MT];
#pragma unroll
        for (int tt = 0; tt < MT; ++tt) h2[tt] = xg[par][tt][lane];
        out = b3[0];
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) out = mlp::mfma_bf(v3[kb], mlp::kblock_operand<MT>(h2, kb), out);
      } else {
        out = xg[par][0][lane];
#pragma unroll
        for (int tt = 1; tt < MT; ++tt) out += xg[par][tt][lane];
      }
      float res[N];
      mlp::broadcast5(out, n, res);
      step<Model, INTEG>(x, v, comp, p, res);
      bool hit;
      float l = Cost::template running<N, M>(x, comp, v, t, p, lds, cs, hit);
      if (p.importance && plain) l += is_term<M>(p, t, v, lds_u + t * M);
      if (p.cosines) l += inflation(p);
      const float y = l - sum_c;
      const float s = sum + y;
      sum_c = (s - sum) - y;
      sum = s;
      if (g == 0) {
#pragma unroll
        for (int i = 0; i < N; ++i) xs[n][i] = x[i];
      }
    }
    // the others take the new state (xs is next written after the next
    // step's second barrier, which every wave reaches after this read)
    __syncthreads();
    if (!leader) {
#pragma unroll
      for (int i = 0; i < N; ++i) x[i] = xs[n][i];
    }
  });
  if (leader) {
    sum = sum + (terminal_cost<Cost, N>(x, T, p, lds, cs) - sum_c);
    if (g == 0 && live) S[k] = __builtin_isfinite(sum) ? sum : __builtin_inff();
  }
}

namespace {

using TileFn = void (*)(DevParams, const float*, const float*, const float*, int64_t, int, int,
                        float*, float*, int);

template <int MT, int INTEG, bool FAST, bool BF>
TileFn pick_cost(uint32_t cost) {
  if (cost == MPPI_COST_TRACK) return rollout_tile_kernel<MT, INTEG, CostTrack, FAST, BF>;
  if (cost == MPPI_COST_QUADRATIC) return rollout_tile_kernel<MT, INTEG, CostQuadratic, FAST, BF>;
  return nullptr;
}

template <int MT, bool BF = false>
TileFn pick_tile(uint32_t integrator, uint32_t cost, bool accurate) {
  if (integrator == MPPI_INT_RK4)
    return accurate ? pick_cost<MT, kRK4, false, BF>(cost) : pick_cost<MT, kRK4, true, BF>(cost);
  if (integrator == MPPI_INT_EULER)
    return accurate ? pick_cost<MT, kEuler, false, BF>(cost)
                    : pick_cost<MT, kEuler, true, BF>(cost);
  return nullptr;
}

template <int MT, int SW, int INTEG, bool FAST, bool BF>
TileFn pick_split_cost(uint32_t cost) {
  if (cost == MPPI_COST_TRACK) return rollout_tile_split_kernel<MT, SW, INTEG, CostTrack, FAST, BF>;
  if (cost == MPPI_COST_QUADRATIC)
    return rollout_tile_split_kernel<MT, SW, INTEG, CostQuadratic, FAST, BF>;
  return nullptr;
}

template <int MT, int SW, bool BF>
TileFn pick_split_bf(uint32_t integrator, uint32_t cost, bool accurate) {
  if (integrator == MPPI_INT_RK4)
    return accurate ? pick_split_cost<MT, SW, kRK4, false, BF>(cost)
                    : pick_split_cost<MT, SW, kRK4, true, BF>(cost);
  if (integrator == MPPI_INT_EULER)
    return accurate ? pick_split_cost<MT, SW, kEuler, false, BF>(cost)
                    : pick_split_cost<MT, SW, kEuler, true, BF>(cost);
  return nullptr;
}

template <int MT, int SW>
TileFn pick_split(uint32_t integrator, uint32_t cost, bool accurate, bool bf) {
  return bf ? pick_split_bf<MT, SW, true>(integrator, cost, accurate)
            : pick_split_bf<MT, SW, false>(integrator, cost, accurate);
}

TileFn select_tile(uint32_t dynamics, uint32_t integrator, uint32_t cost, bool accurate,
                   int hidden, bool bf = false) {
  if (dynamics == MPPI_DYN_BICYCLE) return pick_tile<0>(integrator, cost, accurate);
  if (dynamics != MPPI_DYN_BICYCLE_MLP) return nullptr;
  switch (hidden) {
    case 16: return bf ? pick_tile<1, true>(integrator, cost, accurate)
                       : pick_tile<1>(integrator, cost, accurate);
    case 32: return bf ? pick_tile<2, true>(integrator, cost, accurate)
                       : pick_tile<2>(integrator, cost, accurate);
    case 64: return bf ? pick_tile<4, true>(integrator, cost, accurate)
                       : pick_tile<4>(integrator, cost, accurate);
    default: return nullptr;
  }
}

}  // namespace

bool rollout_tiles_supported(uint32_t dynamics, uint32_t integrator, uint32_t cost, int hidden) {
  return select_tile(dynamics, integrator, cost, false, hidden) != nullptr;
}

hipError_t launch_rollout_tiles(uint32_t dynamics, uint32_t integrator, uint32_t cost,
                                bool accurate_trig, const DevParams& p, const float* d_x0,
                                const float* d_u, const float* d_eps, int64_t ldk, int K, int T,
                                float* d_S, float* d_ckpt, int ckpt_every, hipStream_t stream,
                                int waves) {
  // the split forms: H = 32 over 2 waves; H = 64 over 2 or 4 waves
  const bool mlp = dynamics == MPPI_DYN_BICYCLE_MLP;
  const bool bf = mlp && p.mlp_bf != nullptr;  // BF16 products
  TileFn fn = nullptr;
  if (waves == 1) fn = select_tile(dynamics, integrator, cost, accurate_trig, p.mlp_hidden, bf);
  else if (mlp && p.mlp_hidden == 64 && waves == 4) fn = pick_split<4, 4>(integrator, cost, accurate_trig, bf);
  else if (mlp && p.mlp_hidden == 64 && waves == 2) fn = pick_split<4, 2>(integrator, cost, accurate_trig, bf);
  else if (mlp && p.mlp_hidden == 32 && waves == 2) fn = pick_split<2, 2>(integrator, cost, accurate_trig, bf);
  if (!fn || (d_ckpt && ckpt_every < 1)) return hipErrorInvalidValue;
  const size_t lds = sizeof(float) * static_cast<size_t>(T) * 2;
  if (lds > 48 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       static_cast<int>(lds));
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(fn, dim3(static_cast<unsigned>((K + kTile - 1) / kTile)), dim3(kWave * waves),
                     lds, stream, p, d_x0, d_u, d_eps, ldk, K, T, d_S, d_ckpt, ckpt_every);
  return hipGetLastError();
}

}  // namespace mppi
