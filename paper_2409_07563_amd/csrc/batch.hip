// Batched MPPI: many independent instances (each with its own K, T, lambda,
// sigma, noise stream and cost data) advanced by one launch per phase.
//
// The work lists are host-built tile tables over a device instance table
// (BatchInst): a workgroup picks its tile, reads the instance descriptor with
// wave-uniform scalar loads and runs the same device bodies as the
// single-instance kernels (noise.h, rollout.h, softmin.h).  Sample tiles are
// ordered longest horizon first, so the hardware dispatcher starts the long
// rollouts early and fills the tail with short ones.  The per-iteration launch
// sequence of a batch is captured once in a hipGraph by the host code.
#include "noise.h"
#include "rollout.h"
#include "rowscan.h"
#include "softmin.h"
#include "worklist.h"

namespace mppi {

static_assert(sizeof(WorkItem) == sizeof(int2) && alignof(WorkItem) <= alignof(int2),
              "work lists are uploaded as int2 tables");

// (a1) every normal of a tile's samples; one thread per sample loops
// over the Philox calls of its sample, each call storing four coalesced rows.
__global__ __launch_bounds__(kBatchMaxTile) void batch_noise_kernel(
    const BatchInst* __restrict__ insts, const int2* __restrict__ tiles) {
  const int2 tl = tiles[blockIdx.x];
  const BatchInst& b = insts[tl.x];
  const int k = tl.y * static_cast<int>(blockDim.x) + threadIdx.x;
  if (k >= b.K) return;
  const uint32_t it = b.st->iteration;
  const int ncall = (b.TM + 3) / 4;
  const int m = b.TM / b.T;
  for (int c = 0; c < ncall; ++c)
    noise::emit_call(b.key0, b.key1, it, b.instance, k, c, b.TM, m, b.sigma.v, b.eps, b.ldk,
                     b.p.sigma_t, b.p.mean_sample && k == 0);
}

// (a2) one lane per sample over a tile of samples of one instance;
// the instance's cost data and controls are staged in LDS per workgroup.
template <class Model, int INTEG, class Cost, bool COUNT>
__global__ __launch_bounds__(kBatchMaxTile) void batch_rollout_kernel(
    const BatchInst* __restrict__ insts, const int2* __restrict__ tiles) {
  extern __shared__ float4 lds[];
  const int2 tl = tiles[blockIdx.x];
  const BatchInst& b = insts[tl.x];
  const DevParams& p = b.p;
  const float* lds_u = stage_rollout_lds<Cost>(p, b.u, b.TM, lds);
  const int k = tl.y * static_cast<int>(blockDim.x) + threadIdx.x;
  if (k >= b.K) return;  // no barrier follows
  const RolloutResult r =
      rollout_lane<Model, INTEG, Cost, COUNT>(p, b.x0, lds_u, b.eps + k, b.ldk, b.T, lds,
                                              k < p.n_plain);
  b.S[k] = r.cost;
  if constexpr (COUNT) b.crashes[k] = r.crashes;
}

// (a3)-(a5) one workgroup per instance; (a6) one workgroup per row of the update.
__global__ __launch_bounds__(kWeightsBlock) void batch_weights_kernel(
    const BatchInst* __restrict__ insts) {
  const BatchInst& b = insts[blockIdx.x];
  weights_body(b.S, b.K, b.lambda, b.inv_lambda, b.e, b.st, b.p.n_plain);
}

__global__ __launch_bounds__(kGemvBlock) void batch_gemv_kernel(const BatchInst* __restrict__ insts,
                                                                const int2* __restrict__ tiles) {
  const int2 tl = tiles[blockIdx.x];
  const BatchInst& b = insts[tl.x];
  // the host checks every row tile against T*m before the upload; a row past
  // the instance's would read and write another instance's buffers
  if (tl.y >= b.TM) return;  // uniform over the workgroup: no barrier is skipped by part of it
  gemv_row(b.eps, b.ldk, b.K, b.e, b.st, b.u, b.step, tl.y, false);
}

__global__ void batch_set_iteration_kernel(const BatchInst* __restrict__ insts, int n,
                                           uint32_t iteration) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) insts[i].st->iteration = iteration;
}

// ---------------------------------------------------------------------------
// The one-launch form: a whole iteration of every instance in one launch, no
// workgroup ever waiting for another.  Workgroup q takes sample tile (i, t)
// = fused_items[q] of kBatchMaxTile samples (the list is ordered longest
// horizon first, so the dispatcher starts the long rollouts early) and
//   1. draws the tile's noise in its lanes (the Philox calls of
//      batch_noise_kernel, stored to the noise buffer) and rolls out from it;
//   2. weights the tile's samples against the tile's own minimum m_t
//      (e_k = exp(-(J_k - m_t)/lambda)) and sums them (as the chunked update's
//      chunk weights);
//   3. forms the tile's weighted noise rows N_t[r] = sum_k e_k eps[r][k] from
//      the noise it has just stored (one thread per row);
//   4. counts the tile in the instance's completion counter done[i]; the
//      workgroup that completes the instance's last tile rescales the tiles to
//      the instance's minimum rho (factor exp(-(m_t - rho)/lambda)) and
//      updates u[r] += gamma (sum_t f_t N_t[r] / eta - u[r] W_Z), the
//      statistics and the iteration word, and resets the counter.
// There is no loop over work items in the kernel (a loop whose exit the
// compiler cannot prove uniform, with barriers in its body, can be split so
// that not every path back to a barrier takes the next item).  The costs and
// the noise are bitwise those of the per-phase launches; the update equals
// theirs up to the rounding order of its sums (the arithmetic of the chunked
// update form, with tiles for chunks).
// ---------------------------------------------------------------------------
template <class Model, int INTEG, class Cost, bool COUNT>
__device__ __forceinline__ float tile_rollout_drawn(const BatchInst& b, int tile, float4* lds) {
  constexpr int M = Model::M;
  static_assert(4 % M == 0, "whole steps per Philox call");
  constexpr int SPC = 4 / M;  // steps per Philox call
  const DevParams& p = b.p;
  const float* lds_u = stage_rollout_lds<Cost>(p, b.u, b.TM, lds);
  const int k = tile * kBatchMaxTile + static_cast<int>(threadIdx.x);
  if (k >= b.K) return __builtin_inff();  // no barrier follows in the tile
  const uint32_t it = b.st->iteration;
  const bool zero = p.mean_sample && k == 0;
  LaneRollout<Model, INTEG, Cost, COUNT> lane(p, b.x0, lds, k < p.n_plain);
  // kCalls Philox calls are drawn together (independent chains the
  // scheduler interleaves), then their steps run
  constexpr int kCalls = 4;
  const int ncall = (b.TM + 3) / 4;
  for (int c0 = 0; c0 < ncall; c0 += kCalls) {
    float z[kCalls][4];
#pragma unroll
    for (int g = 0; g < kCalls; ++g)
      if (c0 + g < ncall)
        noise::emit_call(b.key0, b.key1, it, b.instance, k, c0 + g, b.TM, M, b.sigma.v, b.eps,
                         b.ldk, p.sigma_t, zero, z[g]);
#pragma unroll
    for (int g = 0; g < kCalls; ++g)
#pragma unroll
      for (int q = 0; q < SPC; ++q) {
        const int t = (c0 + g) * SPC + q;
        if (t < b.T) lane.step(p, lds_u, lds, t, z[g] + q * M);
      }
  }
  const RolloutResult r = lane.finish(p, b.T, lds);
  b.S[k] = r.cost;
  if constexpr (COUNT) b.crashes[k] = r.crashes;
  return r.cost;
}

// The sum of v over the wave, returned to every lane: a prefix sum over each
// 16-lane row (DPP row_shr 1, 2, 4, 8), then the row totals carried across
// rows (row_bcast 15 into rows 1 and 3, row_bcast 31 into rows 2 and 3), so
// lane 63 holds the total in a fixed order.
template <int CTRL, int ROW_MASK, bool BOUND>
__device__ __forceinline__ float wave_dpp(float x) {
  return __int_as_float(
      __builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROW_MASK, 0xF, BOUND));
}
__device__ __forceinline__ float wave_total(float v) {
  v += wave_dpp<0x111, 0xF, true>(v);   // row_shr:1
  v += wave_dpp<0x112, 0xF, true>(v);   // row_shr:2
  v += wave_dpp<0x114, 0xF, true>(v);   // row_shr:4
  v += wave_dpp<0x118, 0xF, true>(v);   // row_shr:8
  v += wave_dpp<0x142, 0xA, false>(v);  // row_bcast:15 into rows 1 and 3
  v += wave_dpp<0x143, 0xC, false>(v);  // row_bcast:31 into rows 2 and 3
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), kWave - 1));
}

// Steps 2 and 3 for one tile: its minimum and weight sums to tile_stat[t],
// its weighted noise rows to tile_part[t][.].  S_k: this lane's cost (+inf
// past the instance's samples).
__device__ __forceinline__ void tile_softmin_partials(const BatchInst& b, int tile, float S_k) {
  constexpr int NW = kBatchMaxTile / kWave;
  constexpr int kRows = kWave;  // rows per round (one per lane of the combine)
  constexpr int kIn = 8;        // rows whose loads are in flight at once
  __shared__ float lds_m[NW];
  __shared__ float4 lds4[NW];
  __shared__ float part[NW][kRows];
  const float inf = __builtin_inff();
  const int tid = threadIdx.x, lane = tid % kWave, wv = tid / kWave;
  const int k = tile * kBatchMaxTile + tid;
  const bool valid = k < b.K;
  const float mt = block_min<NW>(S_k, lds_m);
  const float ek = (valid && S_k < inf) ? expf((mt - S_k) * b.inv_lambda) : 0.0f;
  float4 v{wave_sum(ek), wave_sum(ek * ek), wave_sum(k >= b.p.n_plain ? ek : 0.0f), 0.0f};
  if (lane == 0) lds4[wv] = v;
  __syncthreads();  // also orders this tile's noise stores before the row reads
  if (tid == 0) {
    v = lds4[0];
#pragma unroll
    for (int i = 1; i < NW; ++i) { v.x += lds4[i].x; v.y += lds4[i].y; v.z += lds4[i].z; }
    b.tile_stat[tile] = float4{mt, v.x, v.y, v.z};
  }
  // N_t[r] = sum_k e_k eps[r][k]: each wave reduces its 64 samples of a row
  // (coalesced 256-byte reads, kIn rows in flight; padding past K is never
  // read), the four wave sums are added in a fixed order
  static_assert(NW == 4, "the wave sums below are added as a fixed tree of four");
  const float* col = b.eps + (valid ? k : 0);
  // uniform bounds (a scalar register) for the loop that holds barriers
  const int TM = __builtin_amdgcn_readfirstlane(b.TM);
  for (int r0 = 0; r0 < TM; r0 += kRows) {
    const int nr = min(kRows, TM - r0);
    for (int rr = 0; rr < nr; rr += kIn) {
      float x[kIn];
#pragma unroll
      for (int q = 0; q < kIn; ++q) {
        const int r = r0 + rr + q;
        x[q] = (valid && rr + q < nr) ? col[static_cast<int64_t>(r) * b.ldk] : 0.0f;
      }
#pragma unroll
      for (int q = 0; q < kIn; ++q) {
        const float t = wave_total(ek * x[q]);
        if (lane == 0 && rr + q < nr) part[wv][rr + q] = t;
      }
    }
    __syncthreads();
    if (tid < nr)
      b.tile_part[static_cast<int64_t>(tile) * TM + r0 + tid] =
          (part[0][tid] + part[1][tid]) + (part[2][tid] + part[3][tid]);
    __syncthreads();  // part is rewritten by the next round
  }
}

// Step 4 for the instance's last tile: rho, the tile factors, eta and the
// statistics, and every row of the update (the chunked update's arithmetic).
__device__ __forceinline__ void instance_combine(const BatchInst& b, int ntile) {
  constexpr int NW = kBatchMaxTile / kWave;
  __shared__ float lds_m[NW];
  __shared__ float4 lds4[NW];
  __shared__ float fsc[kOneLaunchMaxTiles];
  const float inf = __builtin_inff();
  const int tid = threadIdx.x;
  float m = inf;
  for (int c = tid; c < ntile; c += kBatchMaxTile) m = fminf(m, b.tile_stat[c].x);
  const float rho = block_min<NW>(m, lds_m);
  const bool finite = rho < inf;
  float se = 0.0f, se2 = 0.0f, sz = 0.0f;
  for (int c = tid; c < ntile; c += kBatchMaxTile) {
    const float4 q = b.tile_stat[c];
    const float f = (finite && q.x < inf) ? expf((rho - q.x) * b.inv_lambda) : 0.0f;
    fsc[c] = f;
    se += q.y * f;
    se2 += q.z * (f * f);
    sz += q.w * f;
  }
  float4 v{wave_sum(se), wave_sum(se2), wave_sum(sz), 0.0f};
  __syncthreads();
  if (tid % kWave == 0) lds4[tid / kWave] = v;
  __syncthreads();  // also publishes fsc
  v = lds4[0];
#pragma unroll
  for (int i = 1; i < NW; ++i) { v.x += lds4[i].x; v.y += lds4[i].y; v.z += lds4[i].z; }
  const float eta = v.x;
  const float wz = (finite && b.p.n_plain < b.K) ? v.z / eta : 0.0f;
  for (int r = tid; r < b.TM; r += kBatchMaxTile) {
    // the tiles' partials of row r, kIn loads in flight, added in tile order
    constexpr int kIn = 16;
    float tot = 0.0f;
    int c = 0;
    for (; c + kIn <= ntile; c += kIn) {
      float x[kIn];
#pragma unroll
      for (int q = 0; q < kIn; ++q) x[q] = b.tile_part[static_cast<int64_t>(c + q) * b.TM + r];
#pragma unroll
      for (int q = 0; q < kIn; ++q) tot += fsc[c + q] * x[q];
    }
    for (; c < ntile; ++c) tot += fsc[c] * b.tile_part[static_cast<int64_t>(c) * b.TM + r];
    if (eta > 0.0f) {
      float qv = tot / eta;
      if (wz != 0.0f) qv -= b.u[r] * wz;
      b.u[r] = b.u[r] + b.step * qv;
    }
  }
  if (tid == 0) {
    DevState* st = b.st;
    st->wz = wz;
    st->stats[0] = rho;
    st->stats[1] = finite ? eta : 0.0f;
    st->stats[2] = finite ? rho - b.lambda * logf(eta / static_cast<float>(b.K)) : inf;
    st->stats[3] = finite ? (eta * eta) / v.y : 0.0f;
    st->status = finite ? MPPI_OK : MPPI_ENUMERIC;
    st->iteration = st->iteration + 1u;
  }
}

template <class Model, int INTEG, class Cost, bool COUNT>
__global__ __launch_bounds__(kBatchMaxTile) void batch_one_launch_kernel(BatchPlan b) {
  extern __shared__ float4 lds[];
  __shared__ int s_last;
  uint32_t* done = b.done;
  const int2 w = b.fused_items[blockIdx.x];
  const BatchInst& inst = b.insts[w.x];
  const float S_k = tile_rollout_drawn<Model, INTEG, Cost, COUNT>(inst, w.y, lds);
  tile_softmin_partials(inst, w.y, S_k);
  // the tile's partials are visible before it is counted
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  const int ntile = (inst.K + kBatchMaxTile - 1) / kBatchMaxTile;
  if (threadIdx.x == 0) {
    const uint32_t old =
        __hip_atomic_fetch_add(&done[w.x], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    s_last = old + 1u == static_cast<uint32_t>(ntile);
  }
  __syncthreads();
  if (!__builtin_amdgcn_readfirstlane(s_last)) return;  // the whole workgroup
  // this workgroup completed the instance's last tile
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  instance_combine(inst, ntile);
  if (threadIdx.x == 0) __hip_atomic_store(&done[w.x], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// One iteration of a single instance of the double integrator with forward
// Euler and the quadratic cost, in one launch and time-parallel.  With Euler
// the model is linear: the velocity after step t is v_0 + sum_{s<=t} dt a_s
// and the position after step t is p_0 + sum_{s<=t} dt vel_s, two prefix
// sums over time, after which every running cost is evaluated in parallel.
// A sample's horizon is spread over the 16 lanes of a DPP row: lane c owns
// the steps [cC, cC + C), C even, so the Philox calls of its steps (two
// steps of the two controls each) are its own.  A workgroup holds 16
// samples (one tile) and
//   1. each lane draws its steps' noise (exactly as the noise kernel draws
//      it; staged through LDS so that the workgroup stores it in rows of 16
//      consecutive samples) and forms v = mean u + eps;
//   2. the velocities and positions come from two row scans; each lane sums
//      its steps' running costs (Kahan), the row adds the lanes' sums in a
//      fixed order and the terminal cost of the lane that holds x_T;
//   3. the tile's samples are weighted against the tile's minimum, and its
//      weighted noise rows sum_k e_k eps[r][k] formed from the lanes' own
//      steps (xor shuffles over a wave's four samples, then the four waves
//      in a fixed order through LDS);
//   4. the completion counter and the last workgroup's combination are those
//      of the batch's one-launch form (instance_combine).
// ---------------------------------------------------------------------------
constexpr int kDiLanes = 16;                          // lanes per sample
constexpr int kDiSamples = kBatchMaxTile / kDiLanes;  // samples per workgroup

template <int C>
__global__ __launch_bounds__(kBatchMaxTile) void di_iteration_kernel(BatchInst b, uint32_t* done) {
  constexpr int N = 4, M = 2, NW = kBatchMaxTile / kWave;
  static_assert(C % 2 == 0, "whole Philox calls per lane");
  using Cost = CostQuadratic;
  __shared__ float part[NW][kDiLanes * M * C];
  __shared__ float nz[kDiLanes * M * C][kDiSamples + 1];  // [row][sample], padded
  __shared__ float lds_m[NW];
  __shared__ float4 lds4[NW];
  __shared__ int s_last;
  const DevParams& p = b.p;
  const int tid = threadIdx.x, lane = tid % kWave, wv = tid / kWave;
  const int c = tid % kDiLanes;
  const int k = blockIdx.x * kDiSamples + tid / kDiLanes;
  const bool valid = k < b.K;
  const int kk = valid ? k : b.K - 1;  // lanes past K recompute sample K-1, store nothing
  const int T = b.T;
  const uint32_t it = b.st->iteration;  // read before this workgroup is counted
  const bool plain = kk < p.n_plain;
  const float mean = plain ? 1.0f : 0.0f;
  const bool zero = p.mean_sample && kk == 0;
  const int t0 = c * C;

  // 1. the noise of the own steps (rows 2t, 2t + 1), and v
  float eps[C][M], v[C][M];
#pragma unroll
  for (int q = 0; q < C / 2; ++q) {
    const int call = t0 / 2 + q;
    float z[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    if (2 * call < T)
      noise::emit_call(b.key0, b.key1, it, b.instance, kk, call, 0, M, b.sigma.v, b.eps, b.ldk,
                       p.sigma_t, zero, z);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int i = 2 * q + h, t = t0 + i;
#pragma unroll
      for (int j = 0; j < M; ++j) {
        eps[i][j] = z[M * h + j];
        v[i][j] = t < T ? mean * b.u[t * M + j] + eps[i][j] : 0.0f;
        nz[t * M + j][tid / kDiLanes] = eps[i][j];
      }
    }
  }
  __syncthreads();
  for (int idx = tid; idx < b.TM * kDiSamples; idx += kBatchMaxTile) {
    const int r = idx / kDiSamples, sm = idx % kDiSamples;
    const int ks = blockIdx.x * kDiSamples + sm;
    if (ks < b.K) b.eps[static_cast<int64_t>(r) * b.ldk + ks] = nz[r][sm];
  }

  // 2. velocities (increments dt a_t), then positions (increments dt vel_t)
  float vel[M], pos[M];
  {
    float tot[M] = {0.0f, 0.0f};
#pragma unroll
    for (int i = 0; i < C; ++i)
#pragma unroll
      for (int j = 0; j < M; ++j) tot[j] += p.dt * v[i][j];
#pragma unroll
    for (int j = 0; j < M; ++j) vel[j] = b.x0[2 + j] + row_exclusive(tot[j]);
    float pv[M] = {0.0f, 0.0f}, w[M] = {vel[0], vel[1]};
#pragma unroll
    for (int i = 0; i < C; ++i)
#pragma unroll
      for (int j = 0; j < M; ++j) {
        pv[j] += p.dt * w[j];
        w[j] += p.dt * v[i][j];
      }
#pragma unroll
    for (int j = 0; j < M; ++j) pos[j] = b.x0[j] + row_exclusive(pv[j]);
  }
  typename Cost::State cs;
  float sum = 0.0f, sum_c = 0.0f, term = 0.0f;
#pragma unroll
  for (int i = 0; i < C; ++i) {
    const int t = t0 + i;
    if (t < T) {
      // x_{t+1}: the Euler step of the double integrator
      float x[N], comp[N] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int j = 0; j < M; ++j) {
        x[j] = pos[j] + p.dt * vel[j];
        x[2 + j] = vel[j] + p.dt * v[i][j];
      }
      bool hit;
      float l = Cost::template running<N, M>(x, comp, v[i], t, p, nullptr, cs, hit);
      if (p.importance && plain) l += is_term<M>(p, t, v[i], b.u + t * M);
      if (p.cosines) l += inflation(p);
      const float y = l - sum_c;
      const float s2 = sum + y;
      sum_c = (s2 - sum) - y;
      sum = s2;
      if (t == T - 1) term = terminal_cost<Cost, N>(x, T, p, nullptr, cs);
#pragma unroll
      for (int j = 0; j < M; ++j) {
        pos[j] = x[j];
        vel[j] = x[2 + j];
      }
    }
  }
  const int row0 = lane & ~(kDiLanes - 1);
  const float run = __shfl(row_scan(sum - sum_c), row0 + kDiLanes - 1, kWave);
  const float J0 = run + __shfl(term, row0 + (T - 1) / C, kWave);
  const float J = __builtin_isfinite(J0) ? J0 : __builtin_inff();
  if (valid && c == 0) b.S[k] = J;

  // 3. the tile's weights and weighted noise rows
  const int tile = blockIdx.x;
  const float inf = __builtin_inff();
  const float mt = block_min<NW>(valid ? J : inf, lds_m);
  const float ek = (valid && J < inf) ? expf((mt - J) * b.inv_lambda) : 0.0f;
  const float e1 = c == 0 ? ek : 0.0f;  // each sample once
  float4 st4{wave_sum(e1), wave_sum(e1 * e1), wave_sum(kk >= p.n_plain ? e1 : 0.0f), 0.0f};
  if (lane == 0) lds4[wv] = st4;
#pragma unroll
  for (int i = 0; i < C; ++i)
#pragma unroll
    for (int j = 0; j < M; ++j) {
      float y = ek * eps[i][j];
      y += __shfl_xor(y, 16, kWave);
      y += __shfl_xor(y, 32, kWave);
      if (lane < kDiLanes) part[wv][(t0 + i) * M + j] = y;
    }
  __syncthreads();
  if (tid == 0) {
    float4 a = lds4[0];
#pragma unroll
    for (int i = 1; i < NW; ++i) { a.x += lds4[i].x; a.y += lds4[i].y; a.z += lds4[i].z; }
    b.tile_stat[tile] = float4{mt, a.x, a.y, a.z};
  }
  static_assert(NW == 4, "the wave sums are added as a fixed tree of four");
  for (int r = tid; r < b.TM; r += kBatchMaxTile)
    b.tile_part[static_cast<int64_t>(tile) * b.TM + r] =
        (part[0][r] + part[1][r]) + (part[2][r] + part[3][r]);

  // 4. count the tile; the last one combines the tiles
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  const int ntile = static_cast<int>(gridDim.x);
  if (tid == 0) {
    const uint32_t old = __hip_atomic_fetch_add(done, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    s_last = old + 1u == static_cast<uint32_t>(ntile);
  }
  __syncthreads();
  if (!__builtin_amdgcn_readfirstlane(s_last)) return;  // the whole workgroup
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  instance_combine(b, ntile);
  if (tid == 0) __hip_atomic_store(done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

namespace {

using BatchFn = void (*)(const BatchInst*, const int2*);
using OneLaunchFn = void (*)(BatchPlan);

template <class Model, int INTEG, class Cost>
OneLaunchFn pick_one_launch(bool count) {
  if (count) return batch_one_launch_kernel<Model, INTEG, Cost, true>;
  return batch_one_launch_kernel<Model, INTEG, Cost, false>;
}

template <class Model, int INTEG>
OneLaunchFn pick_one_launch_wheeled(uint32_t cost, bool count) {
  switch (cost) {
    case MPPI_COST_PATH_CIRCLES: return pick_one_launch<Model, INTEG, CostPath<true>>(count);
    case MPPI_COST_PATH_COSTMAP: return pick_one_launch<Model, INTEG, CostPath<false>>(count);
    case MPPI_COST_GOAL_CIRCLES: return pick_one_launch<Model, INTEG, CostGoalCircles>(count);
    case MPPI_COST_QUADRATIC: return pick_one_launch<Model, INTEG, CostQuadratic>(count);
    case MPPI_COST_TRACK: return pick_one_launch<Model, INTEG, CostTrack>(count);
    default: return nullptr;
  }
}

template <int INTEG>
OneLaunchFn pick_one_launch_model(uint32_t dynamics, uint32_t cost, bool accurate, bool count) {
  switch (dynamics) {
    case MPPI_DYN_DOUBLE_INTEGRATOR:
      if (cost == MPPI_COST_QUADRATIC)
        return pick_one_launch<DoubleIntegrator, INTEG, CostQuadratic>(count);
      if (cost == MPPI_COST_TRACK) return pick_one_launch<DoubleIntegrator, INTEG, CostTrack>(count);
      return nullptr;
    case MPPI_DYN_BICYCLE:
      return accurate ? pick_one_launch_wheeled<Bicycle<false>, INTEG>(cost, count)
                      : pick_one_launch_wheeled<Bicycle<true>, INTEG>(cost, count);
    case MPPI_DYN_QUADROTOR:
      if (cost == MPPI_COST_HOVER) return pick_one_launch<Quadrotor, INTEG, CostHover>(count);
      if (cost == MPPI_COST_QUADRATIC)
        return pick_one_launch<Quadrotor, INTEG, CostQuadratic>(count);
      if (cost == MPPI_COST_TRACK) return pick_one_launch<Quadrotor, INTEG, CostTrack>(count);
      return nullptr;
    default: return nullptr;
  }
}

OneLaunchFn pick_one_launch_fn(uint32_t dynamics, uint32_t integrator, uint32_t cost,
                                bool accurate, bool count) {
  return integrator == MPPI_INT_EULER
             ? pick_one_launch_model<kEuler>(dynamics, cost, accurate, count)
             : pick_one_launch_model<kRK4>(dynamics, cost, accurate, count);
}

template <class Model, int INTEG, class Cost>
BatchFn pick(bool count) {
  if (count) return batch_rollout_kernel<Model, INTEG, Cost, true>;
  return batch_rollout_kernel<Model, INTEG, Cost, false>;
}

template <class Model, int INTEG>
BatchFn pick_generic(uint32_t cost, bool count) {
  if (cost == MPPI_COST_QUADRATIC) return pick<Model, INTEG, CostQuadratic>(count);
  if (cost == MPPI_COST_TRACK) return pick<Model, INTEG, CostTrack>(count);
  return nullptr;
}

template <class Model, int INTEG>
BatchFn pick_wheeled(uint32_t cost, bool count) {
  switch (cost) {
    case MPPI_COST_PATH_CIRCLES: return pick<Model, INTEG, CostPath<true>>(count);
    case MPPI_COST_PATH_COSTMAP: return pick<Model, INTEG, CostPath<false>>(count);
    case MPPI_COST_GOAL_CIRCLES: return pick<Model, INTEG, CostGoalCircles>(count);
    default: return pick_generic<Model, INTEG>(cost, count);
  }
}

template <int INTEG>
BatchFn pick_model(uint32_t dynamics, uint32_t cost, bool accurate, bool count) {
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

}  // namespace

hipError_t launch_batch_noise(const BatchPlan& b, hipStream_t stream) {
  hipLaunchKernelGGL(batch_noise_kernel, dim3(b.n_sample_tiles), dim3(b.tile), 0, stream,
                     b.insts, b.sample_tiles);
  return hipGetLastError();
}

hipError_t launch_batch_rollout(uint32_t dynamics, uint32_t integrator, uint32_t cost,
                                bool accurate_trig, bool count, const BatchPlan& b,
                                hipStream_t stream) {
  BatchFn fn = integrator == MPPI_INT_EULER ? pick_model<kEuler>(dynamics, cost, accurate_trig, count)
                                            : pick_model<kRK4>(dynamics, cost, accurate_trig, count);
  if (!fn) return hipErrorInvalidValue;
  if (b.rollout_lds > 48 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       static_cast<int>(b.rollout_lds));
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(fn, dim3(b.n_sample_tiles), dim3(b.tile), b.rollout_lds, stream, b.insts,
                     b.sample_tiles);
  return hipGetLastError();
}

hipError_t launch_batch_update(const BatchPlan& b, hipStream_t stream) {
  hipLaunchKernelGGL(batch_weights_kernel, dim3(b.n_inst), dim3(kWeightsBlock), 0, stream, b.insts);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(batch_gemv_kernel, dim3(b.n_row_tiles), dim3(kGemvBlock), 0, stream, b.insts,
                     b.row_tiles);
  return hipGetLastError();
}

bool batch_one_launch_supported(uint32_t dynamics, uint32_t integrator, uint32_t cost) {
  return pick_one_launch_fn(dynamics, integrator, cost, false, false) != nullptr;
}

hipError_t launch_batch_one_launch(uint32_t dynamics, uint32_t integrator, uint32_t cost,
                                   bool accurate_trig, bool count, const BatchPlan& b,
                                   hipStream_t stream) {
  OneLaunchFn fn = pick_one_launch_fn(dynamics, integrator, cost, accurate_trig, count);
  if (!fn || b.n_fused_items < 1) return hipErrorInvalidValue;
  if (b.rollout_lds > 48 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       static_cast<int>(b.rollout_lds));
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(fn, dim3(static_cast<unsigned>(b.n_fused_items)), dim3(kBatchMaxTile),
                     b.rollout_lds, stream, b);
  return hipGetLastError();
}

bool di_iteration_supported(uint32_t dynamics, uint32_t integrator, uint32_t cost, int K, int T) {
  return dynamics == MPPI_DYN_DOUBLE_INTEGRATOR && integrator == MPPI_INT_EULER &&
         cost == MPPI_COST_QUADRATIC && K >= 1 && T >= 1 && T <= 256 &&
         (K + kDiSamples - 1) / kDiSamples <= kOneLaunchMaxTiles;
}

int di_iteration_tiles(int K) { return (K + kDiSamples - 1) / kDiSamples; }

hipError_t launch_di_iteration(const BatchInst& b, uint32_t* d_done, hipStream_t stream) {
  if (!di_iteration_supported(MPPI_DYN_DOUBLE_INTEGRATOR, MPPI_INT_EULER, MPPI_COST_QUADRATIC, b.K,
                              b.T) ||
      b.TM != 2 * b.T)
    return hipErrorInvalidValue;
  // C = 2 ceil(T / 32): 16 lanes cover the horizon in whole Philox calls
  const int C = 2 * ((b.T + 31) / 32);
  using Fn = void (*)(BatchInst, uint32_t*);
  Fn fn = nullptr;
  switch (C) {
    case 2: fn = di_iteration_kernel<2>; break;
    case 4: fn = di_iteration_kernel<4>; break;
    case 6: fn = di_iteration_kernel<6>; break;
    case 8: fn = di_iteration_kernel<8>; break;
    case 10: fn = di_iteration_kernel<10>; break;
    case 12: fn = di_iteration_kernel<12>; break;
    case 14: fn = di_iteration_kernel<14>; break;
    case 16: fn = di_iteration_kernel<16>; break;
    default: return hipErrorInvalidValue;
  }
  hipLaunchKernelGGL(fn, dim3(static_cast<unsigned>(di_iteration_tiles(b.K))), dim3(kBatchMaxTile),
                     0, stream, b, d_done);
  return hipGetLastError();
}

hipError_t launch_batch_set_iteration(const BatchPlan& b, uint32_t iteration, hipStream_t stream) {
  hipLaunchKernelGGL(batch_set_iteration_kernel, dim3((b.n_inst + 255) / 256), dim3(256), 0, stream,
                     b.insts, b.n_inst, iteration);
  return hipGetLastError();
}

}  // namespace mppi
