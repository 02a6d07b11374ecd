// Device bodies of steps (a3)-(a6): baseline, normaliser, weights and control
// update (arXiv 2409.07563, Algorithm 1 and Eq. mppi_update_rule), shared by
// the single-instance kernels (softmin.hip) and the batched kernels
// (batch.hip).  Every reduction has a fixed order (bitwise reproducible).
// The two-pass form:
//  * weights: one workgroup per instance finds rho = min_k J_k, writes
//    e_k = exp(-(J_k - rho)/lambda) (0 for a non-finite J_k), reduces
//    eta = sum e_k and sum e_k^2, and records the statistics;
//  * weighted noise: U[r] = u[r] + (sum_k e_k eps[r][k]) / eta, a matrix-vector
//    product over the [T*m][ldk] noise.  A workgroup of four waves owns a row:
//    its lanes stream the row with 16-byte loads along k (eight in flight per
//    lane), accumulate privately, reduce once per wave and combine the four
//    wave sums in a fixed order, so eps is read exactly once.
// The single-pass form (one_pass_row) folds the weights into the row
// workgroups; the chunked form (chunk_weights, chunked_row) spreads the
// weights over workgroups of 2048 samples, each against its own minimum.
#pragma once

#include "common.h"

namespace mppi {

constexpr int kWeightsBlock = 1024;
constexpr int kGemvBlock = 256;  // one row per workgroup

template <int NW>
__device__ __forceinline__ float block_min(float v, float* lds) {
  v = wave_min(v);
  const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
  __syncthreads();
  if (lane == 0) lds[wv] = v;
  __syncthreads();
  float r = lds[0];
#pragma unroll
  for (int i = 1; i < NW; ++i) r = fminf(r, lds[i]);
  return r;
}

template <int NW>
__device__ __forceinline__ float block_sum(float v, float* lds) {
  v = wave_sum(v);
  const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
  __syncthreads();
  if (lane == 0) lds[wv] = v;
  __syncthreads();
  float r = lds[0];
#pragma unroll
  for (int i = 1; i < NW; ++i) r += lds[i];
  return r;
}

// Sum of two values over the workgroup in one pass (fixed order).
template <int NW>
__device__ __forceinline__ void block_sum2(float& a, float& b, float2* lds) {
  a = wave_sum(a);
  b = wave_sum(b);
  const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
  __syncthreads();
  if (lane == 0) lds[wv] = float2{a, b};
  __syncthreads();
  float2 r = lds[0];
#pragma unroll
  for (int i = 1; i < NW; ++i) { r.x += lds[i].x; r.y += lds[i].y; }
  a = r.x;
  b = r.y;
}

// One workgroup of kWeightsBlock threads per instance.  Also advances the
// instance's iteration word (read by the next sampling step).  The costs are
// taken in chunks of kWeightsChunk per thread, every load of a chunk issued
// before the first is used, so a pass costs a few memory latencies rather than
// one per element; when K fits one chunk (K <= 32768) the costs stay in
// registers between the min pass and the exponential pass.
constexpr int kWeightsChunk = 32;
// Samples k >= n_plain were drawn around zero: their weight mass
// W_Z = sum_{k >= n_plain} w_k goes to st->wz for the update.
// advance: also step the iteration word (otherwise the update's row kernel
// does, after the noise of the next iteration has been drawn from it).
__device__ __forceinline__ void weights_body(const float* __restrict__ S, int K, float lambda,
                                             float inv_lambda, float* __restrict__ e,
                                             DevState* __restrict__ st, int n_plain,
                                             bool advance = true) {
  constexpr int NW = kWeightsBlock / kWave;
  constexpr int kSpan = kWeightsChunk * kWeightsBlock;  // costs per chunk
  __shared__ float lds[NW];
  __shared__ float2 lds2[NW];
  float sv[kWeightsChunk];
  auto load_chunk = [&](int c0) {
#pragma unroll
    for (int q = 0; q < kWeightsChunk; ++q) {
      const int k = c0 + threadIdx.x + q * kWeightsBlock;
      sv[q] = k < K ? S[k] : __builtin_inff();
    }
  };
  float m = __builtin_inff();
  for (int c0 = 0; c0 < K; c0 += kSpan) {
    load_chunk(c0);
#pragma unroll
    for (int q = 0; q < kWeightsChunk; ++q) m = fminf(m, sv[q]);
  }
  const float rho = block_min<NW>(m, lds);
  const bool finite = rho < __builtin_inff();
  float se = 0.0f, se2 = 0.0f, sz = 0.0f;
  for (int c0 = 0; c0 < K; c0 += kSpan) {
    if (K > kSpan) load_chunk(c0);  // one chunk: still in registers
#pragma unroll
    for (int q = 0; q < kWeightsChunk; ++q) {
      const int k = c0 + threadIdx.x + q * kWeightsBlock;
      if (k < K) {
        // non-finite J_k (NaN was turned into +inf by the rollout) gets weight 0
        const float s = sv[q];
        const float ek = (finite && s < __builtin_inff()) ? expf((rho - s) * inv_lambda) : 0.0f;
        e[k] = ek;
        se += ek;
        se2 += ek * ek;
        sz += k >= n_plain ? ek : 0.0f;
      }
    }
  }
  block_sum2<NW>(se, se2, lds2);
  const float eta = se, sum_e2 = se2;
  float wz = 0.0f;
  if (n_plain < K) wz = block_sum<NW>(sz, lds) / eta;  // uniform branch
  if (threadIdx.x == 0) {
    st->wz = finite ? wz : 0.0f;
    st->stats[0] = rho;
    st->stats[1] = finite ? eta : 0.0f;
    st->stats[2] = finite ? rho - lambda * logf(eta / static_cast<float>(K)) : __builtin_inff();
    st->stats[3] = finite ? (eta * eta) / sum_e2 : 0.0f;
    st->status = finite ? MPPI_OK : MPPI_ENUMERIC;
    if (advance) st->iteration = st->iteration + 1u;
  }
}

// Row r of the update, one workgroup of kGemvBlock threads:
// u[r] += step * ((sum_k e_k eps[r][k]) / eta - u[r] W_Z), step the step size
// gamma and W_Z the weight of the samples drawn around zero (whose v - u is
// eps - u).  The row starts 16-byte aligned (ldk is
// a multiple of 64); the last K mod 4 entries go through a scalar tail so the
// unwritten padding of a row is never read.  Eight 16-byte loads of the row
// (and eight of e) are in flight per lane, so a row of up to 8192 samples is
// one memory round trip.  When every cost was non-finite (eta = 0) u is left
// unchanged.
// advance: row 0 steps the iteration word at the end (the single-instance
// update; the weights step then leaves it).
__device__ __forceinline__ void gemv_row(const float* __restrict__ eps, int64_t ldk, int K,
                                         const float* __restrict__ e, DevState* st,
                                         float* __restrict__ u, float step, int r,
                                         bool advance = false) {
  constexpr int NW = kGemvBlock / kWave;
  constexpr int kIn = 8;                     // loads in flight per lane and array
  constexpr int kStride = 4 * kGemvBlock;    // floats per sweep of the workgroup
  __shared__ float part[NW];
  const int tid = threadIdx.x;
  const float* row = eps + static_cast<int64_t>(r) * ldk;
  const int K4 = K & ~3;
  float acc[kIn];
#pragma unroll
  for (int q = 0; q < kIn; ++q) acc[q] = 0.0f;
  int k = 4 * tid;
  for (; k + (kIn - 1) * kStride < K4; k += kIn * kStride) {
    float4 x[kIn], w[kIn];
#pragma unroll
    for (int q = 0; q < kIn; ++q) {
      x[q] = *reinterpret_cast<const float4*>(row + k + q * kStride);
      w[q] = *reinterpret_cast<const float4*>(e + k + q * kStride);
    }
#pragma unroll
    for (int q = 0; q < kIn; ++q)
      acc[q] += w[q].x * x[q].x + w[q].y * x[q].y + w[q].z * x[q].z + w[q].w * x[q].w;
  }
  for (; k < K4; k += kStride) {
    const float4 x = *reinterpret_cast<const float4*>(row + k);
    const float4 w = *reinterpret_cast<const float4*>(e + k);
    acc[0] += w.x * x.x + w.y * x.y + w.z * x.z + w.w * x.w;
  }
  if (K4 + tid < K) acc[0] += e[K4 + tid] * row[K4 + tid];
  const float a = wave_sum(((acc[0] + acc[1]) + (acc[2] + acc[3])) +
                           ((acc[4] + acc[5]) + (acc[6] + acc[7])));
  if (tid % kWave == 0) part[tid / kWave] = a;
  __syncthreads();
  if (tid == 0) {
    float tot = part[0];
#pragma unroll
    for (int i = 1; i < NW; ++i) tot += part[i];
    const float eta = st->stats[1];
    const float wz = st->wz;
    if (eta > 0.0f) {
      float q = tot / eta;
      if (wz != 0.0f) q -= u[r] * wz;
      u[r] = u[r] + step * q;
    }
    if (advance && r == 0) st->iteration = st->iteration + 1u;
  }
}

// The single-pass update of row r (single contexts, K <= kOnePassMaxK): the
// workgroup of row r computes rho, the weights and eta itself from the costs,
// instead of reading them from a weights step, and takes the weighted sum of
// its noise row in the same pass.  Every workgroup runs the same code on the
// same costs, so each finds the same rho, weights and eta (bitwise).  Thread
// t holds samples 4t + 1024q .. + 3 (q < NQ, NQ = ceil(K / 1024)); the noise
// row and the costs are loaded first, all loads in flight together.  Row 0
// records the statistics and the weight mass of the zero-mean samples and
// steps the iteration word.  The weights themselves are not stored (only the
// gradient mode's adjoint reads them, and it uses the two-pass update).

template <int NQ>
__device__ __forceinline__ void one_pass_row(const float* __restrict__ S, int K, float lambda,
                                             float inv_lambda, const float* __restrict__ eps,
                                             int64_t ldk, DevState* st, float* __restrict__ u,
                                             float step, int r, int n_plain) {
  constexpr int NW = kGemvBlock / kWave;
  constexpr int kStride = 4 * kGemvBlock;
  __shared__ float lds[NW];
  __shared__ float4 lds4[NW];
  const int tid = threadIdx.x;
  const float* row = eps + static_cast<int64_t>(r) * ldk;
  const int K4 = K & ~3;
  const float inf = __builtin_inff();
  float4 x[NQ];
  float s[NQ][4];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int k = 4 * tid + q * kStride;
    if (k < K4) {
      x[q] = *reinterpret_cast<const float4*>(row + k);
#pragma unroll
      for (int j = 0; j < 4; ++j) s[q][j] = S[k + j];
    } else {
      x[q] = float4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int j = 0; j < 4; ++j) s[q][j] = inf;
    }
  }
  const int kt = K4 + tid;  // the last K mod 4 samples, one per thread
  const bool tail = kt < K;
  const float xt = tail ? row[kt] : 0.0f;
  const float st_ = tail ? S[kt] : inf;
  float m = st_;
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int j = 0; j < 4; ++j) m = fminf(m, s[q][j]);
  const float rho = block_min<NW>(m, lds);
  const bool finite = rho < inf;
  float dot = 0.0f, se = 0.0f, se2 = 0.0f, sz = 0.0f;
  auto take = [&](int k, float sk, float xk) {
    // non-finite J_k (NaN was turned into +inf by the rollout) gets weight 0
    const float ek = (finite && sk < inf) ? expf((rho - sk) * inv_lambda) : 0.0f;
    se += ek;
    se2 += ek * ek;
    sz += k >= n_plain ? ek : 0.0f;
    dot += ek * xk;
  };
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int k = 4 * tid + q * kStride;
    if (k < K4) {
      take(k, s[q][0], x[q].x);
      take(k + 1, s[q][1], x[q].y);
      take(k + 2, s[q][2], x[q].z);
      take(k + 3, s[q][3], x[q].w);
    }
  }
  if (tail) take(kt, st_, xt);
  // one reduction of (dot, eta, sum e^2, zero-mean mass), fixed order
  float4 v{wave_sum(dot), wave_sum(se), wave_sum(se2), wave_sum(sz)};
  __syncthreads();
  if (tid % kWave == 0) lds4[tid / kWave] = v;
  __syncthreads();
  if (tid != 0) return;
  v = lds4[0];
#pragma unroll
  for (int i = 1; i < NW; ++i) {
    v.x += lds4[i].x; v.y += lds4[i].y; v.z += lds4[i].z; v.w += lds4[i].w;
  }
  const float eta = v.y;
  const float wz = (finite && n_plain < K) ? v.w / eta : 0.0f;
  if (eta > 0.0f) {
    float qv = v.x / eta;
    if (wz != 0.0f) qv -= u[r] * wz;
    u[r] = u[r] + step * qv;
  }
  if (r == 0) {
    st->wz = wz;
    st->stats[0] = rho;
    st->stats[1] = finite ? eta : 0.0f;
    st->stats[2] = finite ? rho - lambda * logf(eta / static_cast<float>(K)) : inf;
    st->stats[3] = finite ? (eta * eta) / v.z : 0.0f;
    st->status = finite ? MPPI_OK : MPPI_ENUMERIC;
    st->iteration = st->iteration + 1u;
  }
}

// The chunked update (single contexts of any size, no gradient mode): the
// weights step is spread over workgroups of kWChunk samples.  Chunk c finds
// its own minimum m_c and writes e'_k = exp(-(J_k - m_c)/lambda) with the
// chunk's sums s_c = sum e'_k, sum e'_k^2 and the zero-mean samples' sum; the
// row workgroups then take rho = min_c m_c, the factors
// f_c = exp(-(m_c - rho)/lambda) (so f_c e'_k is the weight e_k up to
// rounding), eta = sum_c f_c s_c, and the row's sum_c f_c sum_{k in c} e'_k
// eps[r][k].
constexpr int kWChunkBlock = 256;
constexpr int kMaxWChunks = (1 << 20) / kWChunk;  // MPPI's sample limit

__device__ __forceinline__ void chunk_weights(const float* __restrict__ S, int K,
                                              float inv_lambda, float* __restrict__ e,
                                              float4* __restrict__ part, int c, int n_plain) {
  constexpr int NW = kWChunkBlock / kWave;
  constexpr int kPer = kWChunk / kWChunkBlock;
  __shared__ float lds[NW];
  __shared__ float4 lds4[NW];
  const float inf = __builtin_inff();
  const int k0 = c * kWChunk + threadIdx.x;
  float sv[kPer];
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    const int k = k0 + j * kWChunkBlock;
    sv[j] = k < K ? S[k] : inf;
  }
  float m = inf;
#pragma unroll
  for (int j = 0; j < kPer; ++j) m = fminf(m, sv[j]);
  const float mc = block_min<NW>(m, lds);
  float se = 0.0f, se2 = 0.0f, sz = 0.0f;
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    const int k = k0 + j * kWChunkBlock;
    if (k < K) {
      const float ek = sv[j] < inf ? expf((mc - sv[j]) * inv_lambda) : 0.0f;
      e[k] = ek;
      se += ek;
      se2 += ek * ek;
      sz += k >= n_plain ? ek : 0.0f;
    }
  }
  float4 v{wave_sum(se), wave_sum(se2), wave_sum(sz), 0.0f};
  __syncthreads();
  if (threadIdx.x % kWave == 0) lds4[threadIdx.x / kWave] = v;
  __syncthreads();
  if (threadIdx.x != 0) return;
  v = lds4[0];
#pragma unroll
  for (int i = 1; i < NW; ++i) { v.x += lds4[i].x; v.y += lds4[i].y; v.z += lds4[i].z; }
  part[c] = float4{mc, v.x, v.y, v.z};
}

// Row r of the chunked update (kGemvBlock threads); row 0 records the
// statistics and steps the iteration word.
__device__ __forceinline__ void chunked_row(const float* __restrict__ eps, int64_t ldk, int K,
                                           const float* __restrict__ e,
                                           const float4* __restrict__ part, float lambda,
                                           float inv_lambda, DevState* st,
                                           float* __restrict__ u, float step, int r, int n_plain) {
  constexpr int NW = kGemvBlock / kWave;
  constexpr int kIn = 8;
  constexpr int kStride = 4 * kGemvBlock;
  __shared__ float fsc[kMaxWChunks];
  __shared__ float lds[NW];
  __shared__ float4 lds4[NW];
  const int tid = threadIdx.x;
  const float inf = __builtin_inff();
  const int C = (K + kWChunk - 1) / kWChunk;
  // rho, the chunk factors and the sums
  float m = inf;
  for (int c = tid; c < C; c += kGemvBlock) m = fminf(m, part[c].x);
  const float rho = block_min<NW>(m, lds);
  const bool finite = rho < inf;
  float se = 0.0f, se2 = 0.0f, sz = 0.0f;
  for (int c = tid; c < C; c += kGemvBlock) {
    const float4 p = part[c];
    const float f = (finite && p.x < inf) ? expf((rho - p.x) * inv_lambda) : 0.0f;
    fsc[c] = f;
    se += p.y * f;
    se2 += p.z * (f * f);
    sz += p.w * f;
  }
  float4 v{wave_sum(se), wave_sum(se2), wave_sum(sz), 0.0f};
  __syncthreads();
  if (tid % kWave == 0) lds4[tid / kWave] = v;
  __syncthreads();  // also publishes fsc
  v = lds4[0];
#pragma unroll
  for (int i = 1; i < NW; ++i) { v.x += lds4[i].x; v.y += lds4[i].y; v.z += lds4[i].z; }
  const float eta = v.x;
  // the weighted row sum, eight 16-byte loads of the row and of e' in flight
  const float* row = eps + static_cast<int64_t>(r) * ldk;
  const int K4 = K & ~3;
  float acc[kIn];
#pragma unroll
  for (int q = 0; q < kIn; ++q) acc[q] = 0.0f;
  int k = 4 * tid;
  for (; k + (kIn - 1) * kStride < K4; k += kIn * kStride) {
    float4 x[kIn], w[kIn];
#pragma unroll
    for (int q = 0; q < kIn; ++q) {
      x[q] = *reinterpret_cast<const float4*>(row + k + q * kStride);
      w[q] = *reinterpret_cast<const float4*>(e + k + q * kStride);
    }
#pragma unroll
    for (int q = 0; q < kIn; ++q)
      acc[q] += fsc[(k + q * kStride) / kWChunk] *
                (w[q].x * x[q].x + w[q].y * x[q].y + w[q].z * x[q].z + w[q].w * x[q].w);
  }
  for (; k < K4; k += kStride) {
    const float4 x = *reinterpret_cast<const float4*>(row + k);
    const float4 w = *reinterpret_cast<const float4*>(e + k);
    acc[0] += fsc[k / kWChunk] * (w.x * x.x + w.y * x.y + w.z * x.z + w.w * x.w);
  }
  if (K4 + tid < K) acc[0] += fsc[(K4 + tid) / kWChunk] * (e[K4 + tid] * row[K4 + tid]);
  const float a = wave_sum(((acc[0] + acc[1]) + (acc[2] + acc[3])) +
                           ((acc[4] + acc[5]) + (acc[6] + acc[7])));
  // (block_min's reads of lds are two barriers behind)
  if (tid % kWave == 0) lds[tid / kWave] = a;
  __syncthreads();
  if (tid != 0) return;
  float tot = lds[0];
#pragma unroll
  for (int i = 1; i < NW; ++i) tot += lds[i];
  const float wz = (finite && n_plain < K) ? v.z / eta : 0.0f;
  if (eta > 0.0f) {
    float qv = tot / eta;
    if (wz != 0.0f) qv -= u[r] * wz;
    u[r] = u[r] + step * qv;
  }
  if (r == 0) {
    st->wz = wz;
    st->stats[0] = rho;
    st->stats[1] = finite ? eta : 0.0f;
    st->stats[2] = finite ? rho - lambda * logf(eta / static_cast<float>(K)) : inf;
    st->stats[3] = finite ? (eta * eta) / v.y : 0.0f;
    st->status = finite ? MPPI_OK : MPPI_ENUMERIC;
    st->iteration = st->iteration + 1u;
  }
}

}  // namespace mppi
