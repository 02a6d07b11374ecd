// Steps (a3)-(a6): baseline, normaliser, weights and control update
// (arXiv 2409.07563, Algorithm 1 and Eq. mppi_update_rule).
//
// Two kernels, both with a fixed reduction order (bitwise reproducible):
//  * partials: grid (chunk of 256 samples, block of rows).  Each block finds
//    its chunk minimum rho_c, forms e_k = exp(-(J_k - rho_c)/lambda), and
//    reduces eta_c = sum e_k, sum e_k^2 and, for each of its rows r of the
//    [T*m][ldk] noise, N_c[r] = sum_k e_k eps[r][k].  eps is read exactly once
//    overall, coalesced along k.
//  * merge: rho = min_c rho_c, alpha_c = exp(-(rho_c - rho)/lambda),
//    eta = sum_c alpha_c eta_c and U[r] = u[r] + sum_c alpha_c N_c[r] / eta.
// In exact arithmetic this equals the global formulas of Algorithm 1 (the
// per-chunk baseline cancels in the ratio, as the paper notes for rho).
#include "common.h"

namespace mppi {

constexpr int kChunk = 256;   // samples per partial block (one per thread)
constexpr int kRowsPerBlock = 8;
constexpr int kMergeRows = 64;
constexpr int kMaxChunks = 4096;  // K <= 2^20

int softmin_chunks(int K) { return (K + kChunk - 1) / kChunk; }

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

__global__ __launch_bounds__(kChunk) void softmin_partials_kernel(
    const float* __restrict__ S, const float* __restrict__ eps, int64_t ldk, int K, int TM,
    float inv_lambda, float* __restrict__ chunk_min, float* __restrict__ chunk_sum,
    float* __restrict__ chunk_sum2, float* __restrict__ chunk_num) {
  __shared__ float lds[kChunk / kWave];
  const int c = blockIdx.x;
  const int k = c * kChunk + threadIdx.x;
  const float s = k < K ? S[k] : __builtin_inff();
  const float rho_c = block_min<kChunk / kWave>(s, lds);
  // samples with J = +inf (and whole chunks of them) get weight 0
  const float e = (s < __builtin_inff()) ? expf((rho_c - s) * inv_lambda) : 0.0f;
  if (blockIdx.y == 0) {
    const float se = block_sum<kChunk / kWave>(e, lds);
    const float se2 = block_sum<kChunk / kWave>(e * e, lds);
    if (threadIdx.x == 0) {
      chunk_min[c] = rho_c;
      chunk_sum[c] = se;
      chunk_sum2[c] = se2;
    }
  }
  const int r0 = blockIdx.y * kRowsPerBlock;
  const int r1 = min(r0 + kRowsPerBlock, TM);
  for (int r = r0; r < r1; ++r) {
    const float val = k < K ? e * eps[static_cast<int64_t>(r) * ldk + k] : 0.0f;
    const float tot = block_sum<kChunk / kWave>(val, lds);
    if (threadIdx.x == 0) chunk_num[static_cast<int64_t>(c) * TM + r] = tot;
  }
}

// grid: ceil(TM / 64) blocks of 256 threads (4 waves).  Lane = row, wave =
// residue class of the chunk index.
__global__ __launch_bounds__(256) void softmin_merge_kernel(
    const float* __restrict__ chunk_min, const float* __restrict__ chunk_sum,
    const float* __restrict__ chunk_sum2, const float* __restrict__ chunk_num, int nchunk,
    int K, int TM, float lambda, float inv_lambda, float* __restrict__ u,
    DevState* __restrict__ st) {
  __shared__ float alpha[kMaxChunks];
  __shared__ float lds[4];
  __shared__ float part[4][kMergeRows];
  float m = __builtin_inff();
  for (int c = threadIdx.x; c < nchunk; c += 256) m = fminf(m, chunk_min[c]);
  const float rho = block_min<4>(m, lds);
  const bool finite = rho < __builtin_inff();
  float se = 0.0f, se2 = 0.0f;
  for (int c = threadIdx.x; c < nchunk; c += 256) {
    const float rc = chunk_min[c];
    const float a = (finite && rc < __builtin_inff()) ? expf((rho - rc) * inv_lambda) : 0.0f;
    alpha[c] = a;
    se += a * chunk_sum[c];
    se2 += a * a * chunk_sum2[c];
  }
  const float eta = block_sum<4>(se, lds);
  const float sum_e2 = block_sum<4>(se2, lds);  // the barriers also publish alpha[]
  const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
  const int r = blockIdx.x * kMergeRows + lane;
  float acc = 0.0f;
  if (r < TM)
    for (int c = wv; c < nchunk; c += 4) acc += alpha[c] * chunk_num[static_cast<int64_t>(c) * TM + r];
  part[wv][lane] = acc;
  __syncthreads();
  if (wv == 0 && r < TM && finite) {
    const float tot = ((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane];
    u[r] = u[r] + tot / eta;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->stats[0] = rho;
    st->stats[1] = finite ? eta : 0.0f;
    st->stats[2] = finite ? rho - lambda * logf(eta / static_cast<float>(K)) : __builtin_inff();
    st->stats[3] = finite ? (eta * eta) / sum_e2 : 0.0f;
    st->status = finite ? MPPI_OK : MPPI_ENUMERIC;
    st->iteration = st->iteration + 1u;
  }
}

hipError_t launch_softmin_update(const float* d_S, const float* d_eps, int64_t ldk, int K,
                                 int TM, float lambda, const SoftminLayout& L, float* d_u,
                                 DevState* d_state, hipStream_t stream) {
  const float inv_lambda = static_cast<float>(1.0 / static_cast<double>(lambda));
  dim3 g1(L.nchunk, (TM + kRowsPerBlock - 1) / kRowsPerBlock);
  hipLaunchKernelGGL(softmin_partials_kernel, g1, dim3(kChunk), 0, stream, d_S, d_eps, ldk, K, TM,
                     inv_lambda, L.chunk_min, L.chunk_sum, L.chunk_sum2, L.chunk_num);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  dim3 g2((TM + kMergeRows - 1) / kMergeRows);
  hipLaunchKernelGGL(softmin_merge_kernel, g2, dim3(256), 0, stream, L.chunk_min, L.chunk_sum,
                     L.chunk_sum2, L.chunk_num, L.nchunk, K, TM, lambda, inv_lambda, d_u, d_state);
  return hipGetLastError();
}

// w_k = exp(-(J_k - rho)/lambda) / eta from the last merge's rho and eta.
__global__ __launch_bounds__(256) void weights_kernel(const float* __restrict__ S, int K,
                                                      float inv_lambda,
                                                      const DevState* __restrict__ st,
                                                      float* __restrict__ w) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  const float rho = st->stats[0], eta = st->stats[1];
  const float s = S[k];
  w[k] = (eta > 0.0f && s < __builtin_inff()) ? expf((rho - s) * inv_lambda) / eta : 0.0f;
}

hipError_t launch_weights(const float* d_S, int K, float lambda, const DevState* d_state,
                          float* d_w, hipStream_t stream) {
  const float inv_lambda = static_cast<float>(1.0 / static_cast<double>(lambda));
  hipLaunchKernelGGL(weights_kernel, dim3((K + 255) / 256), dim3(256), 0, stream, d_S, K,
                     inv_lambda, d_state, d_w);
  return hipGetLastError();
}

// The iteration word is written by a kernel so that it stays in stream order
// without a host round trip.
__global__ void set_iteration_kernel(DevState* st, uint32_t iteration) {
  st->iteration = iteration;
}

hipError_t launch_set_iteration(DevState* d_state, uint32_t iteration, hipStream_t stream) {
  hipLaunchKernelGGL(set_iteration_kernel, dim3(1), dim3(1), 0, stream, d_state, iteration);
  return hipGetLastError();
}

}  // namespace mppi
