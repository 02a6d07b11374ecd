// Steps (a3)-(a6) for one instance in its three forms (two-pass, single-pass,
// chunked; bodies in softmin.h), the launches that also draw the next
// iteration's noise, the weights for inspection and the iteration word.
#include "noise.h"
#include "softmin.h"

namespace mppi {

int gemv_rows_per_block() { return 1; }

// The update's record on the tape: slot s = *count takes u and the iteration
// word this update's noise was drawn with, then *count = s + 1 (cap + 1 when
// the tape is full).  All threads of the workgroup call it.
__device__ __forceinline__ void tape_record(const TapeRef& tape, const DevState* st) {
  if (!tape.u) return;
  const int s = *tape.count;
  if (s < tape.cap) {
    float* dst = tape.tape_u + static_cast<int64_t>(s) * tape.TM;
    for (int i = threadIdx.x; i < tape.TM; i += blockDim.x) dst[i] = tape.u[i];
    if (threadIdx.x == 0) tape.tape_word[s] = st->iteration;
  }
  __syncthreads();  // every thread has read *count
  if (threadIdx.x == 0) *tape.count = s < tape.cap ? s + 1 : tape.cap + 1;
}

// The weights step (the iteration word is stepped by the update's rows).
__global__ __launch_bounds__(kWeightsBlock) void weights_kernel_one(
    const float* __restrict__ S, int K, float lambda, float inv_lambda, float* __restrict__ e,
    DevState* __restrict__ st, int n_plain, TapeRef tape) {
  tape_record(tape, st);
  weights_body(S, K, lambda, inv_lambda, e, st, n_plain, false);
}

// The weights step of an iteration in workgroup 0 and, in the others, the
// noise of the next iteration into the other noise buffer: two independent
// pieces of work in one launch, so the latency-bound weights step and the
// VALU-bound noise overlap.
__global__ __launch_bounds__(kWeightsBlock) void weights_noise_kernel(
    const float* __restrict__ S, int K, float lambda, float inv_lambda, float* __restrict__ e,
    DevState* __restrict__ st, int n_plain, TapeRef tape, NoiseJob job) {
  if (blockIdx.x == 0) {
    tape_record(tape, st);
    weights_body(S, K, lambda, inv_lambda, e, st, n_plain, false);
    return;
  }
  next_noise(job, blockIdx.x - 1);
}

// The single-pass update: workgroups 0 .. TM-1 take one row each; with a
// next-noise job the workgroups after them draw the next iteration's noise.
template <int NQ>
__global__ __launch_bounds__(kGemvBlock) void one_pass_kernel(
    const float* __restrict__ S, int K, float lambda, float inv_lambda,
    const float* __restrict__ eps, int64_t ldk, DevState* __restrict__ st, float* __restrict__ u,
    float step, int n_plain, int TM, NoiseJob job) {
  if (static_cast<int>(blockIdx.x) < TM) {
    one_pass_row<NQ>(S, K, lambda, inv_lambda, eps, ldk, st, u, step, blockIdx.x, n_plain);
    return;
  }
  next_noise(job, blockIdx.x - TM);
}

hipError_t launch_update_one_pass(const float* d_S, const float* d_eps, int64_t ldk, int K,
                                  int TM, float lambda, float step, float* d_u,
                                  DevState* d_state, hipStream_t stream, int n_plain,
                                  const NoiseJob* next) {
  if (K < 1 || K > kOnePassMaxK) return hipErrorInvalidValue;
  const float inv_lambda = static_cast<float>(1.0 / static_cast<double>(lambda));
  NoiseJob job{};
  int blocks = TM;
  if (next) {
    job = *next;
    blocks += noise_job_blocks(&job, kGemvBlock);
  }
  const int nq = (K + 4 * kGemvBlock - 1) / (4 * kGemvBlock);
  auto go = [&](auto kernel) {
    hipLaunchKernelGGL(kernel, dim3(blocks), dim3(kGemvBlock), 0, stream, d_S, K, lambda,
                       inv_lambda, d_eps, ldk, d_state, d_u, step, n_plain, TM, job);
  };
  if (nq <= 1) go(one_pass_kernel<1>);
  else if (nq <= 2) go(one_pass_kernel<2>);
  else if (nq <= 4) go(one_pass_kernel<4>);
  else if (nq <= 8) go(one_pass_kernel<8>);
  else go(one_pass_kernel<16>);
  return hipGetLastError();
}

// The chunked update's weights step (workgroups 0 .. C-1) and, with a
// next-noise job, the next iteration's noise (the workgroups after).
__global__ __launch_bounds__(kWChunkBlock) void chunk_weights_kernel(
    const float* __restrict__ S, int K, float inv_lambda, float* __restrict__ e,
    float4* __restrict__ part, int n_plain, int C, NoiseJob job) {
  if (static_cast<int>(blockIdx.x) < C) {
    chunk_weights(S, K, inv_lambda, e, part, blockIdx.x, n_plain);
    return;
  }
  next_noise(job, blockIdx.x - C);
}

__global__ __launch_bounds__(kGemvBlock) void chunked_rows_kernel(
    const float* __restrict__ eps, int64_t ldk, int K, const float* __restrict__ e,
    const float4* __restrict__ part, float lambda, float inv_lambda, DevState* __restrict__ st,
    float* __restrict__ u, float step, int n_plain) {
  chunked_row(eps, ldk, K, e, part, lambda, inv_lambda, st, u, step, blockIdx.x, n_plain);
}

hipError_t launch_update_chunked(const float* d_S, const float* d_eps, int64_t ldk, int K,
                                 int TM, float lambda, float step, float* d_e, float4* d_part,
                                 float* d_u, DevState* d_state, hipStream_t stream, int n_plain,
                                 const NoiseJob* next) {
  const int C = (K + kWChunk - 1) / kWChunk;
  if (K < 1 || C > kMaxWChunks) return hipErrorInvalidValue;
  const float inv_lambda = static_cast<float>(1.0 / static_cast<double>(lambda));
  NoiseJob job{};
  int blocks = C;
  if (next) {
    job = *next;
    blocks += noise_job_blocks(&job, kWChunkBlock);
  }
  hipLaunchKernelGGL(chunk_weights_kernel, dim3(blocks), dim3(kWChunkBlock), 0, stream, d_S, K,
                     inv_lambda, d_e, d_part, n_plain, C, job);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(chunked_rows_kernel, dim3(TM), dim3(kGemvBlock), 0, stream, d_eps, ldk, K,
                     d_e, d_part, lambda, inv_lambda, d_state, d_u, step, n_plain);
  return hipGetLastError();
}

__global__ __launch_bounds__(kGemvBlock) void gemv_kernel_one(
    const float* __restrict__ eps, int64_t ldk, int K, const float* __restrict__ e,
    DevState* __restrict__ st, float* __restrict__ u, float step) {
  gemv_row(eps, ldk, K, e, st, u, step, blockIdx.x, true);
}

hipError_t launch_softmin_update(const float* d_S, const float* d_eps, int64_t ldk, int K,
                                 int TM, float lambda, float step, float* d_e, float* d_u,
                                 DevState* d_state, hipStream_t stream, int n_plain,
                                 const TapeRef& tape, const NoiseJob* next) {
  const float inv_lambda = static_cast<float>(1.0 / static_cast<double>(lambda));
  if (next) {
    NoiseJob job = *next;
    const int blocks = 1 + noise_job_blocks(&job, kWeightsBlock);
    hipLaunchKernelGGL(weights_noise_kernel, dim3(blocks), dim3(kWeightsBlock), 0, stream, d_S,
                       K, lambda, inv_lambda, d_e, d_state, n_plain, tape, job);
  } else {
    hipLaunchKernelGGL(weights_kernel_one, dim3(1), dim3(kWeightsBlock), 0, stream, d_S, K,
                       lambda, inv_lambda, d_e, d_state, n_plain, tape);
  }
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(gemv_kernel_one, dim3(TM), dim3(kGemvBlock), 0, stream, d_eps, ldk, K, d_e,
                     d_state, d_u, step);
  return hipGetLastError();
}

// The weights step alone, its statistics going to a scratch state (the
// reverse pass of several iterations rebuilds each iteration's weights
// without touching the context's state).
hipError_t launch_weights_only(const float* d_S, int K, float lambda, float* d_e,
                               DevState* d_scratch_state, hipStream_t stream) {
  const float inv_lambda = static_cast<float>(1.0 / static_cast<double>(lambda));
  hipLaunchKernelGGL(weights_kernel_one, dim3(1), dim3(kWeightsBlock), 0, stream, d_S, K, lambda,
                     inv_lambda, d_e, d_scratch_state, K, TapeRef{});
  return hipGetLastError();
}

// w_k = exp(-(J_k - rho)/lambda) / eta from the last update's rho and eta.
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
