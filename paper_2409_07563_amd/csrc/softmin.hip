// Steps (a3)-(a6) for one instance: the weights and weighted-noise kernels
// (bodies in softmin.h), the weights for inspection and the iteration word.
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

// The weights step of iteration i in workgroup 0 and, in the others, the
// noise of iteration i + 1 (iteration word + 1: the update's rows step the
// word after this kernel) into the other noise buffer: two independent
// pieces of work in one launch, so the latency-bound weights step and the
// VALU-bound noise overlap.  Noise workgroup b covers samples
// (b mod kblocks) * 1024 .. and the Philox calls (b / kblocks) * calls ..
__global__ __launch_bounds__(kWeightsBlock) void weights_noise_kernel(
    const float* __restrict__ S, int K, float lambda, float inv_lambda, float* __restrict__ e,
    DevState* __restrict__ st, int n_plain, TapeRef tape, NoiseJob job) {
  if (blockIdx.x == 0) {
    tape_record(tape, st);
    weights_body(S, K, lambda, inv_lambda, e, st, n_plain, false);
    return;
  }
  const int b = blockIdx.x - 1;
  const int k = (b % job.kblocks) * kWeightsBlock + threadIdx.x;
  if (k >= K) return;
  const uint32_t it = st->iteration + 1u;
  const int ncall = (job.TM + 3) / 4;
  const int c0 = (b / job.kblocks) * job.calls;
  const int m = job.TM / job.T;
  for (int c = c0; c < c0 + job.calls && c < ncall; ++c)
    noise::emit_call(job.key0, job.key1, it, job.instance, k, c, job.TM, m, job.sigma.v, job.eps,
                     job.ldk, job.sigma_t, job.mean_sample && k == 0);
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
    job.kblocks = (K + kWeightsBlock - 1) / kWeightsBlock;
    const int ncall = (job.TM + 3) / 4;
    const int cblocks = (ncall + job.calls - 1) / job.calls;
    hipLaunchKernelGGL(weights_noise_kernel, dim3(1 + job.kblocks * cblocks), dim3(kWeightsBlock),
                       0, stream, d_S, K, lambda, inv_lambda, d_e, d_state, n_plain, tape, job);
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
