// Kernels on the nominal control sequence u between iterations: the MPC
// warm-start shift (arXiv 2409.07563, section "Beginner": a new MPC
// iteration samples around the previous sequence moved forward by the
// optimisation stride) and the reset of gradient mode's differentiation tape
// (the weights kernel records each update's u and Philox iteration word, so
// that the reverse pass can rebuild every iteration).  Both are kernels, so
// they stay in stream order and may be captured in a graph.
#include "common.h"

namespace mppi {

constexpr int kControlsBlock = 256;

// One workgroup: u is staged in LDS (T * m floats), then rewritten.
__device__ __forceinline__ void shift_body(float* __restrict__ u, int T, int m, int steps,
                                           int fill) {
  extern __shared__ float old[];
  const int TM = T * m;
  for (int i = threadIdx.x; i < TM; i += blockDim.x) old[i] = u[i];
  __syncthreads();
  for (int i = threadIdx.x; i < TM; i += blockDim.x) {
    const int t = i / m, j = i - t * m;
    const int src = t + steps;  // steps <= T: no overflow
    float val;
    if (src < T) {
      val = old[src * m + j];
    } else {
      val = fill == 0 ? old[(T - 1) * m + j] : 0.0f;
    }
    u[i] = val;
  }
}

__global__ __launch_bounds__(kControlsBlock) void shift_kernel(float* __restrict__ u, int T, int m,
                                                               int steps, int fill) {
  shift_body(u, T, m, steps, fill);
}

__global__ __launch_bounds__(kControlsBlock) void batch_shift_kernel(
    const BatchInst* __restrict__ insts, int steps, int fill) {
  const BatchInst& b = insts[blockIdx.x];
  const int m = b.TM / b.T;
  shift_body(b.u, b.T, m, steps < b.T ? steps : b.T, fill);
}

namespace {
hipError_t allow_lds(const void* fn, size_t bytes) {
  if (bytes <= 48 * 1024) return hipSuccess;
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                             static_cast<int>(bytes));
}
}  // namespace

hipError_t launch_shift(float* d_u, int T, int m, int steps, int fill, hipStream_t stream) {
  if (steps < 0 || T < 1 || m < 1) return hipErrorInvalidValue;
  if (steps > T) steps = T;
  const size_t lds = sizeof(float) * static_cast<size_t>(T) * m;
  hipError_t e = allow_lds(reinterpret_cast<const void*>(shift_kernel), lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(shift_kernel, dim3(1), dim3(kControlsBlock), lds, stream, d_u, T, m, steps,
                     fill);
  return hipGetLastError();
}

hipError_t launch_batch_shift(const BatchPlan& b, int steps, int fill, hipStream_t stream) {
  if (steps < 0) return hipErrorInvalidValue;
  hipError_t e = allow_lds(reinterpret_cast<const void*>(batch_shift_kernel), b.max_tm_bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(batch_shift_kernel, dim3(b.n_inst), dim3(kControlsBlock), b.max_tm_bytes,
                     stream, b.insts, steps, fill);
  return hipGetLastError();
}

__global__ void tape_reset_kernel(int32_t* count) { *count = 0; }

hipError_t launch_tape_reset(int32_t* d_count, hipStream_t stream) {
  hipLaunchKernelGGL(tape_reset_kernel, dim3(1), dim3(1), 0, stream, d_count);
  return hipGetLastError();
}

}  // namespace mppi
