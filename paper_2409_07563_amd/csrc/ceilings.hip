// Measured ceilings of the chip the MPPI kernels run on: the VALU issue rate
// of independent instruction chains, the latency of one wave's dependent
// rollout chain, and the launch floor of a captured graph.  Measurement only;
// none of it is part of the MPPI method.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/mppi_ceilings.h"

namespace {

thread_local std::string g_err;

int hip_fail(hipError_t e, const char* what) {
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return -3;
}

#define CEIL_TRY(expr, what)                       \
  do {                                             \
    hipError_t e_ = (expr);                        \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

constexpr int kThreads = 256;

// Eight independent chains per thread; the multiplier and addend come from a
// kernel argument so that nothing folds at compile time.
template <int MODE>
__global__ __launch_bounds__(kThreads) void valu_loop_kernel(int iters, float a, float b,
                                                              float* __restrict__ sink) {
  const int gid = blockIdx.x * kThreads + threadIdx.x;
  if constexpr (MODE == 4) {
    uint32_t x[8];
    const uint32_t k = __float_as_uint(a) | 1u;
#pragma unroll
    for (int i = 0; i < 8; ++i) x[i] = static_cast<uint32_t>(gid * 8 + i);
#pragma unroll 4
    for (int it = 0; it < iters; ++it) {
#pragma unroll
      for (int i = 0; i < 8; ++i) x[i] = (i & 1) ? (x[i] + k) : (x[i] ^ k);
      // rotate the roles so that no chain folds into a constant
#pragma unroll
      for (int i = 0; i < 8; ++i) x[i] = (i & 1) ? (x[i] ^ (k << 1)) : (x[i] + (k << 1));
    }
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) s ^= x[i];
    sink[gid] = static_cast<float>(s);
  } else if constexpr (MODE == 3) {
    uint64_t x[8];
    const uint32_t mul = __float_as_uint(a) | 1u;
#pragma unroll
    for (int i = 0; i < 8; ++i) x[i] = static_cast<uint64_t>(gid * 8 + i);
#pragma unroll 4
    for (int it = 0; it < iters; ++it) {
#pragma unroll
      for (int i = 0; i < 8; ++i) x[i] = static_cast<uint64_t>(static_cast<uint32_t>(x[i])) * mul + x[i];
    }
    uint64_t s = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) s ^= x[i];
    sink[gid] = static_cast<float>(static_cast<uint32_t>(s ^ (s >> 32)));
  } else {
    float x[8], y[2];
#pragma unroll
    for (int i = 0; i < 8; ++i) x[i] = static_cast<float>(gid + i) * 1e-6f;
    y[0] = x[0] * 1e-3f;
    y[1] = x[1] * 1e-3f;
#pragma unroll 4
    for (int it = 0; it < iters; ++it) {
      if constexpr (MODE == 0 || MODE == 1) {
#pragma unroll
        for (int i = 0; i < 8; ++i) x[i] = fmaf(x[i], a, b);
      }
      if constexpr (MODE == 1) {
        y[0] = __builtin_amdgcn_exp2f(y[0]);
        y[1] = __builtin_amdgcn_exp2f(y[1]);
      }
      if constexpr (MODE == 2) {
#pragma unroll
        for (int i = 0; i < 8; ++i) x[i] = __builtin_amdgcn_exp2f(x[i]);
      }
    }
    float s = y[0] + y[1];
#pragma unroll
    for (int i = 0; i < 8; ++i) s += x[i];
    sink[gid] = s;
  }
}

// One wave: each lane runs the forward-Euler double integrator through T
// steps (positions advanced with the old velocity), accumulating a quadratic
// cost.  The controls are first staged into LDS with every global load in
// flight at once (one memory round trip), then read four steps at a time, so
// the dependent arithmetic chain, not the memory latency, sets the time.
constexpr int kChainMaxT = 256;
__global__ __launch_bounds__(64) void chain_kernel(int T, const float4* __restrict__ eps4,
                                                    float* __restrict__ out) {
  __shared__ float4 ctl4[kChainMaxT * 32];  // [T][2][64] floats
  const int lane = threadIdx.x;
  const int n4 = T * 32;
  for (int i0 = 0; i0 < n4; i0 += 64 * 16) {
    float4 v[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) v[j] = eps4[min(i0 + j * 64 + lane, n4 - 1)];
    // i0 + 1024 <= 8192 = kChainMaxT * 32: the tail rows land in the
    // array's padding
#pragma unroll
    for (int j = 0; j < 16; ++j) ctl4[i0 + j * 64 + lane] = v[j];
  }
  __syncthreads();
  const float* ctl = reinterpret_cast<const float*>(ctl4);
  const float dt = 0.02f;
  float px = 0.1f * lane, py = -0.05f * lane, vx = 0.0f, vy = 0.0f, J = 0.0f;
#pragma unroll 4
  for (int t = 0; t < T; ++t) {
    const float ax = ctl[t * 128 + lane], ay = ctl[t * 128 + 64 + lane];
    px = fmaf(dt, vx, px);
    py = fmaf(dt, vy, py);
    vx = fmaf(dt, ax, vx);
    vy = fmaf(dt, ay, vy);
    J = fmaf(px, px, J);
    J = fmaf(py, py, J);
  }
  out[lane] = J + px + py + vx + vy;
}

__global__ void empty_kernel() {}

struct Events {
  hipEvent_t a = nullptr, b = nullptr;
  ~Events() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

}  // namespace

extern "C" {

const char* mppi_ceiling_last_error(void) { return g_err.c_str(); }

int mppi_ceiling_valu(int32_t mode, int32_t blocks, int32_t iters, int32_t reps, float* d_sink,
                      void* hip_stream, double* us_out, double* lane_ops_out) {
  if (mode < 0 || mode > 4 || blocks < 1 || iters < 1 || reps < 1 || !d_sink || !us_out ||
      !lane_ops_out) {
    g_err = "mppi_ceiling_valu: invalid argument";
    return -1;
  }
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  void (*fn)(int, float, float, float*) =
      mode == 0 ? valu_loop_kernel<0> : mode == 1 ? valu_loop_kernel<1>
      : mode == 2 ? valu_loop_kernel<2> : mode == 3 ? valu_loop_kernel<3> : valu_loop_kernel<4>;
  const float a = 0.999999f, b = 1e-7f;
  Events ev;
  CEIL_TRY(hipEventCreate(&ev.a), "event");
  CEIL_TRY(hipEventCreate(&ev.b), "event");
  hipLaunchKernelGGL(fn, dim3(blocks), dim3(kThreads), 0, s, iters, a, b, d_sink);
  CEIL_TRY(hipGetLastError(), "launch");
  CEIL_TRY(hipEventRecord(ev.a, s), "record");
  for (int r = 0; r < reps; ++r) hipLaunchKernelGGL(fn, dim3(blocks), dim3(kThreads), 0, s, iters, a, b, d_sink);
  CEIL_TRY(hipGetLastError(), "launch");
  CEIL_TRY(hipEventRecord(ev.b, s), "record");
  CEIL_TRY(hipEventSynchronize(ev.b), "sync");
  float ms = 0.0f;
  CEIL_TRY(hipEventElapsedTime(&ms, ev.a, ev.b), "elapsed");
  *us_out = 1e3 * static_cast<double>(ms) / reps;
  const double per_trip = mode == 1 ? 10.0 : mode == 4 ? 16.0 : 8.0;
  *lane_ops_out = static_cast<double>(blocks) * kThreads * iters * per_trip;
  return 0;
}

int mppi_ceiling_chain(int32_t T, int32_t reps, const float* d_eps, float* d_out,
                       void* hip_stream, double* us_out) {
  if (T < 1 || T > kChainMaxT || reps < 1 || !d_eps || !d_out || !us_out ||
      reinterpret_cast<uintptr_t>(d_eps) % 16) {
    g_err = "mppi_ceiling_chain: invalid argument (T in 1..256, d_eps 16-byte aligned)";
    return -1;
  }
  const float4* eps4 = reinterpret_cast<const float4*>(d_eps);
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  Events ev;
  CEIL_TRY(hipEventCreate(&ev.a), "event");
  CEIL_TRY(hipEventCreate(&ev.b), "event");
  hipLaunchKernelGGL(chain_kernel, dim3(1), dim3(64), 0, s, T, eps4, d_out);
  CEIL_TRY(hipGetLastError(), "launch");
  CEIL_TRY(hipEventRecord(ev.a, s), "record");
  for (int r = 0; r < reps; ++r) hipLaunchKernelGGL(chain_kernel, dim3(1), dim3(64), 0, s, T, eps4, d_out);
  CEIL_TRY(hipGetLastError(), "launch");
  CEIL_TRY(hipEventRecord(ev.b, s), "record");
  CEIL_TRY(hipEventSynchronize(ev.b), "sync");
  float ms = 0.0f;
  CEIL_TRY(hipEventElapsedTime(&ms, ev.a, ev.b), "elapsed");
  *us_out = 1e3 * static_cast<double>(ms) / reps;
  return 0;
}

int mppi_ceiling_graph(int32_t kernels, int32_t iterations, int32_t reps, void* hip_stream,
                       double* us_out) {
  if (kernels < 1 || kernels > 64 || iterations < 1 || iterations > 1024 || reps < 1 ||
      !hip_stream || !us_out) {
    g_err = "mppi_ceiling_graph: invalid argument";
    return -1;
  }
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  CEIL_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "begin capture");
  for (int i = 0; i < iterations; ++i)
    for (int k = 0; k < kernels; ++k) hipLaunchKernelGGL(empty_kernel, dim3(1), dim3(64), 0, s);
  hipError_t e = hipStreamEndCapture(s, &graph);
  if (e != hipSuccess) return hip_fail(e, "end capture");
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return hip_fail(e, "instantiate");
  Events ev;
  int rc = 0;
  float ms = 0.0f;
  if ((e = hipEventCreate(&ev.a)) != hipSuccess || (e = hipEventCreate(&ev.b)) != hipSuccess ||
      (e = hipGraphLaunch(exec, s)) != hipSuccess || (e = hipEventRecord(ev.a, s)) != hipSuccess) {
    rc = hip_fail(e, "graph warm-up");
  } else {
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = hipGraphLaunch(exec, s);
    if (e == hipSuccess) e = hipEventRecord(ev.b, s);
    if (e == hipSuccess) e = hipEventSynchronize(ev.b);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev.a, ev.b);
    if (e != hipSuccess) rc = hip_fail(e, "graph replay");
  }
  (void)hipGraphExecDestroy(exec);
  if (rc == 0) *us_out = 1e3 * static_cast<double>(ms) / reps;
  return rc;
}

}  // extern "C"
