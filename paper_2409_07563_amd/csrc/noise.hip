// Step (a1): fill eps[T][m][ldk] with sigma_j * N(0, 1) draws.
//
// One thread per (sample k, Philox call c): a call yields the four normals
// n = 4c .. 4c+3 of sample k (n = t*m + j).  Lanes of a wave hold consecutive
// samples, so each of the four stores of a wave is one contiguous 256-byte
// row segment of the [T*m][ldk] layout (k fastest).  The kernel is VALU-bound
// (Philox + two Box-Muller pairs, ~50 VALU operations per normal) rather than
// bound by its HBM writes.
#include "common.h"
#include "noise.h"

namespace mppi {

// calls: Philox calls per thread (the calls blockIdx.y * calls + i).
__global__ __launch_bounds__(256) void noise_kernel(uint32_t key0, uint32_t key1,
                                                    const uint32_t* __restrict__ d_iteration,
                                                    uint32_t iteration, uint32_t instance,
                                                    int K, int TM, int m, Sigma8 sigma,
                                                    float* __restrict__ eps, int64_t ldk,
                                                    int calls, const float* __restrict__ sigma_t,
                                                    int mean_sample, uint32_t* d_word_out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  const uint32_t it = d_iteration ? *d_iteration + iteration : iteration;
  if (d_word_out && k == 0 && blockIdx.y == 0) *d_word_out = it;
  const int ncall = (TM + 3) / 4;
  const int c0 = blockIdx.y * calls;
  for (int c = c0; c < c0 + calls && c < ncall; ++c)
    noise::emit_call(key0, key1, it, instance, k, c, TM, m, sigma.v, eps, ldk, sigma_t,
                     mean_sample && k == 0);
}

hipError_t launch_noise(uint64_t seed, const uint32_t* d_iteration, uint32_t iteration,
                        uint32_t instance, int K, int T, int m, const float* sigma,
                        float* d_eps, int64_t ldk, hipStream_t stream, int calls,
                        const float* d_sigma_t, bool mean_sample, uint32_t* d_word_out) {
  if (calls < 1) return hipErrorInvalidValue;
  const int TM = T * m;
  const int ncall = (TM + 3) / 4;
  Sigma8 s{};
  for (int j = 0; j < m; ++j) s.v[j] = sigma[j];
  dim3 grid((K + 255) / 256, (ncall + calls - 1) / calls);
  hipLaunchKernelGGL(noise_kernel, grid, dim3(256), 0, stream, static_cast<uint32_t>(seed),
                     static_cast<uint32_t>(seed >> 32), d_iteration, iteration, instance, K,
                     TM, m, s, d_eps, ldk, calls, d_sigma_t, mean_sample ? 1 : 0, d_word_out);
  return hipGetLastError();
}

// Every possible Box-Muller factor: r[j1-1] for j1 in [1, 2^24], (c, s)[j2]
// for j2 in [0, 2^24).
__global__ __launch_bounds__(256) void noise_tables_kernel(float* __restrict__ r,
                                                           float* __restrict__ c,
                                                           float* __restrict__ s) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= (1u << 24)) return;
  r[j] = noise::radius(j + 1u);
  float cc, ss;
  noise::angle(j, cc, ss);
  c[j] = cc;
  s[j] = ss;
}

hipError_t launch_noise_tables(float* d_r, float* d_c, float* d_s, hipStream_t stream) {
  hipLaunchKernelGGL(noise_tables_kernel, dim3((1u << 24) / 256), dim3(256), 0, stream, d_r,
                     d_c, d_s);
  return hipGetLastError();
}

}  // namespace mppi
