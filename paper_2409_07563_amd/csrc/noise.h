// Gaussian control noise for step (a1) of the MPPI iteration: eps ~ N(0, Sigma)
// (arXiv 2409.07563, Algorithm 1; the paper does not name its generator).
//
// Counter-based so that any sample/time entry can be produced independently
// and reproduced bit for bit on a CPU:
//   * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
//     easy as 1, 2, 3", SC'11): 10 rounds of the 4x32 round function with the
//     multipliers 0xD2511F53 / 0xCD9E8D57 and the key bumped by the Weyl
//     constants 0x9E3779B9 / 0xBB67AE85 between rounds.
//   * Box-Muller (1958) on 24-bit uniforms.  Every operation below is a single
//     IEEE-754 binary32 operation with round-to-nearest-even; contraction is
//     disabled in this file's functions so the compiler cannot fuse or
//     re-associate them.  Range reductions are exact:
//       -2 ln u1, u1 = j1 2^-24, j1 in [1, 2^24]:  j1 = 2^e f with
//         f in [sqrt(1/2), sqrt(2)) read from the float bits of j1, x = f - 1,
//         ln u1 = (e-24) ln2_hi + ((e-24) ln2_lo + x P(x)), P of degree 9
//         (Chebyshev interpolant of log1p(x)/x on [sqrt(1/2)-1, sqrt(2)-1]);
//         the radius is the correctly rounded sqrt.
//       sincos(2 pi u2), u2 = j2 2^-24: quadrant q = (j2 + 2^21) >> 22, the
//         remainder f = (j2 - q 2^22) 2^-24 in [-1/8, 1/8) is exact, and
//         sin / cos of 2 pi f are the order-9 / order-10 Taylor polynomials in
//         f (binary32 coefficients), evaluated in f^2 by Horner with fma.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace mppi {
namespace noise {

struct Words { uint32_t x0, x1, x2, x3; };

__device__ __forceinline__ Words philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                               uint32_t c3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    // one 32 x 32 -> 64-bit product each (v_mad_u64_u32) gives both halves
    const uint64_t p0 = static_cast<uint64_t>(0xD2511F53u) * c0;
    const uint64_t p1 = static_cast<uint64_t>(0xCD9E8D57u) * c2;
    const uint32_t lo0 = static_cast<uint32_t>(p0), hi0 = static_cast<uint32_t>(p0 >> 32);
    const uint32_t lo1 = static_cast<uint32_t>(p1), hi1 = static_cast<uint32_t>(p1 >> 32);
    const uint32_t n0 = hi1 ^ c1 ^ k0;
    const uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    k0 += 0x9E3779B9u;  // the bump after the last round is never used
    k1 += 0xBB67AE85u;
  }
  return Words{c0, c1, c2, c3};
}

// Horner coefficients (binary32).  kLog: log1p(x)/x, constant term first.
__constant__ static const float kLog[10] = {
    0x1.000000p+0f, -0x1.fffff8p-2f, 0x1.55555ep-2f, -0x1.000424p-2f, 0x1.999e86p-3f,
    -0x1.5423b0p-3f, 0x1.22cf10p-3f, -0x1.0fb036p-3f, 0x1.064786p-3f, -0x1.31335ap-4f};
// sin(2 pi f) / f and cos(2 pi f) as polynomials in f^2, constant term first.
__constant__ static const float kSin[5] = {0x1.921fb6p+2f, -0x1.4abbcep+5f, 0x1.466bc6p+6f,
                                           -0x1.32d2ccp+6f, 0x1.507834p+5f};
__constant__ static const float kCos[6] = {0x1.000000p+0f, -0x1.3bd3ccp+4f, 0x1.03c1f0p+6f,
                                           -0x1.55d3c8p+6f, 0x1.e1f506p+5f, -0x1.a6d1f2p+4f};

// sqrt(-2 ln(j1 * 2^-24)), j1 in [1, 2^24]
__device__ __forceinline__ float radius(uint32_t j1) {
#pragma clang fp contract(off)
  const uint32_t b = __float_as_uint(static_cast<float>(j1));  // exact conversion
  const uint32_t mant = b & 0x7FFFFFu;
  const bool high = mant > 0x3504F3u;                          // f > RN(sqrt 2)
  // f in [sqrt(1/2), sqrt(2)): the mantissa with exponent 0, or -1 when high
  const float f = __uint_as_float(mant | (high ? 0x3F000000u : 0x3F800000u));
  const int e = static_cast<int>(b >> 23) - 127 + (high ? 1 : 0);
  const float x = f - 1.0f;
  float p = kLog[9];
#pragma unroll
  for (int i = 8; i >= 0; --i) p = __builtin_fmaf(p, x, kLog[i]);
  const float ke = static_cast<float>(e - 24);
  const float lnu = __builtin_fmaf(ke, 0x1.62e400p-1f, __builtin_fmaf(ke, 0x1.7f7d1cp-20f, x * p));
  return __builtin_sqrtf(-2.0f * lnu);
}

// (cos, sin)(2 pi j2 2^-24), j2 in [0, 2^24)
__device__ __forceinline__ void angle(uint32_t j2, float& c_out, float& s_out) {
#pragma clang fp contract(off)
  const uint32_t q = (j2 + (1u << 21)) >> 22;
  const int32_t rem = static_cast<int32_t>(j2) - static_cast<int32_t>(q << 22);
  const float f = static_cast<float>(rem) * 0x1p-24f;
  const float y = f * f;
  float ps = kSin[4];
#pragma unroll
  for (int i = 3; i >= 0; --i) ps = __builtin_fmaf(ps, y, kSin[i]);
  const float s = f * ps;
  float c = kCos[5];
#pragma unroll
  for (int i = 4; i >= 0; --i) c = __builtin_fmaf(c, y, kCos[i]);
  // rotate by q * pi/2: (c, s) -> (-s, c) per quadrant
  const uint32_t qq = q & 3u;
  const float cs = (qq & 1u) ? s : c;
  const float sn = (qq & 1u) ? c : s;
  c_out = ((qq + 1u) & 2u) ? -cs : cs;  // negated in quadrants 1 and 2
  s_out = (qq & 2u) ? -sn : sn;         // negated in quadrants 2 and 3
}

// The two standard normals of one Box-Muller pair of Philox words.
__device__ __forceinline__ void box_muller(uint32_t a, uint32_t b, float& z0, float& z1) {
#pragma clang fp contract(off)
  const float r = radius((a >> 8) + 1u);
  float c, s;
  angle(b >> 8, c, s);
  z0 = r * c;
  z1 = r * s;
}

// Philox call c of sample k: the four normals n = 4c .. 4c+3 (n = t*m + j),
// scaled by sigma_j (or sigma_t[n] when a per-step table is given) and stored
// at eps[n * ldk + k] (n < TM); zero for every n when `zero` (the noiseless
// mean sample).  out (optional): the four values as stored (entries n >= TM
// are computed but not stored).
__device__ __forceinline__ void emit_call(uint32_t key0, uint32_t key1, uint32_t iteration,
                                          uint32_t instance, int k, int c, int TM, int m,
                                          const float* sigma, float* __restrict__ eps,
                                          int64_t ldk, const float* __restrict__ sigma_t = nullptr,
                                          bool zero = false, float* out = nullptr) {
  const Words w = philox4x32_10(static_cast<uint32_t>(c), static_cast<uint32_t>(k), iteration,
                                instance, key0, key1);
  float z[4];
  box_muller(w.x0, w.x1, z[0], z[1]);
  box_muller(w.x2, w.x3, z[2], z[3]);
  const int n0 = 4 * c;
  // the four deviations of this call (the per-step table is padded to a
  // multiple of four entries, so one aligned 16-byte read covers them)
  float sg[4];
  if (sigma_t) {
    const float4 s4 = *reinterpret_cast<const float4*>(sigma_t + n0);
    sg[0] = s4.x; sg[1] = s4.y; sg[2] = s4.z; sg[3] = s4.w;
  } else {
    int j = n0 % m;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      sg[s] = sigma[j];
      j = (j + 1 == m) ? 0 : j + 1;
    }
  }
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int n = n0 + s;
    const float v = zero ? 0.0f : sg[s] * z[s];
    if (n < TM) eps[static_cast<int64_t>(n) * ldk + k] = v;
    if (out) out[s] = v;
  }
}

}  // namespace noise

// Workgroup b of the noise part of a launch that also draws the next
// iteration's noise: word *job.word_in + 1 (the word of the noise the launch
// reads, plus one) into job.eps, samples (b mod kblocks) * blockDim .. and the
// Philox calls (b / kblocks) * calls ..; workgroup 0 records the word in
// *job.word_out for the launches after.
__device__ __forceinline__ void next_noise(const NoiseJob& job, int b) {
  const uint32_t it = *job.word_in + 1u;
  if (b == 0 && threadIdx.x == 0) *job.word_out = it;
  const int k = (b % job.kblocks) * static_cast<int>(blockDim.x) + threadIdx.x;
  if (k >= job.K) return;
  const int ncall = (job.TM + 3) / 4;
  const int c0 = (b / job.kblocks) * job.calls;
  const int m = job.TM / job.T;
  for (int c = c0; c < c0 + job.calls && c < ncall; ++c)
    noise::emit_call(job.key0, job.key1, it, job.instance, k, c, job.TM, m, job.sigma.v, job.eps,
                     job.ldk, job.sigma_t, job.mean_sample && k == 0);
}

}  // namespace mppi
