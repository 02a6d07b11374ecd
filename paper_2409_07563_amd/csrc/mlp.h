// The MLP residual g(z) = W3 tanh(W2 tanh(W1 z + b1) + b2) + b3 of the
// learned dynamics, z = (x, v) in R^7, H hidden units (H = 16 MT), evaluated
// for 16 samples at a time on the matrix cores with
// v_mfma_f32_16x16x4_f32 (binary32 operands and accumulation).
//
// Lane layout of a wave (64 lanes): n = lane % 16 is the sample of the tile,
// g = lane / 16 the lane's group.  For D[16][16] += A[16][4] B[4][16] a lane
// holds A[n][g], B[g][n] and D[4g + i][n] (i = 0..3).  Activations therefore
// live in the D layout: lane (g, n) holds hidden rows 16t + 4g + i of sample
// n in register (t, i).  The next layer consumes them without any data
// movement by contracting over a permuted hidden index: its K-step (t, i)
// takes row 16t + 4g + i in lane group g, and the weight operand is packed to
// match (A[m][g] = W[16 mt + m][16 t + 4 g + i]).
//
// Operand packs (host-built at context creation, one row of 64 lane values
// per MFMA operand, read as pack[row * 64 + lane]):
//   forward:  W1 (M-tile t, K-step j: inputs 4j + g, input 7 is padding),
//             W2 (t, K-step (tt, i)), W3 (K-step (tt, i), outputs 0..4 of 16),
//             then the biases in the D layout: b1 (t, i), b2 (t, i), b3 (i).
//   adjoint:  W3^T (t, K-step j: outputs 4j + g), W2^T (t, (tt, i)),
//             W1^T (K-step (tt, i), inputs 0..6 of 16).
#pragma once

#include "common.h"

namespace mppi {
namespace mlp {

typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 mfma(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <int MT>
struct Pack {
  // forward rows
  static constexpr int kW1 = 0;
  static constexpr int kW2 = kW1 + 2 * MT;
  static constexpr int kW3 = kW2 + 4 * MT * MT;
  static constexpr int kB1 = kW3 + 4 * MT;
  static constexpr int kB2 = kB1 + 4 * MT;
  static constexpr int kB3 = kB2 + 4 * MT;
  static constexpr int kFwdRows = kB3 + 4;
  // adjoint rows
  static constexpr int kW3t = 0;
  static constexpr int kW2t = kW3t + 2 * MT;
  static constexpr int kW1t = kW2t + 4 * MT * MT;
  static constexpr int kBwdRows = kW1t + 4 * MT;
};

// The forward operands of one lane, register resident.
template <int MT>
struct Weights {
  float w1_[MT][2];
  float w2_[MT][MT][4];
  float w3_[MT][4];
  f4 b1_[MT], b2_[MT], b3_;

  __device__ __forceinline__ void load(const float* __restrict__ pack, int lane) {
    using P = Pack<MT>;
    auto at = [&](int row) { return pack[row * kWave + lane]; };
#pragma unroll
    for (int t = 0; t < MT; ++t) {
      w1_[t][0] = at(P::kW1 + 2 * t);
      w1_[t][1] = at(P::kW1 + 2 * t + 1);
#pragma unroll
      for (int tt = 0; tt < MT; ++tt)
#pragma unroll
        for (int i = 0; i < 4; ++i) w2_[t][tt][i] = at(P::kW2 + (t * MT + tt) * 4 + i);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        w3_[t][i] = at(P::kW3 + 4 * t + i);
        b1_[t][i] = at(P::kB1 + 4 * t + i);
        b2_[t][i] = at(P::kB2 + 4 * t + i);
      }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) b3_[i] = at(P::kB3 + i);
  }
  __device__ __forceinline__ float w1(int t, int j) const { return w1_[t][j]; }
  __device__ __forceinline__ float w2(int t, int tt, int i) const { return w2_[t][tt][i]; }
  __device__ __forceinline__ float w3(int tt, int i) const { return w3_[tt][i]; }
  __device__ __forceinline__ f4 b1(int t) const { return b1_[t]; }
  __device__ __forceinline__ f4 b2(int t) const { return b2_[t]; }
  __device__ __forceinline__ f4 b3() const { return b3_; }
};

// The same operands read from a pack in memory (LDS) at each use.
template <int MT>
struct PackView {
  const float* pk;  // points at pack[0 * 64 + lane]
  using P = Pack<MT>;
  __device__ __forceinline__ float at(int row) const { return pk[row * kWave]; }
  __device__ __forceinline__ f4 at4(int row) const {
    return f4{at(row), at(row + 1), at(row + 2), at(row + 3)};
  }
  __device__ __forceinline__ float w1(int t, int j) const { return at(P::kW1 + 2 * t + j); }
  __device__ __forceinline__ float w2(int t, int tt, int i) const {
    return at(P::kW2 + (t * MT + tt) * 4 + i);
  }
  __device__ __forceinline__ float w3(int tt, int i) const { return at(P::kW3 + 4 * tt + i); }
  __device__ __forceinline__ f4 b1(int t) const { return at4(P::kB1 + 4 * t); }
  __device__ __forceinline__ f4 b2(int t) const { return at4(P::kB2 + 4 * t); }
  __device__ __forceinline__ f4 b3() const { return at4(P::kB3); }
  // adjoint pack (a separate array: pk points at its lane)
  __device__ __forceinline__ float w3t(int t, int j) const { return at(P::kW3t + 2 * t + j); }
  __device__ __forceinline__ float w2t(int t, int tt, int i) const {
    return at(P::kW2t + (t * MT + tt) * 4 + i);
  }
  __device__ __forceinline__ float w1t(int tt, int i) const { return at(P::kW1t + 4 * tt + i); }
};

// The activation from one hardware exp2 and one reciprocal (v_exp_f32,
// v_rcp_f32, about 1 ulp each): with e = e^{-2|a|} = 2^{-2|a| log2 e} in
// (0, 1] and r = 1 / (1 + e),
//   tanh(a) = sign(a) (1 - e) r   (absolute error below 3e-7), and
//   tanh'(a) = 1 - tanh^2(a) = 4 e r^2,
// the latter accurate to a few ulps even where the unit saturates (1 - h^2
// formed from a rounded h would cancel there).  No overflow for any a.
// About 7 instructions against the ~17 of the library tanhf.
__device__ __forceinline__ void act_hw(float a, float& h, float& e, float& r) {
  e = __builtin_amdgcn_exp2f(-2.88539008177792681f * __builtin_fabsf(a));
  r = __builtin_amdgcn_rcpf(1.0f + e);
  h = __builtin_copysignf((1.0f - e) * r, a);
}

__device__ __forceinline__ f4 tanh4(f4 a) {
  f4 h;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    float hi, e, r;
    act_hw(a[i], hi, e, r);
    h[i] = hi;
  }
  return h;
}

// tanh and its derivative
__device__ __forceinline__ void tanh4_d(f4 a, f4& h, f4& d) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    float hi, e, r;
    act_hw(a[i], hi, e, r);
    h[i] = hi;
    d[i] = 4.0f * e * r * r;
  }
}

// The B operand of an input-side K-step: component 4j + g of (x0..x4, v0, v1, 0).
__device__ __forceinline__ float input_operand(const float* x, const float* v, int g, int j) {
  if (j == 0) return g == 0 ? x[0] : g == 1 ? x[1] : g == 2 ? x[2] : x[3];
  return g == 0 ? x[4] : g == 1 ? v[0] : g == 2 ? v[1] : 0.0f;
}

// Hidden activations h1 = tanh(W1 z + b1), h2 = tanh(W2 h1 + b2) of the
// wave's 16 samples, in the D layout; with DERIV also tanh' of both layers;
// with pre1 / pre2 also the pre-activations.
template <int MT, bool DERIV, class WS>
__device__ __forceinline__ void hidden_impl(const WS& W, const float* x, const float* v, int g,
                                            f4 (&h1)[MT], f4 (&h2)[MT], f4* d1, f4* d2,
                                            f4* pre1 = nullptr, f4* pre2 = nullptr) {
  const float z0 = input_operand(x, v, g, 0), z1 = input_operand(x, v, g, 1);
#pragma unroll
  for (int t = 0; t < MT; ++t) {
    const f4 a = mfma(W.w1(t, 1), z1, mfma(W.w1(t, 0), z0, W.b1(t)));
    if (pre1) pre1[t] = a;
    if constexpr (DERIV) tanh4_d(a, h1[t], d1[t]);
    else h1[t] = tanh4(a);
  }
  f4 acc[MT];
#pragma unroll
  for (int t = 0; t < MT; ++t) acc[t] = W.b2(t);
#pragma unroll
  for (int tt = 0; tt < MT; ++tt)
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int t = 0; t < MT; ++t) acc[t] = mfma(W.w2(t, tt, i), h1[tt][i], acc[t]);
#pragma unroll
  for (int t = 0; t < MT; ++t) {
    if (pre2) pre2[t] = acc[t];
    if constexpr (DERIV) tanh4_d(acc[t], h2[t], d2[t]);
    else h2[t] = tanh4(acc[t]);
  }
}

template <int MT, class WS>
__device__ __forceinline__ void hidden(const WS& W, const float* x, const float* v, int g,
                                       f4 (&h1)[MT], f4 (&h2)[MT]) {
  hidden_impl<MT, false>(W, x, v, g, h1, h2, nullptr, nullptr);
}

template <int MT, class WS>
__device__ __forceinline__ void hidden_d(const WS& W, const float* x, const float* v, int g,
                                         f4 (&h1)[MT], f4 (&h2)[MT], f4 (&d1)[MT],
                                         f4 (&d2)[MT]) {
  hidden_impl<MT, true>(W, x, v, g, h1, h2, d1, d2);
}

// Output rows 4g + i of W3 h2 + b3 (rows >= 5 are padding), one accumulator
// per K-tile, combined in a fixed order.
template <int MT, class WS>
__device__ __forceinline__ f4 output(const WS& W, const f4 (&h2)[MT]) {
  f4 acc[MT];
#pragma unroll
  for (int tt = 0; tt < MT; ++tt) {
    acc[tt] = tt == 0 ? W.b3() : f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[tt] = mfma(W.w3(tt, i), h2[tt][i], acc[tt]);
  }
  f4 r = acc[0];
#pragma unroll
  for (int tt = 1; tt < MT; ++tt) r += acc[tt];
  return r;
}

// The five output rows of the lane's own sample n, gathered from the lanes
// that hold them (rows 0..3: group 0, row 4: group 1).
__device__ __forceinline__ void broadcast5(f4 d, int n, float* out) {
  out[0] = __shfl(d[0], n, kWave);
  out[1] = __shfl(d[1], n, kWave);
  out[2] = __shfl(d[2], n, kWave);
  out[3] = __shfl(d[3], n, kWave);
  out[4] = __shfl(d[0], 16 + n, kWave);
}

// g(x, v) for the lane's sample (every group gets all five components).
template <int MT, class WS>
__device__ __forceinline__ void residual(const WS& W, const float* x, const float* v, int g,
                                         int n, float* res) {
  f4 h1[MT], h2[MT];
  hidden<MT>(W, x, v, g, h1, h2);
  broadcast5(output<MT>(W, h2), n, res);
}

// The same, also handing back the pre-activations of both hidden layers.
template <int MT, class WS>
__device__ __forceinline__ void residual_keep(const WS& W, const float* x, const float* v, int g,
                                              int n, float* res, f4 (&pre1)[MT], f4 (&pre2)[MT]) {
  f4 h1[MT], h2[MT];
  hidden_impl<MT, false>(W, x, v, g, h1, h2, nullptr, nullptr, pre1, pre2);
  broadcast5(output<MT>(W, h2), n, res);
}

// Forward mode through g for the tile: the tangent
//   g' = W3 ((W2 ((W1 z') * d1)) * d2)
// of a tangent z' = (xd, 0) of the input (the state moves, the controls are
// held), given the activation derivatives d1, d2 of the forward; gd receives
// the five components of the lane's sample.  The products run in the
// forward's order with zero start values in place of the biases.
template <int MT, class WS>
__device__ __forceinline__ void jvp(const WS& W, const float* xd, int g, int n,
                                    const f4 (&d1)[MT], const f4 (&d2)[MT], float* gd) {
  const f4 zero4{0.0f, 0.0f, 0.0f, 0.0f};
  const float v0[2] = {0.0f, 0.0f};
  const float z0 = input_operand(xd, v0, g, 0), z1 = input_operand(xd, v0, g, 1);
  f4 h1[MT];
#pragma unroll
  for (int t = 0; t < MT; ++t)
    h1[t] = mfma(W.w1(t, 1), z1, mfma(W.w1(t, 0), z0, zero4)) * d1[t];
  f4 acc[MT];
#pragma unroll
  for (int t = 0; t < MT; ++t) acc[t] = zero4;
#pragma unroll
  for (int tt = 0; tt < MT; ++tt)
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int t = 0; t < MT; ++t) acc[t] = mfma(W.w2(t, tt, i), h1[tt][i], acc[t]);
  f4 out[MT];
#pragma unroll
  for (int tt = 0; tt < MT; ++tt) {
    const f4 h2 = acc[tt] * d2[tt];
    out[tt] = zero4;
#pragma unroll
    for (int i = 0; i < 4; ++i) out[tt] = mfma(W.w3(tt, i), h2[i], out[tt]);
  }
  f4 r = out[0];
#pragma unroll
  for (int tt = 1; tt < MT; ++tt) r += out[tt];
  broadcast5(r, n, gd);
}

// Reverse mode through g for the tile: given c = dL/dg (five components per
// lane, for the lane's sample) and the activation derivatives of the forward
// (d1, d2 = tanh' of the two hidden layers),
//   da2 = (W3^T c) * d2,  da1 = (W2^T da2) * d1,
//   dz  = W1^T da1  (rows 4g + i of 16; rows 0..6 are z's components),
// all in the D layout.
template <int MT>
__device__ __forceinline__ void backward(const PackView<MT>& B, const float* c, int g,
                                         const f4 (&d1)[MT], const f4 (&d2)[MT], f4 (&da1)[MT],
                                         f4 (&da2)[MT], f4& dz) {
  const float c0 = g == 0 ? c[0] : g == 1 ? c[1] : g == 2 ? c[2] : c[3];
  const float c1 = g == 0 ? c[4] : 0.0f;
#pragma unroll
  for (int t = 0; t < MT; ++t) {
    const f4 a = mfma(B.w3t(t, 1), c1, mfma(B.w3t(t, 0), c0, f4{0.0f, 0.0f, 0.0f, 0.0f}));
    da2[t] = a * d2[t];
  }
  f4 acc[MT];
#pragma unroll
  for (int t = 0; t < MT; ++t) acc[t] = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int tt = 0; tt < MT; ++tt)
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int t = 0; t < MT; ++t) acc[t] = mfma(B.w2t(t, tt, i), da2[tt][i], acc[t]);
#pragma unroll
  for (int t = 0; t < MT; ++t) da1[t] = acc[t] * d1[t];
  f4 zacc[MT];
#pragma unroll
  for (int tt = 0; tt < MT; ++tt) {
    zacc[tt] = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int i = 0; i < 4; ++i) zacc[tt] = mfma(B.w1t(tt, i), da1[tt][i], zacc[tt]);
  }
  dz = zacc[0];
#pragma unroll
  for (int tt = 1; tt < MT; ++tt) dz += zacc[tt];
}

// ---------------------------------------------------------------------------
// BF16 mode: the three products take bfloat16 operands (weights and the layer
// inputs z, h1, h2, rounded to nearest-even from binary32) with binary32
// accumulation, on v_mfma_f32_16x16x32_bf16; the biases are the accumulators'
// binary32 start values and tanh stays binary32.  A lane holds 8 bfloat16 of
// an operand: lane (g, n) supplies the K-block's contraction slots
// (g, j), j = 0..7, of A row n and of B column n, and the matrix core pairs
// equal slots of A and B, so any fixed map from slots to the contraction
// index that the weight pack and the activations share gives the product.
// K-block kb of a hidden layer covers the previous layer's M-tiles 2kb and
// 2kb+1: slot (g, j) is hidden unit 16(2kb) + 4g + j for j < 4 and
// 16(2kb+1) + 4g + (j - 4) for j >= 4, which are exactly the D registers
// (t, i) lane (g, n) holds for its sample, so the activations feed the next
// layer without data movement (MT odd: the missing tile's slots are zero).
// The input layer has one K-block: slot (0, j) is z_j (j < 7), every other
// slot zero.
//
// Pack (host-built, per lane 16 bytes = 8 bfloat16 per operand row), rows:
//   W1: MT (M-tile t), W2: MT * KB (t, kb), W3: KB (kb, output rows 0..4 of 16)
// with KB = ceil(MT / 2); the biases come from the binary32 pack.
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float fl8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ f4 mfma_bf(bf8 a, bf8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

template <int MT>
struct PackBf {
  static constexpr int KB = (MT + 1) / 2;
  static constexpr int kW1 = 0;
  static constexpr int kW2 = kW1 + MT;
  static constexpr int kW3 = kW2 + MT * KB;
  static constexpr int kRows = kW3 + KB;
};

// the bfloat16 operand rows of one lane, register resident, and the biases
template <int MT>
struct WeightsBf {
  static constexpr int KB = PackBf<MT>::KB;
  bf8 w1_[MT], w2_[MT][KB], w3_[KB];
  f4 b1_[MT], b2_[MT], b3_;
  __device__ __forceinline__ void load(const uint4* __restrict__ bpack,
                                       const float* __restrict__ fpack, int lane) {
    using P = PackBf<MT>;
    auto at = [&](int row) { return __builtin_bit_cast(bf8, bpack[row * kWave + lane]); };
#pragma unroll
    for (int t = 0; t < MT; ++t) {
      w1_[t] = at(P::kW1 + t);
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) w2_[t][kb] = at(P::kW2 + t * KB + kb);
    }
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) w3_[kb] = at(P::kW3 + kb);
    using F = Pack<MT>;
    auto fat = [&](int row) { return fpack[row * kWave + lane]; };
#pragma unroll
    for (int t = 0; t < MT; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        b1_[t][i] = fat(F::kB1 + 4 * t + i);
        b2_[t][i] = fat(F::kB2 + 4 * t + i);
      }
#pragma unroll
    for (int i = 0; i < 4; ++i) b3_[i] = fat(F::kB3 + i);
  }
  __device__ __forceinline__ bf8 w1(int t) const { return w1_[t]; }
  __device__ __forceinline__ bf8 w2(int t, int kb) const { return w2_[t][kb]; }
  __device__ __forceinline__ bf8 w3(int kb) const { return w3_[kb]; }
  __device__ __forceinline__ f4 b1(int t) const { return b1_[t]; }
  __device__ __forceinline__ f4 b2(int t) const { return b2_[t]; }
  __device__ __forceinline__ f4 b3() const { return b3_; }
};

// The same operands read at each use from packs in LDS: the bfloat16 weight
// pack (bp points at row 0 of this lane) and the binary32 pack's biases.
template <int MT>
struct PackViewBf {
  static constexpr int KB = PackBf<MT>::KB;
  const uint4* bp;
  PackView<MT> fv;
  __device__ __forceinline__ bf8 at(int row) const {
    return __builtin_bit_cast(bf8, bp[row * kWave]);
  }
  __device__ __forceinline__ bf8 w1(int t) const { return at(PackBf<MT>::kW1 + t); }
  __device__ __forceinline__ bf8 w2(int t, int kb) const { return at(PackBf<MT>::kW2 + t * KB + kb); }
  __device__ __forceinline__ bf8 w3(int kb) const { return at(PackBf<MT>::kW3 + kb); }
  __device__ __forceinline__ f4 b1(int t) const { return fv.b1(t); }
  __device__ __forceinline__ f4 b2(int t) const { return fv.b2(t); }
  __device__ __forceinline__ f4 b3() const { return fv.b3(); }
};

// The B operand of K-block kb over the activations h (D layout), rounded to
// bfloat16.
template <int MT>
__device__ __forceinline__ bf8 kblock_operand(const f4 (&h)[MT], int kb) {
  fl8 v;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    v[i] = h[2 * kb][i];
    v[4 + i] = 2 * kb + 1 < MT ? h[2 * kb + 1 < MT ? 2 * kb + 1 : 0][i] : 0.0f;
  }
  return __builtin_convertvector(v, bf8);
}

// The input-layer B operand: z = (x0..x4, v0, v1) in lane group 0, rounded.
__device__ __forceinline__ bf8 input_operand_bf(const float* x, const float* v, int g) {
  const fl8 zf = g == 0 ? fl8{x[0], x[1], x[2], x[3], x[4], v[0], v[1], 0.0f}
                        : fl8{0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
  return __builtin_convertvector(zf, bf8);
}

// x rounded to bfloat16 and back (the value a product consumed)
__device__ __forceinline__ float round_bf(float x) {
  return static_cast<float>(static_cast<__bf16>(x));
}
__device__ __forceinline__ f4 round_bf4(f4 x) {
  return f4{round_bf(x[0]), round_bf(x[1]), round_bf(x[2]), round_bf(x[3])};
}

// Hidden activations (and pre-activations) of the tile in BF16 mode
// (WB: WeightsBf or PackViewBf).
template <int MT, class WB>
__device__ __forceinline__ void hidden_bf(const WB& W, const float* x, const float* v, int g,
                                          f4 (&h1)[MT], f4 (&h2)[MT], f4* pre1 = nullptr,
                                          f4* pre2 = nullptr) {
  constexpr int KB = PackBf<MT>::KB;
  const bf8 z = input_operand_bf(x, v, g);
#pragma unroll
  for (int t = 0; t < MT; ++t) {
    const f4 a = mfma_bf(W.w1(t), z, W.b1(t));
    if (pre1) pre1[t] = a;
    h1[t] = tanh4(a);
  }
  bf8 hb[KB];
#pragma unroll
  for (int kb = 0; kb < KB; ++kb) hb[kb] = kblock_operand<MT>(h1, kb);
#pragma unroll
  for (int t = 0; t < MT; ++t) {
    f4 acc = W.b2(t);
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) acc = mfma_bf(W.w2(t, kb), hb[kb], acc);
    if (pre2) pre2[t] = acc;
    h2[t] = tanh4(acc);
  }
}

// Output rows 4g + i of W3 h2 + b3 in BF16 mode.
template <int MT, class WB>
__device__ __forceinline__ f4 output_bf(const WB& W, const f4 (&h2)[MT]) {
  constexpr int KB = PackBf<MT>::KB;
  f4 acc = W.b3();
#pragma unroll
  for (int kb = 0; kb < KB; ++kb) acc = mfma_bf(W.w3(kb), kblock_operand<MT>(h2, kb), acc);
  return acc;
}

template <int MT>
__device__ __forceinline__ void residual(const WeightsBf<MT>& W, const float* x, const float* v,
                                         int g, int n, float* res) {
  f4 h1[MT], h2[MT];
  hidden_bf<MT>(W, x, v, g, h1, h2);
  broadcast5(output_bf<MT>(W, h2), n, res);
}

template <int MT>
__device__ __forceinline__ void residual_keep(const PackViewBf<MT>& W, const float* x,
                                              const float* v, int g, int n, float* res,
                                              f4 (&pre1)[MT], f4 (&pre2)[MT]) {
  f4 h1[MT], h2[MT];
  hidden_bf<MT>(W, x, v, g, h1, h2, pre1, pre2);
  broadcast5(output_bf<MT>(W, h2), n, res);
}

// The binary32 forward pack read with its weights rounded to bfloat16 at each
// use: the BF16 mode's tangents (jvp) take the rounded weights and count the
// roundings of the layer inputs as the identity, as its adjoint does.
template <int MT>
struct RoundedView {
  PackView<MT> fv;
  __device__ __forceinline__ float w1(int t, int j) const { return round_bf(fv.w1(t, j)); }
  __device__ __forceinline__ float w2(int t, int tt, int i) const {
    return round_bf(fv.w2(t, tt, i));
  }
  __device__ __forceinline__ float w3(int tt, int i) const { return round_bf(fv.w3(tt, i)); }
};

}  // namespace mlp
}  // namespace mppi
