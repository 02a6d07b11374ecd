// Step (a9): gradient of a loss L(U) on the controls of one MPPI iteration
// with respect to the dynamics parameters (MLP weights, wheelbase) and the
// diagonal state weights Q of the tracking cost.
//
// With U = u + gamma sum_k w_k eps_k (gamma = 1 in Algorithm 1, else the
// step size of the mirror-descent form), w = softmin(J / lambda) and u
// independent of the parameters theta, G = dL/dU gives
//   dL/dJ_k = a_k = -(gamma w_k / lambda) (g_k - sum_i w_i g_i),  g_k = <G, eps_k>,
//   dL/dtheta = sum_k a_k dJ_k/dtheta,
// and dJ_k/dtheta comes from a reverse sweep of the costate mu_t = dJ_k/dx_t
// through the discrete step (the four RK4 stages and the MLP residual) and
// the tracking cost.  Kernels, in stream order:
//   project:  g_k for blocks of 64 samples, with per-block sums of e_k
//             (binary64: the normaliser eta), the count of samples of nonzero
//             weight and the first sample of weight e_k = 1 (a minimiser);
//   scan:     eta, the block offsets, and the weighted mean of g taken
//             relative to the minimiser's g_ref: d = sum_i w_i (g_i - g_ref);
//   compact:  the list (k, a_k) of samples with nonzero weight, in k order,
//             a_k = -(gamma w_k / lambda) ((g_k - g_ref) - d).  The shift keeps
//             g_k - sum_i w_i g_i accurate when one sample holds almost all
//             the weight (there the plain difference cancels completely);
//   sweep:    per tile of 16 listed samples, segment by segment from the
//             last: the states are rebuilt from the forward's checkpoints
//             (keeping the MLP pre-activations of each step in a per-tile
//             scratch that stays in L2), then the costate runs backwards
//             through them.  The MLP and its
//             transposes run on the matrix cores (mlp.h); the weight
//             gradients are outer products summed over the tile's samples
//             (MFMA with the samples as the contraction index, operands
//             transposed through LDS) and over time in registers.  Each tile
//             writes its partial gradient;
//   reduce:   the partial gradients of the tiles, summed in tile order.
// Every sum has a fixed order, so the gradient is bitwise reproducible.
// Samples of zero weight contribute exactly zero and are skipped.
#include <algorithm>

#include "dynamics.h"
#include "mlp.h"

namespace mppi {

constexpr int kTileS = 16;           // samples per sweep tile (one wave)
constexpr int kProjectBlock = 1024;  // 16 quads of 4 samples x 64 row groups
constexpr int kProjectSamples = 64;

struct BwdBlock {
  double sum_e;
  int count;
  int kmin;  // first sample of the block with e_k = 1, or INT_MAX
};
struct BwdMeta {
  double eta;
  float gref, dbar;
  int count;
};
constexpr int kScanBlock = 1024;
struct BwdItem {
  int k;
  float a;
};

// g_k = sum_r G_r eps_k[r] for the 64 samples of a workgroup: each thread
// reads four adjacent samples (one 16-byte load; ldk is a multiple of 64) of
// every 64th row, and the 64 row-group partials are added in a fixed order.
__global__ __launch_bounds__(kProjectBlock) void adjoint_project_kernel(
    const float* __restrict__ G, const float* __restrict__ eps, int64_t ldk, int K, int TM,
    const float* __restrict__ e, float* __restrict__ gk, BwdBlock* __restrict__ part) {
  constexpr int kQuads = kProjectSamples / 4;
  constexpr int kRowGroups = kProjectBlock / kQuads;
  __shared__ float red[kProjectBlock * 4];  // [row group][sample]
  const int q = threadIdx.x % kQuads, rg = threadIdx.x / kQuads;
  const int k0 = blockIdx.x * kProjectSamples + 4 * q;
  float4 acc = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  if (k0 < K) {
    const float4* col = reinterpret_cast<const float4*>(eps + k0);
    const int64_t ld4 = ldk / 4;
    for (int r = rg; r < TM; r += kRowGroups) {
      const float gr = G[r];
      const float4 v = col[r * ld4];
      acc.x += gr * v.x;
      acc.y += gr * v.y;
      acc.z += gr * v.z;
      acc.w += gr * v.w;
    }
  }
  float* mine = red + rg * kProjectSamples + 4 * q;
  mine[0] = acc.x;
  mine[1] = acc.y;
  mine[2] = acc.z;
  mine[3] = acc.w;
  __syncthreads();
  if (threadIdx.x < kProjectSamples) {
    const int s = threadIdx.x;
    const int k = blockIdx.x * kProjectSamples + s;
    float g = 0.0f;
    for (int i = 0; i < kRowGroups; ++i) g += red[i * kProjectSamples + s];
    const float ek = k < K ? e[k] : 0.0f;
    if (k < K) gk[k] = g;
    // per-block sums over the 64 samples (one wave, fixed shuffle tree)
    int cnt = ek > 0.0f ? 1 : 0;
    int kmin = ek == 1.0f ? k : 0x7FFFFFFF;
    double de = static_cast<double>(ek);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      cnt += __shfl_xor(cnt, o, kWave);
      kmin = min(kmin, __shfl_xor(kmin, o, kWave));
      de += __shfl_xor(de, o, kWave);
    }
    if (s == 0) part[blockIdx.x] = BwdBlock{de, cnt, kmin};
  }
}

__global__ __launch_bounds__(kScanBlock) void adjoint_scan_kernel(
    const BwdBlock* __restrict__ part, int nb, const float* __restrict__ e,
    const float* __restrict__ gk, int K, int* __restrict__ offs, BwdMeta* __restrict__ meta) {
  __shared__ double s_eta;
  __shared__ float s_gref;
  __shared__ float red[kScanBlock / kWave];
  if (threadIdx.x < kWave) {
    // the first wave scans the block counts 64 at a time (exclusive offsets)
    // and sums eta per lane, then over the lanes in a fixed tree
    const int lane = threadIdx.x;
    double eta = 0.0;
    int count = 0, kmin = 0x7FFFFFFF;
    for (int b0 = 0; b0 < nb; b0 += kWave) {
      const int b = b0 + lane;
      BwdBlock q{0.0, 0, 0x7FFFFFFF};
      if (b < nb) q = part[b];
      int incl = q.count;
#pragma unroll
      for (int o = 1; o < kWave; o <<= 1) {
        const int y = __shfl_up(incl, o, kWave);
        if (lane >= o) incl += y;
      }
      if (b < nb) offs[b] = count + incl - q.count;
      count += __shfl(incl, kWave - 1, kWave);
      eta += q.sum_e;
      kmin = min(kmin, q.kmin);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      eta += __shfl_xor(eta, o, kWave);
      kmin = min(kmin, __shfl_xor(kmin, o, kWave));
    }
    if (lane == 0) {
      const bool ok = eta > 0.0 && kmin < K;
      s_eta = ok ? eta : 0.0;
      s_gref = ok ? gk[kmin] : 0.0f;
      meta->eta = s_eta;
      meta->gref = s_gref;
      meta->count = ok ? count : 0;
    }
  }
  __syncthreads();
  // d = sum_i e_i (g_i - g_ref) / eta, fixed partition and tree
  const float gref = s_gref;
  float acc = 0.0f;
  for (int k = threadIdx.x; k < K; k += kScanBlock) {
    const float ek = e[k];
    if (ek > 0.0f) acc += ek * (gk[k] - gref);
  }
  acc = wave_sum(acc);
  if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    float tot = red[0];
    for (int i = 1; i < kScanBlock / kWave; ++i) tot += red[i];
    meta->dbar = s_eta > 0.0 ? static_cast<float>(static_cast<double>(tot) / s_eta) : 0.0f;
  }
}

__global__ __launch_bounds__(kProjectSamples) void adjoint_compact_kernel(
    const float* __restrict__ e, const float* __restrict__ gk, int K, float scale,
    const int* __restrict__ offs, const BwdMeta* __restrict__ meta, BwdItem* __restrict__ list) {
  const int lane = threadIdx.x;
  const int k = blockIdx.x * kProjectSamples + lane;
  const float ek = k < K ? e[k] : 0.0f;
  const bool nz = ek > 0.0f && meta->eta > 0.0;
  const uint64_t mask = __ballot(nz);
  if (!nz) return;
  const int rank = __popcll(mask & ((uint64_t{1} << lane) - 1u));
  const float w = static_cast<float>(static_cast<double>(ek) / meta->eta);
  const float a = -(w * scale) * ((gk[k] - meta->gref) - meta->dbar);  // scale = gamma/lambda
  list[offs[blockIdx.x] + rank] = BwdItem{k, a};
}

// dx += (df/dx)^T c, dL += (df/d wheelbase)^T c and dv += (df/dv)^T c for
// the bicycle derivative f = (s cos psi, s sin psi, s tan(delta) / L, a,
// delta_rate) at x with control v = (a, delta_rate).
template <bool FAST>
__device__ __forceinline__ void bicycle_vjp(const float* x, const float* c, float inv_l,
                                            float* dx, float& dl, float* dv) {
  dv[0] += c[3];
  dv[1] += c[4];
  float sn, cs, sd, cd;
  if constexpr (FAST) {
    sn = __sinf(x[2]);
    cs = __cosf(x[2]);
    sd = __sinf(x[4]);
    cd = __cosf(x[4]);
  } else {
    sincosf(x[2], &sn, &cs);
    sincosf(x[4], &sd, &cd);
  }
  const float rc = FAST ? __builtin_amdgcn_rcpf(cd) : 1.0f / cd;
  const float tn = FAST ? sd * rc : tanf(x[4]);
  const float s = x[3];
  dx[2] += s * (cs * c[1] - sn * c[0]);
  dx[3] += cs * c[0] + sn * c[1] + tn * inv_l * c[2];
  dx[4] += s * (1.0f + tn * tn) * inv_l * c[2];
  dl -= s * tn * inv_l * inv_l * c[2];
}

// mu0 = (dF/dx)^T mu for the RK4 bicycle step from x (control v held),
// gL += (dF/d wheelbase)^T mu and dv += (dF/dv)^T mu: the four stages are
// rebuilt, then transposed in reverse.
template <bool FAST>
__device__ __forceinline__ void rk4_vjp(const DevParams& p, const float* xt, const float* v,
                                        const float* mu, float* mu0, float& gL, float* dv) {
  using Model = Bicycle<FAST>;
  constexpr int N = 5;
  float k1[N], xa[N], k2[N], xb[N], k3[N], xc[N];
  Model::deriv(xt, v, k1, p);
#pragma unroll
  for (int i = 0; i < N; ++i) xa[i] = xt[i] + p.half_dt * k1[i];
  Model::deriv(xa, v, k2, p);
#pragma unroll
  for (int i = 0; i < N; ++i) xb[i] = xt[i] + p.half_dt * k2[i];
  Model::deriv(xb, v, k3, p);
#pragma unroll
  for (int i = 0; i < N; ++i) xc[i] = xt[i] + p.dt * k3[i];
  float cst[N], cx[N];
  const float third_dt = 2.0f * p.sixth_dt;
#pragma unroll
  for (int i = 0; i < N; ++i) { mu0[i] = mu[i]; cst[i] = p.sixth_dt * mu[i]; cx[i] = 0.0f; }
  bicycle_vjp<FAST>(xc, cst, p.inv_wheelbase, cx, gL, dv);  // k4 = f(xc), xc = x + dt k3
#pragma unroll
  for (int i = 0; i < N; ++i) {
    mu0[i] += cx[i];
    cst[i] = third_dt * mu[i] + p.dt * cx[i];
    cx[i] = 0.0f;
  }
  bicycle_vjp<FAST>(xb, cst, p.inv_wheelbase, cx, gL, dv);  // k3 = f(xb), xb = x + dt/2 k2
#pragma unroll
  for (int i = 0; i < N; ++i) {
    mu0[i] += cx[i];
    cst[i] = third_dt * mu[i] + p.half_dt * cx[i];
    cx[i] = 0.0f;
  }
  bicycle_vjp<FAST>(xa, cst, p.inv_wheelbase, cx, gL, dv);  // k2 = f(xa), xa = x + dt/2 k1
#pragma unroll
  for (int i = 0; i < N; ++i) {
    mu0[i] += cx[i];
    cst[i] = p.sixth_dt * mu[i] + p.half_dt * cx[i];
    cx[i] = 0.0f;
  }
  bicycle_vjp<FAST>(xt, cst, p.inv_wheelbase, cx, gL, dv);  // k1 = f(x)
#pragma unroll
  for (int i = 0; i < N; ++i) mu0[i] += cx[i];
}

// d = (df/dx) xd: the bicycle derivative's tangent along xd at x (control
// held), the forward-mode counterpart of bicycle_vjp.
template <bool FAST>
__device__ __forceinline__ void bicycle_jvp(const float* x, const float* xd, float inv_l,
                                            float* d) {
  float sn, cs, sd, cd;
  if constexpr (FAST) {
    sn = __sinf(x[2]);
    cs = __cosf(x[2]);
    sd = __sinf(x[4]);
    cd = __cosf(x[4]);
  } else {
    sincosf(x[2], &sn, &cs);
    sincosf(x[4], &sd, &cd);
  }
  const float rc = FAST ? __builtin_amdgcn_rcpf(cd) : 1.0f / cd;
  const float tn = FAST ? sd * rc : tanf(x[4]);
  const float s = x[3];
  d[0] = cs * xd[3] - s * sn * xd[2];
  d[1] = sn * xd[3] + s * cs * xd[2];
  d[2] = (tn * xd[3] + s * (1.0f + tn * tn) * xd[4]) * inv_l;
  d[3] = 0.0f;
  d[4] = 0.0f;
}

// xn = (dF/dx) xd for the RK4 bicycle step from x (control v held): the
// stages' tangents in the order of the stages.
template <bool FAST>
__device__ __forceinline__ void rk4_jvp(const DevParams& p, const float* xt, const float* v,
                                        const float* xd, float* xn) {
  using Model = Bicycle<FAST>;
  constexpr int N = 5;
  float k[N], xs[N], kd[N], xsd[N], acc[N];
  bicycle_jvp<FAST>(xt, xd, p.inv_wheelbase, kd);  // k1' at x
  Model::deriv(xt, v, k, p);
#pragma unroll
  for (int i = 0; i < N; ++i) {
    acc[i] = kd[i];
    xs[i] = xt[i] + p.half_dt * k[i];
    xsd[i] = xd[i] + p.half_dt * kd[i];
  }
  bicycle_jvp<FAST>(xs, xsd, p.inv_wheelbase, kd);  // k2'
  Model::deriv(xs, v, k, p);
#pragma unroll
  for (int i = 0; i < N; ++i) {
    acc[i] += 2.0f * kd[i];
    xs[i] = xt[i] + p.half_dt * k[i];
    xsd[i] = xd[i] + p.half_dt * kd[i];
  }
  bicycle_jvp<FAST>(xs, xsd, p.inv_wheelbase, kd);  // k3'
  Model::deriv(xs, v, k, p);
#pragma unroll
  for (int i = 0; i < N; ++i) {
    acc[i] += 2.0f * kd[i];
    xs[i] = xt[i] + p.dt * k[i];
    xsd[i] = xd[i] + p.dt * kd[i];
  }
  bicycle_jvp<FAST>(xs, xsd, p.inv_wheelbase, kd);  // k4'
#pragma unroll
  for (int i = 0; i < N; ++i) xn[i] = xd[i] + p.sixth_dt * (acc[i] + kd[i]);
}

// Segment-parallel reverse pass.  The costate carried out of a checkpoint
// segment s (steps t0 .. t1 - 1) is affine in the one carried in at its end:
//   mu_out = P_s^T mu_in + q_s,  P_s = dx_{t1} / dx_{t0},
//   q_s = sum_{t = t0+1 .. t1} (dx_t / dx_{t0})^T c_t,
// c_t the running cost's gradient at x_t.  With few listed samples the
// sequential sweep is latency-bound (one tile walks all T steps twice), so
// for at most tp_tiles tiles:
//   tp kernel:    per (tile, segment, column i) one wave rebuilds the segment
//                 from its checkpoint and carries the tangent of x_{t0} + h e_i
//                 (forward mode through the RK4 stages and the MLP), giving
//                 column i of P_s and component i of q_s; column 0 of the last
//                 segment also keeps x_T;
//   sweep:        per (tile, segment) the usual reverse pass over that
//                 segment alone, from the costate the chain of the later
//                 segments' maps gives (every workgroup forms the chain
//                 itself, from x_T's terminal gradient, in the same order),
//                 on the states and MLP pre-activations the map kernel's
//                 column 0 kept (no rebuild); its partial gradient goes to
//                 its own row;
//   reduce:       sums tiles x segments rows.
// The mode is chosen on the device from the listed count, so no host
// synchronisation is needed.
//
// The parallel units are finer than the checkpoint segments: each segment of
// c steps splits into sub = ceil(c / 5) units of cs = ceil(c / sub) steps (the
// last ones of a ragged final segment may be empty: identity maps).  A unit
// past its segment's start has no checkpoint; its map's waves rebuild the
// segment's earlier steps first (without tangents).  Record per (tile, unit,
// sample): for each column i, P[0..4][i] then q[i] (6 floats); x_T (5, the
// last unit): 35 floats, padded to 36.
constexpr int kTpMaxTiles = kAdjointTilesMax;
// at most this many (tile, unit) rows: the partial gradients and the
// pre-activation scratch grow with them
constexpr int kTpRowBudget = 1280;
constexpr int kTpUnitSteps = 5;

// units per checkpoint segment of c steps, and the steps of a unit
__host__ __device__ inline int tp_sub(int c) { return (c + kTpUnitSteps - 1) / kTpUnitSteps; }
__host__ __device__ inline int tp_unit_steps(int c) { return (c + tp_sub(c) - 1) / tp_sub(c); }

// The most tiles the segment-parallel mode takes for a context of `tiles`
// tiles and nunit units (the scratch is sized for it).
inline int tp_cap(int tiles, int nunit) {
  return std::min(std::min(tiles, kTpMaxTiles), kTpRowBudget / nunit);
}
constexpr int kTpRec = 36;
constexpr int kTpXT = 30;  // offset of x_T in a record
static_assert(kTpXT + 5 <= kTpRec, "record size");

// The unit's forward, kept by the map kernel's column-0 workgroup for the
// unit's sweep (which then skips its rebuild): per (tile, unit, sample) the
// states before each step and after the last ((cs + 1) x 5) and the controls
// (cs x 2), after the records of the same launch; the MLP pre-activations go
// to the unit's row of the pre-activation scratch.
__host__ __device__ inline int tp_state_floats(int c) {
  return (tp_unit_steps(c) + 1) * 5 + tp_unit_steps(c) * 2;
}
__device__ __forceinline__ int64_t tp_states_off(int tp_tiles, int nunit, int c, int row, int n) {
  return static_cast<int64_t>(tp_tiles) * nunit * kTileS * kTpRec +
         (static_cast<int64_t>(row) * kTileS + n) * tp_state_floats(c);
}

// Which units a workgroup of the sweep handles: in the segment-parallel mode
// one (tile, unit) pair, units of `sub` per segment; otherwise one tile and
// every segment (units = segments).
struct SegSel {
  int tile, lo, hi, sub;
  bool par;
};

__device__ __forceinline__ SegSel seg_select(int nseg, int c, int tp_tiles, int count) {
  SegSel s;
  s.par = tp_tiles > 0 && count <= tp_tiles * kTileS;
  if (s.par) {
    s.sub = tp_sub(c);
    const int nunit = nseg * s.sub;
    s.tile = blockIdx.x / nunit;
    s.lo = s.hi = blockIdx.x % nunit;
  } else {
    s.sub = 1;
    s.tile = blockIdx.x;
    s.lo = 0;
    s.hi = nseg - 1;
  }
  return s;
}

// Steps [t0, t0 + len) of unit u (sub units per segment of c steps).
__device__ __forceinline__ void unit_steps(int u, int sub, int c, int T, int& seg, int& h,
                                           int& t0, int& len) {
  seg = u / sub;
  h = u % sub;
  const int cs = (c + sub - 1) / sub;
  const int seg_len = min(c, T - seg * c);
  t0 = seg * c + min(h * cs, seg_len);
  len = max(0, min(cs, seg_len - h * cs));
}

// The costate carried into unit `unit` (< nunit - 1) for the lane's sample n of
// tile `tile`: the terminal gradient at x_T, then the maps of units
// nunit - 1 .. unit + 1 in that order.
__device__ __forceinline__ void tp_chain(const DevParams& p, const float* __restrict__ tp,
                                         int tile, int nunit, int unit, int n, int T, float a,
                                         float* mu) {
  constexpr int N = 5;
  const float* last = tp + (static_cast<int64_t>(tile * nunit + nunit - 1) * kTileS + n) * kTpRec;
  const float* r = p.ref + static_cast<int64_t>(T) * N;
#pragma unroll
  for (int i = 0; i < N; ++i) mu[i] = a * 2.0f * p.w[16] * p.w[i] * (last[kTpXT + i] - r[i]);
  for (int s = nunit - 1; s > unit; --s) {
    const float* rec = tp + (static_cast<int64_t>(tile * nunit + s) * kTileS + n) * kTpRec;
    float m[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
      float acc = rec[i * 6 + 5];
#pragma unroll
      for (int j = 0; j < N; ++j) acc = fmaf(rec[i * 6 + j], mu[j], acc);
      m[i] = acc;
    }
#pragma unroll
    for (int i = 0; i < N; ++i) mu[i] = m[i];
  }
}

// The state at a segment's start: its checkpoint.
__device__ __forceinline__ void load_checkpoint(const float* __restrict__ ckpt, int64_t ldk, int k,
                                                int seg, float* x, float* comp) {
  constexpr int N = 5;
  const float* ck = ckpt + static_cast<int64_t>(seg) * 7 * ldk + k;
#pragma unroll
  for (int i = 0; i < N; ++i) { x[i] = ck[i * ldk]; comp[i] = 0.0f; }
  comp[0] = ck[5 * ldk];
  comp[1] = ck[6 * ldk];
}

// The unit's states (len + 1) and controls (len) of one sample as the map
// kernel kept them, into the sweep's per-sample arrays.
__device__ __forceinline__ void copy_unit_forward(const float* __restrict__ st, int c, int len,
                                                  float* xs, float* vs) {
  const int cs = tp_unit_steps(c);
  for (int j = 0; j <= len; ++j)
#pragma unroll
    for (int i = 0; i < 5; ++i) xs[j * 5 + i] = st[j * 5 + i];
  for (int j = 0; j < len; ++j)
#pragma unroll
    for (int q = 0; q < 2; ++q) vs[j * 2 + q] = st[(cs + 1) * 5 + j * 2 + q];
}

// Row `row` of the partial gradients holds dL/du only for the steps of its
// segment: zero the other steps' columns (segment-parallel mode).
__device__ __forceinline__ void tp_zero_du(float* __restrict__ row, int du_off, int T, int t0,
                                           int len, int tid, int nthreads) {
  constexpr int M = 2;
  for (int i = tid; i < T * M; i += nthreads) {
    const int t = i / M;
    if (t < t0 || t >= t0 + len) row[du_off + i] = 0.0f;
  }
}

// BF: the rebuild on the bfloat16 products (as the sweep's), the tangents
// through the rounded weights with the roundings of the layer inputs taken as
// the identity.
template <int MT, bool FAST, bool BF = false>
__global__ __launch_bounds__(kWave) void adjoint_tp_kernel(
    DevParams p, const float* __restrict__ u, const float* __restrict__ eps, int64_t ldk, int T,
    const float* __restrict__ ckpt, int c, const BwdItem* __restrict__ list,
    const BwdMeta* __restrict__ meta, int tp_tiles, float* __restrict__ tp,
    mlp::f4* __restrict__ pre) {
  using Model = Bicycle<FAST>;
  using f4 = mlp::f4;
  constexpr int N = 5, M = 2;
  const int count = meta->count;
  if (count > tp_tiles * kTileS) return;  // the sequential sweep runs instead
  const int nseg = (T + c - 1) / c, sub = tp_sub(c), nunit = nseg * sub;
  const int col = blockIdx.x % N, tu = blockIdx.x / N;
  const int unit = tu % nunit, tile = tu / nunit;
  const int base = tile * kTileS;
  if (base >= count) return;  // wave-uniform
  extern __shared__ float4 lds4[];
  const float* lds = reinterpret_cast<const float*>(lds4);
  const int lane = threadIdx.x, n = lane % kTileS, g = lane / kTileS;
  constexpr int kFwd = MT ? mlp::Pack<MT>::kFwdRows * kWave : 0;  // floats
  if constexpr (MT > 0) {
    const float4* src = reinterpret_cast<const float4*>(p.mlp);
    for (int i = lane; i < kFwd / 4; i += kWave) lds4[i] = src[i];
    if constexpr (BF) {
      const float4* src_h = reinterpret_cast<const float4*>(p.mlp_bf);
      for (int i = lane; i < mlp::PackBf<MT>::kRows * kWave; i += kWave)
        lds4[kFwd / 4 + i] = src_h[i];
    }
    __syncthreads();
  }
  const mlp::PackView<MT ? MT : 1> WF{lds + lane};
  const mlp::PackViewBf<MT ? MT : 1> WFB{reinterpret_cast<const uint4*>(lds + kFwd) + lane, WF};
  const int idx = base + n;
  const bool valid = idx < count;
  const BwdItem item = list[valid ? idx : base];
  const float a = valid ? item.a : 0.0f;
  const float* e = eps + item.k;
  int seg, h, t0, len;
  unit_steps(unit, sub, c, T, seg, h, t0, len);
  float x[N], comp[N], xd[N];
  const float* ck = ckpt + static_cast<int64_t>(seg) * 7 * ldk + item.k;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    x[i] = ck[i * ldk];
    comp[i] = 0.0f;
    xd[i] = i == col ? 1.0f : 0.0f;
  }
  comp[0] = ck[5 * ldk];
  comp[1] = ck[6 * ldk];
  // the segment's steps before the unit: the sweep's rebuild, no tangent
  for (int t = seg * c; t < t0; ++t) {
    float v[M];
#pragma unroll
    for (int k = 0; k < M; ++k) v[k] = u[t * M + k] + e[static_cast<int64_t>(t * M + k) * ldk];
    if constexpr (MT > 0) {
      f4 a1[MT], a2[MT];
      float res[N];
      if constexpr (BF) mlp::residual_keep<MT>(WFB, x, v, g, n, res, a1, a2);
      else mlp::residual_keep<MT>(WF, x, v, g, n, res, a1, a2);
      step<Model, kRK4>(x, v, comp, p, res);
    } else {
      step<Model, kRK4>(x, v, comp, p);
    }
  }
  float* rec = tp + (static_cast<int64_t>(tile * nunit + unit) * kTileS + n) * kTpRec;
  float q = 0.0f;
  // column 0 keeps the unit's forward for its sweep
  const int row = tile * nunit + unit, cs = tp_unit_steps(c);
  float* st = tp + tp_states_off(tp_tiles, nunit, c, row, n);
  mlp::f4* my_pre = pre + static_cast<int64_t>(row) * cs * 2 * (MT ? MT : 1) * kWave + lane;
  for (int j = 0; j < len; ++j) {
    const int t = t0 + j;
    float v[M];
#pragma unroll
    for (int k = 0; k < M; ++k) v[k] = u[t * M + k] + e[static_cast<int64_t>(t * M + k) * ldk];
    if (col == 0 && g == 0) {
#pragma unroll
      for (int i = 0; i < N; ++i) st[j * N + i] = x[i];
#pragma unroll
      for (int k = 0; k < M; ++k) st[(cs + 1) * N + j * M + k] = v[k];
    }
    float xn[N];
    rk4_jvp<FAST>(p, x, v, xd, xn);
    if constexpr (MT > 0) {
      f4 d1[MT], d2[MT], a1[MT], a2[MT];
      float res[N], gd[N];
      if constexpr (BF) {
        f4 hh;
        mlp::residual_keep<MT>(WFB, x, v, g, n, res, a1, a2);
#pragma unroll
        for (int t2 = 0; t2 < MT; ++t2) {
          mlp::tanh4_d(a1[t2], hh, d1[t2]);
          mlp::tanh4_d(a2[t2], hh, d2[t2]);
        }
        mlp::jvp<MT>(mlp::RoundedView<MT>{WF}, xd, g, n, d1, d2, gd);
      } else {
        f4 h1[MT], h2[MT];
        mlp::hidden_impl<MT, true>(WF, x, v, g, h1, h2, d1, d2, a1, a2);
        mlp::broadcast5(mlp::output<MT>(WF, h2), n, res);
        mlp::jvp<MT>(WF, xd, g, n, d1, d2, gd);
      }
      if (col == 0) {
        f4* ps = my_pre + static_cast<int64_t>(j) * 2 * MT * kWave;
#pragma unroll
        for (int t2 = 0; t2 < MT; ++t2) {
          ps[t2 * kWave] = a1[t2];
          ps[(MT + t2) * kWave] = a2[t2];
        }
      }
#pragma unroll
      for (int i = 0; i < N; ++i) xn[i] += p.dt * gd[i];
      step<Model, kRK4>(x, v, comp, p, res);
    } else {
      step<Model, kRK4>(x, v, comp, p);
    }
    // the running cost's gradient at x_{t+1} along the tangent
    const float* r = p.ref + static_cast<int64_t>(t + 1) * N;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      xd[i] = xn[i];
      q = fmaf(a * 2.0f * p.w[i] * (x[i] - r[i]), xd[i], q);
    }
  }
  if (g == 0) {
#pragma unroll
    for (int i = 0; i < N; ++i) rec[col * 6 + i] = xd[i];
    rec[col * 6 + 5] = q;
    if (col == 0) {
#pragma unroll
      for (int i = 0; i < N; ++i) st[len * N + i] = x[i];
    }
    if (unit == nunit - 1 && col == 0) {  // after the last step: x_T
#pragma unroll
      for (int i = 0; i < N; ++i) rec[kTpXT + i] = x[i];
    }
  }
}

// The map kernel with the MLP of the tile split over SW waves (binary32
// products): wave w owns the hidden M-tiles w TW .. w TW + TW - 1 of every
// product, forward and tangent, with its operand slices in registers; the
// h1 and h1' tiles and the output partials meet in LDS (double-buffered by
// step parity, two barriers per step).  The products accumulate in the order
// of the one-wave kernel's; the bicycle step and its tangent are repeated by
// every wave.  Used for H = 64 whatever the sweep's split, so the sweeps of
// every split read the same records.  BF: the forward on the bfloat16
// products as the split sweep's rebuild takes them (h2 tiles exchanged, every
// wave forms the output over all K-blocks), the tangents through the rounded
// weights.
template <int MT, int SW, bool FAST, bool BF = false>
__global__ __launch_bounds__(kWave * SW) void adjoint_tp_split_kernel(
    DevParams p, const float* __restrict__ u, const float* __restrict__ eps, int64_t ldk, int T,
    const float* __restrict__ ckpt, int c, const BwdItem* __restrict__ list,
    const BwdMeta* __restrict__ meta, int tp_tiles, float* __restrict__ tp,
    mlp::f4* __restrict__ pre) {
  static_assert(MT % SW == 0, "tiles per wave");
  constexpr int TW = MT / SW;
  using Model = Bicycle<FAST>;
  using f4 = mlp::f4;
  using PK = mlp::Pack<MT>;
  constexpr int N = 5, M = 2;
  const int count = meta->count;
  if (count > tp_tiles * kTileS) return;  // the sequential sweep runs instead
  const int nseg = (T + c - 1) / c, sub = tp_sub(c), nunit = nseg * sub;
  const int col = blockIdx.x % N, tu = blockIdx.x / N;
  const int unit = tu % nunit, tile = tu / nunit;
  const int base = tile * kTileS;
  if (base >= count) return;  // workgroup-uniform
  extern __shared__ float4 lds4[];
  f4* xa = reinterpret_cast<f4*>(lds4);  // [2][MT][64] each: h1, h1', output, tangent output
  f4* xt1 = xa + 2 * MT * kWave;
  f4* xb = xt1 + 2 * MT * kWave;
  f4* xt3 = xb + 2 * MT * kWave;
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  const int n = lane % kTileS, g = lane / kTileS;
  const int q0 = w * TW;
  auto xch = [&](f4* buf, int par, int q) -> f4& { return buf[(par * MT + q) * kWave + lane]; };

  // this wave's forward operand slices (BF: the binary32 weights rounded to
  // bfloat16 for the tangents, the bfloat16 rows for the forward)
  const float* pf = p.mlp + lane;
  auto wt = [&](int row) {
    const float w8 = pf[row * kWave];
    return BF ? mlp::round_bf(w8) : w8;
  };
  float fw1[TW][2], fw2[TW][MT][4], fw3[TW][4];
  f4 fb1[TW], fb2[TW], fb3[TW];
  constexpr int KB = mlp::PackBf<MT>::KB;
  constexpr int TWB = BF ? TW : 1, KBB = BF ? KB : 1;
  mlp::bf8 v1[TWB], v2[TWB][KBB], v3[KBB];
#pragma unroll
  for (int q = 0; q < TW; ++q) {
    const int t = q0 + q;
    if constexpr (BF) {
      using PB = mlp::PackBf<MT>;
      const uint4* bp = p.mlp_bf + lane;
      v1[q] = __builtin_bit_cast(mlp::bf8, bp[(PB::kW1 + t) * kWave]);
#pragma unroll
      for (int kb = 0; kb < KB; ++kb)
        v2[q][kb] = __builtin_bit_cast(mlp::bf8, bp[(PB::kW2 + t * KB + kb) * kWave]);
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) fw1[q][j] = wt(PK::kW1 + 2 * t + j);
#pragma unroll
    for (int tt = 0; tt < MT; ++tt)
#pragma unroll
      for (int i = 0; i < 4; ++i) fw2[q][tt][i] = wt(PK::kW2 + (t * MT + tt) * 4 + i);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      fw3[q][i] = wt(PK::kW3 + 4 * t + i);
      fb1[q][i] = pf[(PK::kB1 + 4 * t + i) * kWave];
      fb2[q][i] = pf[(PK::kB2 + 4 * t + i) * kWave];
      fb3[q][i] = (BF || t == 0) ? pf[(PK::kB3 + i) * kWave] : 0.0f;
    }
  }
  if constexpr (BF) {
    using PB = mlp::PackBf<MT>;
#pragma unroll
    for (int kb = 0; kb < KB; ++kb)
      v3[kb] = __builtin_bit_cast(mlp::bf8, p.mlp_bf[(PB::kW3 + kb) * kWave + lane]);
  }

  const int idx = base + n;
  const bool valid = idx < count;
  const BwdItem item = list[valid ? idx : base];
  const float a = valid ? item.a : 0.0f;
  const float* e = eps + item.k;
  int seg, h, t0, len;
  unit_steps(unit, sub, c, T, seg, h, t0, len);
  float x[N], comp[N], xd[N];
  const float* ck = ckpt + static_cast<int64_t>(seg) * 7 * ldk + item.k;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    x[i] = ck[i * ldk];
    comp[i] = 0.0f;
    xd[i] = i == col ? 1.0f : 0.0f;
  }
  comp[0] = ck[5 * ldk];
  comp[1] = ck[6 * ldk];
  const f4 zero4{0.0f, 0.0f, 0.0f, 0.0f};
  const float v0[2] = {0.0f, 0.0f};
  int par = 0;
  float q = 0.0f;
  // column 0 keeps the unit's forward for its sweep
  const int row = tile * nunit + unit, cs = tp_unit_steps(c);
  float* st = tp + tp_states_off(tp_tiles, nunit, c, row, n);
  f4* my_pre = pre + static_cast<int64_t>(row) * cs * 2 * MT * kWave + lane;
  const bool keep = col == 0;
  // one step: the MLP forward (and with TAN its tangent along xd), then the
  // RK4 step (and the tangent's); every wave runs it (barriers inside)
  auto one_step = [&](int t, bool tan) {
    float v[M];
#pragma unroll
    for (int k = 0; k < M; ++k) v[k] = u[t * M + k] + e[static_cast<int64_t>(t * M + k) * ldk];
    f4* ps = my_pre + static_cast<int64_t>(t - t0) * 2 * MT * kWave;
    if (tan && keep && w == 0 && g == 0) {
#pragma unroll
      for (int i = 0; i < N; ++i) st[(t - t0) * N + i] = x[i];
#pragma unroll
      for (int k = 0; k < M; ++k) st[(cs + 1) * N + (t - t0) * M + k] = v[k];
    }
    float xn[N];
    if (tan) rk4_jvp<FAST>(p, x, v, xd, xn);
    const float z0 = mlp::input_operand(x, v, g, 0), z1 = mlp::input_operand(x, v, g, 1);
    const float y0 = mlp::input_operand(xd, v0, g, 0), y1 = mlp::input_operand(xd, v0, g, 1);
    mlp::bf8 zb;
    if constexpr (BF) zb = mlp::input_operand_bf(x, v, g);
#pragma unroll
    for (int qq = 0; qq < TW; ++qq) {
      f4 a1;
      if constexpr (BF) a1 = mlp::mfma_bf(v1[qq], zb, fb1[qq]);
      else a1 = mlp::mfma(fw1[qq][1], z1, mlp::mfma(fw1[qq][0], z0, fb1[qq]));
      if (tan && keep) ps[(q0 + qq) * kWave] = a1;
      f4 h1, d1;
      mlp::tanh4_d(a1, h1, d1);
      xch(xa, par, q0 + qq) = h1;
      if (tan)
        xch(xt1, par, q0 + qq) = mlp::mfma(fw1[qq][1], y1, mlp::mfma(fw1[qq][0], y0, zero4)) * d1;
    }
    __syncthreads();
    f4 acc[TW], acct[TW];
#pragma unroll
    for (int qq = 0; qq < TW; ++qq) { acc[qq] = fb2[qq]; acct[qq] = zero4; }
    if constexpr (BF) {
      f4 h1a[MT];
#pragma unroll
      for (int tt = 0; tt < MT; ++tt) h1a[tt] = xch(xa, par, tt);
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) {
        const mlp::bf8 hb = mlp::kblock_operand<MT>(h1a, kb);
#pragma unroll
        for (int qq = 0; qq < TW; ++qq) acc[qq] = mlp::mfma_bf(v2[qq][kb], hb, acc[qq]);
      }
    } else {
#pragma unroll
      for (int tt = 0; tt < MT; ++tt) {
        const f4 hh = xch(xa, par, tt);
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int qq = 0; qq < TW; ++qq) acc[qq] = mlp::mfma(fw2[qq][tt][i], hh[i], acc[qq]);
      }
    }
    if (tan) {
#pragma unroll
      for (int tt = 0; tt < MT; ++tt) {
        const f4 ht = xch(xt1, par, tt);
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int qq = 0; qq < TW; ++qq) acct[qq] = mlp::mfma(fw2[qq][tt][i], ht[i], acct[qq]);
      }
    }
#pragma unroll
    for (int qq = 0; qq < TW; ++qq) {
      if (tan && keep) ps[(MT + q0 + qq) * kWave] = acc[qq];
      f4 h2, d2;
      mlp::tanh4_d(acc[qq], h2, d2);
      if constexpr (BF) {
        xch(xb, par, q0 + qq) = h2;  // the h2 tiles: every wave forms the output
      } else {
        f4 part = fb3[qq];
#pragma unroll
        for (int i = 0; i < 4; ++i) part = mlp::mfma(fw3[qq][i], h2[i], part);
        xch(xb, par, q0 + qq) = part;
      }
      if (tan) {
        const f4 h2t = acct[qq] * d2;
        f4 pt = zero4;
#pragma unroll
        for (int i = 0; i < 4; ++i) pt = mlp::mfma(fw3[qq][i], h2t[i], pt);
        xch(xt3, par, q0 + qq) = pt;
      }
    }
    __syncthreads();
    f4 out;
    if constexpr (BF) {
      f4 h2a[MT];
#pragma unroll
      for (int tt = 0; tt < MT; ++tt) h2a[tt] = xch(xb, par, tt);
      out = fb3[0];
#pragma unroll
      for (int kb = 0; kb < KB; ++kb)
        out = mlp::mfma_bf(v3[kb], mlp::kblock_operand<MT>(h2a, kb), out);
    } else {
      out = xch(xb, par, 0);
#pragma unroll
      for (int tt = 1; tt < MT; ++tt) out += xch(xb, par, tt);
    }
    float res[N];
    mlp::broadcast5(out, n, res);
    if (tan) {
      f4 ot = xch(xt3, par, 0);
#pragma unroll
      for (int tt = 1; tt < MT; ++tt) ot += xch(xt3, par, tt);
      float gd[N];
      mlp::broadcast5(ot, n, gd);
#pragma unroll
      for (int i = 0; i < N; ++i) xn[i] += p.dt * gd[i];
    }
    par ^= 1;
    step<Model, kRK4>(x, v, comp, p, res);
    if (tan) {
      const float* r = p.ref + static_cast<int64_t>(t + 1) * N;
#pragma unroll
      for (int i = 0; i < N; ++i) {
        xd[i] = xn[i];
        q = fmaf(a * 2.0f * p.w[i] * (x[i] - r[i]), xd[i], q);
      }
    }
  };
  // the segment's steps before the unit: the sweep's rebuild, no tangent
  for (int t = seg * c; t < t0; ++t) one_step(t, false);
  float* rec = tp + (static_cast<int64_t>(tile * nunit + unit) * kTileS + n) * kTpRec;
  for (int t = t0; t < t0 + len; ++t) one_step(t, true);
  if (w == 0 && g == 0) {
#pragma unroll
    for (int i = 0; i < N; ++i) rec[col * 6 + i] = xd[i];
    rec[col * 6 + 5] = q;
    if (keep) {
#pragma unroll
      for (int i = 0; i < N; ++i) st[len * N + i] = x[i];
    }
    if (unit == nunit - 1 && col == 0) {  // after the last step: x_T
#pragma unroll
      for (int i = 0; i < N; ++i) rec[kTpXT + i] = x[i];
    }
  }
}

template <int MT, bool BF = false>
struct SweepLds {
  static constexpr int P = 64 * MT + 16;  // transposition row stride (16 mod 32: no bank conflicts)
  static constexpr int kFwd = MT ? mlp::Pack<MT>::kFwdRows * kWave : 0;
  static constexpr int kBwd = MT ? mlp::Pack<MT>::kBwdRows * kWave : 0;
  // BF16 mode: the bfloat16 weight pack (16 bytes per lane and row)
  static constexpr int kBf = (MT && BF) ? mlp::PackBf<MT ? MT : 1>::kRows * kWave * 4 : 0;
  static constexpr int kTb = MT ? kTileS * P : 0;
  static size_t bytes(int c) {
    return sizeof(float) * (kFwd + kBwd + kBf + kTb + kTileS * ((c + 1) * 5 + c * 2));
  }
};

// Sum over the 16 lanes of a lane group (fixed xor tree).
__device__ __forceinline__ float group_sum(float v) {
  v += __shfl_xor(v, 8, kWave);
  v += __shfl_xor(v, 4, kWave);
  v += __shfl_xor(v, 2, kWave);
  v += __shfl_xor(v, 1, kWave);
  return v;
}

// The tile's share of dL/du_t = sum_k a_k dJ_k/du_t for one step: dv holds
// the a_k-weighted (dF/dv)^T mu of the lane's sample; the control term of the
// running cost (2 R v) and, with the importance-sampling term, its
// derivative in u through v = u + eps and directly (lambda Sigma^-1 v) are
// added, then the 16 samples of the tile are summed (fixed xor tree) and
// lane 0 writes out[0..1].  Every lane of the wave must call it.
// ic: the constant importance coefficients, read once per kernel by the caller.
__device__ __forceinline__ void du_step(const DevParams& p, const float* ic, int t, float a,
                                        const float* v, float* dv, int lane, float* out) {
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    float d = dv[q] + a * (2.0f * p.w[8 + q] * v[q]);
    if (p.importance) {
      // a branch, not a pointer select: a pointer that may name the
      // by-value array becomes a generic (flat) load, whose wait also drains
      // the loads the sweep requests ahead
      const float cq = p.is_coef_t ? p.is_coef_t[2 * t + q] : ic[q];
      d += a * (cq * v[q]);
    }
    const float sum = group_sum(d);
    if (lane == 0) out[q] = sum;
  }
}

// BF: the forward rebuild takes the BF16 products (mlp::hidden_bf), and the
// weight gradients take the rounded layer inputs (the roundings count as the
// identity; the adjoint's transposed pack holds the rounded weights).
template <int MT, bool FAST, bool BF = false>
__global__ __launch_bounds__(kWave) void adjoint_sweep_kernel(
    DevParams p, const float* __restrict__ u, const float* __restrict__ eps, int64_t ldk, int T,
    const float* __restrict__ ckpt, int c, const BwdItem* __restrict__ list,
    const BwdMeta* __restrict__ meta, float* __restrict__ partial, int64_t ngp, int du_off,
    mlp::f4* __restrict__ pre, const float* __restrict__ tp, int tp_tiles) {
  using Model = Bicycle<FAST>;
  using L = SweepLds<MT, BF>;
  using f4 = mlp::f4;
  constexpr int N = 5, M = 2, H = 16 * MT;
  const int nseg = (T + c - 1) / c;
  const SegSel sel = seg_select(nseg, c, tp_tiles, meta->count);
  const int nunit = nseg * sel.sub;
  const int base = sel.tile * kTileS;
  if (base >= meta->count) return;  // wave-uniform
  extern __shared__ float4 lds4[];
  float* lds = reinterpret_cast<float*>(lds4);
  const int lane = threadIdx.x, n = lane % kTileS, g = lane / kTileS;
  if constexpr (MT > 0) {
    const float4* src_f = reinterpret_cast<const float4*>(p.mlp);
    const float4* src_b = reinterpret_cast<const float4*>(p.mlp_bwd);
    for (int i = lane; i < L::kFwd / 4; i += kWave) lds4[i] = src_f[i];
    for (int i = lane; i < L::kBwd / 4; i += kWave) lds4[L::kFwd / 4 + i] = src_b[i];
    if constexpr (BF) {
      const float4* src_h = reinterpret_cast<const float4*>(p.mlp_bf);
      for (int i = lane; i < L::kBf / 4; i += kWave) lds4[(L::kFwd + L::kBwd) / 4 + i] = src_h[i];
    }
  }
  const mlp::PackView<MT ? MT : 1> WF{lds + lane};
  const mlp::PackView<MT ? MT : 1> WB{lds + L::kFwd + lane};
  const mlp::PackViewBf<MT ? MT : 1> WFB{
      reinterpret_cast<const uint4*>(lds + L::kFwd + L::kBwd) + lane, WF};
  float* tb = lds + L::kFwd + L::kBwd + L::kBf;
  float* xs = tb + L::kTb + n * ((c + 1) * N);                     // [c+1][5] of sample n
  float* vs = tb + L::kTb + kTileS * (c + 1) * N + n * (c * M);    // [c][2] of sample n
  __syncthreads();

  // this tile's pre-activation scratch: [c steps][2 layers][MT][64 lanes] f4
  // (a row holds c steps, or a unit's steps in the segment-parallel mode)
  const int pre_steps = sel.par ? tp_unit_steps(c) : c;
  mlp::f4* my_pre =
      pre + static_cast<int64_t>(blockIdx.x) * pre_steps * 2 * (MT ? MT : 1) * kWave + lane;
  const int idx = base + n;
  const bool valid = idx < meta->count;
  const BwdItem item = list[valid ? idx : base];
  const int k = item.k;
  const float a = valid ? item.a : 0.0f;  // padding lanes rebuild a listed sample, weight 0
  const float* e = eps + k;

  // accumulators: weight gradients (D layout), biases, Q, wheelbase
  f4 dW1[MT ? MT : 1], dW2[MT ? MT : 1][MT ? MT : 1], dW3[MT ? MT : 1];
  f4 db1[MT ? MT : 1], db2[MT ? MT : 1];
  float db3[N], gQ[N], gL = 0.0f, mu[N];
  const f4 zero4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int t = 0; t < (MT ? MT : 1); ++t) {
    dW1[t] = dW3[t] = db1[t] = db2[t] = zero4;
#pragma unroll
    for (int q = 0; q < (MT ? MT : 1); ++q) dW2[t][q] = zero4;
  }
#pragma unroll
  for (int i = 0; i < N; ++i) { db3[i] = 0.0f; gQ[i] = 0.0f; mu[i] = 0.0f; }
  const float ic[2] = {p.is_coef[0], p.is_coef[1]};

  if (sel.par) {
    if (sel.hi < nunit - 1) tp_chain(p, tp, sel.tile, nunit, sel.hi, n, T, a, mu);
    if (du_off >= 0) {
      int sg, hp, ut0, ulen;
      unit_steps(sel.hi, sel.sub, c, T, sg, hp, ut0, ulen);
      tp_zero_du(partial + static_cast<int64_t>(blockIdx.x) * ngp, du_off, T, ut0, ulen,
                 threadIdx.x, blockDim.x);
    }
  }
  for (int ui = sel.hi; ui >= sel.lo; --ui) {
    int seg, hp, t0, len;
    unit_steps(ui, sel.sub, c, T, seg, hp, t0, len);
    if (sel.par) {
      // the unit's states, controls and pre-activations as the map kernel kept them
      if (g == 0) copy_unit_forward(tp + tp_states_off(tp_tiles, nunit, c, sel.tile * nunit + ui, n),
                                    c, len, xs, vs);
    } else {
      // rebuild x_{t0} .. x_{t0+len} from the checkpoint
      float x[N], comp[N];
      load_checkpoint(ckpt, ldk, k, seg, x, comp);
      // u and the noise of a step are requested one step ahead
      float un[M], en[M];
      auto fetch_v = [&](int t) {
  #pragma unroll
        for (int q = 0; q < M; ++q) {
          un[q] = u[t * M + q];
          en[q] = e[static_cast<int64_t>(t * M + q) * ldk];
        }
      };
      if (len > 0) fetch_v(t0);
      for (int j = 0; j < len; ++j) {
        const int t = t0 + j;
        float v[M];
  #pragma unroll
        for (int q = 0; q < M; ++q) v[q] = un[q] + en[q];
        if (j + 1 < len) fetch_v(t + 1);
        if (g == 0) {
  #pragma unroll
          for (int i = 0; i < N; ++i) xs[j * N + i] = x[i];
  #pragma unroll
          for (int q = 0; q < M; ++q) vs[j * M + q] = v[q];
        }
        if constexpr (MT > 0) {
          float res[N];
          f4 a1[MT], a2[MT];
          if constexpr (BF) mlp::residual_keep<MT>(WFB, x, v, g, n, res, a1, a2);
          else mlp::residual_keep<MT>(WF, x, v, g, n, res, a1, a2);
          f4* ps = my_pre + static_cast<int64_t>(j) * 2 * MT * kWave;
  #pragma unroll
          for (int t2 = 0; t2 < MT; ++t2) {
            ps[t2 * kWave] = a1[t2];
            ps[(MT + t2) * kWave] = a2[t2];
          }
          step<Model, kRK4>(x, v, comp, p, res);
        } else {
          step<Model, kRK4>(x, v, comp, p);
        }
      }
      if (g == 0) {
  #pragma unroll
        for (int i = 0; i < N; ++i) xs[len * N + i] = x[i];
      }
    }
    __syncthreads();
    if (ui == nunit - 1) {  // terminal cost w16 sum_i Q_i (x_T - r_T)^2
      const float* r = p.ref + static_cast<int64_t>(T) * N;
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const float d = xs[len * N + i] - r[i];
        mu[i] = a * 2.0f * p.w[16] * p.w[i] * d;
        gQ[i] += a * p.w[16] * d * d;
      }
    }
    // the reference state after each step, requested one step ahead
    float rn[N];
    auto fetch_r = [&](int j) {
      const float* r = p.ref + static_cast<int64_t>(t0 + j + 1) * N;
#pragma unroll
      for (int i = 0; i < N; ++i) rn[i] = r[i];
    };
    if (len > 0) fetch_r(len - 1);
    for (int j = len - 1; j >= 0; --j) {
      const int t = t0 + j;
      // running cost at x_{t+1}
      float r[N];
#pragma unroll
      for (int i = 0; i < N; ++i) r[i] = rn[i];
      if (j > 0) fetch_r(j - 1);
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const float d = xs[(j + 1) * N + i] - r[i];
        mu[i] += a * 2.0f * p.w[i] * d;
        gQ[i] += a * d * d;
      }
      float xt[N], v[M];
#pragma unroll
      for (int i = 0; i < N; ++i) xt[i] = xs[j * N + i];
#pragma unroll
      for (int q = 0; q < M; ++q) v[q] = vs[j * M + q];
      float mu0[N], dv[M] = {0.0f, 0.0f};
      rk4_vjp<FAST>(p, xt, v, mu, mu0, gL, dv);

      if constexpr (MT > 0) {
        // residual dt g(z): c = dt mu_{t+1}
        f4 h1[MT], h2[MT], d1[MT], d2[MT], da1[MT], da2[MT], dz;
        {
          const f4* ps = my_pre + static_cast<int64_t>(j) * 2 * MT * kWave;
#pragma unroll
          for (int t2 = 0; t2 < MT; ++t2) {
            mlp::tanh4_d(ps[t2 * kWave], h1[t2], d1[t2]);
            mlp::tanh4_d(ps[(MT + t2) * kWave], h2[t2], d2[t2]);
          }
        }
        float cg[N];
#pragma unroll
        for (int i = 0; i < N; ++i) cg[i] = p.dt * mu[i];
        mlp::backward<MT>(WB, cg, g, d1, d2, da1, da2, dz);
        float dzs[N];
        mlp::broadcast5(dz, n, dzs);
#pragma unroll
        for (int i = 0; i < N; ++i) mu0[i] += dzs[i];
        dv[0] += __shfl(dz[1], 16 + n, kWave);  // z rows 5, 6: the controls
        dv[1] += __shfl(dz[2], 16 + n, kWave);
#pragma unroll
        for (int t2 = 0; t2 < MT; ++t2) { db1[t2] += da1[t2]; db2[t2] += da2[t2]; }
#pragma unroll
        for (int i = 0; i < N; ++i) db3[i] += cg[i];
        // weight gradients: transpose the tile's activations through LDS so
        // the samples become the MFMA contraction index
        float* row = tb + n * L::P;
#pragma unroll
        for (int t2 = 0; t2 < MT; ++t2) {
          *reinterpret_cast<f4*>(row + 16 * t2 + 4 * g) = BF ? mlp::round_bf4(h1[t2]) : h1[t2];
          *reinterpret_cast<f4*>(row + H + 16 * t2 + 4 * g) = BF ? mlp::round_bf4(h2[t2]) : h2[t2];
          *reinterpret_cast<f4*>(row + 2 * H + 16 * t2 + 4 * g) = da1[t2];
          *reinterpret_cast<f4*>(row + 3 * H + 16 * t2 + 4 * g) = da2[t2];
        }
        // rows 4H .. 4H+7: z = (x, v, 0); rows 4H+8 .. 4H+15: c (5) and zeros
        f4 zc = g == 0 ? f4{xt[0], xt[1], xt[2], xt[3]}
              : g == 1 ? f4{xt[4], v[0], v[1], 0.0f}
              : g == 2 ? f4{cg[0], cg[1], cg[2], cg[3]}
                       : f4{cg[4], 0.0f, 0.0f, 0.0f};
        if (BF && g < 2) zc = mlp::round_bf4(zc);
        *reinterpret_cast<f4*>(row + 4 * H + 4 * g) = zc;
        __syncthreads();
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const float* tq = tb + (4 * s + g) * L::P;
          float ah[MT], ad2[MT], ad1[MT], bh2[MT];
#pragma unroll
          for (int t2 = 0; t2 < MT; ++t2) {
            ah[t2] = tq[16 * t2 + n];
            bh2[t2] = tq[H + 16 * t2 + n];
            ad1[t2] = tq[2 * H + 16 * t2 + n];
            ad2[t2] = tq[3 * H + 16 * t2 + n];
          }
          const float bz = tq[4 * H + n];
          const float ac = n < 8 ? tq[4 * H + 8 + n] : 0.0f;
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) {
#pragma unroll
            for (int nt = 0; nt < MT; ++nt) dW2[mt][nt] = mlp::mfma(ad2[mt], ah[nt], dW2[mt][nt]);
            dW1[mt] = mlp::mfma(ad1[mt], bz, dW1[mt]);
            dW3[mt] = mlp::mfma(ac, bh2[mt], dW3[mt]);
          }
        }
        __syncthreads();
      }
      if (du_off >= 0)
        du_step(p, ic, t, a, v, dv, lane, partial + blockIdx.x * ngp + du_off + t * M);
#pragma unroll
      for (int i = 0; i < N; ++i) mu[i] = mu0[i];
    }
    __syncthreads();  // xs / vs are rewritten by the next segment
  }

  // this tile's partial gradient: [W1 | b1 | W2 | b2 | W3 | b3 | Q | wheelbase]
  float* out = partial + static_cast<int64_t>(blockIdx.x) * ngp;
  const int offQ = MT ? 14 * H + H * H + 5 : 0;
  if constexpr (MT > 0) {
    const int oB1 = 7 * H, oW2 = 8 * H, oB2 = 8 * H + H * H, oW3 = 9 * H + H * H,
              oB3 = 14 * H + H * H;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = 16 * mt + 4 * g + i;
        if (n < 7) out[r * 7 + n] = dW1[mt][i];
#pragma unroll
        for (int nt = 0; nt < MT; ++nt) out[oW2 + r * H + 16 * nt + n] = dW2[mt][nt][i];
        const int o = 4 * g + i;
        if (o < 5) out[oW3 + o * H + 16 * mt + n] = dW3[mt][i];
        const float s1 = group_sum(db1[mt][i]);
        const float s2 = group_sum(db2[mt][i]);
        if (n == 0) { out[oB1 + r] = s1; out[oB2 + r] = s2; }
      }
    }
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const float s3 = group_sum(db3[i]);
      if (lane == 0) out[oB3 + i] = s3;
    }
  }
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const float sq = group_sum(gQ[i]);
    if (lane == 0) out[offQ + i] = sq;
  }
  const float sl = group_sum(gL);
  if (lane == 0) out[offQ + N] = sl;
}

// The sweep with the tile's MLP split over SW waves of one workgroup (SW = 2
// or 4, H = 16 MT): wave w owns the TW = MT / SW hidden M-tiles q0 = w TW, ...
// in every product, with its operand slices in registers (the weight packs
// need no LDS):
//   forward rebuild: h1 of the own tiles, then h2 of the own tiles over all of
//     h1 (h1 tiles exchanged through LDS), output partials of the own K-tiles
//     (exchanged);
//   reverse: da2 of the own tiles = (W3^T c) d2; da1 of the own tiles =
//     (W2^T da2) d1 over all da2 tiles (exchanged); dz partials of the own
//     K-tiles (exchanged); dW2 / dW1 rows and dW3 columns of the own tiles as
//     outer products over the tile's samples (the activations of all waves
//     meet in the shared transposition buffer).
// Every accumulation runs in the order of the one-wave sweep, so the
// gradient is bitwise the same; the bicycle step and its transpose are
// repeated by every wave.
template <int MT, int SW>
struct SplitLds {
  static constexpr int P = 64 * MT + 16;
  static size_t bytes(int c) {
    return sizeof(float) * (kTileS * P + kTileS * ((c + 1) * 5 + c * 2)) +
           sizeof(mlp::f4) * 2 * 2 * MT * kWave;
  }
};

// BF: the forward rebuild on the bfloat16 products as the split forward
// kernel takes them (h2 tiles exchanged, the output over every K-block in
// order), and the weight gradients over the rounded layer inputs.
template <int MT, int SW, bool FAST, bool BF = false>
__global__ __launch_bounds__(kWave * SW) void adjoint_sweep_split_kernel(
    DevParams p, const float* __restrict__ u, const float* __restrict__ eps, int64_t ldk, int T,
    const float* __restrict__ ckpt, int c, const BwdItem* __restrict__ list,
    const BwdMeta* __restrict__ meta, float* __restrict__ partial, int64_t ngp, int du_off,
    mlp::f4* __restrict__ pre, const float* __restrict__ tp, int tp_tiles) {
  static_assert(MT % SW == 0, "tiles per wave");
  constexpr int TW = MT / SW;
  using Model = Bicycle<FAST>;
  using f4 = mlp::f4;
  using PK = mlp::Pack<MT>;
  constexpr int N = 5, M = 2, H = 16 * MT, PS = SplitLds<MT, SW>::P;
  const int nseg = (T + c - 1) / c;
  const SegSel sel = seg_select(nseg, c, tp_tiles, meta->count);
  const int nunit = nseg * sel.sub;
  const int base = sel.tile * kTileS;
  if (base >= meta->count) return;  // workgroup-uniform
  extern __shared__ float4 lds4[];
  float* tb = reinterpret_cast<float*>(lds4);                             // [16][PS]
  float* st_x = tb + kTileS * PS;                                         // states
  f4* xa = reinterpret_cast<f4*>(st_x + kTileS * ((c + 1) * N + c * M));  // [2][MT][64]
  f4* xb = xa + 2 * MT * kWave;                                           // [2][MT][64]
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  const int n = lane % kTileS, g = lane / kTileS;
  const int q0 = w * TW;
  float* xs = st_x + n * ((c + 1) * N);
  float* vs = st_x + kTileS * (c + 1) * N + n * (c * M);
  auto xch = [&](f4* buf, int par, int q) -> f4& { return buf[(par * MT + q) * kWave + lane]; };

  // this wave's operand slices
  const float* pf = p.mlp + lane;
  const float* pb = p.mlp_bwd + lane;
  constexpr int KB = mlp::PackBf<MT>::KB;
  constexpr int TWF = BF ? 1 : TW, MTF = BF ? 1 : MT;
  constexpr int TWB = BF ? TW : 1, KBB = BF ? KB : 1;
  float fw1[TWF][2], fw2[TWF][MTF][4], fw3[TWF][4], bw3t[TW][2], bw2t[TW][MT][4], bw1t[TW][4];
  mlp::bf8 v1[TWB], v2[TWB][KBB], v3[KBB];
  f4 fb1[TW], fb2[TW], fb3[TW];
#pragma unroll
  for (int q = 0; q < TW; ++q) {
    const int t = q0 + q;
    if constexpr (BF) {
      using PB = mlp::PackBf<MT>;
      const uint4* bp = p.mlp_bf + lane;
      v1[q] = __builtin_bit_cast(mlp::bf8, bp[(PB::kW1 + t) * kWave]);
#pragma unroll
      for (int kb = 0; kb < KB; ++kb)
        v2[q][kb] = __builtin_bit_cast(mlp::bf8, bp[(PB::kW2 + t * KB + kb) * kWave]);
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      if constexpr (!BF) fw1[q][j] = pf[(PK::kW1 + 2 * t + j) * kWave];
      bw3t[q][j] = pb[(PK::kW3t + 2 * t + j) * kWave];
    }
#pragma unroll
    for (int tt = 0; tt < MT; ++tt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        if constexpr (!BF) fw2[q][tt][i] = pf[(PK::kW2 + (t * MT + tt) * 4 + i) * kWave];
        bw2t[q][tt][i] = pb[(PK::kW2t + (t * MT + tt) * 4 + i) * kWave];
      }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if constexpr (!BF) fw3[q][i] = pf[(PK::kW3 + 4 * t + i) * kWave];
      bw1t[q][i] = pb[(PK::kW1t + 4 * t + i) * kWave];
      fb1[q][i] = pf[(PK::kB1 + 4 * t + i) * kWave];
      fb2[q][i] = pf[(PK::kB2 + 4 * t + i) * kWave];
      fb3[q][i] = (BF || t == 0) ? pf[(PK::kB3 + i) * kWave] : 0.0f;
    }
  }
  if constexpr (BF) {
    using PB = mlp::PackBf<MT>;
#pragma unroll
    for (int kb = 0; kb < KB; ++kb)
      v3[kb] = __builtin_bit_cast(mlp::bf8, p.mlp_bf[(PB::kW3 + kb) * kWave + lane]);
  }

  // this tile's pre-activation scratch: [c steps][2 layers][MT][64 lanes] f4
  const int pre_steps = sel.par ? tp_unit_steps(c) : c;
  f4* my_pre = pre + static_cast<int64_t>(blockIdx.x) * pre_steps * 2 * MT * kWave + lane;
  const int idx = base + n;
  const bool valid = idx < meta->count;
  const BwdItem item = list[valid ? idx : base];
  const int k = item.k;
  const float a = valid ? item.a : 0.0f;
  const float* e = eps + k;

  const f4 zero4{0.0f, 0.0f, 0.0f, 0.0f};
  f4 dW1[TW], dW3[TW], db1[TW], db2[TW], dW2[TW][MT];
#pragma unroll
  for (int q = 0; q < TW; ++q) {
    dW1[q] = dW3[q] = db1[q] = db2[q] = zero4;
#pragma unroll
    for (int nt = 0; nt < MT; ++nt) dW2[q][nt] = zero4;
  }
  float db3[N], gQ[N], gL = 0.0f, mu[N];
#pragma unroll
  for (int i = 0; i < N; ++i) { db3[i] = 0.0f; gQ[i] = 0.0f; mu[i] = 0.0f; }
  const float ic[2] = {p.is_coef[0], p.is_coef[1]};
  int par = 0;

  if (sel.par) {
    if (sel.hi < nunit - 1) tp_chain(p, tp, sel.tile, nunit, sel.hi, n, T, a, mu);
    if (du_off >= 0) {
      int sg, hp, ut0, ulen;
      unit_steps(sel.hi, sel.sub, c, T, sg, hp, ut0, ulen);
      tp_zero_du(partial + static_cast<int64_t>(blockIdx.x) * ngp, du_off, T, ut0, ulen,
                 threadIdx.x, blockDim.x);
    }
  }
  for (int ui = sel.hi; ui >= sel.lo; --ui) {
    int seg, hp, t0, len;
    unit_steps(ui, sel.sub, c, T, seg, hp, t0, len);
    if (sel.par) {
      // the unit's states, controls and pre-activations as the map kernel kept them
      if (w == 0 && g == 0)
        copy_unit_forward(tp + tp_states_off(tp_tiles, nunit, c, sel.tile * nunit + ui, n), c,
                          len, xs, vs);
    } else {
      float x[N], comp[N];
      load_checkpoint(ckpt, ldk, k, seg, x, comp);
      // u and the noise of a step are requested one step ahead, so their
      // latency hides behind the previous step's work (barriers wait for LDS
      // only, not for these loads)
      float un[M], en[M];
      auto fetch_v = [&](int t) {
  #pragma unroll
        for (int q = 0; q < M; ++q) {
          un[q] = u[t * M + q];
          en[q] = e[static_cast<int64_t>(t * M + q) * ldk];
        }
      };
      if (len > 0) fetch_v(t0);
      for (int j = 0; j < len; ++j) {
        const int t = t0 + j;
        float v[M];
  #pragma unroll
        for (int q = 0; q < M; ++q) v[q] = un[q] + en[q];
        if (j + 1 < len) fetch_v(t + 1);
        if (w == 0 && g == 0) {
  #pragma unroll
          for (int i = 0; i < N; ++i) xs[j * N + i] = x[i];
  #pragma unroll
          for (int q = 0; q < M; ++q) vs[j * M + q] = v[q];
        }
        // MLP forward, split (as the split forward kernel)
        f4* ps = my_pre + static_cast<int64_t>(j) * 2 * MT * kWave;
        if constexpr (BF) {
          const mlp::bf8 zb = mlp::input_operand_bf(x, v, g);
  #pragma unroll
          for (int q = 0; q < TW; ++q) {
            const f4 a1 = mlp::mfma_bf(v1[q], zb, fb1[q]);
            ps[(q0 + q) * kWave] = a1;
            xch(xa, par, q0 + q) = mlp::tanh4(a1);
          }
        } else {
          const float z0 = mlp::input_operand(x, v, g, 0), z1 = mlp::input_operand(x, v, g, 1);
  #pragma unroll
          for (int q = 0; q < TW; ++q) {
            const f4 a1 = mlp::mfma(fw1[q][1], z1, mlp::mfma(fw1[q][0], z0, fb1[q]));
            ps[(q0 + q) * kWave] = a1;
            xch(xa, par, q0 + q) = mlp::tanh4(a1);
          }
        }
        __syncthreads();
        f4 acc[TW];
  #pragma unroll
        for (int q = 0; q < TW; ++q) acc[q] = fb2[q];
        f4 out;
        if constexpr (BF) {
          f4 h1a[MT];
  #pragma unroll
          for (int tt = 0; tt < MT; ++tt) h1a[tt] = xch(xa, par, tt);
  #pragma unroll
          for (int kb = 0; kb < KB; ++kb) {
            const mlp::bf8 hb = mlp::kblock_operand<MT>(h1a, kb);
  #pragma unroll
            for (int q = 0; q < TW; ++q) acc[q] = mlp::mfma_bf(v2[q][kb], hb, acc[q]);
          }
  #pragma unroll
          for (int q = 0; q < TW; ++q) {
            ps[(MT + q0 + q) * kWave] = acc[q];
            xch(xb, par, q0 + q) = mlp::tanh4(acc[q]);
          }
          __syncthreads();
          f4 h2a[MT];
  #pragma unroll
          for (int tt = 0; tt < MT; ++tt) h2a[tt] = xch(xb, par, tt);
          out = fb3[0];
  #pragma unroll
          for (int kb = 0; kb < KB; ++kb) out = mlp::mfma_bf(v3[kb], mlp::kblock_operand<MT>(h2a, kb), out);
        } else {
  #pragma unroll
          for (int tt = 0; tt < MT; ++tt) {
            const f4 h = xch(xa, par, tt);
  #pragma unroll
            for (int i = 0; i < 4; ++i)
  #pragma unroll
              for (int q = 0; q < TW; ++q) acc[q] = mlp::mfma(fw2[q][tt][i], h[i], acc[q]);
          }
  #pragma unroll
          for (int q = 0; q < TW; ++q) {
            ps[(MT + q0 + q) * kWave] = acc[q];
            const f4 h2 = mlp::tanh4(acc[q]);
            f4 part = fb3[q];
  #pragma unroll
            for (int i = 0; i < 4; ++i) part = mlp::mfma(fw3[q][i], h2[i], part);
            xch(xb, par, q0 + q) = part;
          }
          __syncthreads();
          out = xch(xb, par, 0);
  #pragma unroll
          for (int tt = 1; tt < MT; ++tt) out += xch(xb, par, tt);
        }
        par ^= 1;
        float res[N];
        mlp::broadcast5(out, n, res);
        step<Model, kRK4>(x, v, comp, p, res);
      }
      if (w == 0 && g == 0) {
  #pragma unroll
        for (int i = 0; i < N; ++i) xs[len * N + i] = x[i];
      }
    }
    __syncthreads();
    if (ui == nunit - 1) {
      const float* r = p.ref + static_cast<int64_t>(T) * N;
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const float d = xs[len * N + i] - r[i];
        mu[i] = a * 2.0f * p.w[16] * p.w[i] * d;
        gQ[i] += a * p.w[16] * d * d;
      }
    }
    // the reference state after the step and the step's MLP pre-activations,
    // requested one step ahead like the forward's noise
    float rn[N];
    f4 pn1[TW], pn2[TW];
    auto fetch_r = [&](int j) {
      const float* r = p.ref + static_cast<int64_t>(t0 + j + 1) * N;
#pragma unroll
      for (int i = 0; i < N; ++i) rn[i] = r[i];
      const f4* ps = my_pre + static_cast<int64_t>(j) * 2 * MT * kWave;
#pragma unroll
      for (int q = 0; q < TW; ++q) {
        pn1[q] = ps[(q0 + q) * kWave];
        pn2[q] = ps[(MT + q0 + q) * kWave];
      }
    };
    if (len > 0) fetch_r(len - 1);
    for (int j = len - 1; j >= 0; --j) {
      const int t = t0 + j;
      float r[N];
      f4 pa1[TW], pa2[TW];
#pragma unroll
      for (int i = 0; i < N; ++i) r[i] = rn[i];
#pragma unroll
      for (int q = 0; q < TW; ++q) {
        pa1[q] = pn1[q];
        pa2[q] = pn2[q];
      }
      if (j > 0) fetch_r(j - 1);
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const float d = xs[(j + 1) * N + i] - r[i];
        mu[i] += a * 2.0f * p.w[i] * d;
        gQ[i] += a * d * d;
      }
      float xt[N], v[M];
#pragma unroll
      for (int i = 0; i < N; ++i) xt[i] = xs[j * N + i];
#pragma unroll
      for (int q = 0; q < M; ++q) v[q] = vs[j * M + q];
      float mu0[N], dv[M] = {0.0f, 0.0f};
      rk4_vjp<FAST>(p, xt, v, mu, mu0, gL, dv);
      // the MLP residual dt g(z): c = dt mu_{t+1}
      f4 h1[TW], d1[TW], h2[TW], d2[TW];
#pragma unroll
      for (int q = 0; q < TW; ++q) {
        mlp::tanh4_d(pa1[q], h1[q], d1[q]);
        mlp::tanh4_d(pa2[q], h2[q], d2[q]);
      }
      float cg[N];
#pragma unroll
      for (int i = 0; i < N; ++i) cg[i] = p.dt * mu[i];
      const float c0 = g == 0 ? cg[0] : g == 1 ? cg[1] : g == 2 ? cg[2] : cg[3];
      const float c1 = g == 0 ? cg[4] : 0.0f;
      f4 da2[TW];
#pragma unroll
      for (int q = 0; q < TW; ++q) {
        da2[q] = mlp::mfma(bw3t[q][1], c1, mlp::mfma(bw3t[q][0], c0, zero4)) * d2[q];
        xch(xa, par, q0 + q) = da2[q];
      }
      __syncthreads();
      f4 acc[TW];
#pragma unroll
      for (int q = 0; q < TW; ++q) acc[q] = zero4;
#pragma unroll
      for (int tt = 0; tt < MT; ++tt) {
        const f4 d = xch(xa, par, tt);
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int q = 0; q < TW; ++q) acc[q] = mlp::mfma(bw2t[q][tt][i], d[i], acc[q]);
      }
      float* row = tb + n * PS;
      f4 da1[TW];
#pragma unroll
      for (int q = 0; q < TW; ++q) {
        da1[q] = acc[q] * d1[q];
        f4 zp = zero4;
#pragma unroll
        for (int i = 0; i < 4; ++i) zp = mlp::mfma(bw1t[q][i], da1[q][i], zp);
        xch(xb, par, q0 + q) = zp;
        // the transposition buffer: the own rows
        const int qt = q0 + q;
        *reinterpret_cast<f4*>(row + 16 * qt + 4 * g) = BF ? mlp::round_bf4(h1[q]) : h1[q];
        *reinterpret_cast<f4*>(row + H + 16 * qt + 4 * g) = BF ? mlp::round_bf4(h2[q]) : h2[q];
        *reinterpret_cast<f4*>(row + 2 * H + 16 * qt + 4 * g) = da1[q];
        *reinterpret_cast<f4*>(row + 3 * H + 16 * qt + 4 * g) = da2[q];
      }
      if (w == 0) {  // z and c
        f4 zc = g == 0 ? f4{xt[0], xt[1], xt[2], xt[3]}
              : g == 1 ? f4{xt[4], v[0], v[1], 0.0f}
              : g == 2 ? f4{cg[0], cg[1], cg[2], cg[3]}
                       : f4{cg[4], 0.0f, 0.0f, 0.0f};
        if (BF && g < 2) zc = mlp::round_bf4(zc);
        *reinterpret_cast<f4*>(row + 4 * H + 4 * g) = zc;
      }
      __syncthreads();
      f4 dz = xch(xb, par, 0);
#pragma unroll
      for (int tt = 1; tt < MT; ++tt) dz += xch(xb, par, tt);
      par ^= 1;
      float dzs[N];
      mlp::broadcast5(dz, n, dzs);
#pragma unroll
      for (int i = 0; i < N; ++i) mu0[i] += dzs[i];
      dv[0] += __shfl(dz[1], 16 + n, kWave);  // z rows 5, 6: the controls
      dv[1] += __shfl(dz[2], 16 + n, kWave);
#pragma unroll
      for (int q = 0; q < TW; ++q) {
        db1[q] += da1[q];
        db2[q] += da2[q];
      }
      if (w == 0) {
#pragma unroll
        for (int i = 0; i < N; ++i) db3[i] += cg[i];
      }
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) {
        const float* tq = tb + (4 * s4 + g) * PS;
        const float bz = tq[4 * H + n];
        const float ac = n < 8 ? tq[4 * H + 8 + n] : 0.0f;
        float bh1[MT];
#pragma unroll
        for (int nt = 0; nt < MT; ++nt) bh1[nt] = tq[16 * nt + n];
#pragma unroll
        for (int q = 0; q < TW; ++q) {
          const int qt = q0 + q;
          const float ad2 = tq[3 * H + 16 * qt + n];
          const float ad1 = tq[2 * H + 16 * qt + n];
          const float bh2 = tq[H + 16 * qt + n];
#pragma unroll
          for (int nt = 0; nt < MT; ++nt) dW2[q][nt] = mlp::mfma(ad2, bh1[nt], dW2[q][nt]);
          dW1[q] = mlp::mfma(ad1, bz, dW1[q]);
          dW3[q] = mlp::mfma(ac, bh2, dW3[q]);
        }
      }
      __syncthreads();  // the transposition buffer is rewritten by the next step
      if (du_off >= 0 && w == 0)
        du_step(p, ic, t, a, v, dv, lane, partial + blockIdx.x * ngp + du_off + t * M);
#pragma unroll
      for (int i = 0; i < N; ++i) mu[i] = mu0[i];
    }
    __syncthreads();  // xs / vs are rewritten by the next segment
  }

  // this tile's partial gradient: [W1 | b1 | W2 | b2 | W3 | b3 | Q | wheelbase]
  float* out = partial + static_cast<int64_t>(blockIdx.x) * ngp;
  const int oB1 = 7 * H, oW2 = 8 * H, oB2 = 8 * H + H * H, oW3 = 9 * H + H * H,
            oB3 = 14 * H + H * H, offQ = 14 * H + H * H + 5;
#pragma unroll
  for (int q = 0; q < TW; ++q) {
    const int qt = q0 + q;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = 16 * qt + 4 * g + i;
      if (n < 7) out[r * 7 + n] = dW1[q][i];
#pragma unroll
      for (int nt = 0; nt < MT; ++nt) out[oW2 + r * H + 16 * nt + n] = dW2[q][nt][i];
      const int o = 4 * g + i;
      if (o < 5) out[oW3 + o * H + 16 * qt + n] = dW3[q][i];
      const float s1 = group_sum(db1[q][i]);
      const float s2 = group_sum(db2[q][i]);
      if (n == 0) { out[oB1 + r] = s1; out[oB2 + r] = s2; }
    }
  }
  if (w == 0) {
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const float s3 = group_sum(db3[i]);
      if (lane == 0) out[oB3 + i] = s3;
      const float sq = group_sum(gQ[i]);
      if (lane == 0) out[offQ + i] = sq;
    }
    const float sl = group_sum(gL);
    if (lane == 0) out[offQ + N] = sl;
  }
}

// Column j of the sum over the swept tiles of partial[tile][j]: 64 columns
// per workgroup, the tiles split over 16 lanes per column (tile = p mod 16),
// the 16 partial sums combined in a fixed order.  Columns j < ngrad are the
// gradient (grad[j] = sum, or += with accumulate); columns ngrad.. (ncols >
// ngrad) are dL/du, added to G[j - ngrad].  In the segment-parallel mode the
// rows are the (tile, unit) pairs.
constexpr int kReduceCols = 64, kReduceParts = 16;
__global__ __launch_bounds__(kReduceCols * kReduceParts) void adjoint_reduce_kernel(
    const float* __restrict__ partial, int64_t ngp, int ngrad, int ncols,
    const BwdMeta* __restrict__ meta, float* __restrict__ grad, int accumulate,
    float* __restrict__ G, int tp_tiles, int nunit) {
  __shared__ float red[kReduceParts][kReduceCols];
  const int c = threadIdx.x % kReduceCols, part = threadIdx.x / kReduceCols;
  const int j = blockIdx.x * kReduceCols + c;
  const int count = meta->count;
  const int tiles = (count + kTileS - 1) / kTileS *
                    (tp_tiles > 0 && count <= tp_tiles * kTileS ? nunit : 1);
  float s = 0.0f;
  if (j < ncols) {
    int w = part;
    float s1 = 0.0f;
    for (; w + kReduceParts < tiles; w += 2 * kReduceParts) {
      s += partial[static_cast<int64_t>(w) * ngp + j];
      s1 += partial[static_cast<int64_t>(w + kReduceParts) * ngp + j];
    }
    if (w < tiles) s += partial[static_cast<int64_t>(w) * ngp + j];
    s += s1;
  }
  red[part][c] = s;
  __syncthreads();
  if (part == 0 && j < ncols) {
    float t = red[0][c];
#pragma unroll
    for (int q = 1; q < kReduceParts; ++q) t += red[q][c];
    if (j < ngrad) {
      grad[j] = accumulate ? grad[j] + t : t;
    } else {
      G[j - ngrad] += t;
    }
  }
}

// ---- host side ----------------------------------------------------------------
int adjoint_grad_len(uint32_t dynamics, int hidden) {
  const int H = dynamics == MPPI_DYN_BICYCLE_MLP ? hidden : 0;
  return (H ? 14 * H + H * H + 5 : 0) + 6;
}

AdjointScratch adjoint_scratch_layout(int K, int ngrad, int hidden, int ckpt_every, int TM) {
  AdjointScratch s{};
  const int nb = (K + kProjectSamples - 1) / kProjectSamples;
  const int tiles = (K + kTileS - 1) / kTileS;
  s.ngp = (ngrad + TM + 63) / 64 * 64;  // the gradient, then dL/du
  size_t off = 0;
  auto take = [&](size_t b) { size_t o = off; off = (off + b + 255) / 256 * 256; return o; };
  s.gk = take(sizeof(float) * K);
  s.part = take(sizeof(BwdBlock) * nb);
  s.offs = take(sizeof(int) * nb);
  s.meta = take(sizeof(BwdMeta));
  s.list = take(sizeof(BwdItem) * K);
  // rows: one per tile, or per (tile, unit) in the segment-parallel mode
  const int nunit = (TM / 2 + ckpt_every - 1) / ckpt_every * tp_sub(ckpt_every);
  const int tp_max = tp_cap(tiles, nunit);
  const size_t rows = std::max(static_cast<size_t>(tiles), static_cast<size_t>(tp_max) * nunit);
  s.partial = take(sizeof(float) * rows * s.ngp);
  // pre-activations of one segment per tile row (c steps), or of one unit per
  // (tile, unit) row: steps x 2 layers x H/16 x 64 lanes x 4
  const size_t pre_steps = std::max(static_cast<size_t>(tiles) * ckpt_every,
                                    static_cast<size_t>(tp_max) * nunit * tp_unit_steps(ckpt_every));
  s.pre = take(sizeof(float) * 4 * pre_steps * 2 * (hidden > 0 ? hidden / 16 : 0) * kWave);
  // the unit records, then the units' kept forward (states and controls)
  s.tp = take(sizeof(float) * static_cast<size_t>(tp_max) * nunit * kTileS *
              (kTpRec + tp_state_floats(ckpt_every)));
  s.total = off;
  return s;
}

size_t adjoint_lds_bytes(int hidden, int ckpt_every, bool bf) {
  switch (hidden) {
    case 0: return SweepLds<0>::bytes(ckpt_every);
    case 16: return bf ? SweepLds<1, true>::bytes(ckpt_every) : SweepLds<1>::bytes(ckpt_every);
    case 32: return bf ? SweepLds<2, true>::bytes(ckpt_every) : SweepLds<2>::bytes(ckpt_every);
    case 64: return bf ? SweepLds<4, true>::bytes(ckpt_every) : SweepLds<4>::bytes(ckpt_every);
    default: return 0;
  }
}

namespace {
using SweepFn = void (*)(DevParams, const float*, const float*, int64_t, int, const float*, int,
                         const BwdItem*, const BwdMeta*, float*, int64_t, int, mlp::f4*,
                         const float*, int);
using TpFn = void (*)(DevParams, const float*, const float*, int64_t, int, const float*, int,
                      const BwdItem*, const BwdMeta*, int, float*, mlp::f4*);
template <int MT, bool BF = false>
TpFn pick_tp(bool accurate) {
  return accurate ? adjoint_tp_kernel<MT, false, BF> : adjoint_tp_kernel<MT, true, BF>;
}
template <int MT, bool BF = false>
SweepFn pick_sweep(bool accurate) {
  return accurate ? adjoint_sweep_kernel<MT, false, BF> : adjoint_sweep_kernel<MT, true, BF>;
}
template <int MT, int SW>
SweepFn pick_split_sweep(bool accurate, bool bf) {
  if (bf)
    return accurate ? adjoint_sweep_split_kernel<MT, SW, false, true>
                    : adjoint_sweep_split_kernel<MT, SW, true, true>;
  return accurate ? adjoint_sweep_split_kernel<MT, SW, false>
                  : adjoint_sweep_split_kernel<MT, SW, true>;
}
}  // namespace

hipError_t launch_adjoint(const DevParams& p, bool accurate_trig, int hidden, const float* d_G,
                          const float* d_u, const float* d_eps, int64_t ldk, int K, int T,
                          const float* d_e, float lambda, float step, const float* d_ckpt,
                          int ckpt_every, char* d_scratch, const AdjointScratch& s, int ngrad,
                          float* d_grad, hipStream_t stream, int waves, bool accumulate,
                          float* d_G_acc, int tp_tiles) {
  SweepFn fn = nullptr;
  const bool bf = hidden > 0 && p.mlp_bf != nullptr;  // BF16 products
  const int tiles = (K + kTileS - 1) / kTileS;
  const int nunit = (T + ckpt_every - 1) / ckpt_every * tp_sub(ckpt_every);
  // segment-parallel mode: up to tp tiles
  const int tp = std::min(std::max(tp_tiles, 0), tp_cap(tiles, nunit));
  TpFn tfn = nullptr;
  int twaves = 1;
  size_t tlds = 0;  // the forward pack (binary32), then the bfloat16 pack
  switch (hidden) {
    case 0: tfn = pick_tp<0>(accurate_trig); break;
    case 16:
      tfn = bf ? pick_tp<1, true>(accurate_trig) : pick_tp<1>(accurate_trig);
      tlds = mlp::Pack<1>::kFwdRows + (bf ? 4 * mlp::PackBf<1>::kRows : 0);
      break;
    case 32:
      tfn = bf ? pick_tp<2, true>(accurate_trig) : pick_tp<2>(accurate_trig);
      tlds = mlp::Pack<2>::kFwdRows + (bf ? 4 * mlp::PackBf<2>::kRows : 0);
      break;
    case 64:
      tfn = bf ? pick_tp<4, true>(accurate_trig) : pick_tp<4>(accurate_trig);
      tlds = mlp::Pack<4>::kFwdRows + (bf ? 4 * mlp::PackBf<4>::kRows : 0);
      break;
    default: break;
  }
  tlds *= sizeof(float) * kWave;
  if (hidden == 64) {  // the MLP split over 4 waves
    if (bf)
      tfn = accurate_trig ? adjoint_tp_split_kernel<4, 4, false, true>
                          : adjoint_tp_split_kernel<4, 4, true, true>;
    else
      tfn = accurate_trig ? adjoint_tp_split_kernel<4, 4, false>
                          : adjoint_tp_split_kernel<4, 4, true>;
    twaves = 4;
    tlds = sizeof(mlp::f4) * 4 * 2 * 4 * kWave;
  }
  if (tp > 0 && tfn && tlds > 48 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(tfn),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       static_cast<int>(tlds));
    if (e != hipSuccess) return e;
  }
  size_t lds = adjoint_lds_bytes(hidden, ckpt_every, bf);
  if (waves > 1) {
    if (hidden == 64 && waves == 4) {
      fn = pick_split_sweep<4, 4>(accurate_trig, bf);
      lds = SplitLds<4, 4>::bytes(ckpt_every);
    } else if (hidden == 64 && waves == 2) {
      fn = pick_split_sweep<4, 2>(accurate_trig, bf);
      lds = SplitLds<4, 2>::bytes(ckpt_every);
    } else if (hidden == 32 && waves == 2) {
      fn = pick_split_sweep<2, 2>(accurate_trig, bf);
      lds = SplitLds<2, 2>::bytes(ckpt_every);
    } else {
      return hipErrorInvalidValue;
    }
  } else {
    switch (hidden) {
      case 0: fn = pick_sweep<0>(accurate_trig); break;
      case 16: fn = bf ? pick_sweep<1, true>(accurate_trig) : pick_sweep<1>(accurate_trig); break;
      case 32: fn = bf ? pick_sweep<2, true>(accurate_trig) : pick_sweep<2>(accurate_trig); break;
      case 64: fn = bf ? pick_sweep<4, true>(accurate_trig) : pick_sweep<4>(accurate_trig); break;
      default: return hipErrorInvalidValue;
    }
  }
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  if (lds > 48 * 1024) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       static_cast<int>(lds));
    if (e != hipSuccess) return e;
  }
  float* gk = reinterpret_cast<float*>(d_scratch + s.gk);
  BwdBlock* part = reinterpret_cast<BwdBlock*>(d_scratch + s.part);
  int* offs = reinterpret_cast<int*>(d_scratch + s.offs);
  BwdMeta* meta = reinterpret_cast<BwdMeta*>(d_scratch + s.meta);
  BwdItem* list = reinterpret_cast<BwdItem*>(d_scratch + s.list);
  float* partial = reinterpret_cast<float*>(d_scratch + s.partial);
  mlp::f4* pre = reinterpret_cast<mlp::f4*>(d_scratch + s.pre);
  const int nb = (K + kProjectSamples - 1) / kProjectSamples;
  const int TM = T * 2;
  hipLaunchKernelGGL(adjoint_project_kernel, dim3(nb), dim3(kProjectBlock), 0, stream, d_G, d_eps,
                     ldk, K, TM, d_e, gk, part);
  hipLaunchKernelGGL(adjoint_scan_kernel, dim3(1), dim3(kScanBlock), 0, stream, part, nb, d_e, gk,
                     K, offs, meta);
  hipLaunchKernelGGL(adjoint_compact_kernel, dim3(nb), dim3(kProjectSamples), 0, stream, d_e, gk,
                     K, static_cast<float>(static_cast<double>(step) / static_cast<double>(lambda)),
                     offs, meta, list);
  const int du_off = d_G_acc ? ngrad : -1;
  const int ncols = ngrad + (d_G_acc ? TM : 0);
  if (ncols > s.ngp) return hipErrorInvalidValue;
  float* tpbuf = reinterpret_cast<float*>(d_scratch + s.tp);
  if (tp > 0) {
    if (!tfn) return hipErrorInvalidValue;
    hipLaunchKernelGGL(tfn, dim3(tp * nunit * 5), dim3(kWave * twaves), tlds, stream, p, d_u,
                       d_eps, ldk, T, d_ckpt, ckpt_every, list, meta, tp, tpbuf, pre);
  }
  const int rows = std::max(tiles, tp * nunit);
  hipLaunchKernelGGL(fn, dim3(rows), dim3(kWave * waves), lds, stream, p, d_u, d_eps, ldk, T,
                     d_ckpt, ckpt_every, list, meta, partial, s.ngp, du_off, pre, tpbuf, tp);
  hipLaunchKernelGGL(adjoint_reduce_kernel, dim3((ncols + kReduceCols - 1) / kReduceCols),
                     dim3(kReduceCols * kReduceParts), 0, stream, partial, s.ngp, ngrad, ncols,
                     meta, d_grad, accumulate ? 1 : 0, d_G_acc, tp, nunit);
  return hipGetLastError();
}

}  // namespace mppi
