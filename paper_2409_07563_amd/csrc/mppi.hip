// Host side of the C ABI declared in include/mppi.h: argument validation,
// workspace carving, parameter upload, the circle grid, batch work lists and
// the launch sequence of MPPI iterations (arXiv 2409.07563, Algorithm 1),
// captured once per iteration count in a hipGraph.  No device allocation
// happens here; all device memory is the caller's workspace.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "common.h"
#include "mlp.h"
#include "worklist.h"

using namespace mppi;

namespace {

thread_local std::string g_last_error = "";

// The workspace of mppi_create_static: a fixed array every GPU this library
// runs on holds (its own copy at its own address) until the process ends.  In
// host code the name only stands for the array; its device address comes from
// hipGetSymbolAddress on that device, kept per device below.
constexpr size_t kStaticWorkspaceBytes = MPPI_STATIC_WORKSPACE_BYTES;
static __device__ __align__(256) char scratch[kStaticWorkspaceBytes];
constexpr int kMaxStaticDevices = 64;
struct StaticWorkspace {
  char* ptr = nullptr;  // device address on that device (set on first use)
  bool busy = false;    // a live context holds it
};
std::mutex g_static_mu;
StaticWorkspace g_static[kMaxStaticDevices];

mppi_status fail(mppi_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
mppi_status fail(mppi_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

mppi_status hip_fail(hipError_t e, const char* what) {
  return fail(MPPI_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(expr)                                 \
  do {                                                \
    hipError_t e_ = (expr);                           \
    if (e_ != hipSuccess) return hip_fail(e_, #expr); \
  } while (0)

int model_dims(uint32_t dyn, int* n, int* m) {
  switch (dyn) {
    case MPPI_DYN_DOUBLE_INTEGRATOR: *n = 4; *m = 2; return 1;
    case MPPI_DYN_BICYCLE: *n = 5; *m = 2; return 1;
    case MPPI_DYN_QUADROTOR: *n = 13; *m = 4; return 1;
    case MPPI_DYN_BICYCLE_MLP: *n = 5; *m = 2; return 1;
    default: return 0;
  }
}

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Per-instance workspace slice (byte offsets from the slice base, 256-aligned).
struct Layout {
  int64_t ldk;  // noise row stride (K rounded up to a wave)
  // single contexts whose two buffers fit the cache: two noise buffers, so
  // that an update can draw the next iteration's noise while the weighted sum
  // still reads this one's (eps2 == eps otherwise)
  size_t eps, eps2, e;
  size_t words;  // single contexts: the iteration word each noise buffer was drawn with
  size_t wpart;  // single contexts: the chunked update's per-chunk sums
  size_t ref, stage, costmap, mlp, mlp_bwd, mlp_bf;
  size_t sigma_t, is_coef_t;  // per-step noise deviations and importance coefficients
  // MPPI_F_REQUIRES_GRAD: checkpoints [nseg][7][ldk], the rollout's controls,
  // the adjoint's scratch
  size_t ckpt, u_roll, adj;
  AdjointScratch adj_layout;
  // the differentiation tape: u [tape_len][T*m], iteration words, the count,
  // the reverse pass's dL/du and its scratch state
  size_t tape_u, tape_word, tape_count, tape_G, tape_state;
  // split rollout form: the trajectory buffer [T][traj_words][ldk] and the
  // cost chunks' partial sums and counts
  size_t traj, split_part;
  int traj_words;  // 0: no split form for this instance
  size_t total;
};

int mlp_hidden_of(const mppi_config* c, const mppi_params* p) {
  return c->dynamics == MPPI_DYN_BICYCLE_MLP ? p->mlp_hidden : 0;
}
int pack_rows(int hidden, bool bwd) {
  switch (hidden) {
    case 16: return bwd ? mlp::Pack<1>::kBwdRows : mlp::Pack<1>::kFwdRows;
    case 32: return bwd ? mlp::Pack<2>::kBwdRows : mlp::Pack<2>::kFwdRows;
    case 64: return bwd ? mlp::Pack<4>::kBwdRows : mlp::Pack<4>::kFwdRows;
    default: return 0;
  }
}
bool wants_grad(const mppi_config* c) { return (c->flags & MPPI_F_REQUIRES_GRAD) != 0; }
// Updates the reverse pass of mppi_backward_iters can reach back through.
int tape_len_of(const mppi_params* p) { return p->tape_len > 0 ? p->tape_len : 16; }
// Samples k >= n_plain are drawn around zero: the last floor(fraction K), at
// most K - 1 when sample 0 is the noiseless mean.
int n_plain_of(const mppi_config* c) {
  const int K = c->num_samples;
  int64_t nz = static_cast<int64_t>(floor(static_cast<double>(c->zero_mean_fraction) * K));
  if (nz > K) nz = K;
  if ((c->flags & MPPI_F_MEAN_SAMPLE) && nz > K - 1) nz = K - 1;
  if (nz < 0) nz = 0;
  return K - static_cast<int>(nz);
}
// The step size gamma of the update (1: Algorithm 1).
float step_size(const mppi_config& c) {
  return (c.flags & MPPI_F_STEP_SIZE) ? c.step_size : 1.0f;
}
int ckpt_every_of(const mppi_params* p) { return p->checkpoint_every ? p->checkpoint_every : 10; }

bool bf16_of(const mppi_config* c) { return (c->flags & MPPI_F_BF16_MLP) != 0; }
// rows of the bfloat16 weight pack (mlp::PackBf)
int bf_pack_rows(int hidden) {
  const int MT = hidden / 16, KB = (MT + 1) / 2;
  return MT + MT * KB + KB;
}

// binary32 -> bfloat16 bits, round to nearest, ties to even (a NaN stays a
// quiet NaN)
uint16_t bf16_bits(float x) {
  uint32_t b;
  memcpy(&b, &x, 4);
  if ((b & 0x7F800000u) == 0x7F800000u && (b & 0x7FFFFFu)) return static_cast<uint16_t>((b >> 16) | 0x40u);
  b += 0x7FFFu + ((b >> 16) & 1u);
  return static_cast<uint16_t>(b >> 16);
}
float bf16_round(float x) {
  const uint32_t b = static_cast<uint32_t>(bf16_bits(x)) << 16;
  float r;
  memcpy(&r, &b, 4);
  return r;
}

// The MFMA operand packs of the MLP (lane layout in mlp.h) from the weight
// blob W1[H][7] b1[H] W2[H][H] b2[H] W3[5][H] b3[5].  bf (BF16 mode, optional):
// also the bfloat16 weight pack, and the adjoint's pack takes the rounded
// weights (the products' derivatives use the weights the forward used).
void build_mlp_packs(const float* blob_in, int H, std::vector<float4>* fwd,
                     std::vector<float4>* bwd, std::vector<uint4>* bf = nullptr) {
  const int MT = H / 16;
  std::vector<float> rounded;
  const float* blob = blob_in;
  if (bf) {
    const int nw = 14 * H + H * H + 5;
    rounded.assign(blob_in, blob_in + nw);
    const int oW2 = 8 * H, oW3 = 9 * H + H * H;
    for (int i = 0; i < 7 * H; ++i) rounded[i] = bf16_round(rounded[i]);
    for (int i = 0; i < H * H; ++i) rounded[oW2 + i] = bf16_round(rounded[oW2 + i]);
    for (int i = 0; i < 5 * H; ++i) rounded[oW3 + i] = bf16_round(rounded[oW3 + i]);
    blob = rounded.data();
  }
  const float* W1 = blob;
  const float* b1 = W1 + 7 * H;
  const float* W2 = b1 + H;
  const float* b2 = W2 + H * H;
  const float* W3 = b2 + H;
  const float* b3 = W3 + 5 * H;
  if (bf) {
    // slot (g, j) of K-block kb: hidden unit 16(2kb) + 4g + j (j < 4) or
    // 16(2kb+1) + 4g + j - 4; -1 where the tile does not exist
    auto unit = [&](int kb, int g, int j) {
      const int tile = 2 * kb + (j >> 2);
      return tile < MT ? 16 * tile + 4 * g + (j & 3) : -1;
    };
    const int KB = (MT + 1) / 2;
    bf->assign(static_cast<size_t>(bf_pack_rows(H)) * kWave, uint4{0, 0, 0, 0});
    for (int l = 0; l < kWave; ++l) {
      const int n = l % 16, g = l / 16;
      int r = 0;
      auto put = [&](const float* v8) {
        uint32_t w[4];
        for (int q = 0; q < 4; ++q)
          w[q] = static_cast<uint32_t>(bf16_bits(v8[2 * q])) |
                 (static_cast<uint32_t>(bf16_bits(v8[2 * q + 1])) << 16);
        (*bf)[static_cast<size_t>(r++) * kWave + l] = uint4{w[0], w[1], w[2], w[3]};
      };
      float v8[8];
      for (int t = 0; t < MT; ++t) {  // W1: z slot (0, j) = z_j
        for (int j = 0; j < 8; ++j) {
          const int k = 8 * g + j;
          v8[j] = k < 7 ? W1[(16 * t + n) * 7 + k] : 0.0f;
        }
        put(v8);
      }
      for (int t = 0; t < MT; ++t)
        for (int kb = 0; kb < KB; ++kb) {
          for (int j = 0; j < 8; ++j) {
            const int u = unit(kb, g, j);
            v8[j] = u >= 0 ? W2[(16 * t + n) * H + u] : 0.0f;
          }
          put(v8);
        }
      for (int kb = 0; kb < KB; ++kb) {
        for (int j = 0; j < 8; ++j) {
          const int u = unit(kb, g, j);
          v8[j] = (u >= 0 && n < 5) ? W3[n * H + u] : 0.0f;
        }
        put(v8);
      }
    }
  }
  const int fr = pack_rows(H, false), br = pack_rows(H, true);
  std::vector<float> f(static_cast<size_t>(fr) * kWave, 0.0f), b(static_cast<size_t>(br) * kWave, 0.0f);
  for (int l = 0; l < kWave; ++l) {
    const int n = l % 16, g = l / 16;
    int r = 0;
    auto F = [&](float v) { f[static_cast<size_t>(r++) * kWave + l] = v; };
    for (int t = 0; t < MT; ++t)
      for (int j = 0; j < 2; ++j) F(4 * j + g < 7 ? W1[(16 * t + n) * 7 + 4 * j + g] : 0.0f);
    for (int t = 0; t < MT; ++t)
      for (int tt = 0; tt < MT; ++tt)
        for (int i = 0; i < 4; ++i) F(W2[(16 * t + n) * H + 16 * tt + 4 * g + i]);
    for (int tt = 0; tt < MT; ++tt)
      for (int i = 0; i < 4; ++i) F(n < 5 ? W3[n * H + 16 * tt + 4 * g + i] : 0.0f);
    for (int t = 0; t < MT; ++t)
      for (int i = 0; i < 4; ++i) F(b1[16 * t + 4 * g + i]);
    for (int t = 0; t < MT; ++t)
      for (int i = 0; i < 4; ++i) F(b2[16 * t + 4 * g + i]);
    for (int i = 0; i < 4; ++i) F(4 * g + i < 5 ? b3[4 * g + i] : 0.0f);
    r = 0;
    auto B = [&](float v) { b[static_cast<size_t>(r++) * kWave + l] = v; };
    for (int t = 0; t < MT; ++t)
      for (int j = 0; j < 2; ++j) B(4 * j + g < 5 ? W3[(4 * j + g) * H + 16 * t + n] : 0.0f);
    for (int t = 0; t < MT; ++t)
      for (int tt = 0; tt < MT; ++tt)
        for (int i = 0; i < 4; ++i) B(W2[(16 * tt + 4 * g + i) * H + 16 * t + n]);
    for (int tt = 0; tt < MT; ++tt)
      for (int i = 0; i < 4; ++i) B(n < 7 ? W1[(16 * tt + 4 * g + i) * 7 + n] : 0.0f);
  }
  fwd->assign(reinterpret_cast<const float4*>(f.data()),
              reinterpret_cast<const float4*>(f.data()) + f.size() / 4);
  bwd->assign(reinterpret_cast<const float4*>(b.data()),
              reinterpret_cast<const float4*>(b.data()) + b.size() / 4);
}

bool uses_circles(uint32_t cost) {
  return cost == MPPI_COST_PATH_CIRCLES || cost == MPPI_COST_GOAL_CIRCLES;
}
bool uses_spline(uint32_t cost) {
  return cost == MPPI_COST_PATH_CIRCLES || cost == MPPI_COST_PATH_COSTMAP;
}

mppi_status validate(const mppi_config* c, const mppi_params* p, int* n_out, int* m_out) {
  if (!c || !p) return fail(MPPI_EINVAL, "config and params must not be NULL");
  if (c->abi_version != MPPI_ABI_VERSION)
    return fail(MPPI_EINVAL, "abi_version %u, library speaks %u", c->abi_version, MPPI_ABI_VERSION);
  int n, m;
  if (!model_dims(c->dynamics, &n, &m)) return fail(MPPI_EINVAL, "unknown dynamics %u", c->dynamics);
  if (c->state_dim != n || c->control_dim != m)
    return fail(MPPI_EINVAL, "state/control dims %d/%d do not match the dynamics (%d/%d)",
                c->state_dim, c->control_dim, n, m);
  if (c->integrator > MPPI_INT_RK4) return fail(MPPI_EINVAL, "unknown integrator %u", c->integrator);
  if (c->cost > MPPI_COST_GOAL_CIRCLES) return fail(MPPI_EINVAL, "unknown cost %u", c->cost);
  if (c->num_samples < 1 || c->num_samples > (1 << 20))
    return fail(MPPI_EINVAL, "num_samples %d outside [1, 2^20]", c->num_samples);
  if (c->horizon < 1 || c->horizon > 4096)
    return fail(MPPI_EINVAL, "horizon %d outside [1, 4096]", c->horizon);
  if (!(c->dt > 0.0f) || !isfinite(c->dt)) return fail(MPPI_EINVAL, "dt must be finite and > 0");
  if (!(c->lambda > 0.0f) || !isfinite(c->lambda))
    return fail(MPPI_EINVAL, "lambda must be finite and > 0");
  for (int j = 0; j < m; ++j)
    if (!(c->sigma[j] >= 0.0f) || !isfinite(c->sigma[j]))
      return fail(MPPI_EINVAL, "sigma[%d] must be finite and >= 0", j);
  if (c->flags & MPPI_F_IMPORTANCE_SAMPLING)
    for (int j = 0; j < m; ++j)
      if (!(c->sigma[j] > 0.0f))
        return fail(MPPI_EINVAL, "MPPI_F_IMPORTANCE_SAMPLING needs sigma[%d] > 0", j);
  if ((c->flags & MPPI_F_STEP_SIZE) && (!(c->step_size >= 0.0f) || !isfinite(c->step_size)))
    return fail(MPPI_EINVAL, "step_size must be finite and >= 0");
  if (!(c->zero_mean_fraction >= 0.0f && c->zero_mean_fraction <= 1.0f))
    return fail(MPPI_EINVAL, "zero_mean_fraction must be in [0, 1]");
  if (wants_grad(c) && c->zero_mean_fraction != 0.0f)
    return fail(MPPI_EUNSUPPORTED, "MPPI_F_REQUIRES_GRAD needs zero_mean_fraction = 0");
  if (p->sigma_t)
    for (int64_t i = 0; i < (int64_t)c->horizon * m; ++i) {
      const float sg = p->sigma_t[i];
      if (!(sg >= 0.0f) || !isfinite(sg)) return fail(MPPI_EINVAL, "sigma_t[%lld] must be finite and >= 0", (long long)i);
      if ((c->flags & MPPI_F_IMPORTANCE_SAMPLING) && !(sg > 0.0f))
        return fail(MPPI_EINVAL, "MPPI_F_IMPORTANCE_SAMPLING needs sigma_t[%lld] > 0", (long long)i);
    }
  if (bf16_of(c) && c->dynamics != MPPI_DYN_BICYCLE_MLP)
    return fail(MPPI_EINVAL, "MPPI_F_BF16_MLP is for BICYCLE_MLP dynamics");
  if (c->dynamics == MPPI_DYN_BICYCLE_MLP) {
    if (!p->mlp) return fail(MPPI_EINVAL, "MLP dynamics need the weight blob");
    if (p->mlp_hidden != 16 && p->mlp_hidden != 32 && p->mlp_hidden != 64)
      return fail(MPPI_EUNSUPPORTED, "MLP hidden width %d: built for 16, 32 and 64",
                  p->mlp_hidden);
    if (!rollout_tiles_supported(c->dynamics, c->integrator, c->cost, p->mlp_hidden))
      return fail(MPPI_EUNSUPPORTED, "cost %u is not built for MLP dynamics", c->cost);
  } else if (!rollout_supported(c->dynamics, c->integrator, c->cost)) {
    return fail(MPPI_EUNSUPPORTED, "cost %u is not defined for dynamics %u", c->cost, c->dynamics);
  }
  if ((c->dynamics == MPPI_DYN_BICYCLE || c->dynamics == MPPI_DYN_BICYCLE_MLP) &&
      !(p->wheelbase > 0.0f))
    return fail(MPPI_EINVAL, "wheelbase must be > 0");
  if (wants_grad(c)) {
    if (!((c->dynamics == MPPI_DYN_BICYCLE || c->dynamics == MPPI_DYN_BICYCLE_MLP) &&
          c->integrator == MPPI_INT_RK4 && c->cost == MPPI_COST_TRACK))
      return fail(MPPI_EUNSUPPORTED, "MPPI_F_REQUIRES_GRAD needs the bicycle (with or without "
                  "the MLP residual), RK4 and the TRACK cost");
    if (p->checkpoint_every < 0 || p->checkpoint_every > 64)
      return fail(MPPI_EINVAL, "checkpoint_every %d outside [0, 64]", p->checkpoint_every);
    if (p->tape_len < 0 || p->tape_len > 1024)
      return fail(MPPI_EINVAL, "tape_len %d outside [0, 1024]", p->tape_len);
  }
  if (p->cost_cosines < 0 || p->cost_cosines > 65536)
    return fail(MPPI_EINVAL, "cost_cosines %d outside [0, 65536]", p->cost_cosines);
  if (c->dynamics == MPPI_DYN_QUADROTOR) {
    if (!(p->mass > 0.0f)) return fail(MPPI_EINVAL, "mass must be > 0");
    for (int i = 0; i < 3; ++i)
      if (!(p->inertia[i] > 0.0f)) return fail(MPPI_EINVAL, "inertia[%d] must be > 0", i);
  }
  // cost data
  int need_ref = 0;
  switch (c->cost) {
    case MPPI_COST_QUADRATIC: need_ref = n; break;
    case MPPI_COST_HOVER: need_ref = 11; break;
    case MPPI_COST_TRACK: need_ref = (c->horizon + 1) * n; break;
    case MPPI_COST_GOAL_CIRCLES: need_ref = 2; break;
    default: break;
  }
  if (need_ref && (!p->ref || p->ref_len < need_ref))
    return fail(MPPI_EINVAL, "cost needs ref with >= %d floats (got %d)", need_ref, p->ref_len);
  if (uses_spline(c->cost)) {
    if (p->num_segments < 1 || p->num_segments > 1024 || !p->knots || !p->coef)
      return fail(MPPI_EINVAL, "path cost needs 1..1024 spline segments with knots and coef");
    for (int s = 0; s < p->num_segments; ++s)
      if (!(p->knots[s + 1] > p->knots[s]))
        return fail(MPPI_EINVAL, "spline knots must increase (knot %d)", s + 1);
  }
  if (uses_circles(c->cost)) {
    if (p->num_circles < 0 || p->num_circles > 2048)
      return fail(MPPI_EINVAL, "num_circles %d outside [0, 2048]", p->num_circles);
    if (p->num_circles > 0 && (!p->cx || !p->cy || !p->r2))
      return fail(MPPI_EINVAL, "circle arrays must not be NULL");
  }
  if (c->cost == MPPI_COST_PATH_COSTMAP) {
    if (p->map_w < 2 || p->map_h < 2 || !p->costmap || !(p->map_res > 0.0f))
      return fail(MPPI_EINVAL, "costmap needs map_w, map_h >= 2, map_res > 0 and data");
    if ((int64_t)p->map_w * p->map_h > (int64_t)1 << 26)
      return fail(MPPI_EINVAL, "costmap larger than 2^26 cells");
  }
  *n_out = n;
  *m_out = m;
  return MPPI_OK;
}

// The split rollout form exists for single, non-MLP, non-gradient contexts
// whose cost kernel fits the LDS.
bool split_form_for(const mppi_config* c, const mppi_params* p, bool batch) {
  if (batch || wants_grad(c) || mlp_hidden_of(c, p) ||
      !rollout_split_supported(c->dynamics, c->integrator, c->cost))
    return false;
  return true;
}

// The next iteration's noise is drawn ahead by the update only while both
// noise buffers fit in half of the 256 MiB last-level cache: beyond, the
// second buffer's writes would evict the noise that the rollout has just read
// and the weighted sum reads next (measured: the 210 MB buffers of a
// K = 65536, T = 200, m = 4 problem lose more to HBM re-reads than the
// overlap gains).
constexpr size_t kDrawAheadMaxBytes = size_t(64) << 20;  // per buffer

bool draw_ahead_for(int TM, int64_t ldk, bool batch) {
  return !batch && sizeof(float) * static_cast<size_t>(TM) * static_cast<size_t>(ldk) <=
                       kDrawAheadMaxBytes;
}

Layout make_layout(const mppi_config* c, const mppi_params* p, int n, int m, bool batch) {
  (void)n;
  Layout L{};
  const int K = c->num_samples, T = c->horizon, TM = T * m;
  L.ldk = (K + kWave - 1) / kWave * kWave;
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes); return o; };
  L.eps = take(sizeof(float) * (size_t)TM * L.ldk);
  L.eps2 = draw_ahead_for(TM, L.ldk, batch) ? take(sizeof(float) * (size_t)TM * L.ldk) : L.eps;
  L.words = take(2 * sizeof(uint32_t));
  L.wpart = take(sizeof(float4) * ((K + kWChunk - 1) / kWChunk));
  L.e = take(sizeof(float) * L.ldk);
  L.ref = take(sizeof(float) * (size_t)(p->ref ? p->ref_len : 1));
  const int S = uses_spline(c->cost) ? p->num_segments : 0;
  const size_t cells =
      c->cost == MPPI_COST_PATH_COSTMAP ? (size_t)p->map_w * (size_t)p->map_h : 1;
  // room for the costmap's bitmap (staged when the map is two-valued and the
  // bitmap fits the LDS)
  const size_t map_bits = c->cost == MPPI_COST_PATH_COSTMAP && (cells + 7) / 8 <= kMaxRolloutLds
                              ? sizeof(float4) * ((cells + 127) / 128)
                              : 0;
  L.stage = take((uses_circles(c->cost) ? kMaxGridBytes : sizeof(float4)) +
                 sizeof(float4) * (S + (S + 1 + 3) / 4) + map_bits);
  L.costmap = take(sizeof(float) * cells);
  if (p->sigma_t) {
    L.sigma_t = take(sizeof(float) * ((TM + 3) / 4 * 4));  // read four at a time
    L.is_coef_t = take(sizeof(float) * TM);
  }
  const int H = mlp_hidden_of(c, p);
  L.mlp = take(sizeof(float) * kWave * (H ? pack_rows(H, false) : 1));
  L.mlp_bwd = take(sizeof(float) * kWave * (H ? pack_rows(H, true) : 1));
  L.mlp_bf = take(sizeof(uint4) * kWave * (H && bf16_of(c) ? bf_pack_rows(H) : 1));
  if (wants_grad(c)) {
    const int ce = ckpt_every_of(p);
    const int nseg = (T + ce - 1) / ce;
    L.ckpt = take(sizeof(float) * 7 * static_cast<size_t>(nseg) * L.ldk);
    L.u_roll = take(sizeof(float) * TM);
    L.adj_layout = adjoint_scratch_layout(K, adjoint_grad_len(c->dynamics, H), H, ce, TM);
    L.adj = take(L.adj_layout.total);
    const int tl = tape_len_of(p);
    L.tape_u = take(sizeof(float) * static_cast<size_t>(tl) * TM);
    L.tape_word = take(sizeof(uint32_t) * tl);
    L.tape_count = take(sizeof(int32_t));
    L.tape_G = take(sizeof(float) * TM);
    L.tape_state = take(sizeof(DevState));
  }
  if (split_form_for(c, p, batch)) {
    L.traj_words = split_traj_words(c->dynamics, c->cost);
    L.traj = take(sizeof(float) * static_cast<size_t>(T) * L.traj_words * L.ldk);
    L.split_part = take(2 * sizeof(float) * kSplitMaxChunks * static_cast<size_t>(L.ldk));
  }
  L.total = off;
  return L;
}

// Uniform grid over the circles for the rollout's crash test.  Each circle is
// listed in every cell that its bounding box, inflated by delta = 1e-3 cells,
// touches; the kernel computes a point's cell in binary32 with an error far
// below delta, so the list of the computed cell holds every circle that
// contains the point.  The cell size starts near two circle radii (about one
// listed circle per cell) and grows until the grid fits kMaxGridBytes of LDS.
struct Grid {
  std::vector<float4> words;  // offsets (uint32, padded to float4) then entries
  int nx = 1, ny = 1, off4 = 1;
  float x0 = 0.0f, y0 = 0.0f, inv_cell = 1.0f;
};

bool build_grid(const float* cx, const float* cy, const float* r2, int N, Grid* g) {
  g->words.assign(1, float4{0, 0, 0, 0});  // one empty cell: offsets {0, 0}
  g->nx = g->ny = 1;
  g->off4 = 1;
  if (N == 0) return true;
  double xmin = 1e300, xmax = -1e300, ymin = 1e300, ymax = -1e300, rmax = 0.0;
  std::vector<double> r(N);
  for (int i = 0; i < N; ++i) {
    r[i] = sqrt(fmax(static_cast<double>(r2[i]), 0.0));
    rmax = fmax(rmax, r[i]);
    xmin = fmin(xmin, cx[i] - r[i]); xmax = fmax(xmax, cx[i] + r[i]);
    ymin = fmin(ymin, cy[i] - r[i]); ymax = fmax(ymax, cy[i] + r[i]);
  }
  const double span = fmax(xmax - xmin, ymax - ymin);
  double cell = fmax(2.0 * rmax, sqrt((xmax - xmin) * (ymax - ymin) / (4.0 * N)));
  cell = fmax(cell, 1e-3 * (1.0 + fabs(xmin) + fabs(xmax) + fabs(ymin) + fabs(ymax)));
  cell = fmax(cell, span / 256.0);
  for (int attempt = 0; attempt < 64; ++attempt, cell *= 1.5) {
    const float inv = static_cast<float>(1.0 / cell);
    const double c = 1.0 / static_cast<double>(inv);  // the cell size the kernel sees
    const float fx0 = static_cast<float>(xmin - 0.5 * c), fy0 = static_cast<float>(ymin - 0.5 * c);
    const int nx = static_cast<int>(floor((xmax - fx0) / c)) + 2;
    const int ny = static_cast<int>(floor((ymax - fy0) / c)) + 2;
    if (nx > 256 || ny > 256) continue;
    const int ncell = nx * ny;
    const double delta = 1e-3 * c;
    auto span_of = [&](double lo, double hi, double o, int n, int* a, int* b) {
      *a = static_cast<int>(floor((lo - delta - o) / c));
      *b = static_cast<int>(floor((hi + delta - o) / c));
      *a = *a < 0 ? 0 : (*a > n - 1 ? n - 1 : *a);
      *b = *b < 0 ? 0 : (*b > n - 1 ? n - 1 : *b);
    };
    std::vector<uint32_t> count(ncell + 1, 0);
    for (int i = 0; i < N; ++i) {
      int ax, bx, ay, by;
      span_of(cx[i] - r[i], cx[i] + r[i], fx0, nx, &ax, &bx);
      span_of(cy[i] - r[i], cy[i] + r[i], fy0, ny, &ay, &by);
      for (int iy = ay; iy <= by; ++iy)
        for (int ix = ax; ix <= bx; ++ix) ++count[iy * nx + ix + 1];
    }
    for (int q = 0; q < ncell; ++q) count[q + 1] += count[q];
    const uint32_t nent = count[ncell];
    const int off4 = (ncell + 1 + 3) / 4;
    if (16.0 * (off4 + static_cast<double>(nent)) > kMaxGridBytes) continue;
    std::vector<float4> words(off4 + nent, float4{0, 0, 0, 0});
    uint32_t* off = reinterpret_cast<uint32_t*>(words.data());
    for (int q = 0; q <= ncell; ++q) off[q] = count[q];
    std::vector<uint32_t> fill(count.begin(), count.end() - 1);
    for (int i = 0; i < N; ++i) {
      int ax, bx, ay, by;
      span_of(cx[i] - r[i], cx[i] + r[i], fx0, nx, &ax, &bx);
      span_of(cy[i] - r[i], cy[i] + r[i], fy0, ny, &ay, &by);
      for (int iy = ay; iy <= by; ++iy)
        for (int ix = ax; ix <= bx; ++ix)
          words[off4 + fill[iy * nx + ix]++] = float4{cx[i], cy[i], r2[i], 0.0f};
    }
    g->words.swap(words);
    g->nx = nx; g->ny = ny; g->off4 = off4;
    g->x0 = fx0; g->y0 = fy0; g->inv_cell = inv;
    return true;
  }
  return false;
}


// One MPPI problem instance inside a context: its configuration, its slice
// of the workspace and the device-side constants its kernels take.
struct Instance {
  mppi_config cfg;
  int n, m, K, T, TM;
  Layout L;
  char* base;  // the instance's workspace slice
  DevParams dp;
  int lanes;   // lanes per sample of the single-instance rollout (1, 4, 8, 16)
  bool split;  // the split rollout form is available
  bool ahead_ok;  // a second noise buffer: updates draw the next iteration's noise
  bool grad;   // MPPI_F_REQUIRES_GRAD
  int tape_cap;  // gradient mode: tape slots
  int hidden, ckpt_every, n_theta;
  // views into the context's packed regions
  DevState* st;
  float* x0;
  float* u;
  float* S;
  int32_t* crashes;
  int64_t off_x0, off_u, off_S;
  int cur;  // the noise buffer of the current iteration (0: eps, 1: eps2)

  template <class X>
  X* at(size_t off) const { return reinterpret_cast<X*>(base + off); }
  float* eps() const { return at<float>(cur ? L.eps2 : L.eps); }
  float* eps_other() const { return at<float>(cur ? L.eps : L.eps2); }
  uint32_t* word(int buf) const { return at<uint32_t>(L.words) + buf; }
  float* e() const { return at<float>(L.e); }
};

// Context-level layout: packed per-instance regions first (so the packed host
// views of set_state / set_controls / get_controls / costs are single copies),
// then the batch tables, then the instance slices.
struct CtxLayout {
  size_t states, x0, u, S, crashes, insts, sample_tiles, row_tiles, one_items, done;
  size_t tile_part, tile_stat;  // the one-launch form's tile partials (packed)
  bool one_single;  // a single context with the one-launch form (its tiles of 16 samples)
  std::vector<size_t> slice;
  size_t total;
  int n_sample_tiles, n_row_tiles;
  int64_t n_one_items;  // tiles of kBatchMaxTile samples
  int64_t n_tile_part;  // floats of tile partial rows: sum_i ntile_i T_i m_i
};

// A single context whose iteration also runs as one time-parallel launch
// (launch_di_iteration).
bool one_single_for(const mppi_config* c) {
  return !wants_grad(c) && di_iteration_supported(c->dynamics, c->integrator, c->cost,
                                                  c->num_samples, c->horizon);
}

CtxLayout make_ctx_layout(const mppi_config* cfgs, const mppi_params* params, int n_inst,
                          bool batch) {
  CtxLayout C{};
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes); return o; };
  int64_t nx = 0, nu = 0, nS = 0;
  C.n_sample_tiles = C.n_row_tiles = 0;
  C.n_one_items = 0;
  C.n_tile_part = 0;
  for (int i = 0; i < n_inst; ++i) {
    int n, m;
    model_dims(cfgs[i].dynamics, &n, &m);
    nx += n;
    nu += (int64_t)cfgs[i].horizon * m;
    nS += cfgs[i].num_samples;
    const int TM = cfgs[i].horizon * m;
    C.n_sample_tiles += (cfgs[i].num_samples + kBatchMinTile - 1) / kBatchMinTile;
    C.n_row_tiles += (TM + gemv_rows_per_block() - 1) / gemv_rows_per_block();
    const int64_t ntile = (cfgs[i].num_samples + kBatchMaxTile - 1) / kBatchMaxTile;
    C.n_one_items += ntile;
    C.n_tile_part += ntile * TM;
  }
  C.states = take(sizeof(DevState) * n_inst);
  C.x0 = take(sizeof(float) * (nx + MPPI_MAX_STATE));
  C.u = take(sizeof(float) * nu);
  C.S = take(sizeof(float) * (nS + kWave));
  C.crashes = take(sizeof(int32_t) * (nS + kWave));
  C.one_single = !batch && one_single_for(&cfgs[0]);
  if (C.one_single) {
    const int64_t nt = di_iteration_tiles(cfgs[0].num_samples);
    C.done = take(sizeof(uint32_t));
    C.tile_part = take(sizeof(float) * nt * cfgs[0].horizon * 2);
    C.tile_stat = take(sizeof(float4) * nt);
  }
  if (batch) {
    C.insts = take(sizeof(BatchInst) * n_inst);
    C.sample_tiles = take(sizeof(int2) * C.n_sample_tiles);
    C.row_tiles = take(sizeof(int2) * C.n_row_tiles);
    C.one_items = take(sizeof(int2) * C.n_one_items);
    C.done = take(sizeof(uint32_t) * n_inst);
    C.tile_part = take(sizeof(float) * C.n_tile_part);
    C.tile_stat = take(sizeof(float4) * C.n_one_items);
  }
  C.slice.resize(n_inst);
  for (int i = 0; i < n_inst; ++i) {
    int n, m;
    model_dims(cfgs[i].dynamics, &n, &m);
    C.slice[i] = take(make_layout(&cfgs[i], &params[i], n, m, batch).total);
  }
  C.total = off;
  return C;
}

}  // namespace

struct mppi_ctx {
  std::vector<Instance> inst;
  bool batch = false;
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  CtxLayout C;
  BatchPlan plan{};
  int64_t n_x0 = 0, n_u = 0, n_S = 0;
  bool have_state = false;
  bool have_noise = false;
  bool have_costs = false;
  bool rollout_fresh = false;  // the costs are this iteration's rollout
  bool grad_ready = false;     // an update followed a fresh rollout
  bool tape_external = false;  // an update since the tape's reset used mppi_set_costs
  // single contexts: the last mppi_iterate's final update drew the noise of
  // the current iteration word into the other buffer, and nothing since has
  // changed the word or the buffers (the next mppi_iterate starts from it)
  bool ahead = false;
  // device whose static workspace this context holds (mppi_create_static),
  // else -1
  int static_device = -1;
  // mppi_iterate launch sequences, keyed by (iterations, first noise buffer,
  // whether its noise was drawn ahead)
  std::map<int64_t, hipGraphExec_t> graphs;
  mppi_tuning tune{};                     // launch shapes (lanes: instance 0's choice)
  ~mppi_ctx() { drop_graphs(); }
  void drop_graphs() {
    for (auto& g : graphs) (void)hipGraphExecDestroy(g.second);
    graphs.clear();
  }
  const Instance& one() const { return inst[0]; }
};

namespace {
// The tape starts over: the next update's u no longer depends on the
// parameters through earlier updates (new controls, state or parameters).
hipError_t tape_reset(mppi_ctx* c) {
  if (c->batch || !c->one().grad) return hipSuccess;
  c->tape_external = false;
  return launch_tape_reset(c->one().at<int32_t>(c->one().L.tape_count), c->stream);
}

// The single-pass update exists for single, non-gradient contexts with up to
// kOnePassMaxK samples, the chunked one for single, non-gradient contexts (the
// gradient mode's adjoint reads the weights the two-pass update stores).
bool chunked_for(const mppi_ctx* c) { return !c->batch && !c->one().grad; }
bool one_pass_for(const mppi_ctx* c) { return chunked_for(c) && c->one().K <= kOnePassMaxK; }

}  // namespace

namespace {

// Uploads one instance's parameter arrays into its slice and fills its
// device constants.  Enqueued on `stream`; the caller synchronises.
mppi_status setup_instance(const mppi_config* cfg, const mppi_params* p, bool batch, char* slice,
                           hipStream_t stream, Instance* I, std::vector<std::vector<float4>>* keep) {
  int n, m;
  mppi_status st = validate(cfg, p, &n, &m);
  if (st != MPPI_OK) return st;
  I->cfg = *cfg;
  I->n = n; I->m = m; I->K = cfg->num_samples; I->T = cfg->horizon; I->TM = I->T * m;
  I->L = make_layout(cfg, p, n, m, batch);
  I->base = slice;

  // the staged cost block: circle grid, then spline coefficient rows, then knots
  const int S = uses_spline(cfg->cost) ? p->num_segments : 0;
  const int N = uses_circles(cfg->cost) ? p->num_circles : 0;
  Grid grid;
  if (!build_grid(p->cx, p->cy, p->r2, N, &grid))
    return fail(MPPI_EUNSUPPORTED, "circle grid does not fit %d bytes of LDS", kMaxGridBytes);
  keep->emplace_back(grid.words);
  std::vector<float4>& stage = keep->back();
  const int spline_coef4 = static_cast<int>(stage.size());
  for (int s = 0; s < S; ++s)
    stage.push_back(float4{p->coef[4 * s], p->coef[4 * s + 1], p->coef[4 * s + 2], p->coef[4 * s + 3]});
  const int spline_knot4 = static_cast<int>(stage.size());
  if (S > 0) {
    std::vector<float> kn(((S + 1 + 3) / 4) * 4, 0.0f);
    memcpy(kn.data(), p->knots, sizeof(float) * (S + 1));
    for (size_t q = 0; q < kn.size(); q += 4)
      stage.push_back(float4{kn[q], kn[q + 1], kn[q + 2], kn[q + 3]});
  }
  // a costmap of at most two distinct values (compared bit for bit) is also
  // staged as a bitmap, when it fits beside the rest of the stage
  int map_bits4 = -1;
  float map_v[2] = {0.0f, 0.0f};
  if (cfg->cost == MPPI_COST_PATH_COSTMAP) {
    const int64_t cells = static_cast<int64_t>(p->map_w) * p->map_h;
    uint32_t vals[2];
    int nval = 0;
    for (int64_t q = 0; q < cells && nval <= 2; ++q) {
      uint32_t b;
      memcpy(&b, p->costmap + q, 4);
      if (nval > 0 && b == vals[0]) continue;
      if (nval > 1 && b == vals[1]) continue;
      if (nval < 2) vals[nval] = b;
      ++nval;
    }
    const size_t words4 = static_cast<size_t>((cells + 127) / 128);
    const size_t need = rollout_lds_bytes(cfg->dynamics, cfg->cost,
                                          static_cast<int>(stage.size() + words4), I->T);
    if (nval <= 2 && need <= kMaxRolloutLds) {
      memcpy(&map_v[0], &vals[0], 4);
      memcpy(&map_v[1], nval == 2 ? &vals[1] : &vals[0], 4);
      map_bits4 = static_cast<int>(stage.size());
      std::vector<uint32_t> bits(4 * words4, 0u);
      for (int64_t q = 0; q < cells; ++q) {
        uint32_t b;
        memcpy(&b, p->costmap + q, 4);
        if (nval == 2 && b == vals[1]) bits[q >> 5] |= 1u << (q & 31);
      }
      for (size_t w = 0; w < words4; ++w) {
        float4 f;
        memcpy(&f, bits.data() + 4 * w, 16);
        stage.push_back(f);
      }
    }
  }
  const size_t lds_need =
      rollout_lds_bytes(cfg->dynamics, cfg->cost, static_cast<int>(stage.size()), I->T);
  if (lds_need > kMaxRolloutLds)
    return fail(MPPI_EUNSUPPORTED, "cost data plus T*m controls exceed %zu bytes of LDS",
                kMaxRolloutLds);
  // the split form's cost kernel also holds 16 x 64 partial sums and counts
  I->split = I->L.traj_words > 0 && lds_need + 2 * 16 * 64 * 4 <= kMaxRolloutLds;
  I->ahead_ok = I->L.eps2 != I->L.eps;
  keep->emplace_back();
  std::vector<float4>& ref4 = keep->back();
  const int ref_len = p->ref ? p->ref_len : 1;
  ref4.resize((ref_len + 3) / 4, float4{0, 0, 0, 0});
  if (p->ref) memcpy(ref4.data(), p->ref, sizeof(float) * p->ref_len);

  auto up = [&](size_t off, const void* src, size_t bytes) -> hipError_t {
    return hipMemcpyAsync(slice + off, src, bytes, hipMemcpyHostToDevice, stream);
  };
  hipError_t e = up(I->L.ref, ref4.data(), sizeof(float) * ref_len);
  if (e == hipSuccess) e = up(I->L.stage, stage.data(), sizeof(float4) * stage.size());
  if (e == hipSuccess && cfg->cost == MPPI_COST_PATH_COSTMAP)
    e = up(I->L.costmap, p->costmap, sizeof(float) * (size_t)p->map_w * p->map_h);
  if (e == hipSuccess && p->sigma_t) {
    keep->emplace_back();
    // sigma_t padded with zeros to a multiple of four, then lambda / sigma_t^2
    std::vector<float4>& tab = keep->back();
    const int TM = I->TM, TM4 = (TM + 3) / 4 * 4;
    tab.assign((static_cast<size_t>(TM4) + TM + 3) / 4, float4{0, 0, 0, 0});
    float* f = reinterpret_cast<float*>(tab.data());
    for (int i = 0; i < TM; ++i) {
      const double sg = p->sigma_t[i];
      f[i] = p->sigma_t[i];
      f[TM4 + i] = (cfg->flags & MPPI_F_IMPORTANCE_SAMPLING)
                       ? static_cast<float>(static_cast<double>(cfg->lambda) / (sg * sg))
                       : 0.0f;
    }
    e = up(I->L.sigma_t, f, sizeof(float) * TM4);
    if (e == hipSuccess) e = up(I->L.is_coef_t, f + TM4, sizeof(float) * TM);
  }
  I->hidden = mlp_hidden_of(cfg, p);
  I->grad = wants_grad(cfg);
  I->tape_cap = I->grad ? tape_len_of(p) : 0;
  I->ckpt_every = ckpt_every_of(p);
  I->n_theta = adjoint_grad_len(cfg->dynamics, I->hidden);
  if (e == hipSuccess && I->hidden) {
    keep->emplace_back();
    std::vector<float4>& fwd = keep->back();
    keep->emplace_back();
    std::vector<float4>& bwd = keep->back();
    std::vector<uint4> bfp;
    build_mlp_packs(p->mlp, I->hidden, &fwd, &bwd, bf16_of(cfg) ? &bfp : nullptr);
    e = up(I->L.mlp, fwd.data(), sizeof(float4) * fwd.size());
    if (e == hipSuccess) e = up(I->L.mlp_bwd, bwd.data(), sizeof(float4) * bwd.size());
    if (e == hipSuccess && !bfp.empty()) {
      // staged through the kept buffers so the asynchronous copy's source lives on
      keep->emplace_back(bfp.size());
      memcpy(keep->back().data(), bfp.data(), sizeof(uint4) * bfp.size());
      e = up(I->L.mlp_bf, keep->back().data(), sizeof(uint4) * bfp.size());
    }
  }
  if (e != hipSuccess) return hip_fail(e, "parameter upload");

  // rollout variant: four lanes per sample while one lane per sample would
  // leave most SIMDs idle
  I->lanes = rollout_quad_available(cfg->dynamics, cfg->integrator) &&
                     !(cfg->flags & MPPI_F_ROLLOUT_LANE) &&
                     ((cfg->flags & MPPI_F_ROLLOUT_QUAD) || I->K <= 32768)
                 ? 4 : 1;

  DevParams& d = I->dp;
  memset(&d, 0, sizeof d);
  d.dt = cfg->dt;
  d.half_dt = 0.5f * cfg->dt;
  d.sixth_dt = static_cast<float>(static_cast<double>(cfg->dt) / 6.0);
  d.inv_wheelbase = p->wheelbase > 0.0f ? static_cast<float>(1.0 / p->wheelbase) : 0.0f;
  d.inv_mass = p->mass > 0.0f ? static_cast<float>(1.0 / p->mass) : 0.0f;
  d.gravity = p->gravity;
  for (int i = 0; i < 3; ++i) {
    d.inertia[i] = p->inertia[i];
    d.inv_inertia[i] = p->inertia[i] > 0.0f ? static_cast<float>(1.0 / p->inertia[i]) : 0.0f;
  }
  memcpy(d.w, p->w, sizeof d.w);
  d.ref = I->at<float>(I->L.ref);
  d.mlp_hidden = I->hidden;
  d.mlp = I->hidden ? I->at<float>(I->L.mlp) : nullptr;
  d.mlp_bwd = I->hidden ? I->at<float>(I->L.mlp_bwd) : nullptr;
  d.mlp_bf = I->hidden && bf16_of(cfg) ? I->at<uint4>(I->L.mlp_bf) : nullptr;
  d.cosines = p->cost_cosines;
  d.n_plain = n_plain_of(cfg);
  d.mean_sample = (cfg->flags & MPPI_F_MEAN_SAMPLE) ? 1 : 0;
  d.sigma_t = p->sigma_t ? I->at<float>(I->L.sigma_t) : nullptr;
  d.is_coef_t =
      p->sigma_t && (cfg->flags & MPPI_F_IMPORTANCE_SAMPLING) ? I->at<float>(I->L.is_coef_t) : nullptr;
  d.importance = (cfg->flags & MPPI_F_IMPORTANCE_SAMPLING) ? 1 : 0;
  for (int j = 0; j < m && d.importance; ++j) {
    const double sg = cfg->sigma[j];
    d.is_coef[j] = static_cast<float>(static_cast<double>(cfg->lambda) / (sg * sg));
  }
  d.nseg = S;
  d.ncirc = N;
  d.stage = I->at<float4>(I->L.stage);
  d.stage_words4 = static_cast<int>(stage.size());
  d.spline_coef4 = spline_coef4;
  d.spline_knot4 = spline_knot4;
  d.grid_nx = grid.nx;
  d.grid_ny = grid.ny;
  d.grid_off4 = grid.off4;
  d.grid_x0 = grid.x0;
  d.grid_y0 = grid.y0;
  d.grid_inv_cell = grid.inv_cell;
  if (cfg->cost == MPPI_COST_PATH_COSTMAP) {
    d.map_w = p->map_w;
    d.map_h = p->map_h;
    d.map_x0 = p->map_x0;
    d.map_y0 = p->map_y0;
    d.map_res = p->map_res;
    d.map_inv_res = static_cast<float>(1.0 / static_cast<double>(p->map_res));
    d.costmap = I->at<float>(I->L.costmap);
  }
  d.map_bits4 = map_bits4;
  d.map_v0 = map_v[0];
  d.map_v1 = map_v[1];
  return MPPI_OK;
}

// The sample tiles of a batch, `tile` samples each, longest horizon first
// (stable: instance order within a horizon).  Checked against the instances'
// sample counts and the table's capacity before the upload (the launch grid
// is the checked length); uploads and waits.
mppi_status upload_sample_tiles(mppi_ctx* c, int tile) {
  const int n_inst = static_cast<int>(c->inst.size());
  if (tile < kBatchMinTile || tile > kBatchMaxTile || tile % kBatchMinTile)
    return fail(MPPI_EINVAL, "batch tile %d outside %d..%d", tile, kBatchMinTile, kBatchMaxTile);
  std::vector<int32_t> K(n_inst), T(n_inst);
  for (int i = 0; i < n_inst; ++i) { K[i] = c->inst[i].K; T[i] = c->inst[i].T; }
  const std::vector<WorkItem> tiles = build_sample_tiles(K.data(), T.data(), n_inst, tile);
  const std::string bad = check_work_list(tiles.data(), static_cast<int64_t>(tiles.size()),
                                          c->C.n_sample_tiles, tile, K.data(), n_inst);
  if (!bad.empty()) return fail(MPPI_EINVAL, "sample work list: %s", bad.c_str());
  hipError_t e = hipMemcpyAsync(c->ws + c->C.sample_tiles, tiles.data(),
                                sizeof(WorkItem) * tiles.size(), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(e, "sample work list upload");
  c->plan.n_sample_tiles = static_cast<int>(tiles.size());
  c->plan.tile = tile;
  return MPPI_OK;
}

mppi_status create_ctx(const mppi_config* cfgs, const mppi_params* params, int n_inst, bool batch,
                       void* d_workspace, size_t workspace_bytes, void* hip_stream,
                       mppi_ctx** out) {
  if (!out) return fail(MPPI_EINVAL, "out must not be NULL");
  *out = nullptr;
  if (!cfgs || !params || n_inst < 1 || n_inst > 65536)
    return fail(MPPI_EINVAL, "need 1..65536 configurations and parameter sets");
  for (int i = 0; i < n_inst; ++i) {
    int n, m;
    mppi_status s = validate(&cfgs[i], &params[i], &n, &m);
    if (s != MPPI_OK) return s;
    if (batch && (cfgs[i].dynamics == MPPI_DYN_BICYCLE_MLP || wants_grad(&cfgs[i])))
      return fail(MPPI_EUNSUPPORTED, "batch contexts run neither MLP dynamics nor "
                  "MPPI_F_REQUIRES_GRAD");
    if (batch && (cfgs[i].dynamics != cfgs[0].dynamics || cfgs[i].integrator != cfgs[0].integrator ||
                  cfgs[i].cost != cfgs[0].cost || cfgs[i].flags != cfgs[0].flags))
      return fail(MPPI_EINVAL, "batch instance %d differs from instance 0 in dynamics, "
                  "integrator, cost or flags", i);
  }
  const CtxLayout C = make_ctx_layout(cfgs, params, n_inst, batch);
  if (!d_workspace) return fail(MPPI_EINVAL, "workspace must not be NULL");
  if (reinterpret_cast<uintptr_t>(d_workspace) % kAlign)
    return fail(MPPI_EINVAL, "workspace must be %zu-byte aligned", kAlign);
  if (workspace_bytes < C.total)
    return fail(MPPI_ENOMEM, "workspace of %zu bytes, need %zu", workspace_bytes, C.total);

  mppi_ctx* c = new mppi_ctx();
  c->batch = batch;
  c->ws = static_cast<char*>(d_workspace);
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->C = C;
  c->inst.resize(n_inst);
  std::vector<std::vector<float4>> keep;
  keep.reserve(8 * n_inst);
  std::vector<DevState> states(n_inst);
  int64_t ox = 0, ou = 0, oS = 0;
  for (int i = 0; i < n_inst; ++i) {
    Instance& I = c->inst[i];
    mppi_status s =
        setup_instance(&cfgs[i], &params[i], batch, c->ws + C.slice[i], c->stream, &I, &keep);
    if (s != MPPI_OK) { (void)hipStreamSynchronize(c->stream); delete c; return s; }
    I.st = reinterpret_cast<DevState*>(c->ws + C.states) + i;
    I.x0 = reinterpret_cast<float*>(c->ws + C.x0) + ox;
    I.u = reinterpret_cast<float*>(c->ws + C.u) + ou;
    I.S = reinterpret_cast<float*>(c->ws + C.S) + oS;
    I.crashes = reinterpret_cast<int32_t*>(c->ws + C.crashes) + oS;
    I.off_x0 = ox; I.off_u = ou; I.off_S = oS;
    I.cur = 0;
    ox += I.n; ou += I.TM; oS += I.K;
    states[i] = DevState{};
    states[i].status = MPPI_OK;
  }
  c->n_x0 = ox; c->n_u = ou; c->n_S = oS;
  hipError_t e = hipMemcpyAsync(c->ws + C.states, states.data(), sizeof(DevState) * n_inst,
                                hipMemcpyHostToDevice, c->stream);
  std::vector<float> zeros(ou, 0.0f);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->ws + C.u, zeros.data(), sizeof(float) * ou, hipMemcpyHostToDevice, c->stream);

  // batch tables
  std::vector<BatchInst> bi;
  std::vector<WorkItem> row_tiles, one_items;
  if (batch && e == hipSuccess) {
    size_t lds = 0;
    int64_t part_off = 0, stat_off = 0;
    bool one_ok = true;  // every instance within the one-launch form's tile limit
    for (int i = 0; i < n_inst; ++i) {
      const Instance& I = c->inst[i];
      BatchInst b{};
      b.p = I.dp;
      b.x0 = I.x0; b.u = I.u; b.eps = I.eps(); b.S = I.S;
      b.crashes = (cfgs[i].flags & MPPI_F_DEBUG) && uses_circles(cfgs[i].cost) ? I.crashes : nullptr;
      b.ldk = I.L.ldk; b.K = I.K; b.T = I.T; b.TM = I.TM;
      b.lambda = cfgs[i].lambda;
      b.inv_lambda = static_cast<float>(1.0 / static_cast<double>(cfgs[i].lambda));
      b.step = step_size(cfgs[i]);
      b.key0 = static_cast<uint32_t>(cfgs[i].seed);
      b.key1 = static_cast<uint32_t>(cfgs[i].seed >> 32);
      b.instance = cfgs[i].instance;
      for (int j = 0; j < I.m; ++j) b.sigma.v[j] = cfgs[i].sigma[j];
      b.e = I.e();
      b.st = I.st;
      b.tile_part = reinterpret_cast<float*>(c->ws + C.tile_part) + part_off;
      b.tile_stat = reinterpret_cast<float4*>(c->ws + C.tile_stat) + stat_off;
      const int64_t ntile_i = (I.K + kBatchMaxTile - 1) / kBatchMaxTile;
      part_off += ntile_i * I.TM;
      stat_off += ntile_i;
      one_ok = one_ok && ntile_i <= kOneLaunchMaxTiles;
      bi.push_back(b);
      lds = std::max(lds, rollout_lds_bytes(cfgs[i].dynamics, cfgs[i].cost, I.dp.stage_words4, I.T));
    }
    const int rpb = gemv_rows_per_block();
    std::vector<int32_t> TM(n_inst);
    for (int i = 0; i < n_inst; ++i) TM[i] = c->inst[i].TM;
    row_tiles = build_row_tiles(TM.data(), n_inst, rpb);
    const std::string bad = check_work_list(row_tiles.data(),
                                            static_cast<int64_t>(row_tiles.size()),
                                            C.n_row_tiles, rpb, TM.data(), n_inst);
    if (!bad.empty()) {
      (void)hipStreamSynchronize(c->stream);
      delete c;
      return fail(MPPI_EINVAL, "row work list: %s", bad.c_str());
    }
    e = hipMemcpyAsync(c->ws + C.insts, bi.data(), sizeof(BatchInst) * n_inst,
                       hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(c->ws + C.row_tiles, row_tiles.data(),
                         sizeof(WorkItem) * row_tiles.size(), hipMemcpyHostToDevice, c->stream);
    BatchPlan& P = c->plan;
    P.insts = reinterpret_cast<const BatchInst*>(c->ws + C.insts);
    P.sample_tiles = reinterpret_cast<const int2*>(c->ws + C.sample_tiles);
    P.row_tiles = reinterpret_cast<const int2*>(c->ws + C.row_tiles);
    P.n_row_tiles = static_cast<int>(row_tiles.size());
    P.n_inst = n_inst;
    P.rollout_lds = lds;
    size_t tm = 0;
    for (int i = 0; i < n_inst; ++i) tm = std::max(tm, sizeof(float) * c->inst[i].TM);
    P.max_tm_bytes = tm;
    // the one-launch form: its tiles (longest horizon first, checked) and
    // zeroed per-instance tile counters, where the combination has a kernel
    // and every instance at most kOneLaunchMaxTiles tiles
    P.fused_items = reinterpret_cast<const int2*>(c->ws + C.one_items);
    P.n_fused_items = 0;
    P.done = reinterpret_cast<uint32_t*>(c->ws + C.done);
    if (e == hipSuccess) e = hipMemsetAsync(P.done, 0, sizeof(uint32_t) * n_inst, c->stream);
    if (one_ok && batch_one_launch_supported(cfgs[0].dynamics, cfgs[0].integrator, cfgs[0].cost) &&
        e == hipSuccess) {
      std::vector<int32_t> Kv(n_inst), Tv(n_inst);
      for (int i = 0; i < n_inst; ++i) { Kv[i] = c->inst[i].K; Tv[i] = c->inst[i].T; }
      one_items = build_sample_tiles(Kv.data(), Tv.data(), n_inst, kBatchMaxTile);
      const std::string bad2 = check_work_list(one_items.data(),
                                               static_cast<int64_t>(one_items.size()),
                                               C.n_one_items, kBatchMaxTile, Kv.data(), n_inst);
      if (!bad2.empty()) {
        (void)hipStreamSynchronize(c->stream);
        delete c;
        return fail(MPPI_EINVAL, "one-launch work list: %s", bad2.c_str());
      }
      e = hipMemcpyAsync(c->ws + C.one_items, one_items.data(),
                         sizeof(WorkItem) * one_items.size(), hipMemcpyHostToDevice, c->stream);
      P.n_fused_items = static_cast<int>(one_items.size());
    }
  }
  // a single context's one-launch form: its zeroed tile counter
  if (C.one_single && e == hipSuccess)
    e = hipMemsetAsync(c->ws + C.done, 0, sizeof(uint32_t), c->stream);
  const hipError_t e2 = hipStreamSynchronize(c->stream);  // host staging buffers die here
  if (e == hipSuccess) e = e2;
  // default launch shapes: four lanes per sample where one lane per sample
  // would leave most SIMDs idle
  const Instance& I0 = c->inst[0];
  const bool tiles = I0.hidden || I0.grad;
  c->tune.lanes_per_sample = tiles ? 16 : (batch ? 1 : I0.lanes);
  // MLP dynamics: the tile's MLP split over H/16 waves where that form exists
  c->tune.rollout_block = I0.hidden >= 32 ? 4 * I0.hidden : 64;
  c->tune.batch_tile = kBatchMaxTile;
  c->tune.noise_calls = 1;
  c->tune.rollout_form = MPPI_ROLLOUT_FUSED;
  c->tune.cost_waves = 8;
  c->tune.batch_form = MPPI_BATCH_PHASES;
  c->tune.adjoint_tiles = kAdjointTilesDefault;
  c->tune.update_form = one_pass_for(c)  ? MPPI_UPDATE_ONE_PASS
                        : chunked_for(c) ? MPPI_UPDATE_CHUNKED
                                         : MPPI_UPDATE_TWO_PASS;
  if (e == hipSuccess) e = tape_reset(c);
  if (e != hipSuccess) { delete c; return hip_fail(e, "context upload"); }
  if (batch) {
    const mppi_status st = upload_sample_tiles(c, c->tune.batch_tile);
    if (st != MPPI_OK) { delete c; return st; }
  }
  *out = c;
  g_last_error.clear();
  return MPPI_OK;
}

// ---- the phases of one iteration on a context -------------------------------
hipError_t phase_sample(mppi_ctx* c) {
  if (c->batch) return launch_batch_noise(c->plan, c->stream);
  const Instance& I = c->one();
  return launch_noise(I.cfg.seed, &I.st->iteration, 0u, I.cfg.instance, I.K, I.T, I.m,
                      I.cfg.sigma, I.eps(), I.L.ldk, c->stream, c->tune.noise_calls, I.dp.sigma_t,
                      I.dp.mean_sample != 0, I.word(I.cur));
}

// The next iteration's noise, into the buffer after the current one.
NoiseJob next_noise_job(const mppi_ctx* c) {
  const Instance& I = c->one();
  NoiseJob job{};
  job.key0 = static_cast<uint32_t>(I.cfg.seed);
  job.key1 = static_cast<uint32_t>(I.cfg.seed >> 32);
  job.instance = I.cfg.instance;
  job.word_in = I.word(I.cur);
  job.word_out = I.word(I.cur ^ 1);
  job.K = I.K;
  job.T = I.T;
  job.TM = I.TM;
  for (int j = 0; j < I.m; ++j) job.sigma.v[j] = I.cfg.sigma[j];
  job.eps = I.eps_other();
  job.ldk = I.L.ldk;
  job.sigma_t = I.dp.sigma_t;
  job.mean_sample = I.dp.mean_sample != 0;
  job.calls = c->tune.noise_calls;
  return job;
}

// The rollout launch that can also draw the next iteration's noise: the
// fused kernels of a single context (not the MLP tiles or the split form).
bool rollout_draws_noise(const mppi_ctx* c) {
  const Instance& I = c->one();
  return !c->batch && !(I.hidden || I.grad) && c->tune.rollout_form != MPPI_ROLLOUT_SPLIT;
}

// next: also draw the next iteration's noise (rollout_draws_noise only).
hipError_t phase_rollout(mppi_ctx* c, bool next = false) {
  const Instance& I = c->one();
  const bool count = (I.cfg.flags & MPPI_F_DEBUG) && uses_circles(I.cfg.cost);
  const bool accurate = (I.cfg.flags & MPPI_F_ACCURATE_TRIG) != 0;
  if (c->batch)
    return launch_batch_rollout(I.cfg.dynamics, I.cfg.integrator, I.cfg.cost, accurate, count,
                                c->plan, c->stream);
  if (I.hidden || I.grad) {
    float* ckpt = I.grad ? I.at<float>(I.L.ckpt) : nullptr;
    if (I.grad) {
      hipError_t e = hipMemcpyAsync(I.at<float>(I.L.u_roll), I.u, sizeof(float) * I.TM,
                                    hipMemcpyDeviceToDevice, c->stream);
      if (e != hipSuccess) return e;
    }
    return launch_rollout_tiles(I.cfg.dynamics, I.cfg.integrator, I.cfg.cost, accurate, I.dp, I.x0,
                                I.u, I.eps(), I.L.ldk, I.K, I.T, I.S, ckpt, I.ckpt_every,
                                c->stream, c->tune.rollout_block / kWave);
  }
  if (c->tune.rollout_form == MPPI_ROLLOUT_SPLIT)
    return launch_rollout_split(I.cfg.dynamics, I.cfg.integrator, I.cfg.cost, accurate, I.lanes,
                                I.dp, I.x0, I.u, I.eps(), I.L.ldk, I.K, I.T, I.at<float>(I.L.traj),
                                I.at<float>(I.L.split_part), I.S, count ? I.crashes : nullptr,
                                c->stream,
                                c->tune.rollout_block, c->tune.cost_waves);
  NoiseJob job{};
  if (next) job = next_noise_job(c);
  if (c->tune.rollout_form == MPPI_ROLLOUT_SCAN)
    return launch_rollout_scan(I.cfg.dynamics, I.cfg.integrator, I.cfg.cost, accurate, I.dp, I.x0,
                               I.u, I.eps(), I.L.ldk, I.K, I.T, I.S, count ? I.crashes : nullptr,
                               c->stream, c->tune.rollout_block, next ? &job : nullptr,
                               c->tune.lanes_per_sample);
  return launch_rollout(I.cfg.dynamics, I.cfg.integrator, I.cfg.cost, accurate, I.lanes, I.dp, I.x0,
                        I.u, I.eps(), I.L.ldk, I.K, I.T, I.S, count ? I.crashes : nullptr,
                        c->stream, c->tune.rollout_block, next ? &job : nullptr);
}

// next: the weights launch also draws the next iteration's noise into the
// other buffer (the caller then switches buffers).
hipError_t phase_update(mppi_ctx* c, bool next = false) {
  if (c->batch) return launch_batch_update(c->plan, c->stream);
  const Instance& I = c->one();
  TapeRef tape;
  if (I.grad) {
    tape.u = I.u;
    tape.TM = I.TM;
    tape.tape_u = I.at<float>(I.L.tape_u);
    tape.tape_word = I.at<uint32_t>(I.L.tape_word);
    tape.count = I.at<int32_t>(I.L.tape_count);
    tape.cap = I.tape_cap;
  }
  NoiseJob job{};
  if (next) job = next_noise_job(c);
  if (c->tune.update_form == MPPI_UPDATE_ONE_PASS)
    return launch_update_one_pass(I.S, I.eps(), I.L.ldk, I.K, I.TM, I.cfg.lambda,
                                  step_size(I.cfg), I.u, I.st, c->stream, I.dp.n_plain,
                                  next ? &job : nullptr);
  if (c->tune.update_form == MPPI_UPDATE_CHUNKED)
    return launch_update_chunked(I.S, I.eps(), I.L.ldk, I.K, I.TM, I.cfg.lambda,
                                 step_size(I.cfg), I.e(), I.at<float4>(I.L.wpart), I.u, I.st,
                                 c->stream, I.dp.n_plain, next ? &job : nullptr);
  return launch_softmin_update(I.S, I.eps(), I.L.ldk, I.K, I.TM, I.cfg.lambda, step_size(I.cfg),
                               I.e(), I.u, I.st, c->stream, I.dp.n_plain, tape,
                               next ? &job : nullptr);
}

// The one-launch form of a single context: its descriptor (the batch's
// instance descriptor, with tiles of 16 samples).
BatchInst single_inst(const mppi_ctx* c) {
  const Instance& I = c->one();
  BatchInst b{};
  b.p = I.dp;
  b.x0 = I.x0; b.u = I.u; b.eps = I.eps(); b.S = I.S;
  b.crashes = nullptr;
  b.ldk = I.L.ldk; b.K = I.K; b.T = I.T; b.TM = I.TM;
  b.lambda = I.cfg.lambda;
  b.inv_lambda = static_cast<float>(1.0 / static_cast<double>(I.cfg.lambda));
  b.step = step_size(I.cfg);
  b.key0 = static_cast<uint32_t>(I.cfg.seed);
  b.key1 = static_cast<uint32_t>(I.cfg.seed >> 32);
  b.instance = I.cfg.instance;
  for (int j = 0; j < I.m; ++j) b.sigma.v[j] = I.cfg.sigma[j];
  b.e = I.e();
  b.st = I.st;
  b.tile_part = reinterpret_cast<float*>(c->ws + c->C.tile_part);
  b.tile_stat = reinterpret_cast<float4*>(c->ws + c->C.tile_stat);
  return b;
}

bool one_launch_single(const mppi_ctx* c) {
  return !c->batch && c->tune.batch_form == MPPI_BATCH_ONE_LAUNCH;
}

// Iteration i of mppi_iterate.  A single context with two noise buffers
// draws the noise of the first iteration only, and not even that when it was
// drawn ahead; every update draws the next iteration's noise into the other
// buffer (after the last one, the noise of the next call's first iteration)
// and switches buffers.  Other contexts sample in every iteration.
hipError_t phase_iteration(mppi_ctx* c, int i, bool ahead) {
  hipError_t e = hipSuccess;
  if (one_launch_single(c))
    return launch_di_iteration(single_inst(c), reinterpret_cast<uint32_t*>(c->ws + c->C.done),
                               c->stream);
  if (c->batch && c->tune.batch_form == MPPI_BATCH_ONE_LAUNCH) {
    const Instance& I = c->one();
    const bool count = (I.cfg.flags & MPPI_F_DEBUG) && uses_circles(I.cfg.cost);
    const bool accurate = (I.cfg.flags & MPPI_F_ACCURATE_TRIG) != 0;
    return launch_batch_one_launch(I.cfg.dynamics, I.cfg.integrator, I.cfg.cost, accurate, count,
                                   c->plan, c->stream);
  }
  if (c->batch || !c->one().ahead_ok) {
    e = phase_sample(c);
    if (e == hipSuccess) e = phase_rollout(c);
    return e == hipSuccess ? phase_update(c) : e;
  }
  if (i == 0 && !ahead) e = phase_sample(c);
  // the next noise in the rollout's launch where it can go there (its
  // workgroups fill the issue slots the latency-bound rollout leaves), else
  // in the update's
  const bool in_rollout = rollout_draws_noise(c);
  if (e == hipSuccess) e = phase_rollout(c, in_rollout);
  if (e == hipSuccess) e = phase_update(c, !in_rollout);
  c->inst[0].cur ^= 1;
  return e;
}

}  // namespace

extern "C" {

const char* mppi_last_error(void) { return g_last_error.c_str(); }

size_t mppi_workspace_bytes(const mppi_config* cfg, const mppi_params* params) {
  int n, m;
  if (validate(cfg, params, &n, &m) != MPPI_OK) return 0;
  return make_ctx_layout(cfg, params, 1, false).total;
}

size_t mppi_batch_workspace_bytes(const mppi_config* cfgs, const mppi_params* params, int32_t n) {
  if (!cfgs || !params || n < 1 || n > 65536) {
    fail(MPPI_EINVAL, "need 1..65536 configurations and parameter sets");
    return 0;
  }
  for (int i = 0; i < n; ++i) {
    int ns, ms;
    if (validate(&cfgs[i], &params[i], &ns, &ms) != MPPI_OK) return 0;
  }
  return make_ctx_layout(cfgs, params, n, true).total;
}

mppi_status mppi_create(const mppi_config* cfg, const mppi_params* p, void* d_workspace,
                        size_t workspace_bytes, void* hip_stream, mppi_ctx** out) {
  return create_ctx(cfg, p, 1, false, d_workspace, workspace_bytes, hip_stream, out);
}

mppi_status mppi_create_batch(const mppi_config* cfgs, const mppi_params* params, int32_t n,
                              void* d_workspace, size_t workspace_bytes, void* hip_stream,
                              mppi_ctx** out) {
  return create_ctx(cfgs, params, n, true, d_workspace, workspace_bytes, hip_stream, out);
}

mppi_status mppi_create_static(const mppi_config* cfg, const mppi_params* p, void* hip_stream,
                               mppi_ctx** out) {
  if (!out) return fail(MPPI_EINVAL, "out must not be NULL");
  *out = nullptr;
  const size_t need = mppi_workspace_bytes(cfg, p);
  if (need == 0) return MPPI_EINVAL;  // message set by the size query
  if (need > kStaticWorkspaceBytes)
    return fail(MPPI_ENOMEM, "this configuration needs a workspace of %zu bytes; the static "
                "workspace holds %zu (use mppi_create with a workspace of your own)",
                need, kStaticWorkspaceBytes);
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "current device");
  if (dev < 0 || dev >= kMaxStaticDevices)
    return fail(MPPI_EUNSUPPORTED, "device %d: static workspaces exist for devices 0..%d", dev,
                kMaxStaticDevices - 1);
  if (hip_stream) {
    int sdev = -1;
    e = hipStreamGetDevice(static_cast<hipStream_t>(hip_stream), &sdev);
    if (e != hipSuccess) return hip_fail(e, "stream device");
    if (sdev != dev)
      return fail(MPPI_EINVAL, "the stream belongs to device %d but device %d is current", sdev,
                  dev);
  }
  char* ws = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_static_mu);
    StaticWorkspace& W = g_static[dev];
    if (W.busy)
      return fail(MPPI_ESTATE, "device %d's static workspace belongs to a live context; "
                  "destroy that context first", dev);
    if (!W.ptr) {
      // the array's device address on the current device (each GPU holds its
      // own copy); taken once per device and kept
      void* ptr = nullptr;
      e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
      if (e != hipSuccess) return hip_fail(e, "static workspace address");
      if (!ptr || reinterpret_cast<uintptr_t>(ptr) % kAlign)
        return fail(MPPI_EDEVICE, "static workspace at %p is not %zu-byte aligned", ptr, kAlign);
      W.ptr = static_cast<char*>(ptr);
    }
    W.busy = true;
    ws = W.ptr;
  }
  const mppi_status st = create_ctx(cfg, p, 1, false, ws, kStaticWorkspaceBytes, hip_stream, out);
  if (st != MPPI_OK) {
    std::lock_guard<std::mutex> lock(g_static_mu);
    g_static[dev].busy = false;
    return st;
  }
  (*out)->static_device = dev;
  return MPPI_OK;
}

void mppi_destroy(mppi_ctx* ctx) {
  if (!ctx) return;
  const int dev = ctx->static_device;
  if (dev >= 0) {
    // the next static context reuses the array: the work enqueued on it ends first
    (void)hipStreamSynchronize(ctx->stream);
    delete ctx;
    std::lock_guard<std::mutex> lock(g_static_mu);
    g_static[dev].busy = false;
    return;
  }
  delete ctx;
}

int32_t mppi_num_instances(const mppi_ctx* c) { return c ? static_cast<int32_t>(c->inst.size()) : 0; }

mppi_status mppi_offsets(const mppi_ctx* c, int32_t what, int64_t* host_offsets) {
  if (!c || !host_offsets) return fail(MPPI_EINVAL, "ctx and host_offsets must not be NULL");
  int64_t acc = 0;
  for (size_t i = 0; i < c->inst.size(); ++i) {
    const Instance& I = c->inst[i];
    host_offsets[i] = acc;
    switch (what) {
      case MPPI_PACKED_STATE: acc += I.n; break;
      case MPPI_PACKED_CONTROLS: acc += I.TM; break;
      case MPPI_PACKED_SAMPLES: acc += I.K; break;
      case MPPI_PACKED_NOISE: acc += static_cast<int64_t>(I.TM) * I.K; break;
      default: return fail(MPPI_EINVAL, "unknown packed array %d", what);
    }
  }
  host_offsets[c->inst.size()] = acc;
  return MPPI_OK;
}

mppi_status mppi_get_tuning(const mppi_ctx* c, mppi_tuning* out) {
  if (!c || !out) return fail(MPPI_EINVAL, "ctx and out must not be NULL");
  *out = c->tune;
  return MPPI_OK;
}

mppi_status mppi_set_tuning(mppi_ctx* c, const mppi_tuning* t) {
  if (!c || !t) return fail(MPPI_EINVAL, "ctx and t must not be NULL");
  c->ahead = false;  // the word or a noise buffer may change
  auto shape = [](int v) { return v == 64 || v == 128 || v == 256; };
  if (!shape(t->rollout_block) || !shape(t->batch_tile))
    return fail(MPPI_EINVAL, "rollout_block and batch_tile must be 64, 128 or 256");
  if (t->noise_calls != 1 && t->noise_calls != 2 && t->noise_calls != 4)
    return fail(MPPI_EINVAL, "noise_calls must be 1, 2 or 4");
  const int cw = t->cost_waves;
  if (cw < 1 || cw > kSplitMaxWaves * kSplitMaxChunks || (cw & (cw - 1)))
    return fail(MPPI_EINVAL, "cost_waves must be a power of two from 1 to %d",
                kSplitMaxWaves * kSplitMaxChunks);
  if (t->rollout_form != MPPI_ROLLOUT_FUSED && t->rollout_form != MPPI_ROLLOUT_SPLIT &&
      t->rollout_form != MPPI_ROLLOUT_SCAN)
    return fail(MPPI_EINVAL, "rollout_form must be MPPI_ROLLOUT_FUSED, MPPI_ROLLOUT_SPLIT or "
                "MPPI_ROLLOUT_SCAN");
  if (t->update_form != MPPI_UPDATE_TWO_PASS && t->update_form != MPPI_UPDATE_ONE_PASS &&
      t->update_form != MPPI_UPDATE_CHUNKED)
    return fail(MPPI_EINVAL, "update_form must be MPPI_UPDATE_TWO_PASS, MPPI_UPDATE_ONE_PASS "
                "or MPPI_UPDATE_CHUNKED");
  if (t->batch_form != MPPI_BATCH_PHASES && t->batch_form != MPPI_BATCH_ONE_LAUNCH)
    return fail(MPPI_EINVAL, "batch_form must be MPPI_BATCH_PHASES or MPPI_BATCH_ONE_LAUNCH");
  if (t->adjoint_tiles < 0 || t->adjoint_tiles > kAdjointTilesMax)
    return fail(MPPI_EINVAL, "adjoint_tiles must be 0 .. %d", kAdjointTilesMax);
  if (t->batch_form == MPPI_BATCH_ONE_LAUNCH && !c->batch) {
    if (!c->C.one_single)
      return fail(MPPI_EUNSUPPORTED, "the one-launch form of a single context exists for the "
                  "double integrator with forward Euler and the quadratic cost, at most %d "
                  "samples and 256 steps (no gradient mode)", kOneLaunchMaxTiles * 16);
  } else if (t->batch_form == MPPI_BATCH_ONE_LAUNCH) {
    if (c->plan.n_fused_items < 1)
      return fail(MPPI_EUNSUPPORTED, "no one-launch kernel for this batch's dynamics and cost, "
                  "or an instance with more than %d samples", kOneLaunchMaxTiles * kBatchMaxTile);
    if (t->batch_tile != kBatchMaxTile || t->update_form != MPPI_UPDATE_TWO_PASS)
      return fail(MPPI_EUNSUPPORTED, "the one-launch form needs batch_tile %d and the "
                  "two-pass update setting", kBatchMaxTile);
  }
  if (t->update_form == MPPI_UPDATE_ONE_PASS && !one_pass_for(c))
    return fail(MPPI_EUNSUPPORTED, "the single-pass update exists for single contexts with at "
                "most %d samples (no gradient mode)", kOnePassMaxK);
  if (t->update_form == MPPI_UPDATE_CHUNKED && !chunked_for(c))
    return fail(MPPI_EUNSUPPORTED, "the chunked update exists for single contexts (no gradient "
                "mode)");
  Instance& I = c->inst[0];
  if (t->rollout_form == MPPI_ROLLOUT_SPLIT) {
    if (c->batch || !I.split)
      return fail(MPPI_EUNSUPPORTED, "the split rollout form exists for single contexts with "
                  "double-integrator, bicycle or quadrotor dynamics (no gradient mode)");
    if (t->lanes_per_sample != 1 &&
        !(t->lanes_per_sample == 4 && rollout_quad_available(I.cfg.dynamics, I.cfg.integrator)))
      return fail(MPPI_EUNSUPPORTED, "split form: lanes_per_sample 1, or 4 for the bicycle "
                  "with RK4");
  }
  if (t->rollout_form == MPPI_ROLLOUT_SCAN) {
    if (c->batch || I.hidden || I.grad ||
        !rollout_scan_supported(I.cfg.dynamics, I.cfg.integrator, I.cfg.cost, I.T,
                                t->lanes_per_sample == 32 ? 32 : 16))
      return fail(MPPI_EUNSUPPORTED, "the scan rollout form exists for single contexts with "
                  "bicycle dynamics, RK4 and at most 256 steps (no gradient mode)");
    if (t->lanes_per_sample != 16 && t->lanes_per_sample != 32)
      return fail(MPPI_EINVAL, "scan form: lanes_per_sample must be 16 or 32");
  }
  if (I.hidden || I.grad) {
    // waves per 16-sample tile: 1, or the MLP split over 2 (H = 32, 64) or 4 (H = 64)
    const int waves = t->rollout_block / kWave;
    const bool split_ok = (I.hidden == 64 && (waves == 2 || waves == 4)) ||
                          (I.hidden == 32 && waves == 2);
    if (t->lanes_per_sample != 16 || !(t->rollout_block == 64 || split_ok))
      return fail(MPPI_EUNSUPPORTED, "MLP dynamics and gradient mode use 16 lanes per sample "
                  "and 64-thread workgroups, or 128 / 256 threads with the MLP split over "
                  "2 (H = 32, 64) or 4 (H = 64) waves");
  } else if (t->lanes_per_sample == 4 || t->lanes_per_sample == 8 ||
             t->lanes_per_sample == 16) {
    if (c->batch || !rollout_quad_available(I.cfg.dynamics, I.cfg.integrator))
      return fail(MPPI_EUNSUPPORTED, "4, 8 or 16 lanes per sample exist for a single bicycle "
                  "instance with RK4 only");
  } else if (t->lanes_per_sample != 1 &&
             !(t->lanes_per_sample == 32 && t->rollout_form == MPPI_ROLLOUT_SCAN)) {
    return fail(MPPI_EINVAL, "lanes_per_sample must be 1, 4, 8 or 16 (or 32 in the scan form)");
  }
  if (c->batch && t->batch_tile != c->plan.tile) {
    const mppi_status st = upload_sample_tiles(c, t->batch_tile);
    if (st != MPPI_OK) return st;
  }
  if (!(I.hidden || I.grad)) I.lanes = t->lanes_per_sample;
  c->tune = *t;
  c->drop_graphs();
  return MPPI_OK;
}

mppi_status mppi_autotune(mppi_ctx* c, int32_t reps, char* report, size_t report_len) {
  if (!c) return fail(MPPI_EINVAL, "ctx must not be NULL");
  c->ahead = false;  // the word or a noise buffer may change
  if (!c->have_state) return fail(MPPI_ESTATE, "mppi_set_state must come before mppi_autotune");
  if (reps < 1) reps = 1;
  std::string text;
  hipEvent_t a = nullptr, b = nullptr;
  HIP_TRY(hipEventCreate(&a));
  hipError_t e = hipEventCreate(&b);
  auto done = [&](mppi_status st) {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (report && report_len) {
      snprintf(report, report_len, "%s", text.c_str());
    }
    return st;
  };
  if (e != hipSuccess) return done(hip_fail(e, "hipEventCreate"));
  // seconds per launch of fn, after one warm-up launch
  auto time_it = [&](auto fn, double* us) -> hipError_t {
    hipError_t err = fn();
    if (err == hipSuccess) err = hipEventRecord(a, c->stream);
    for (int r = 0; r < reps && err == hipSuccess; ++r) err = fn();
    if (err == hipSuccess) err = hipEventRecord(b, c->stream);
    if (err == hipSuccess) err = hipEventSynchronize(b);
    float ms = 0.0f;
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, a, b);
    *us = 1e3 * ms / reps;
    return err;
  };
  auto line = [&](const char* phase, const mppi_tuning& t, double us) {
    char buf[208];
    snprintf(buf, sizeof buf,
             "%s lanes=%d block=%d tile=%d calls=%d form=%d waves=%d update=%d batch=%d %.2f\n",
             phase, t.lanes_per_sample, t.rollout_block, t.batch_tile, t.noise_calls,
             t.rollout_form, t.cost_waves, t.update_form, t.batch_form, us);
    text += buf;
  };
  // Each group of candidates shapes one phase; the candidates of a group are
  // timed round-robin in kRounds rounds and each keeps its best round, so a
  // drift of the clock or of the caches does not decide the choice.
  constexpr int kRounds = 3;
  mppi_tuning best = c->tune;
  const Instance& I = c->one();
  const bool tiles = I.hidden || I.grad;
  struct Cand {
    mppi_tuning t;
    double us;
  };
  // margin: a later candidate replaces the one kept so far only if it is
  // faster by more than this fraction (the first candidate is the default)
  auto search = [&](const char* phase, std::vector<mppi_tuning> cands, auto fn,
                    mppi_tuning* chosen, double margin = 0.0) -> mppi_status {
    std::vector<Cand> cs;
    for (const mppi_tuning& t : cands) cs.push_back(Cand{t, 1e300});
    for (int r = 0; r < kRounds; ++r)
      for (Cand& cd : cs) {
        mppi_status st = mppi_set_tuning(c, &cd.t);
        if (st != MPPI_OK) return st;
        double us = 0.0;
        hipError_t err = time_it(fn, &us);
        if (err != hipSuccess) return hip_fail(err, "autotune launch");
        cd.us = std::min(cd.us, us);
      }
    const Cand* b = &cs[0];
    for (const Cand& cd : cs) {
      line(phase, cd.t, cd.us);
      if (cd.us < b->us * (1.0 - margin)) b = &cd;
    }
    *chosen = b->t;
    return MPPI_OK;
  };
  auto sample_rollout = [&] {
    hipError_t err = phase_sample(c);
    return err == hipSuccess ? phase_rollout(c) : err;
  };
  mppi_status st;
  if (c->batch) {
    // the tile size shapes both the noise and the rollout launch
    std::vector<mppi_tuning> cands;
    for (int tile : {64, 128, 256}) {
      mppi_tuning t = c->tune;
      t.batch_tile = tile;
      cands.push_back(t);
    }
    st = search("sample+rollout", cands, sample_rollout, &best);
    if (st != MPPI_OK) return done(st);
    if (c->plan.n_fused_items > 0) {
      // a whole iteration in each batch form; u and the instances' scalars
      // (iteration words) are put back afterwards
      std::vector<float> u_save(static_cast<size_t>(c->n_u));
      std::vector<DevState> st_save(c->inst.size());
      e = hipMemcpyAsync(u_save.data(), c->ws + c->C.u, sizeof(float) * u_save.size(),
                         hipMemcpyDeviceToHost, c->stream);
      if (e == hipSuccess)
        e = hipMemcpyAsync(st_save.data(), c->ws + c->C.states, sizeof(DevState) * st_save.size(),
                           hipMemcpyDeviceToHost, c->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
      if (e != hipSuccess) return done(hip_fail(e, "autotune save"));
      std::vector<mppi_tuning> forms;
      mppi_tuning a = best;
      a.batch_form = MPPI_BATCH_PHASES;
      forms.push_back(a);
      mppi_tuning b2 = best;
      b2.batch_tile = kBatchMaxTile;
      b2.update_form = MPPI_UPDATE_TWO_PASS;
      b2.batch_form = MPPI_BATCH_ONE_LAUNCH;
      forms.push_back(b2);
      // timed as mppi_iterate runs them: one iteration replayed from its graph
      // (the one-launch form is kept only when clearly faster: 5 %)
      st = search("iteration", forms, [&] {
        return mppi_iterate(c, 1) == MPPI_OK ? hipSuccess : hipErrorLaunchFailure;
      }, &best, 0.05);
      e = hipMemcpyAsync(c->ws + c->C.u, u_save.data(), sizeof(float) * u_save.size(),
                         hipMemcpyHostToDevice, c->stream);
      if (e == hipSuccess)
        e = hipMemcpyAsync(c->ws + c->C.states, st_save.data(), sizeof(DevState) * st_save.size(),
                           hipMemcpyHostToDevice, c->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
      if (st != MPPI_OK) return done(st);
      if (e != hipSuccess) return done(hip_fail(e, "autotune restore"));
    }
  } else {
    std::vector<mppi_tuning> cands;
    for (int calls : {1, 2, 4}) {
      mppi_tuning t = c->tune;
      t.noise_calls = calls;
      cands.push_back(t);
    }
    mppi_tuning pick;
    st = search("sample", cands, [&] { return phase_sample(c); }, &pick);
    if (st != MPPI_OK) return done(st);
    best.noise_calls = pick.noise_calls;
    st = mppi_set_tuning(c, &best);
    if (st != MPPI_OK) return done(st);
    cands.clear();
    if (tiles && I.hidden >= 32) {
      for (int block : {64, 128, 256}) {
        if (block == 256 && I.hidden != 64) continue;
        mppi_tuning t = best;
        t.rollout_block = block;
        cands.push_back(t);
      }
    } else if (!tiles) {
      const bool quad_ok = rollout_quad_available(I.cfg.dynamics, I.cfg.integrator);
      for (int lanes : {1, 4, 8, 16}) {
        if (lanes > 1 && !quad_ok) continue;
        for (int block : {64, 128, 256}) {
          mppi_tuning t = best;
          t.rollout_form = MPPI_ROLLOUT_FUSED;
          t.lanes_per_sample = lanes;
          t.rollout_block = block;
          cands.push_back(t);
        }
      }
      // the time-parallel scan form
      for (int lanes : {16, 32}) {
        if (!rollout_scan_supported(I.cfg.dynamics, I.cfg.integrator, I.cfg.cost, I.T, lanes))
          continue;
        for (int block : {64, 128, 256}) {
          mppi_tuning t = best;
          t.rollout_form = MPPI_ROLLOUT_SCAN;
          t.lanes_per_sample = lanes;
          t.rollout_block = block;
          cands.push_back(t);
        }
      }
      // the split form (section "Choosing between the Split and Combined
      // Kernels": both are timed, the faster is kept)
      if (I.split)
        for (int lanes : {1, 4}) {
          if (lanes > 1 && !quad_ok) continue;
          for (int block : {64, 128, 256})
            for (int waves : {2, 4, 8, 16, 32, 64, 128}) {
              mppi_tuning t = best;
              t.rollout_form = MPPI_ROLLOUT_SPLIT;
              t.lanes_per_sample = lanes;
              t.rollout_block = block;
              t.cost_waves = waves;
              cands.push_back(t);
            }
        }
    }
    if (!cands.empty()) {
      e = phase_sample(c);  // the rollouts read this iteration's noise
      if (e != hipSuccess) return done(hip_fail(e, "autotune launch"));
      st = search("rollout", cands, [&] { return phase_rollout(c); }, &pick);
      if (st != MPPI_OK) return done(st);
      best.lanes_per_sample = pick.lanes_per_sample;
      best.rollout_block = pick.rollout_block;
      best.rollout_form = pick.rollout_form;
      best.cost_waves = pick.cost_waves;
    }
    if (c->C.one_single) {
      // a whole iteration in each form (the per-phase launches in the shapes
      // chosen above, and the one-launch form); u, the iteration word and
      // the current noise buffer are put back afterwards
      std::vector<float> u_save(static_cast<size_t>(c->n_u));
      DevState st_save{};
      const int cur_save = c->inst[0].cur;
      e = hipMemcpyAsync(u_save.data(), c->ws + c->C.u, sizeof(float) * u_save.size(),
                         hipMemcpyDeviceToHost, c->stream);
      if (e == hipSuccess)
        e = hipMemcpyAsync(&st_save, c->ws + c->C.states, sizeof(DevState), hipMemcpyDeviceToHost,
                           c->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
      if (e != hipSuccess) return done(hip_fail(e, "autotune save"));
      std::vector<mppi_tuning> forms;
      mppi_tuning a = best;
      a.batch_form = MPPI_BATCH_PHASES;
      forms.push_back(a);
      mppi_tuning b2 = best;
      b2.batch_form = MPPI_BATCH_ONE_LAUNCH;
      forms.push_back(b2);
      // timed as mppi_iterate runs them: one iteration replayed from its graph
      // (the one-launch form is kept only when clearly faster: 5 %)
      st = search("iteration", forms, [&] {
        return mppi_iterate(c, 1) == MPPI_OK ? hipSuccess : hipErrorLaunchFailure;
      }, &best, 0.05);
      c->inst[0].cur = cur_save;
      c->ahead = false;
      e = hipMemcpyAsync(c->ws + c->C.u, u_save.data(), sizeof(float) * u_save.size(),
                         hipMemcpyHostToDevice, c->stream);
      if (e == hipSuccess)
        e = hipMemcpyAsync(c->ws + c->C.states, &st_save, sizeof(DevState), hipMemcpyHostToDevice,
                           c->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
      if (st != MPPI_OK) return done(st);
      if (e != hipSuccess) return done(hip_fail(e, "autotune restore"));
    }
  }
  st = mppi_set_tuning(c, &best);
  if (st != MPPI_OK) return done(st);
  // the noise and cost buffers now hold this iteration's sampling and rollout
  e = phase_sample(c);
  if (e == hipSuccess) e = phase_rollout(c);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return done(hip_fail(e, "autotune launch"));
  c->have_noise = c->have_costs = c->rollout_fresh = true;
  c->grad_ready = false;
  line("chosen", best, 0.0);
  return done(MPPI_OK);
}

mppi_status mppi_set_state(mppi_ctx* c, const float* d_x0) {
  if (!c || !d_x0) return fail(MPPI_EINVAL, "ctx and d_x0 must not be NULL");
  HIP_TRY(hipMemcpyAsync(c->ws + c->C.x0, d_x0, sizeof(float) * c->n_x0, hipMemcpyDeviceToDevice,
                         c->stream));
  HIP_TRY(tape_reset(c));
  c->have_state = true;
  return MPPI_OK;
}

mppi_status mppi_set_controls(mppi_ctx* c, const float* d_u) {
  if (!c || !d_u) return fail(MPPI_EINVAL, "ctx and d_u must not be NULL");
  HIP_TRY(hipMemcpyAsync(c->ws + c->C.u, d_u, sizeof(float) * c->n_u, hipMemcpyDeviceToDevice,
                         c->stream));
  HIP_TRY(tape_reset(c));
  return MPPI_OK;
}

mppi_status mppi_shift(mppi_ctx* c, int32_t steps, int32_t fill) {
  if (!c) return fail(MPPI_EINVAL, "ctx must not be NULL");
  if (steps < 0) return fail(MPPI_EINVAL, "steps must be >= 0");
  if (fill != MPPI_SHIFT_HOLD && fill != MPPI_SHIFT_ZERO)
    return fail(MPPI_EINVAL, "fill must be MPPI_SHIFT_HOLD or MPPI_SHIFT_ZERO");
  if (c->batch) {
    HIP_TRY(launch_batch_shift(c->plan, steps, fill, c->stream));
  } else {
    const Instance& I = c->one();
    HIP_TRY(launch_shift(I.u, I.T, I.m, steps, fill, c->stream));
  }
  HIP_TRY(tape_reset(c));
  return MPPI_OK;
}

mppi_status mppi_set_iteration(mppi_ctx* c, uint32_t iteration) {
  if (!c) return fail(MPPI_EINVAL, "ctx must not be NULL");
  c->ahead = false;  // the word or a noise buffer may change
  if (c->batch) {
    HIP_TRY(launch_batch_set_iteration(c->plan, iteration, c->stream));
  } else {
    HIP_TRY(launch_set_iteration(c->one().st, iteration, c->stream));
  }
  return MPPI_OK;
}

mppi_status mppi_sample(mppi_ctx* c) {
  if (!c) return fail(MPPI_EINVAL, "ctx must not be NULL");
  c->ahead = false;  // the word or a noise buffer may change
  HIP_TRY(phase_sample(c));
  c->have_noise = true;
  c->rollout_fresh = c->grad_ready = false;
  return MPPI_OK;
}

mppi_status mppi_rollout(mppi_ctx* c) {
  if (!c) return fail(MPPI_EINVAL, "ctx must not be NULL");
  c->ahead = false;  // the word or a noise buffer may change
  if (!c->have_state) return fail(MPPI_ESTATE, "mppi_set_state must come before a rollout");
  if (!c->have_noise) return fail(MPPI_ESTATE, "mppi_sample must come before a rollout");
  hipError_t e = phase_rollout(c);
  if (e != hipSuccess) return hip_fail(e, "rollout launch");
  c->have_costs = true;
  c->rollout_fresh = true;
  c->grad_ready = false;  // the costs and checkpoints no longer match the last update
  return MPPI_OK;
}

mppi_status mppi_set_costs(mppi_ctx* c, const float* d_costs) {
  if (!c || !d_costs) return fail(MPPI_EINVAL, "ctx and d_costs must not be NULL");
  c->ahead = false;  // the word or a noise buffer may change
  HIP_TRY(hipMemcpyAsync(c->ws + c->C.S, d_costs, sizeof(float) * c->n_S, hipMemcpyDeviceToDevice,
                         c->stream));
  c->have_costs = true;
  c->rollout_fresh = c->grad_ready = false;
  return MPPI_OK;
}

mppi_status mppi_update(mppi_ctx* c) {
  if (!c) return fail(MPPI_EINVAL, "ctx must not be NULL");
  c->ahead = false;  // the word or a noise buffer may change
  if (!c->have_noise || !c->have_costs)
    return fail(MPPI_ESTATE, "mppi_update needs noise and costs of the current iteration");
  hipError_t e = phase_update(c);
  if (e != hipSuccess) return hip_fail(e, "update launch");
  c->grad_ready = c->rollout_fresh;
  if (!c->rollout_fresh) c->tape_external = true;
  return MPPI_OK;
}

mppi_status mppi_iterate(mppi_ctx* c, int32_t num_iters) {
  if (!c) return fail(MPPI_EINVAL, "ctx must not be NULL");
  if (num_iters < 1) return fail(MPPI_EINVAL, "num_iters must be >= 1");
  if (!c->have_state) return fail(MPPI_ESTATE, "mppi_set_state must come before mppi_iterate");
  // A single context's sequence starts in the buffer after the current one
  // (holding noise drawn ahead, if any) and ends with the last iteration's
  // noise current and the next call's drawn ahead in the other buffer.
  const bool single = !c->batch && c->one().ahead_ok && !one_launch_single(c);
  const bool ahead = single && c->ahead;
  const int start = single ? c->inst[0].cur ^ 1 : 0;
  const int last = start ^ ((num_iters - 1) & 1);
  c->ahead = false;
  auto finish = [&] {
    if (single) c->inst[0].cur = last;
    c->ahead = single;
    c->have_noise = c->have_costs = c->rollout_fresh = c->grad_ready = true;
    return MPPI_OK;
  };
  // the launch sequence of num_iters iterations, captured once and replayed
  // as a graph; one iteration (one to four launches) is launched directly,
  // which reaches the GPU sooner than a graph launch, and the null stream
  // cannot be captured
  if (single) c->inst[0].cur = start;
  if (c->stream == nullptr || num_iters == 1) {
    for (int i = 0; i < num_iters; ++i) {
      hipError_t e = phase_iteration(c, i, ahead);
      if (e != hipSuccess) {
        if (single) c->inst[0].cur = last;
        return hip_fail(e, "iteration launch");
      }
    }
    return finish();
  }
  const int64_t key = static_cast<int64_t>(num_iters) * 4 + start * 2 + (ahead ? 1 : 0);
  auto it = c->graphs.find(key);
  if (it == c->graphs.end()) {
    hipGraph_t g = nullptr;
    HIP_TRY(hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed));
    hipError_t e = hipSuccess;
    for (int i = 0; i < num_iters && e == hipSuccess; ++i) e = phase_iteration(c, i, ahead);
    const hipError_t ec = hipStreamEndCapture(c->stream, &g);
    if (single) c->inst[0].cur = last;
    if (e != hipSuccess || ec != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return hip_fail(e != hipSuccess ? e : ec, "iteration capture");
    }
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return hip_fail(e, "graph instantiation");
    it = c->graphs.emplace(key, exec).first;
  }
  HIP_TRY(hipGraphLaunch(it->second, c->stream));
  return finish();
}

mppi_status mppi_get_controls(mppi_ctx* c, float* d_U) {
  if (!c || !d_U) return fail(MPPI_EINVAL, "ctx and d_U must not be NULL");
  HIP_TRY(hipMemcpyAsync(d_U, c->ws + c->C.u, sizeof(float) * c->n_u, hipMemcpyDeviceToDevice,
                         c->stream));
  return MPPI_OK;
}

mppi_status mppi_get_debug(mppi_ctx* c, int32_t what, void* d_dst) {
  if (!c || !d_dst) return fail(MPPI_EINVAL, "ctx and d_dst must not be NULL");
  switch (what) {
    case MPPI_DEBUG_NOISE: {
      char* dst = static_cast<char*>(d_dst);
      for (const Instance& I : c->inst) {
        HIP_TRY(hipMemcpy2DAsync(dst, sizeof(float) * I.K, I.eps(), sizeof(float) * I.L.ldk,
                                 sizeof(float) * I.K, I.TM, hipMemcpyDeviceToDevice, c->stream));
        dst += sizeof(float) * static_cast<size_t>(I.TM) * I.K;
      }
      return MPPI_OK;
    }
    case MPPI_DEBUG_COSTS:
      HIP_TRY(hipMemcpyAsync(d_dst, c->ws + c->C.S, sizeof(float) * c->n_S,
                             hipMemcpyDeviceToDevice, c->stream));
      return MPPI_OK;
    case MPPI_DEBUG_WEIGHTS:
      for (const Instance& I : c->inst) {
        hipError_t e = launch_weights(I.S, I.K, I.cfg.lambda, I.st,
                                      static_cast<float*>(d_dst) + I.off_S, c->stream);
        if (e != hipSuccess) return hip_fail(e, "weights launch");
      }
      return MPPI_OK;
    case MPPI_DEBUG_STATS:
      HIP_TRY(hipMemcpyAsync(d_dst, c->ws + c->C.states, sizeof(DevState) * c->inst.size(),
                             hipMemcpyDeviceToDevice, c->stream));
      return MPPI_OK;
    case MPPI_DEBUG_CRASHES:
      if (!(c->one().cfg.flags & MPPI_F_DEBUG) || !uses_circles(c->one().cfg.cost))
        return fail(MPPI_ESTATE, "crash counts need MPPI_F_DEBUG and a circles cost");
      HIP_TRY(hipMemcpyAsync(d_dst, c->ws + c->C.crashes, sizeof(int32_t) * c->n_S,
                             hipMemcpyDeviceToDevice, c->stream));
      return MPPI_OK;
    default:
      return fail(MPPI_EINVAL, "unknown debug buffer %d", what);
  }
}

int32_t mppi_theta_len(const mppi_ctx* c) {
  if (!c) { fail(MPPI_EINVAL, "ctx must not be NULL"); return 0; }
  if (c->batch || !c->one().grad) {
    fail(MPPI_ESTATE, "the context was created without MPPI_F_REQUIRES_GRAD");
    return 0;
  }
  return c->one().n_theta;
}

mppi_status mppi_set_theta(mppi_ctx* c, const float* host_theta) {
  if (!c || !host_theta) return fail(MPPI_EINVAL, "ctx and host_theta must not be NULL");
  c->ahead = false;  // the word or a noise buffer may change
  if (c->batch || !c->one().grad)
    return fail(MPPI_ESTATE, "the context was created without MPPI_F_REQUIRES_GRAD");
  Instance& I = c->inst[0];
  for (int i = 0; i < I.n_theta; ++i)
    if (!isfinite(host_theta[i])) return fail(MPPI_EINVAL, "theta[%d] is not finite", i);
  const int nmlp = I.n_theta - I.n - 1;
  const float wheelbase = host_theta[nmlp + I.n];
  if (!(wheelbase > 0.0f)) return fail(MPPI_EINVAL, "wheelbase must be > 0");
  if (I.hidden) {
    std::vector<float4> fwd, bwd;
    std::vector<uint4> bfp;
    build_mlp_packs(host_theta, I.hidden, &fwd, &bwd, bf16_of(&I.cfg) ? &bfp : nullptr);
    HIP_TRY(hipMemcpyAsync(I.at<char>(I.L.mlp), fwd.data(), sizeof(float4) * fwd.size(),
                           hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(I.at<char>(I.L.mlp_bwd), bwd.data(), sizeof(float4) * bwd.size(),
                           hipMemcpyHostToDevice, c->stream));
    if (!bfp.empty())
      HIP_TRY(hipMemcpyAsync(I.at<char>(I.L.mlp_bf), bfp.data(), sizeof(uint4) * bfp.size(),
                             hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
  }
  for (int i = 0; i < I.n; ++i) I.dp.w[i] = host_theta[nmlp + i];
  I.dp.inv_wheelbase = static_cast<float>(1.0 / wheelbase);
  // the kernels take the constants by value: recapture graphs on next use
  c->drop_graphs();
  HIP_TRY(tape_reset(c));
  return MPPI_OK;
}

mppi_status mppi_backward(mppi_ctx* c, const float* d_dL_dU, float* d_grad) {
  if (!c || !d_dL_dU || !d_grad) return fail(MPPI_EINVAL, "ctx, d_dL_dU and d_grad must not be NULL");
  if (c->batch || !c->one().grad)
    return fail(MPPI_ESTATE, "the context was created without MPPI_F_REQUIRES_GRAD");
  if (!c->grad_ready)
    return fail(MPPI_ESTATE, "mppi_backward needs an update that followed this iteration's "
                "rollout (none since the last mppi_sample, mppi_rollout or mppi_set_costs)");
  const Instance& I = c->one();
  hipError_t e = launch_adjoint(I.dp, (I.cfg.flags & MPPI_F_ACCURATE_TRIG) != 0, I.hidden, d_dL_dU,
                                I.at<float>(I.L.u_roll), I.eps(), I.L.ldk, I.K, I.T, I.e(),
                                I.cfg.lambda, step_size(I.cfg), I.at<float>(I.L.ckpt),
                                I.ckpt_every,
                                I.at<char>(I.L.adj), I.L.adj_layout, I.n_theta, d_grad, c->stream,
                                c->tune.rollout_block / kWave, false, nullptr,
                                c->tune.adjoint_tiles);
  if (e != hipSuccess) return hip_fail(e, "adjoint launch");
  return MPPI_OK;
}

mppi_status mppi_backward_iters(mppi_ctx* c, const float* d_dL_dU, float* d_grad,
                                float* d_dL_du0) {
  if (!c || !d_dL_dU || !d_grad)
    return fail(MPPI_EINVAL, "ctx, d_dL_dU and d_grad must not be NULL");
  c->ahead = false;  // the word or a noise buffer may change
  if (c->batch || !c->one().grad)
    return fail(MPPI_ESTATE, "the context was created without MPPI_F_REQUIRES_GRAD");
  if (c->tape_external)
    return fail(MPPI_ESTATE, "an update since the tape's start used mppi_set_costs");
  const Instance& I = c->one();
  int32_t n = 0;
  HIP_TRY(hipMemcpyAsync(&n, I.at<int32_t>(I.L.tape_count), sizeof n, hipMemcpyDeviceToHost,
                         c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (n < 1) return fail(MPPI_ESTATE, "no update since the tape's start");
  if (n > I.tape_cap)
    return fail(MPPI_ESTATE, "more than tape_len = %d updates since the tape's start",
                I.tape_cap);
  const bool accurate = (I.cfg.flags & MPPI_F_ACCURATE_TRIG) != 0;
  const int waves = c->tune.rollout_block / kWave;
  float* G = I.at<float>(I.L.tape_G);
  float* ckpt = I.at<float>(I.L.ckpt);
  DevState* scratch_state = I.at<DevState>(I.L.tape_state);
  HIP_TRY(hipMemcpyAsync(G, d_dL_dU, sizeof(float) * I.TM, hipMemcpyDeviceToDevice, c->stream));
  // the last taped iteration is still in the buffers (noise, checkpoints,
  // costs, weights) when its update came right after its rollout and nothing
  // has run since
  const bool last_in_place = c->grad_ready;
  for (int i = n - 1; i >= 0; --i) {
    const float* u_i = I.at<float>(I.L.tape_u) + static_cast<int64_t>(i) * I.TM;
    hipError_t e = hipSuccess;
    if (!(i == n - 1 && last_in_place)) {
      // rebuild iteration i from its tape entry: noise, checkpointing rollout, weights
      e = launch_noise(I.cfg.seed, I.at<uint32_t>(I.L.tape_word) + i, 0u, I.cfg.instance, I.K,
                       I.T, I.m, I.cfg.sigma, I.eps(), I.L.ldk, c->stream, c->tune.noise_calls,
                       I.dp.sigma_t, I.dp.mean_sample != 0);
      if (e == hipSuccess)
        e = launch_rollout_tiles(I.cfg.dynamics, I.cfg.integrator, I.cfg.cost, accurate, I.dp,
                                 I.x0, u_i, I.eps(), I.L.ldk, I.K, I.T, I.S, ckpt, I.ckpt_every,
                                 c->stream, waves);
      if (e == hipSuccess)
        e = launch_weights_only(I.S, I.K, I.cfg.lambda, I.e(), scratch_state, c->stream);
    }
    // then its reverse pass: grad (+)= sum_k a_k dJ_k/dtheta, G += sum_k a_k dJ_k/du_i
    if (e == hipSuccess)
      e = launch_adjoint(I.dp, accurate, I.hidden, G, u_i, I.eps(), I.L.ldk, I.K, I.T, I.e(),
                         I.cfg.lambda, step_size(I.cfg), ckpt, I.ckpt_every, I.at<char>(I.L.adj),
                         I.L.adj_layout, I.n_theta, d_grad, c->stream, waves, i != n - 1, G,
                         c->tune.adjoint_tiles);
    if (e != hipSuccess) return hip_fail(e, "reverse pass launch");
  }
  if (d_dL_du0)
    HIP_TRY(hipMemcpyAsync(d_dL_du0, G, sizeof(float) * I.TM, hipMemcpyDeviceToDevice,
                           c->stream));
  // the noise, cost and weight buffers now hold the first taped iteration's
  c->rollout_fresh = c->grad_ready = false;
  return MPPI_OK;
}

mppi_status mppi_noise(uint64_t seed, uint32_t iteration, uint32_t instance, int32_t K, int32_t T,
                       int32_t m, const float* sigma, float* d_eps, int64_t ldk,
                       void* hip_stream) {
  if (!sigma || !d_eps) return fail(MPPI_EINVAL, "sigma and d_eps must not be NULL");
  if (K < 1 || T < 1 || m < 1 || m > MPPI_MAX_CONTROL || ldk < K)
    return fail(MPPI_EINVAL, "need K, T >= 1, 1 <= m <= %d, ldk >= K", MPPI_MAX_CONTROL);
  if ((int64_t)T * m > 4 * 65535) return fail(MPPI_EINVAL, "T*m larger than 262140");
  hipError_t e = launch_noise(seed, nullptr, iteration, instance, K, T, m, sigma, d_eps, ldk,
                              static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return hip_fail(e, "noise launch");
  return MPPI_OK;
}

mppi_status mppi_noise_tables(float* d_r, float* d_c, float* d_s, void* hip_stream) {
  if (!d_r || !d_c || !d_s) return fail(MPPI_EINVAL, "table pointers must not be NULL");
  hipError_t e = launch_noise_tables(d_r, d_c, d_s, static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return hip_fail(e, "noise table launch");
  return MPPI_OK;
}

}  // extern "C"
