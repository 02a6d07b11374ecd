// Host side of the C ABI declared in include/mppi.h: argument validation,
// workspace carving, parameter upload and the launch sequence of one MPPI
// iteration (arXiv 2409.07563, Algorithm 1).  No device allocation happens
// here; all device memory is the caller's workspace.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <string>
#include <vector>

#include "common.h"

using namespace mppi;

namespace {

thread_local std::string g_last_error = "";

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

// Workspace layout (byte offsets from the workspace base), all 256-aligned.
struct Layout {
  int64_t ldk;  // noise row stride (K rounded up to a wave)
  int nchunk;
  size_t state, x0, u, eps, S, crashes, weights;
  size_t chunk_min, chunk_sum, chunk_sum2, chunk_num;
  size_t ref, stage, costmap, mlp;
  size_t total;
};

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
  if (c->dynamics == MPPI_DYN_BICYCLE_MLP)
    return fail(MPPI_EUNSUPPORTED, "MLP residual dynamics are not built in this version");
  if (!rollout_supported(c->dynamics, c->integrator, c->cost))
    return fail(MPPI_EUNSUPPORTED, "cost %u is not defined for dynamics %u", c->cost, c->dynamics);
  if ((c->dynamics == MPPI_DYN_BICYCLE) && !(p->wheelbase > 0.0f))
    return fail(MPPI_EINVAL, "wheelbase must be > 0");
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

Layout make_layout(const mppi_config* c, const mppi_params* p, int n, int m) {
  Layout L{};
  const int K = c->num_samples, T = c->horizon, TM = T * m;
  L.ldk = (K + kWave - 1) / kWave * kWave;
  L.nchunk = softmin_chunks(K);
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes); return o; };
  L.state = take(sizeof(DevState));
  L.x0 = take(sizeof(float) * MPPI_MAX_STATE);
  L.u = take(sizeof(float) * TM);
  L.eps = take(sizeof(float) * (size_t)TM * L.ldk);
  L.S = take(sizeof(float) * L.ldk);
  L.crashes = take(sizeof(int32_t) * L.ldk);
  L.weights = take(sizeof(float) * L.ldk);
  L.chunk_min = take(sizeof(float) * L.nchunk);
  L.chunk_sum = take(sizeof(float) * L.nchunk);
  L.chunk_sum2 = take(sizeof(float) * L.nchunk);
  L.chunk_num = take(sizeof(float) * (size_t)L.nchunk * TM);
  L.ref = take(sizeof(float) * (size_t)(p->ref ? p->ref_len : 1));
  const int S = uses_spline(c->cost) ? p->num_segments : 0;
  L.stage = take((uses_circles(c->cost) ? kMaxGridBytes : sizeof(float4)) +
                 sizeof(float4) * (S + (S + 1 + 3) / 4));
  const size_t cells =
      c->cost == MPPI_COST_PATH_COSTMAP ? (size_t)p->map_w * (size_t)p->map_h : 1;
  L.costmap = take(sizeof(float) * cells);
  L.mlp = take(sizeof(float));
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

}  // namespace

struct mppi_ctx {
  mppi_config cfg;
  int n, m, K, T, TM;
  Layout L;
  char* ws;
  hipStream_t stream;
  DevParams dp;
  bool quad = false;  // four lanes per sample in the rollout
  bool have_state = false;
  bool have_noise = false;
  bool have_costs = false;

  template <class X>
  X* at(size_t off) const { return reinterpret_cast<X*>(ws + off); }
  DevState* state() const { return at<DevState>(L.state); }
  SoftminLayout softmin() const {
    return SoftminLayout{at<float>(L.chunk_min), at<float>(L.chunk_sum), at<float>(L.chunk_sum2),
                         at<float>(L.chunk_num), L.nchunk};
  }
};

extern "C" {

const char* mppi_last_error(void) { return g_last_error.c_str(); }

size_t mppi_workspace_bytes(const mppi_config* cfg, const mppi_params* params) {
  int n, m;
  if (validate(cfg, params, &n, &m) != MPPI_OK) return 0;
  return make_layout(cfg, params, n, m).total;
}

mppi_status mppi_create(const mppi_config* cfg, const mppi_params* p, void* d_workspace,
                        size_t workspace_bytes, void* hip_stream, mppi_ctx** out) {
  if (!out) return fail(MPPI_EINVAL, "out must not be NULL");
  *out = nullptr;
  int n, m;
  mppi_status st = validate(cfg, p, &n, &m);
  if (st != MPPI_OK) return st;
  const Layout L = make_layout(cfg, p, n, m);
  if (!d_workspace) return fail(MPPI_EINVAL, "workspace must not be NULL");
  if (reinterpret_cast<uintptr_t>(d_workspace) % kAlign)
    return fail(MPPI_EINVAL, "workspace must be %zu-byte aligned", kAlign);
  if (workspace_bytes < L.total)
    return fail(MPPI_ENOMEM, "workspace of %zu bytes, need %zu", workspace_bytes, L.total);

  mppi_ctx* c = new mppi_ctx();
  c->cfg = *cfg;
  c->n = n; c->m = m; c->K = cfg->num_samples; c->T = cfg->horizon; c->TM = c->T * m;
  c->L = L;
  c->ws = static_cast<char*>(d_workspace);
  c->stream = static_cast<hipStream_t>(hip_stream);

  // host staging of the parameter arrays in their device formats
  std::vector<float> ref(p->ref ? p->ref_len : 1, 0.0f);
  if (p->ref) memcpy(ref.data(), p->ref, sizeof(float) * p->ref_len);
  // the staged cost block: circle grid, then spline coefficient rows, then knots
  const int S = uses_spline(cfg->cost) ? p->num_segments : 0;
  const int N = uses_circles(cfg->cost) ? p->num_circles : 0;
  Grid grid;
  if (!build_grid(p->cx, p->cy, p->r2, N, &grid)) {
    delete c;
    return fail(MPPI_EUNSUPPORTED, "circle grid does not fit %d bytes of LDS", kMaxGridBytes);
  }
  std::vector<float4> stage(grid.words);
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
  if (rollout_lds_bytes(cfg->dynamics, cfg->cost, static_cast<int>(stage.size()), c->T) >
      kMaxRolloutLds) {
    delete c;
    return fail(MPPI_EUNSUPPORTED, "cost data plus T*m controls exceed %zu bytes of LDS",
                kMaxRolloutLds);
  }

  auto fail_free = [&](mppi_status s) { delete c; return s; };
  auto up = [&](size_t off, const void* src, size_t bytes) -> hipError_t {
    return hipMemcpyAsync(c->ws + off, src, bytes, hipMemcpyHostToDevice, c->stream);
  };
  hipError_t e = hipSuccess;
  DevState st0{};
  st0.status = MPPI_OK;
  if (e == hipSuccess) e = up(L.state, &st0, sizeof st0);
  std::vector<float> zeros_u(c->TM, 0.0f);
  if (e == hipSuccess) e = up(L.u, zeros_u.data(), sizeof(float) * c->TM);
  if (e == hipSuccess) e = up(L.ref, ref.data(), sizeof(float) * ref.size());
  if (e == hipSuccess) e = up(L.stage, stage.data(), sizeof(float4) * stage.size());
  if (e == hipSuccess && cfg->cost == MPPI_COST_PATH_COSTMAP)
    e = up(L.costmap, p->costmap, sizeof(float) * (size_t)p->map_w * p->map_h);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return fail_free(hip_fail(e, "parameter upload"));

  // rollout variant: four lanes per sample while one lane per sample would
  // leave most SIMDs idle
  c->quad = rollout_quad_available(cfg->dynamics, cfg->integrator) &&
            !(cfg->flags & MPPI_F_ROLLOUT_LANE) &&
            ((cfg->flags & MPPI_F_ROLLOUT_QUAD) || c->K <= 32768);

  DevParams& d = c->dp;
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
  d.ref = c->at<float>(L.ref);
  d.nseg = S;
  d.ncirc = N;
  d.stage = c->at<float4>(L.stage);
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
    d.costmap = c->at<float>(L.costmap);
  }
  *out = c;
  g_last_error.clear();
  return MPPI_OK;
}

void mppi_destroy(mppi_ctx* ctx) { delete ctx; }

mppi_status mppi_set_state(mppi_ctx* c, const float* d_x0) {
  if (!c || !d_x0) return fail(MPPI_EINVAL, "ctx and d_x0 must not be NULL");
  HIP_TRY(hipMemcpyAsync(c->at<float>(c->L.x0), d_x0, sizeof(float) * c->n,
                         hipMemcpyDeviceToDevice, c->stream));
  c->have_state = true;
  return MPPI_OK;
}

mppi_status mppi_set_controls(mppi_ctx* c, const float* d_u) {
  if (!c || !d_u) return fail(MPPI_EINVAL, "ctx and d_u must not be NULL");
  HIP_TRY(hipMemcpyAsync(c->at<float>(c->L.u), d_u, sizeof(float) * c->TM,
                         hipMemcpyDeviceToDevice, c->stream));
  return MPPI_OK;
}

mppi_status mppi_set_iteration(mppi_ctx* c, uint32_t iteration) {
  if (!c) return fail(MPPI_EINVAL, "ctx must not be NULL");
  HIP_TRY(launch_set_iteration(c->state(), iteration, c->stream));
  return MPPI_OK;
}

mppi_status mppi_sample(mppi_ctx* c) {
  if (!c) return fail(MPPI_EINVAL, "ctx must not be NULL");
  HIP_TRY(launch_noise(c->cfg.seed, &c->state()->iteration, 0u, c->cfg.instance, c->K, c->T, c->m,
                       c->cfg.sigma, c->at<float>(c->L.eps), c->L.ldk, c->stream));
  c->have_noise = true;
  return MPPI_OK;
}

mppi_status mppi_rollout(mppi_ctx* c) {
  if (!c) return fail(MPPI_EINVAL, "ctx must not be NULL");
  if (!c->have_state) return fail(MPPI_ESTATE, "mppi_set_state must come before a rollout");
  if (!c->have_noise) return fail(MPPI_ESTATE, "mppi_sample must come before a rollout");
  int32_t* crashes = (c->cfg.flags & MPPI_F_DEBUG) && uses_circles(c->cfg.cost)
                         ? c->at<int32_t>(c->L.crashes)
                         : nullptr;
  hipError_t e = launch_rollout(c->cfg.dynamics, c->cfg.integrator, c->cfg.cost,
                                (c->cfg.flags & MPPI_F_ACCURATE_TRIG) != 0, c->quad, c->dp,
                                c->at<float>(c->L.x0), c->at<float>(c->L.u),
                                c->at<float>(c->L.eps), c->L.ldk, c->K, c->T,
                                c->at<float>(c->L.S), crashes, c->stream);
  if (e != hipSuccess) return hip_fail(e, "rollout launch");
  c->have_costs = true;
  return MPPI_OK;
}

mppi_status mppi_set_costs(mppi_ctx* c, const float* d_costs) {
  if (!c || !d_costs) return fail(MPPI_EINVAL, "ctx and d_costs must not be NULL");
  HIP_TRY(hipMemcpyAsync(c->at<float>(c->L.S), d_costs, sizeof(float) * c->K,
                         hipMemcpyDeviceToDevice, c->stream));
  c->have_costs = true;
  return MPPI_OK;
}

mppi_status mppi_update(mppi_ctx* c) {
  if (!c) return fail(MPPI_EINVAL, "ctx must not be NULL");
  if (!c->have_noise || !c->have_costs)
    return fail(MPPI_ESTATE, "mppi_update needs noise and costs of the current iteration");
  hipError_t e = launch_softmin_update(c->at<float>(c->L.S), c->at<float>(c->L.eps), c->L.ldk, c->K,
                                       c->TM, c->cfg.lambda, c->softmin(), c->at<float>(c->L.u),
                                       c->state(), c->stream);
  if (e != hipSuccess) return hip_fail(e, "update launch");
  return MPPI_OK;
}

mppi_status mppi_iterate(mppi_ctx* c, int32_t num_iters) {
  if (!c) return fail(MPPI_EINVAL, "ctx must not be NULL");
  if (num_iters < 1) return fail(MPPI_EINVAL, "num_iters must be >= 1");
  if (!c->have_state) return fail(MPPI_ESTATE, "mppi_set_state must come before mppi_iterate");
  for (int i = 0; i < num_iters; ++i) {
    mppi_status s;
    if ((s = mppi_sample(c)) != MPPI_OK) return s;
    if ((s = mppi_rollout(c)) != MPPI_OK) return s;
    if ((s = mppi_update(c)) != MPPI_OK) return s;
  }
  return MPPI_OK;
}

mppi_status mppi_get_controls(mppi_ctx* c, float* d_U) {
  if (!c || !d_U) return fail(MPPI_EINVAL, "ctx and d_U must not be NULL");
  HIP_TRY(hipMemcpyAsync(d_U, c->at<float>(c->L.u), sizeof(float) * c->TM,
                         hipMemcpyDeviceToDevice, c->stream));
  return MPPI_OK;
}

mppi_status mppi_get_debug(mppi_ctx* c, int32_t what, void* d_dst) {
  if (!c || !d_dst) return fail(MPPI_EINVAL, "ctx and d_dst must not be NULL");
  switch (what) {
    case MPPI_DEBUG_NOISE:
      HIP_TRY(hipMemcpy2DAsync(d_dst, sizeof(float) * c->K, c->at<float>(c->L.eps),
                               sizeof(float) * c->L.ldk, sizeof(float) * c->K, c->TM,
                               hipMemcpyDeviceToDevice, c->stream));
      return MPPI_OK;
    case MPPI_DEBUG_COSTS:
      HIP_TRY(hipMemcpyAsync(d_dst, c->at<float>(c->L.S), sizeof(float) * c->K,
                             hipMemcpyDeviceToDevice, c->stream));
      return MPPI_OK;
    case MPPI_DEBUG_WEIGHTS: {
      hipError_t e = launch_weights(c->at<float>(c->L.S), c->K, c->cfg.lambda, c->state(),
                                    static_cast<float*>(d_dst), c->stream);
      if (e != hipSuccess) return hip_fail(e, "weights launch");
      return MPPI_OK;
    }
    case MPPI_DEBUG_STATS:
      HIP_TRY(hipMemcpyAsync(d_dst, c->state(), sizeof(DevState), hipMemcpyDeviceToDevice,
                             c->stream));
      return MPPI_OK;
    case MPPI_DEBUG_CRASHES:
      if (!(c->cfg.flags & MPPI_F_DEBUG) || !uses_circles(c->cfg.cost))
        return fail(MPPI_ESTATE, "crash counts need MPPI_F_DEBUG and a circles cost");
      HIP_TRY(hipMemcpyAsync(d_dst, c->at<int32_t>(c->L.crashes), sizeof(int32_t) * c->K,
                             hipMemcpyDeviceToDevice, c->stream));
      return MPPI_OK;
    default:
      return fail(MPPI_EINVAL, "unknown debug buffer %d", what);
  }
}

mppi_status mppi_backward(mppi_ctx* c, const float* d_dL_dU, float* d_grad) {
  (void)d_dL_dU;
  (void)d_grad;
  if (!c) return fail(MPPI_EINVAL, "ctx must not be NULL");
  return fail(MPPI_EUNSUPPORTED, "mppi_backward is not built in this version");
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
