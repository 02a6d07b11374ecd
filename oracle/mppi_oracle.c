/*
 * MPPI reference oracle — TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, double-precision CPU evaluation of one MPPI iteration as
 * stated in arXiv 2409.07563 ("MPPI-Generic"), Section II-C, Algorithm 1 and
 * the update rule Eq. (mppi_update_rule).  Only the tests, the smoke check and
 * the benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header or constant generator with the GPU library: every piece below is
 * written from the paper and from the published definitions it names.
 *
 * Build: gcc -O2 -std=c11 -fno-fast-math -ffp-contract=off -shared -fPIC.
 * -ffp-contract=off matters for the noise transform: it is specified as an
 * exact sequence of binary32 operations and must not be re-associated or
 * contracted.
 *
 * Contents
 *   1. Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).
 *   2. The Gaussian noise definition: Box-Muller (1958) with a binary32 recipe
 *      for -2 ln u1 and sincos(2 pi u2) (see orc_bm_radius / orc_bm_angle).
 *   3. Models x_{t+1} = F(x_t, v_t): double integrator (Euler), kinematic
 *      bicycle (RK4), quadrotor (RK4 + quaternion renormalisation), bicycle
 *      with an MLP residual.  Eq. (dynamics), Section II.
 *   4. Costs l(x, v) and phi(x).  Eq. (2) / Algorithm 1.
 *   5. Algorithm 1: rollouts (cost after each step, terminal cost on the last
 *      state), baseline rho = min J, normaliser eta, weights w, and the
 *      control update U_t = u_t + sum_m w^m eps^m_t.
 *   6. Free-energy statistics (Section II-B, Eq. free_energy).
 *
 * Readings of the paper used here:
 *   - The running cost is charged on the post-step state and the sampled
 *     control, l(x_{t+1}, v_t), for t = 0..T-1, and phi on x_T (Algorithm 1;
 *     the combined-kernel description in Section III-C agrees).
 *   - The importance-sampling term is disabled (beta = 0, Section II-C).
 *   - The update uses U = u + sum w eps (Algorithm 1), equal in exact
 *     arithmetic to sum w v (Eq. mppi_update_rule) because sum w = 1.
 *   - A non-finite rollout cost counts as +inf (weight 0).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* 1. Philox4x32-10                                                          */
/* ------------------------------------------------------------------------ */

/* Round multipliers and Weyl key increments of Philox4x32 as published by
 * Salmon et al. (SC'11, Section 4). */
#define PHILOX_M4x32_0 0xD2511F53u
#define PHILOX_M4x32_1 0xCD9E8D57u
#define PHILOX_W32_0 0x9E3779B9u
#define PHILOX_W32_1 0xBB67AE85u

static void philox_round(uint32_t c[4], const uint32_t k[2]) {
  uint64_t p0 = (uint64_t)PHILOX_M4x32_0 * (uint64_t)c[0];
  uint64_t p1 = (uint64_t)PHILOX_M4x32_1 * (uint64_t)c[2];
  uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
  uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
  uint32_t n0 = hi1 ^ c[1] ^ k[0];
  uint32_t n1 = lo1;
  uint32_t n2 = hi0 ^ c[3] ^ k[1];
  uint32_t n3 = lo0;
  c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
}

/* Philox4x32 with R rounds: the key is bumped by the Weyl constants between
 * rounds.  out may alias ctr. */
void orc_philox4x32(const uint32_t ctr[4], const uint32_t key[2], int rounds,
                    uint32_t out[4]) {
  uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
  uint32_t k[2] = {key[0], key[1]};
  for (int r = 0; r < rounds; ++r) {
    if (r > 0) { k[0] += PHILOX_W32_0; k[1] += PHILOX_W32_1; }
    philox_round(c, k);
  }
  out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; out[3] = c[3];
}

/* ------------------------------------------------------------------------ */
/* 2. Gaussian noise definition                                              */
/* ------------------------------------------------------------------------ */
/*
 * The paper samples eps ~ N(0, Sigma) (Algorithm 1, Section II-C) without
 * naming a generator.  The noise used on both sides of the parity tests is
 * defined as follows (binary32, round-to-nearest-even, no contraction):
 *
 *   normal index within sample k:  n = t*m + j       (t < T, j < m)
 *   Philox call:   c = n / 4,  counter = (c, k, iter, instance),
 *                  key = (seed & 0xffffffff, seed >> 32),  10 rounds -> x[4]
 *   slot s = n % 4 uses the pair (a, b) = (x[2*(s/2)], x[2*(s/2)+1]) and
 *   takes the cosine branch when s is even, the sine branch when odd.
 *   Box-Muller: j1 = (a >> 8) + 1 in [1, 2^24], u1 = j1 * 2^-24 in (0, 1]
 *               j2 = b >> 8 in [0, 2^24),      u2 = j2 * 2^-24 in [0, 1)
 *               z = sqrt(-2 ln u1) * {cos, sin}(2 pi u2)
 *   eps[t][j][k] = sigma_j * z                     (one binary32 multiply)
 *
 * -2 ln u1 and sincos(2 pi u2) are evaluated with exact range reductions and
 * fixed polynomials (coefficients below, binary32):
 *   ln:  j1 = 2^e * f with f in [sqrt(1/2), sqrt(2)) (exact, from the float
 *        bits of j1); x = f - 1 (exact);  p = Horner(LNC, x) with fmaf;
 *        ln u1 = fmaf(e - 24, LN2_HI, fmaf(e - 24, LN2_LO, x * p)).
 *        LNC is the degree-9 Chebyshev interpolant of log1p(x)/x on
 *        [sqrt(1/2)-1, sqrt(2)-1], monomial coefficients rounded to binary32.
 *        r = sqrtf(-2 * ln u1)   (correctly rounded square root).
 *   sincos: q = (j2 + 2^21) >> 22;  i = j2 - q*2^22 in [-2^21, 2^21);
 *        f = (float)i * 2^-24 in [-1/8, 1/8) (exact);  y = f*f;
 *        sin(2 pi f) = f * Horner(SC, y);  cos(2 pi f) = Horner(CC, y);
 *        SC / CC are the Taylor coefficients of sin / cos of 2 pi f in f
 *        (orders 1..9 / 0..10), rounded to binary32.  The quadrant q & 3
 *        rotates (c, s) by multiples of pi/2 (exact sign/swap).
 */
static const float LNC[10] = {
    0x1.000000p+0f,  -0x1.fffff8p-2f, 0x1.55555ep-2f,  -0x1.000424p-2f,
    0x1.999e86p-3f,  -0x1.5423b0p-3f, 0x1.22cf10p-3f,  -0x1.0fb036p-3f,
    0x1.064786p-3f,  -0x1.31335ap-4f};
static const float SC[5] = {0x1.921fb6p+2f, -0x1.4abbcep+5f, 0x1.466bc6p+6f,
                            -0x1.32d2ccp+6f, 0x1.507834p+5f};
static const float CC[6] = {0x1.000000p+0f,  -0x1.3bd3ccp+4f, 0x1.03c1f0p+6f,
                            -0x1.55d3c8p+6f, 0x1.e1f506p+5f,  -0x1.a6d1f2p+4f};
/* ln 2 split so that e * LN2_HI is exact for |e| < 2^8. */
static const float LN2_HI = 0x1.62e400p-1f;
static const float LN2_LO = 0x1.7f7d1cp-20f;

static float bits_to_float(uint32_t u) { float f; memcpy(&f, &u, 4); return f; }
static uint32_t float_to_bits(float f) { uint32_t u; memcpy(&u, &f, 4); return u; }

/* sqrt(-2 ln(j1 * 2^-24)) for j1 in [1, 2^24]. */
float orc_bm_radius(uint32_t j1) {
  float fj = (float)j1; /* exact: j1 <= 2^24 */
  uint32_t bits = float_to_bits(fj);
  int e = (int)(bits >> 23) - 127;
  uint32_t mant = bits & 0x7FFFFFu;
  float f = bits_to_float(mant | 0x3F800000u); /* [1, 2) */
  if (mant > 0x3504F3u) { /* f > sqrt(2) (0x3FB504F3 = RN(sqrt 2)) */
    f = f * 0.5f;         /* exact */
    e += 1;
  }
  float x = f - 1.0f; /* exact (Sterbenz) */
  float p = LNC[9];
  for (int i = 8; i >= 0; --i) p = fmaf(p, x, LNC[i]);
  float lnf = x * p;
  float ke = (float)(e - 24);
  float ln = fmaf(ke, LN2_HI, fmaf(ke, LN2_LO, lnf));
  return sqrtf(-2.0f * ln);
}

/* (cos, sin)(2 pi j2 2^-24) for j2 in [0, 2^24). */
void orc_bm_angle(uint32_t j2, float* c_out, float* s_out) {
  uint32_t q = (j2 + (1u << 21)) >> 22;
  int32_t i = (int32_t)j2 - (int32_t)(q << 22);
  float f = (float)i * 0x1p-24f;
  float y = f * f;
  float ps = SC[4];
  for (int k = 3; k >= 0; --k) ps = fmaf(ps, y, SC[k]);
  float s = f * ps;
  float c = CC[5];
  for (int k = 4; k >= 0; --k) c = fmaf(c, y, CC[k]);
  switch (q & 3u) {
    case 0: *c_out = c; *s_out = s; break;
    case 1: *c_out = -s; *s_out = c; break;
    case 2: *c_out = -c; *s_out = -s; break;
    default: *c_out = s; *s_out = -c; break;
  }
}

void orc_box_muller(uint32_t a, uint32_t b, float* z0, float* z1) {
  float r = orc_bm_radius((a >> 8) + 1u);
  float c, s;
  orc_bm_angle(b >> 8, &c, &s);
  *z0 = r * c;
  *z1 = r * s;
}

/* Standard normal number n of sample k (see the definition above). */
static float std_normal(uint64_t seed, uint32_t k, uint32_t iter, uint32_t inst,
                        uint32_t n) {
  uint32_t ctr[4] = {n >> 2, k, iter, inst};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t x[4];
  orc_philox4x32(ctr, key, 10, x);
  uint32_t s = n & 3u;
  uint32_t pr = s >> 1;
  float z0, z1;
  orc_box_muller(x[2 * pr], x[2 * pr + 1], &z0, &z1);
  return (s & 1u) ? z1 : z0;
}

/* eps[t][j][k], row stride ldk >= K. */
void orc_noise(uint64_t seed, uint32_t iter, uint32_t inst, int32_t K, int32_t T,
               int32_t m, const float* sigma, int64_t ldk, float* eps) {
  for (int32_t t = 0; t < T; ++t)
    for (int32_t j = 0; j < m; ++j)
      for (int32_t k = 0; k < K; ++k) {
        uint32_t n = (uint32_t)(t * m + j);
        eps[((int64_t)t * m + j) * ldk + k] =
            sigma[j] * std_normal(seed, (uint32_t)k, iter, inst, n);
      }
}

/* ------------------------------------------------------------------------ */
/* Problem description                                                       */
/* ------------------------------------------------------------------------ */
enum { ORC_DI = 0, ORC_BICYCLE = 1, ORC_QUAD = 2, ORC_BICYCLE_MLP = 3 };
enum { ORC_EULER = 0, ORC_RK4 = 1 };
enum {
  ORC_COST_QUADRATIC = 0,
  ORC_COST_PATH_CIRCLES = 1,
  ORC_COST_PATH_COSTMAP = 2,
  ORC_COST_HOVER = 3,
  ORC_COST_TRACK = 4,
  ORC_COST_GOAL_CIRCLES = 5
};

typedef struct {
  int32_t model, integrator, cost;
  int32_t K, T, n, m;
  double dt, lambda;
  float sigma[8];
  uint64_t seed;
  uint32_t instance;
  /* dynamics constants */
  double wheelbase, mass, inertia[3], gravity;
  int32_t mlp_hidden;
  const double* mlp; /* W1[H][7] b1[H] W2[H][H] b2[H] W3[5][H] b3[5] */
  /* cost constants; meaning of w[] depends on the cost kind (see costs) */
  double w[32];
  const double* ref; /* goal / waypoint data or reference trajectory */
  int32_t ref_len;
  int32_t nseg; /* natural cubic spline y = s(x): knots[nseg+1], coef[nseg][4] */
  const double* knots;
  const double* coef;
  int32_t ncirc; /* circles: centres and squared radii */
  const double* cx;
  const double* cy;
  const double* r2;
  int32_t map_w, map_h; /* costmap [map_h][map_w], cell centres on a grid */
  double map_x0, map_y0, map_res;
  const double* map;
  /* importance-sampling term in the weights (1) or not (0), and the step
   * size of the update (1: the plain MPPI update) */
  int32_t is_beta;
  double gamma;
  /* cosines chained ahead of every running cost, scaled by zero (the cost
   * complexity experiment of the Results section); 0 = none */
  int32_t cost_cosines;
  /* sampling options (section "Sampling Distributions"): a per-step standard
   * deviation table sigma_t[T][m] (NULL: sigma for every step); sample 0 drawn
   * without noise (the mean itself); a fraction of the samples drawn around
   * zero instead of u (the last floor(zero_frac K) samples, at most K - 1 of
   * them when sample 0 is the noiseless mean) */
  const float* sigma_t;
  int32_t mean_sample;
  double zero_frac;
  /* bicycle with an MLP residual: the three matrix products take bfloat16
   * operands (0: binary64 operands).  The weights and each product's input
   * (z, h1, h2) are rounded to binary32 and then to the nearest bfloat16,
   * ties to even (bf16_of); biases, sums and tanh stay binary64.  The
   * backward pass takes the roundings as the identity: it differentiates
   * with the rounded weights and inputs. */
  int32_t mlp_bf16;
} orc_problem;

/* Samples k >= orc_plain_count(P) are drawn around zero. */
static int32_t orc_plain_count(const orc_problem* P) {
  int32_t nz = (int32_t)floor(P->zero_frac * (double)P->K);
  if (nz > P->K) nz = P->K;
  if (P->mean_sample && nz > P->K - 1) nz = P->K - 1;
  if (nz < 0) nz = 0;
  return P->K - nz;
}

/* The standard deviation of control j at step t. */
static float orc_sigma(const orc_problem* P, int32_t t, int j) {
  return P->sigma_t ? P->sigma_t[(int64_t)t * P->m + j] : P->sigma[j];
}

/* The perturbations of one iteration with the sampling options:
 * eps[t][j][k] = sigma_{t,j} z (one binary32 product of the standard normal
 * z of the noise definition), and eps[.][.][0] = 0 for the noiseless mean
 * sample. */
void orc_sample(const orc_problem* P, uint32_t iter, int64_t ldk, float* eps) {
  const int32_t K = P->K, T = P->T, m = P->m;
  for (int32_t t = 0; t < T; ++t)
    for (int32_t j = 0; j < m; ++j) {
      const float sg = orc_sigma(P, t, j);
      for (int32_t k = 0; k < K; ++k) {
        const uint32_t n = (uint32_t)(t * m + j);
        const float z = std_normal(P->seed, (uint32_t)k, iter, P->instance, n);
        eps[((int64_t)t * m + j) * ldk + k] = (P->mean_sample && k == 0) ? 0.0f : sg * z;
      }
    }
}

/* ------------------------------------------------------------------------ */
/* 3. Models                                                                 */
/* ------------------------------------------------------------------------ */

/* Kinematic bicycle: state (px, py, yaw, speed, steer), control (accel,
 * steer rate).  d/dt = (s cos yaw, s sin yaw, s tan(steer)/L, a, steer_rate). */
static void bicycle_deriv(const orc_problem* P, const double* x, const double* v,
                          double* d) {
  d[0] = x[3] * cos(x[2]);
  d[1] = x[3] * sin(x[2]);
  d[2] = x[3] * tan(x[4]) / P->wheelbase;
  d[3] = v[0];
  d[4] = v[1];
}

/* Rigid-body quadrotor: state p(3), q = (w, x, y, z) (Hamilton), v(3) world
 * frame, omega(3) body frame; control (thrust F, torques tx, ty, tz).
 *   p' = v;  q' = 1/2 q (x) (0, omega);  v' = R(q) (0, 0, F) / mass - (0, 0, g)
 *   omega' = J^-1 (tau - omega x (J omega)),  J = diag(inertia). */
static void quad_deriv(const orc_problem* P, const double* x, const double* v,
                       double* d) {
  const double qw = x[3], qx = x[4], qy = x[5], qz = x[6];
  const double wx = x[10], wy = x[11], wz = x[12];
  d[0] = x[7];
  d[1] = x[8];
  d[2] = x[9];
  d[3] = 0.5 * (-qx * wx - qy * wy - qz * wz);
  d[4] = 0.5 * (qw * wx + qy * wz - qz * wy);
  d[5] = 0.5 * (qw * wy + qz * wx - qx * wz);
  d[6] = 0.5 * (qw * wz + qx * wy - qy * wx);
  /* third column of the rotation matrix of q */
  const double r13 = 2.0 * (qx * qz + qw * qy);
  const double r23 = 2.0 * (qy * qz - qw * qx);
  const double r33 = 1.0 - 2.0 * (qx * qx + qy * qy);
  const double a = v[0] / P->mass;
  d[7] = r13 * a;
  d[8] = r23 * a;
  d[9] = r33 * a - P->gravity;
  const double J0 = P->inertia[0], J1 = P->inertia[1], J2 = P->inertia[2];
  const double h0 = J0 * wx, h1 = J1 * wy, h2 = J2 * wz; /* J omega */
  const double c0 = wy * h2 - wz * h1;                  /* omega x J omega */
  const double c1 = wz * h0 - wx * h2;
  const double c2 = wx * h1 - wy * h0;
  d[10] = (v[1] - c0) / J0;
  d[11] = (v[2] - c1) / J1;
  d[12] = (v[3] - c2) / J2;
}

static void deriv(const orc_problem* P, const double* x, const double* v,
                  double* d) {
  switch (P->model) {
    case ORC_DI: /* (px, py, vx, vy), control (ax, ay) */
      d[0] = x[2]; d[1] = x[3]; d[2] = v[0]; d[3] = v[1];
      break;
    case ORC_BICYCLE:
    case ORC_BICYCLE_MLP:
      bicycle_deriv(P, x, v, d);
      break;
    case ORC_QUAD:
      quad_deriv(P, x, v, d);
      break;
  }
}

/* The bfloat16 value nearest to x: x rounded to binary32 (nearest, ties to
 * even), then to 8 significand bits with binary32's exponent range, the
 * discarded low 16 bits of the binary32 encoding compared with half of the
 * kept unit, ties to the even kept value.  A carry out of the significand
 * moves up one binade (to infinity past the largest finite value); NaN and
 * infinities pass through. */
double orc_bf16(double x) {
  const float f = (float)x;
  uint32_t b;
  memcpy(&b, &f, sizeof b);
  if ((b & 0x7f800000u) == 0x7f800000u) return (double)f;
  const uint32_t low = b & 0xffffu;
  uint32_t r = b & 0xffff0000u;
  if (low > 0x8000u || (low == 0x8000u && (r & 0x10000u) != 0u)) r += 0x10000u;
  float y;
  memcpy(&y, &r, sizeof y);
  return (double)y;
}

/* An operand of one of the MLP's products: rounded in the bfloat16 option. */
static double mlp_op(const orc_problem* P, double x) {
  return P->mlp_bf16 ? orc_bf16(x) : x;
}

/* The MLP residual g([x; v]) = W3 tanh(W2 tanh(W1 z + b1) + b2) + b3,
 * z = (x[0..5), v[0..2)); in the bfloat16 option every product operand goes
 * through mlp_op. */
static void mlp_residual(const orc_problem* P, const double* x, const double* v,
                         double* g) {
  const int H = P->mlp_hidden;
  const double* W1 = P->mlp;
  const double* b1 = W1 + H * 7;
  const double* W2 = b1 + H;
  const double* b2 = W2 + H * H;
  const double* W3 = b2 + H;
  const double* b3 = W3 + 5 * H;
  double z[7] = {x[0], x[1], x[2], x[3], x[4], v[0], v[1]};
  double h1[256], h2[256];
  for (int i = 0; i < H; ++i) {
    double a = b1[i];
    for (int j = 0; j < 7; ++j) a += mlp_op(P, W1[i * 7 + j]) * mlp_op(P, z[j]);
    h1[i] = tanh(a);
  }
  for (int i = 0; i < H; ++i) {
    double a = b2[i];
    for (int j = 0; j < H; ++j) a += mlp_op(P, W2[i * H + j]) * mlp_op(P, h1[j]);
    h2[i] = tanh(a);
  }
  for (int i = 0; i < 5; ++i) {
    double a = b3[i];
    for (int j = 0; j < H; ++j) a += mlp_op(P, W3[i * H + j]) * mlp_op(P, h2[j]);
    g[i] = a;
  }
}

/* One step x <- F(x, v): forward Euler or classic RK4 with v held over the
 * step; quaternion renormalised after the step; MLP residual dt * g(x_t, v_t)
 * on the pre-step state. */
void orc_step(const orc_problem* P, double* x, const double* v) {
  const int n = P->n;
  const double dt = P->dt;
  double x0[16] = {0};
  for (int i = 0; i < n; ++i) x0[i] = x[i];
  if (P->integrator == ORC_EULER) {
    double d[16];
    deriv(P, x0, v, d);
    for (int i = 0; i < n; ++i) x[i] = x0[i] + dt * d[i];
  } else {
    double k1[16] = {0}, k2[16] = {0}, k3[16] = {0}, k4[16] = {0}, xs[16] = {0};
    deriv(P, x0, v, k1);
    for (int i = 0; i < n; ++i) xs[i] = x0[i] + 0.5 * dt * k1[i];
    deriv(P, xs, v, k2);
    for (int i = 0; i < n; ++i) xs[i] = x0[i] + 0.5 * dt * k2[i];
    deriv(P, xs, v, k3);
    for (int i = 0; i < n; ++i) xs[i] = x0[i] + dt * k3[i];
    deriv(P, xs, v, k4);
    for (int i = 0; i < n; ++i)
      x[i] = x0[i] + dt / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
  }
  if (P->model == ORC_QUAD) {
    double nq = sqrt(x[3] * x[3] + x[4] * x[4] + x[5] * x[5] + x[6] * x[6]);
    for (int i = 3; i < 7; ++i) x[i] /= nq;
  }
  if (P->model == ORC_BICYCLE_MLP) {
    double g[5];
    mlp_residual(P, x0, v, g);
    for (int i = 0; i < 5; ++i) x[i] += dt * g[i];
  }
}

/* ------------------------------------------------------------------------ */
/* 4. Costs                                                                  */
/* ------------------------------------------------------------------------ */

/* Natural cubic spline y = s(x) with x clamped to the knot range.
 * Segment i covers [knots[i], knots[i+1]); y = a + b d + c d^2 + e d^3 with
 * d = x - knots[i]. Returns s(x) and s'(x). */
static void spline_eval(const orc_problem* P, double px, double* y, double* dy) {
  const int S = P->nseg;
  double x = px;
  if (x < P->knots[0]) x = P->knots[0];
  if (x > P->knots[S]) x = P->knots[S];
  int i = 0;
  while (i + 1 < S && x >= P->knots[i + 1]) ++i;
  const double* c = P->coef + 4 * i;
  const double d = x - P->knots[i];
  *y = c[0] + d * (c[1] + d * (c[2] + d * c[3]));
  *dy = c[1] + d * (2.0 * c[2] + 3.0 * d * c[3]);
}

/* Crash indicator: the point lies in (or on) some circle.  *margin receives
 * the smallest relative distance |d^2 - r^2| / r^2 over all circles, which
 * says how close this decision was to flipping. */
static int circles_hit(const orc_problem* P, double px, double py,
                       double* margin) {
  int hit = 0;
  for (int i = 0; i < P->ncirc; ++i) {
    const double dx = px - P->cx[i], dy = py - P->cy[i];
    const double d2 = dx * dx + dy * dy;
    if (d2 <= P->r2[i]) hit = 1;
    const double mg = fabs(d2 - P->r2[i]) / P->r2[i];
    if (mg < *margin) *margin = mg;
  }
  return hit;
}

/* Bilinear interpolation of the costmap between cell centres, clamped to the
 * edge cells.  Cell (ix, iy) has its centre at
 * (x0 + (ix + 1/2) res, y0 + (iy + 1/2) res). */
static double costmap_eval_grad(const orc_problem* P, double px, double py, double* slope);
static double costmap_eval(const orc_problem* P, double px, double py) {
  double slope;
  return costmap_eval_grad(P, px, py, &slope);
}

/* Value and |dM/dx| + |dM/dy| of the bilinear costmap (0 along clamped
 * directions). */
static double costmap_eval_grad(const orc_problem* P, double px, double py, double* slope) {
  const int W = P->map_w, H = P->map_h;
  double gx = (px - P->map_x0) / P->map_res - 0.5;
  double gy = (py - P->map_y0) / P->map_res - 0.5;
  const int clamp_x = gx < 0.0 || gx > W - 1, clamp_y = gy < 0.0 || gy > H - 1;
  if (gx < 0.0) gx = 0.0;
  if (gx > W - 1) gx = W - 1;
  if (gy < 0.0) gy = 0.0;
  if (gy > H - 1) gy = H - 1;
  int ix = (int)floor(gx), iy = (int)floor(gy);
  if (ix > W - 2) ix = W - 2;
  if (iy > H - 2) iy = H - 2;
  const double fx = gx - ix, fy = gy - iy;
  const double* m = P->map;
  const double m00 = m[iy * W + ix], m01 = m[iy * W + ix + 1];
  const double m10 = m[(iy + 1) * W + ix], m11 = m[(iy + 1) * W + ix + 1];
  const double dmx = ((1.0 - fy) * (m01 - m00) + fy * (m11 - m10)) / P->map_res;
  const double dmy = ((1.0 - fx) * (m10 - m00) + fx * (m11 - m01)) / P->map_res;
  *slope = (clamp_x ? 0.0 : fabs(dmx)) + (clamp_y ? 0.0 : fabs(dmy));
  return (1.0 - fx) * (1.0 - fy) * m00 + fx * (1.0 - fy) * m01 +
         (1.0 - fx) * fy * m10 + fx * fy * m11;
}

/* Path-tracking terms for the bicycle: lateral error to the spline measured
 * along y, heading error to the spline tangent, speed error. */
static double path_terms(const orc_problem* P, const double* x) {
  double y, dy;
  spline_eval(P, x[0], &y, &dy);
  const double e = x[1] - y;
  const double eh = x[2] - atan(dy);
  const double es = x[3] - P->w[3];
  return P->w[0] * e * e + P->w[1] * eh * eh + P->w[2] * es * es;
}

static double quad_state_terms(const orc_problem* P, const double* x) {
  const double* pw = P->ref;     /* waypoint (3) */
  const double* qr = P->ref + 3; /* reference attitude (4) */
  double cp = 0, cv = 0, cw = 0;
  for (int i = 0; i < 3; ++i) {
    cp += (x[i] - pw[i]) * (x[i] - pw[i]);
    cv += x[7 + i] * x[7 + i];
    cw += x[10 + i] * x[10 + i];
  }
  const double dq = x[3] * qr[0] + x[4] * qr[1] + x[5] * qr[2] + x[6] * qr[3];
  return P->w[0] * cp + P->w[1] * cv + P->w[2] * cw + P->w[3] * (1.0 - dq * dq);
}

/*
 * Running cost l(x_{t+1}, v_t) (t = step index, x = post-step state).
 *   QUADRATIC:    sum_i w[i] (x_i - g_i)^2 + sum_j w[8+j] v_j^2, g = ref[0..n)
 *   PATH_*:       w = (w_lat, w_head, w_speed, v_ref, r_a, r_steer, crash,
 *                 terminal_scale): path terms + r_a a^2 + r_steer v1^2 +
 *                 crash * [inside a circle]  (CIRCLES) or + costmap(p) (COSTMAP)
 *   HOVER:        w = (w_p, w_v, w_w, w_q, w_u, w_box, box, terminal_scale),
 *                 ref = (waypoint 3, q_ref 4, u_hover 4):  state terms +
 *                 w_u |v - u_hover|^2 + w_box sum_i max(0, |p_i| - box)^2
 *   TRACK:        sum_i w[i] (x_i - ref[(t+1) n + i])^2 + sum_j w[8+j] v_j^2
 *   GOAL_CIRCLES: w = (w_goal, r_a, r_steer, crash, terminal_scale),
 *                 ref = goal (2): w_goal |p - goal|^2 + controls + crash term
 */
static double running_cost(const orc_problem* P, const double* x,
                           const double* v, int t, double* margin,
                           int* crashed, double* slope) {
  const int n = P->n, m = P->m;
  /* the inflation: cost_cosines nested cosines of 1, times zero */
  double infl = 0.0;
  if (P->cost_cosines > 0) {
    double z = 1.0;
    for (int32_t i = 0; i < P->cost_cosines; ++i) z = cos(z);
    infl = 0.0 * z;
  }
  double c = 0.0;
  switch (P->cost) {
    case ORC_COST_QUADRATIC:
      for (int i = 0; i < n; ++i) c += P->w[i] * (x[i] - P->ref[i]) * (x[i] - P->ref[i]);
      for (int j = 0; j < m; ++j) c += P->w[8 + j] * v[j] * v[j];
      break;
    case ORC_COST_PATH_CIRCLES:
    case ORC_COST_PATH_COSTMAP:
      c = path_terms(P, x) + P->w[4] * v[0] * v[0] + P->w[5] * v[1] * v[1];
      if (P->cost == ORC_COST_PATH_CIRCLES) {
        if (circles_hit(P, x[0], x[1], margin)) { c += P->w[6]; ++*crashed; }
      } else {
        double sl;
        c += costmap_eval_grad(P, x[0], x[1], &sl);
        *slope += sl;
      }
      break;
    case ORC_COST_HOVER: {
      c = quad_state_terms(P, x);
      const double* uh = P->ref + 7;
      for (int j = 0; j < 4; ++j) c += P->w[4] * (v[j] - uh[j]) * (v[j] - uh[j]);
      for (int i = 0; i < 3; ++i) {
        const double o = fabs(x[i]) - P->w[6];
        if (o > 0.0) c += P->w[5] * o * o;
      }
      break;
    }
    case ORC_COST_TRACK: {
      const double* xr = P->ref + (int64_t)(t + 1) * n;
      for (int i = 0; i < n; ++i) c += P->w[i] * (x[i] - xr[i]) * (x[i] - xr[i]);
      for (int j = 0; j < m; ++j) c += P->w[8 + j] * v[j] * v[j];
      break;
    }
    case ORC_COST_GOAL_CIRCLES: {
      const double dx = x[0] - P->ref[0], dy = x[1] - P->ref[1];
      c = P->w[0] * (dx * dx + dy * dy) + P->w[1] * v[0] * v[0] + P->w[2] * v[1] * v[1];
      if (circles_hit(P, x[0], x[1], margin)) { c += P->w[3]; ++*crashed; }
      break;
    }
  }
  return c + infl;
}

/* Terminal cost phi(x_T). */
static double terminal_cost(const orc_problem* P, const double* x) {
  const int n = P->n;
  double c = 0.0;
  switch (P->cost) {
    case ORC_COST_QUADRATIC:
      for (int i = 0; i < n; ++i) c += P->w[16 + i] * (x[i] - P->ref[i]) * (x[i] - P->ref[i]);
      break;
    case ORC_COST_PATH_CIRCLES:
    case ORC_COST_PATH_COSTMAP:
      c = P->w[7] * path_terms(P, x);
      break;
    case ORC_COST_HOVER:
      c = P->w[7] * quad_state_terms(P, x);
      break;
    case ORC_COST_TRACK: {
      const double* xr = P->ref + (int64_t)P->T * n;
      for (int i = 0; i < n; ++i) c += P->w[i] * (x[i] - xr[i]) * (x[i] - xr[i]);
      c *= P->w[16];
      break;
    }
    case ORC_COST_GOAL_CIRCLES: {
      const double dx = x[0] - P->ref[0], dy = x[1] - P->ref[1];
      c = P->w[4] * P->w[0] * (dx * dx + dy * dy);
      break;
    }
  }
  return c;
}

/* ------------------------------------------------------------------------ */
/* 5. Algorithm 1                                                            */
/* ------------------------------------------------------------------------ */

/* Rollout costs J^k for every sample (the inner loops of Algorithm 1):
 * x <- x0; for t: v = u_t + eps_t; x <- F(x, v); J += l(x, v); then J += phi(x).
 * eps is [T][m][ldk].  margin[k] / crashes[k] (optional) receive the smallest
 * crash-decision margin and the number of crashed steps; slope[k] (optional)
 * the sum over steps of the costmap's |dM/dx| + |dM/dy| at the visited
 * positions (how strongly the cost reacts to a position error). */
/* The importance-sampling term of one step (section "MPPI-Generic's MPPI
 * Implementation" and Eq. information_theoretic_weighting): the sampling
 * distribution N(u_t, Sigma_t) against the base distribution N(0, Sigma_t)
 * gives ln p/s = -(v - u/2)' Sigma_t^-1 u, and the weights use
 * J - lambda beta ln p/s, i.e. J plus lambda (v - u/2)' Sigma_t^-1 u (Sigma_t
 * diagonal).  u_t is the mean the sample was drawn around (zero for the
 * zero-mean samples, whose term then vanishes: their density is the base
 * one). */
static double is_term(const orc_problem* P, int32_t t, const double* u_t, const double* v) {
  double s = 0.0;
  for (int j = 0; j < P->m; ++j) {
    const double sg = (double)orc_sigma(P, t, j);
    s += (v[j] - 0.5 * u_t[j]) * u_t[j] / (sg * sg);
  }
  return P->lambda * s;
}

/* S[k]: the cost J of sample k's rollout (Algorithm 1) with
 * v = u + eps_k (v = eps_k for the zero-mean samples), plus the
 * importance-sampling term when P->is_beta is set. */
void orc_rollout_costs(const orc_problem* P, const double* x0, const double* u,
                       const float* eps, int64_t ldk, double* S, double* margin,
                       int32_t* crashes, double* slope) {
  const int n = P->n, m = P->m;
  const int32_t n_plain = orc_plain_count(P);
  for (int32_t k = 0; k < P->K; ++k) {
    double x[16], v[8], mean[8];
    for (int i = 0; i < n; ++i) x[i] = x0[i];
    double J = 0.0, mg = INFINITY, sl = 0.0;
    int cr = 0;
    for (int32_t t = 0; t < P->T; ++t) {
      for (int j = 0; j < m; ++j) {
        mean[j] = k < n_plain ? u[t * m + j] : 0.0;
        v[j] = mean[j] + (double)eps[((int64_t)t * m + j) * ldk + k];
      }
      orc_step(P, x, v);
      J += running_cost(P, x, v, t, &mg, &cr, &sl);
      if (P->is_beta) J += is_term(P, t, mean, v);
    }
    J += terminal_cost(P, x);
    if (!isfinite(J)) J = INFINITY;
    S[k] = J;
    if (margin) margin[k] = mg;
    if (crashes) crashes[k] = cr;
    if (slope) slope[k] = sl;
  }
}

/* Baseline, normaliser, weights and control update (the last two loops of
 * Algorithm 1):  rho = min J;  eta = sum exp(-(J - rho)/lambda);
 * w = exp(-(J - rho)/lambda)/eta;  U_t = u_t + gamma sum_k w_k eps_{k,t}
 * (gamma = 1: Algorithm 1; otherwise the step size of the dynamic
 * mirror-descent form U = (1 - gamma) u + gamma sum_k w_k v_k, section
 * "Comparisons to sampling-efficient algorithms").
 * stats = (rho, eta, free-energy estimate rho - lambda ln(eta/K),
 * effective sample size 1/sum w^2).  Returns 0, or -6 when every J is
 * non-finite (then w = 0 and U = u). */
int orc_softmin_update(const orc_problem* P, const double* S, const float* eps,
                       int64_t ldk, const double* u, double* w, double* U,
                       double* stats) {
  const int32_t K = P->K, T = P->T, m = P->m;
  const double lam = P->lambda;
  double rho = INFINITY;
  for (int32_t k = 0; k < K; ++k)
    if (S[k] < rho) rho = S[k];
  if (!isfinite(rho)) {
    for (int32_t k = 0; k < K; ++k) w[k] = 0.0;
    for (int32_t i = 0; i < T * m; ++i) U[i] = u[i];
    if (stats) { stats[0] = rho; stats[1] = 0; stats[2] = INFINITY; stats[3] = 0; }
    return -6;
  }
  double eta = 0.0;
  for (int32_t k = 0; k < K; ++k) eta += exp(-(S[k] - rho) / lam);
  double sw2 = 0.0;
  for (int32_t k = 0; k < K; ++k) {
    w[k] = exp(-(S[k] - rho) / lam) / eta;
    sw2 += w[k] * w[k];
  }
  /* U = u + gamma sum_k w_k (v_k - u): v_k - u = eps_k for the samples
   * drawn around u, eps_k - u for those drawn around zero */
  const int32_t n_plain = orc_plain_count(P);
  for (int32_t t = 0; t < T; ++t)
    for (int32_t j = 0; j < m; ++j) {
      double acc = 0.0;
      const float* row = eps + ((int64_t)t * m + j) * ldk;
      const double ut = u[t * m + j];
      for (int32_t k = 0; k < K; ++k)
        acc += w[k] * (k < n_plain ? (double)row[k] : (double)row[k] - ut);
      U[t * m + j] = ut + P->gamma * acc;
    }
  if (stats) {
    stats[0] = rho;
    stats[1] = eta;
    stats[2] = rho - lam * log(eta / K);
    stats[3] = 1.0 / sw2;
  }
  return 0;
}

/* I iterations of Algorithm 1 with warm start u <- U and fresh noise per
 * iteration (Philox iteration word iter0 + i).  u is updated in place.
 * Optional outputs hold the last iteration's eps/S/w/stats. */
int orc_mppi(const orc_problem* P, const double* x0, double* u, int32_t iters,
             uint32_t iter0, float* eps_out, double* S_out, double* w_out,
             double* stats_out) {
  const int32_t K = P->K, T = P->T, m = P->m;
  float* eps = eps_out ? eps_out : (float*)malloc(sizeof(float) * (size_t)T * m * K);
  double* S = S_out ? S_out : (double*)malloc(sizeof(double) * (size_t)K);
  double* w = w_out ? w_out : (double*)malloc(sizeof(double) * (size_t)K);
  double* U = (double*)malloc(sizeof(double) * (size_t)T * m);
  int rc = 0;
  for (int32_t i = 0; i < iters; ++i) {
    orc_sample(P, iter0 + (uint32_t)i, K, eps);
    orc_rollout_costs(P, x0, u, eps, K, S, NULL, NULL, NULL);
    rc = orc_softmin_update(P, S, eps, K, u, w, U, stats_out);
    for (int32_t q = 0; q < T * m; ++q) u[q] = U[q];
  }
  free(U);
  if (!eps_out) free(eps);
  if (!S_out) free(S);
  if (!w_out) free(w);
  return rc;
}

/* The MPC warm start between calls (section "Beginner", the plant's
 * optimisation stride): the nominal sequence moves `steps` steps forward,
 * u[t] <- u[t + steps]; the steps past the horizon take the last control
 * (fill 0) or zero (fill 1).  u is [T][m], updated in place. */
void orc_shift(const orc_problem* P, double* u, int32_t steps, int32_t fill) {
  const int32_t T = P->T, m = P->m;
  double* old = (double*)malloc(sizeof(double) * (size_t)T * m);
  for (int32_t q = 0; q < T * m; ++q) old[q] = u[q];
  for (int32_t t = 0; t < T; ++t)
    for (int j = 0; j < m; ++j) {
      const int64_t src = (int64_t)t + steps;
      double val;
      if (src < T) val = old[src * m + j];
      else val = fill == 0 ? old[(int64_t)(T - 1) * m + j] : 0.0;
      u[(int64_t)t * m + j] = val;
    }
  free(old);
}

/* Deterministic rollout of one control sequence; xs receives [T+1][n]. */
void orc_trajectory(const orc_problem* P, const double* x0, const double* v_seq,
                    double* xs) {
  const int n = P->n, m = P->m;
  double x[16];
  for (int i = 0; i < n; ++i) { x[i] = x0[i]; xs[i] = x0[i]; }
  for (int32_t t = 0; t < P->T; ++t) {
    orc_step(P, x, v_seq + t * m);
    for (int i = 0; i < n; ++i) xs[(t + 1) * n + i] = x[i];
  }
}

/* Cost of one control sequence (the inner loop of Algorithm 1 for one m). */
double orc_sequence_cost(const orc_problem* P, const double* x0,
                         const double* v_seq) {
  const int n = P->n, m = P->m;
  double x[16], mg = INFINITY, sl = 0.0;
  int cr = 0;
  for (int i = 0; i < n; ++i) x[i] = x0[i];
  double J = 0.0;
  for (int32_t t = 0; t < P->T; ++t) {
    orc_step(P, x, v_seq + t * m);
    J += running_cost(P, x, v_seq + t * m, t, &mg, &cr, &sl);
  }
  return J + terminal_cost(P, x);
}

/* Test support for orc_cost_condition: the cost of one control sequence with
 * delta added to component i of x_s (the state after step s, 1 <= s <= T)
 * right after the step that produces it, before its running cost (and, for
 * s = T, the terminal cost) is charged; the perturbation then propagates
 * through every later step.  Central differences of this function in delta
 * give dJ/dx_{s,i}, the sensitivities that orc_cost_condition forms with its
 * adjoint. */
double orc_sequence_cost_injected(const orc_problem* P, const double* x0, const double* v_seq,
                                  int32_t s, int32_t i, double delta) {
  const int n = P->n, m = P->m;
  double x[16], mg = INFINITY, sl = 0.0;
  int cr = 0;
  for (int q = 0; q < n; ++q) x[q] = x0[q];
  double J = 0.0;
  for (int32_t t = 0; t < P->T; ++t) {
    orc_step(P, x, v_seq + t * m);
    if (t + 1 == s) x[i] += delta;
    J += running_cost(P, x, v_seq + t * m, t, &mg, &cr, &sl);
  }
  return J + terminal_cost(P, x);
}

/* Single-point evaluations used by unit tests of the model and cost pieces. */
double orc_eval_running_cost(const orc_problem* P, const double* x,
                             const double* v, int32_t t) {
  double mg = INFINITY, sl = 0.0;
  int cr = 0;
  return running_cost(P, x, v, t, &mg, &cr, &sl);
}
double orc_eval_terminal_cost(const orc_problem* P, const double* x) {
  return terminal_cost(P, x);
}
void orc_eval_deriv(const orc_problem* P, const double* x, const double* v,
                    double* d) {
  deriv(P, x, v, d);
}
void orc_eval_spline(const orc_problem* P, double px, double* y, double* dy) {
  spline_eval(P, px, y, dy);
}
double orc_eval_costmap(const orc_problem* P, double px, double py) {
  return costmap_eval(P, px, py);
}

/* Bulk helpers for the tests: the transform's radius factor for every
 * j1 in [1, 2^24] (r[j1 - 1]) and the angle factors for every j2 in [0, 2^24). */
void orc_bm_tables(float* r, float* c, float* s) {
  for (uint32_t j = 0; j < (1u << 24); ++j) {
    r[j] = orc_bm_radius(j + 1u);
    orc_bm_angle(j, &c[j], &s[j]);
  }
}

/* Philox4x32-10 blocks for n counters (ctr[n][4]) under one key. */
void orc_philox_many(int64_t n, const uint32_t* ctr, const uint32_t key[2],
                     uint32_t* out) {
  for (int64_t i = 0; i < n; ++i) orc_philox4x32(ctr + 4 * i, key, 10, out + 4 * i);
}

/* ------------------------------------------------------------------------ */
/* 7. Gradient of a loss on the updated controls (differentiable MPPI)       */
/* ------------------------------------------------------------------------ */
/*
 * For one iteration U = u + sum_k w_k eps_k with w = softmin(J / lambda) and
 * u independent of theta, a loss L(U) with G = dL/dU has
 *   dL/dJ_k = -(w_k / lambda) (g_k - sum_i w_i g_i),  g_k = <G, eps_k>
 * (the baseline rho cancels), and dL/dtheta = sum_k (dL/dJ_k) dJ_k/dtheta.
 * dJ_k/dtheta comes from the discrete adjoint of the rollout: the costate
 * mu_t = dJ/dx_t is swept backwards through every RK4 stage and the MLP
 * residual of the actual discrete map (not a continuous adjoint ODE).
 * Parameter layout of grad: [MLP blob (W1 b1 W2 b2 W3 b3) | Q diag (n) |
 * wheelbase]; supported for the bicycle models with the TRACK cost.
 */

/* Jacobian-transpose product of the bicycle derivative at (x, v):
 * dx += (df/dx)^T c, and dL += (df/dwheelbase)^T c. */
static void bicycle_deriv_vjp(const orc_problem* P, const double* x, const double* c,
                              double* dx, double* dL, double* dv) {
  const double psi = x[2], s = x[3], d = x[4], Lw = P->wheelbase;
  const double cp = cos(psi), sp = sin(psi), td = tan(d), sec2 = 1.0 + td * td;
  dx[2] += -s * sp * c[0] + s * cp * c[1];
  dx[3] += cp * c[0] + sp * c[1] + td / Lw * c[2];
  dx[4] += s * sec2 / Lw * c[2];
  *dL += -s * td / (Lw * Lw) * c[2];
  /* speed' = accel = v0, steer' = steer rate = v1 */
  if (dv) { dv[0] += c[3]; dv[1] += c[4]; }
}

/* MLP residual forward with the activations kept for its backward (tanh
 * outputs before any bfloat16 rounding). */
static void mlp_forward_keep(const orc_problem* P, const double* z, double* h1, double* h2,
                             double* g) {
  const int H = P->mlp_hidden;
  const double* W1 = P->mlp;
  const double* b1 = W1 + H * 7;
  const double* W2 = b1 + H;
  const double* b2 = W2 + H * H;
  const double* W3 = b2 + H;
  const double* b3 = W3 + 5 * H;
  for (int i = 0; i < H; ++i) {
    double a = b1[i];
    for (int j = 0; j < 7; ++j) a += mlp_op(P, W1[i * 7 + j]) * mlp_op(P, z[j]);
    h1[i] = tanh(a);
  }
  for (int i = 0; i < H; ++i) {
    double a = b2[i];
    for (int j = 0; j < H; ++j) a += mlp_op(P, W2[i * H + j]) * mlp_op(P, h1[j]);
    h2[i] = tanh(a);
  }
  for (int i = 0; i < 5; ++i) {
    double a = b3[i];
    for (int j = 0; j < H; ++j) a += mlp_op(P, W3[i * H + j]) * mlp_op(P, h2[j]);
    g[i] = a;
  }
}

/* Backward of g(z): dz += (dg/dz)^T cg, dmlp += (dg/dtheta)^T cg.  In the
 * bfloat16 option the roundings count as the identity: the products'
 * derivatives take the rounded weights and inputs, tanh' the unrounded
 * outputs.  sens (optional) += sum over the product inputs o of
 * |dJ/do| |o| (o = z, h1, h2 as the products consume them, dJ/do with cg =
 * dJ/dg): the first-order change of J when every such input moves by its own
 * size. */
static void mlp_vjp(const orc_problem* P, const double* z, const double* cg, double* dz,
                    double* dmlp, double* sens) {
  const int H = P->mlp_hidden;
  double h1[256], h2[256], g[5], da2[256], da1[256];
  mlp_forward_keep(P, z, h1, h2, g);
  const double* W1 = P->mlp;
  const double* W2 = W1 + H * 7 + H;
  const double* W3 = W2 + H * H + H;
  double* dW1 = dmlp;
  double* db1 = dW1 + H * 7;
  double* dW2 = db1 + H;
  double* db2 = dW2 + H * H;
  double* dW3 = db2 + H;
  double* db3 = dW3 + 5 * H;
  for (int i = 0; i < 5; ++i) {
    db3[i] += cg[i];
    for (int j = 0; j < H; ++j) dW3[i * H + j] += cg[i] * mlp_op(P, h2[j]);
  }
  for (int j = 0; j < H; ++j) {
    double s = 0.0;
    for (int i = 0; i < 5; ++i) s += mlp_op(P, W3[i * H + j]) * cg[i];
    if (sens) *sens += fabs(s) * fabs(mlp_op(P, h2[j]));
    da2[j] = s * (1.0 - h2[j] * h2[j]);
  }
  for (int i = 0; i < H; ++i) {
    db2[i] += da2[i];
    for (int j = 0; j < H; ++j) dW2[i * H + j] += da2[i] * mlp_op(P, h1[j]);
  }
  for (int j = 0; j < H; ++j) {
    double s = 0.0;
    for (int i = 0; i < H; ++i) s += mlp_op(P, W2[i * H + j]) * da2[i];
    if (sens) *sens += fabs(s) * fabs(mlp_op(P, h1[j]));
    da1[j] = s * (1.0 - h1[j] * h1[j]);
  }
  for (int i = 0; i < H; ++i) {
    db1[i] += da1[i];
    for (int j = 0; j < 7; ++j) dW1[i * 7 + j] += da1[i] * mlp_op(P, z[j]);
  }
  for (int j = 0; j < 7; ++j) {
    double s = 0.0;
    for (int i = 0; i < H; ++i) s += mlp_op(P, W1[i * 7 + j]) * da1[i];
    if (sens) *sens += fabs(s) * fabs(mlp_op(P, z[j]));
    dz[j] += s;
  }
}

/* Test support: mlp_vjp alone, dz[7] and dmlp (the weight blob's layout)
 * accumulated from z[7] and cg[5] = dJ/dg. */
void orc_mlp_vjp(const orc_problem* P, const double* z, const double* cg, double* dz,
                 double* dmlp) {
  mlp_vjp(P, z, cg, dz, dmlp, NULL);
}

/* Backward of one step x1 = F(x0, v): given mu1 = dJ/dx1, returns
 * mu0 = (dF/dx0)^T mu1 and accumulates (dF/dtheta)^T mu1 into grad and, when
 * dv is given, (dF/dv)^T mu1 into dv. */
static void step_vjp(const orc_problem* P, const double* x0, const double* v, const double* mu1,
                     double* mu0, double* grad_mlp, double* grad_L, double* dv, double* sens) {
  const int n = 5;
  const double h = P->dt;
  double k1[5], k2[5], k3[5], x2[5], x3[5], x4[5];
  deriv(P, x0, v, k1);
  for (int i = 0; i < n; ++i) x2[i] = x0[i] + 0.5 * h * k1[i];
  deriv(P, x2, v, k2);
  for (int i = 0; i < n; ++i) x3[i] = x0[i] + 0.5 * h * k2[i];
  deriv(P, x3, v, k3);
  for (int i = 0; i < n; ++i) x4[i] = x0[i] + h * k3[i];
  double ck1[5], ck2[5], ck3[5], ck4[5], cx[5];
  for (int i = 0; i < n; ++i) {
    mu0[i] = mu1[i];
    ck1[i] = h / 6.0 * mu1[i];
    ck2[i] = h / 3.0 * mu1[i];
    ck3[i] = h / 3.0 * mu1[i];
    ck4[i] = h / 6.0 * mu1[i];
  }
  /* k4 = f(x4), x4 = x0 + h k3 */
  for (int i = 0; i < n; ++i) cx[i] = 0.0;
  bicycle_deriv_vjp(P, x4, ck4, cx, grad_L, dv);
  for (int i = 0; i < n; ++i) { mu0[i] += cx[i]; ck3[i] += h * cx[i]; }
  /* k3 = f(x3), x3 = x0 + h/2 k2 */
  for (int i = 0; i < n; ++i) cx[i] = 0.0;
  bicycle_deriv_vjp(P, x3, ck3, cx, grad_L, dv);
  for (int i = 0; i < n; ++i) { mu0[i] += cx[i]; ck2[i] += 0.5 * h * cx[i]; }
  /* k2 = f(x2), x2 = x0 + h/2 k1 */
  for (int i = 0; i < n; ++i) cx[i] = 0.0;
  bicycle_deriv_vjp(P, x2, ck2, cx, grad_L, dv);
  for (int i = 0; i < n; ++i) { mu0[i] += cx[i]; ck1[i] += 0.5 * h * cx[i]; }
  /* k1 = f(x0) */
  for (int i = 0; i < n; ++i) cx[i] = 0.0;
  bicycle_deriv_vjp(P, x0, ck1, cx, grad_L, dv);
  for (int i = 0; i < n; ++i) mu0[i] += cx[i];
  /* residual dt * g([x0; v]) */
  if (P->model == ORC_BICYCLE_MLP) {
    double z[7] = {x0[0], x0[1], x0[2], x0[3], x0[4], v[0], v[1]};
    double cg[5], dz[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int i = 0; i < 5; ++i) cg[i] = h * mu1[i];
    mlp_vjp(P, z, cg, dz, grad_mlp, sens);
    for (int i = 0; i < 5; ++i) mu0[i] += dz[i];
    if (dv) { dv[0] += dz[5]; dv[1] += dz[6]; }
  }
}

static int backward_supported(const orc_problem* P) {
  return (P->model == ORC_BICYCLE || P->model == ORC_BICYCLE_MLP) && P->cost == ORC_COST_TRACK &&
         P->integrator == ORC_RK4 && orc_plain_count(P) == P->K;
}

/* One iteration's reverse pass (accumulating): grad += dL/dtheta at fixed u,
 * du += sum_k a_k dJ_k/du (the dependence of the costs on the nominal
 * sequence u, through v = u + eps and, with the importance-sampling term,
 * directly), with a_k = dL/dJ_k; grad_abs / du_abs += the matching sums of
 * |terms| (rel_k-scaled for grad_abs).  The arguments are those of
 * orc_backward. */
static int backward_one(const orc_problem* P, const double* x0, const double* u, const float* eps,
                        const double* G, const double* S_in, const double* rel, double* grad,
                        double* grad_abs, double* du, double* du_abs, double* U_out,
                        double* S_out, double* w_out) {
  const int32_t K = P->K, T = P->T, m = P->m, n = P->n;
  const int H = P->mlp_hidden;
  const int nmlp = P->model == ORC_BICYCLE_MLP ? 7 * H + H + H * H + H + 5 * H + 5 : 0;
  const int ngrad = nmlp + n + 1;
  double* S = (double*)calloc((size_t)K, sizeof(double));
  double* w = (double*)malloc(sizeof(double) * K);
  double* U = (double*)malloc(sizeof(double) * T * m);
  double stats[4];
  if (S_in)
    for (int32_t k = 0; k < K; ++k) S[k] = S_in[k];
  else
    orc_rollout_costs(P, x0, u, eps, K, S, NULL, NULL, NULL);
  int rc = orc_softmin_update(P, S, eps, K, u, w, U, stats);
  double* dk = (double*)malloc(sizeof(double) * ngrad); /* dJ_k/dtheta of one sample */
  double* dku = (double*)malloc(sizeof(double) * T * m); /* dJ_k/du of one sample */
  if (rc == 0) {
    /* g_k = <G, eps_k>; dL/dJ_k = -(w_k/lambda) (g_k - sum_i w_i g_i), written
     * as -(w_k/lambda) sum_i w_i (g_k - g_i) (the weights sum to one) so that
     * no cancellation occurs when one sample holds almost all the weight */
    double* g = (double*)malloc(sizeof(double) * K);
    double* ak = (double*)malloc(sizeof(double) * K);
    for (int32_t k = 0; k < K; ++k) {
      double acc = 0.0;
      for (int32_t r = 0; r < T * m; ++r) acc += G[r] * (double)eps[(int64_t)r * K + k];
      g[k] = acc;
    }
    for (int32_t k = 0; k < K; ++k) {
      double d = 0.0;
      if (w[k] != 0.0)
        for (int32_t i = 0; i < K; ++i) d += w[i] * (g[k] - g[i]);
      ak[k] = -(P->gamma * w[k] / P->lambda) * d; /* U - u = gamma sum w eps */
    }
    double* xs = (double*)malloc(sizeof(double) * (T + 1) * n);
    double* vs = (double*)malloc(sizeof(double) * T * m);
    double* gmlp = dk;
    double* gQ = dk + nmlp;
    double* gL = dk + nmlp + n;
    for (int32_t k = 0; k < K; ++k) {
      const double a = ak[k];
      if (a == 0.0) continue;
      for (int i = 0; i < ngrad; ++i) dk[i] = 0.0;
      for (int i = 0; i < T * m; ++i) dku[i] = 0.0;
      for (int i = 0; i < n; ++i) xs[i] = x0[i];
      for (int32_t t = 0; t < T; ++t) {
        for (int j = 0; j < m; ++j) vs[t * m + j] = u[t * m + j] + (double)eps[((int64_t)t * m + j) * K + k];
        for (int i = 0; i < n; ++i) xs[(t + 1) * n + i] = xs[t * n + i];
        orc_step(P, xs + (t + 1) * n, vs + t * m);
      }
      /* terminal and running costs: phi = w16 sum Q_i e_i^2 at x_T, l_t at x_{t+1} */
      /* dJ_k/dtheta with mu_t = dJ_k/dx_t (a_k is applied afterwards) */
      double mu[5], mu0[5];
      const double* xT = xs + T * n;
      const double* rT = P->ref + (int64_t)T * n;
      for (int i = 0; i < n; ++i) {
        const double e = xT[i] - rT[i];
        mu[i] = 2.0 * P->w[16] * P->w[i] * e;
        gQ[i] += P->w[16] * e * e;
      }
      for (int32_t t = T - 1; t >= 0; --t) {
        /* running cost l_t on x_{t+1} */
        const double* x1 = xs + (t + 1) * n;
        const double* r1 = P->ref + (int64_t)(t + 1) * n;
        for (int i = 0; i < n; ++i) {
          const double e = x1[i] - r1[i];
          mu[i] += 2.0 * P->w[i] * e;
          gQ[i] += e * e;
        }
        /* dJ/dv_t: the control term of l_t, then the step */
        double* dv = dku + t * m;
        for (int j = 0; j < m; ++j) dv[j] = 2.0 * P->w[8 + j] * vs[t * m + j];
        step_vjp(P, xs + t * n, vs + t * m, mu, mu0, gmlp, gL, dv, NULL);
        /* the importance-sampling term lambda (v - u/2)' Sigma^-1 u with
         * v = u + eps: its derivative in u is lambda Sigma^-1 v */
        if (P->is_beta)
          for (int j = 0; j < m; ++j)
            dv[j] += P->lambda * vs[t * m + j] /
                     ((double)orc_sigma(P, t, j) * (double)orc_sigma(P, t, j));
        for (int i = 0; i < n; ++i) mu[i] = mu0[i];
      }
      for (int i = 0; i < ngrad; ++i) {
        grad[i] += a * dk[i];
        if (grad_abs) grad_abs[i] += fabs(a * dk[i]) * (rel ? rel[k] : 1.0);
      }
      for (int i = 0; i < T * m; ++i) {
        if (du) du[i] += a * dku[i];
        if (du_abs) du_abs[i] += fabs(a * dku[i]);
      }
    }
    free(xs);
    free(vs);
    free(g);
    free(ak);
  }
  if (U_out) for (int i = 0; i < T * m; ++i) U_out[i] = U[i];
  if (S_out) for (int k = 0; k < K; ++k) S_out[k] = S[k];
  if (w_out) for (int k = 0; k < K; ++k) w_out[k] = w[k];
  free(dk);
  free(dku);
  free(S);
  free(w);
  free(U);
  return rc;
}

/* grad <- dL/dtheta for L with dL/dU = G (layout above), for one iteration
 * from u (which does not depend on theta); also returns the forward's U, S
 * and w.  S_in (optional): costs to form the weights from in place of the
 * rollout's own (the sweeps still differentiate the rollouts).  grad_abs
 * (optional): sum over samples of rel_k |a_k dJ_k/dtheta| (rel_k = 1 when rel
 * is NULL), the scale of the rounding error of the sum when sample k's terms
 * carry relative error rel_k.  du (optional): sum_k a_k dJ_k/du, the part of
 * dL/du that passes through the costs (dL/du = G + du), with du_abs the sum
 * of |terms|.  Returns 0, -1 if unsupported, -6 if all J are non-finite. */
int orc_backward(const orc_problem* P, const double* x0, const double* u, const float* eps,
                 const double* G, const double* S_in, const double* rel, double* grad,
                 double* grad_abs, double* U_out, double* S_out, double* w_out, double* du,
                 double* du_abs) {
  if (!backward_supported(P)) return -1;
  const int ngrad = (P->model == ORC_BICYCLE_MLP ? 14 * P->mlp_hidden +
                     P->mlp_hidden * P->mlp_hidden + 5 : 0) + P->n + 1;
  for (int i = 0; i < ngrad; ++i) {
    grad[i] = 0.0;
    if (grad_abs) grad_abs[i] = 0.0;
  }
  for (int i = 0; i < P->T * P->m; ++i) {
    if (du) du[i] = 0.0;
    if (du_abs) du_abs[i] = 0.0;
  }
  return backward_one(P, x0, u, eps, G, S_in, rel, grad, grad_abs, du, du_abs, U_out, S_out,
                      w_out);
}

/* The gradient through `iters` warm-started iterations (Algorithm 1's outer
 * loop, iteration words iter0, iter0 + 1, ...) from the nominal sequence u0:
 * with u_{i+1} = u_i + gamma sum_k w_k(u_i, theta) eps_k and a loss on u_I
 * given by G = dL/du_I, the reverse pass runs the iterations backwards,
 *   grad += sum_k a_k dJ_k/dtheta,   G <- G + sum_k a_k dJ_k/du_i,
 * with a_k the softmin Jacobian of iteration i applied to the current G.
 * Outputs: grad (dL/dtheta), grad_abs (sum of |terms| over all iterations,
 * optional), du0 (dL/du0, optional), U_out (u_I, optional).  Returns 0, -1 if
 * unsupported, or the first nonzero status of an iteration. */
int orc_backward_iters(const orc_problem* P, const double* x0, const double* u0, int32_t iters,
                       uint32_t iter0, const double* G, double* grad, double* grad_abs,
                       double* du0, double* U_out) {
  if (!backward_supported(P) || iters < 1) return -1;
  const int32_t K = P->K, T = P->T, m = P->m, TM = T * m;
  const int ngrad = (P->model == ORC_BICYCLE_MLP ? 14 * P->mlp_hidden +
                     P->mlp_hidden * P->mlp_hidden + 5 : 0) + P->n + 1;
  double* tape = (double*)malloc(sizeof(double) * (size_t)(iters + 1) * TM);
  float* eps = (float*)malloc(sizeof(float) * (size_t)TM * K);
  double* S = (double*)malloc(sizeof(double) * K);
  double* w = (double*)malloc(sizeof(double) * K);
  double stats[4];
  int rc = 0;
  for (int i = 0; i < TM; ++i) tape[i] = u0[i];
  for (int32_t it = 0; it < iters; ++it) {
    const double* u = tape + (size_t)it * TM;
    double* U = tape + (size_t)(it + 1) * TM;
    orc_sample(P, iter0 + (uint32_t)it, K, eps);
    orc_rollout_costs(P, x0, u, eps, K, S, NULL, NULL, NULL);
    const int r = orc_softmin_update(P, S, eps, K, u, w, U, stats);
    if (r && !rc) rc = r;
  }
  for (int i = 0; i < ngrad; ++i) {
    grad[i] = 0.0;
    if (grad_abs) grad_abs[i] = 0.0;
  }
  double* Gc = (double*)malloc(sizeof(double) * TM);
  double* du = (double*)malloc(sizeof(double) * TM);
  for (int i = 0; i < TM; ++i) Gc[i] = G[i];
  for (int32_t it = iters - 1; it >= 0; --it) {
    orc_sample(P, iter0 + (uint32_t)it, K, eps);
    for (int i = 0; i < TM; ++i) du[i] = 0.0;
    const int r = backward_one(P, x0, tape + (size_t)it * TM, eps, Gc, NULL, NULL, grad, grad_abs,
                               du, NULL, NULL, NULL, NULL);
    if (r && !rc) rc = r;
    for (int i = 0; i < TM; ++i) Gc[i] += du[i];
  }
  if (du0) for (int i = 0; i < TM; ++i) du0[i] = Gc[i];
  if (U_out) for (int i = 0; i < TM; ++i) U_out[i] = tape[(size_t)iters * TM + i];
  free(Gc);
  free(du);
  free(tape);
  free(eps);
  free(S);
  free(w);
  return rc;
}

/* Sensitivity of each sample's cost to the rounding of its trajectory:
 * cond[k] = sum_{t=1..T} sum_i |dJ_k/dx_{t,i}| |x_{t,i}|, the first-order
 * change of J_k when every state component at every step is perturbed by one
 * unit in the last place relative to its size.  A binary32 rollout commits a
 * few such roundings per component and step, so its cost can differ from the
 * binary64 one by a small multiple of 2^-24 cond[k] whatever the kernel does.
 * cond_bf (optional, the bfloat16 option of the MLP): cond_bf[k] = sum over
 * steps and over the inputs o of the MLP's products (z, h1, h2 after their
 * rounding) of |dJ_k/do| |o|, the first-order change of J_k when every such
 * operand moves by its own size.  An operand whose rounding decision goes the
 * other way moves by one bfloat16 unit in the last place, at most 2^-7 of its
 * size.  Same models, integrator and cost as orc_backward; returns -1
 * otherwise. */
int orc_cost_condition(const orc_problem* P, const double* x0, const double* u, const float* eps,
                       int64_t ldk, double* cond, double* cond_bf) {
  if ((P->model != ORC_BICYCLE && P->model != ORC_BICYCLE_MLP) || P->cost != ORC_COST_TRACK ||
      P->integrator != ORC_RK4)
    return -1;
  const int32_t K = P->K, T = P->T, m = P->m, n = P->n;
  const int H = P->mlp_hidden;
  const int nmlp = P->model == ORC_BICYCLE_MLP ? 7 * H + H + H * H + H + 5 * H + 5 : 0;
  double* scratch = (double*)malloc(sizeof(double) * (nmlp + 1));
  double* xs = (double*)malloc(sizeof(double) * (T + 1) * n);
  double* vs = (double*)malloc(sizeof(double) * T * m);
  for (int32_t k = 0; k < K; ++k) {
    for (int i = 0; i < n; ++i) xs[i] = x0[i];
    for (int32_t t = 0; t < T; ++t) {
      for (int j = 0; j < m; ++j) vs[t * m + j] = u[t * m + j] + (double)eps[((int64_t)t * m + j) * ldk + k];
      for (int i = 0; i < n; ++i) xs[(t + 1) * n + i] = xs[t * n + i];
      orc_step(P, xs + (t + 1) * n, vs + t * m);
    }
    double mu[5], mu0[5], c = 0.0, cb = 0.0;
    const double* xT = xs + T * n;
    const double* rT = P->ref + (int64_t)T * n;
    for (int i = 0; i < n; ++i) mu[i] = 2.0 * P->w[16] * P->w[i] * (xT[i] - rT[i]);
    for (int32_t t = T - 1; t >= 0; --t) {
      const double* x1 = xs + (t + 1) * n;
      const double* r1 = P->ref + (int64_t)(t + 1) * n;
      for (int i = 0; i < n; ++i) mu[i] += 2.0 * P->w[i] * (x1[i] - r1[i]);
      for (int i = 0; i < n; ++i) c += fabs(mu[i]) * fabs(x1[i]);
      step_vjp(P, xs + t * n, vs + t * m, mu, mu0, scratch, scratch + nmlp, NULL,
               cond_bf ? &cb : NULL);
      for (int i = 0; i < n; ++i) mu[i] = mu0[i];
    }
    cond[k] = c;
    if (cond_bf) cond_bf[k] = cb;
  }
  free(scratch);
  free(xs);
  free(vs);
  return 0;
}
