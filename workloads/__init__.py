"""Seeded synthetic MPPI workloads.

This module only *builds inputs*: initial states, nominal controls, model
constants and cost data (spline, circles, costmap, MLP weights, reference
trajectories).  It holds none of the MPPI arithmetic; both the GPU library and
the CPU oracle consume what it returns.  Every array is binary32, the precision
the GPU path computes in; the oracle widens the same values to binary64.

The paper benchmarks on a wheeled robot with a costmap obstacle cost, T = 100,
dt = 0.02 (Section V, Table 1) and uses no dataset.  The workloads here are
synthetic stand-ins of the same class:

  c1  double integrator 4/2, Euler dt 0.02, K 1024, T 100, quadratic goal cost
  c2  kinematic bicycle 5/2, RK4 dt 0.02, K 8192, T 100, 10 warm-started
      iterations, spline path tracking + 200 circular obstacles (analytic
      crash indicator, or the same scene rasterised into a 512x512 costmap)
  c3  quadrotor 13/4, RK4 dt 0.01, K 65536, T 200, hover-at-waypoint cost
  c4  256 independent bicycle instances with uneven K and T
  c5  bicycle + MLP residual dynamics, tracking cost (differentiable case)

Setup randomness uses numpy's PCG64 with seed 2000 + config id; the MPPI noise
seed (drawn by the method itself, on both sides, from the Philox counter) is
1000 + config id.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

F32 = np.float32

MODELS = {"double_integrator": (4, 2), "bicycle": (5, 2), "quadrotor": (13, 4),
          "bicycle_mlp": (5, 2)}
COSTS = ("quadratic", "path_circles", "path_costmap", "hover", "track",
         "goal_circles")


@dataclasses.dataclass
class Workload:
    name: str
    model: str
    integrator: str
    cost: str
    K: int
    T: int
    dt: float
    lam: float
    sigma: np.ndarray
    seed: int
    x0: np.ndarray
    u0: np.ndarray
    w: np.ndarray
    iters: int = 1
    instance: int = 0
    is_beta: int = 0      # importance-sampling term in the weights (0 or 1)
    gamma: float = 1.0    # step size of the update (1: plain MPPI)
    cost_cosines: int = 0 # cosines chained ahead of each running cost, times 0
    mean_sample: int = 0  # sample 0 drawn without noise (v = u)
    zero_frac: float = 0.0  # fraction of the samples drawn around zero
    sigma_t: Optional[np.ndarray] = None  # per-step noise std [T][m] (None: sigma)
    wheelbase: float = 0.0
    mass: float = 0.0
    inertia: tuple = (0.0, 0.0, 0.0)
    gravity: float = 0.0
    mlp: Optional[np.ndarray] = None
    mlp_hidden: int = 0
    mlp_bf16: int = 0     # MLP products on bfloat16 operands (binary32 accumulation)
    ref: Optional[np.ndarray] = None
    knots: Optional[np.ndarray] = None
    coef: Optional[np.ndarray] = None
    cx: Optional[np.ndarray] = None
    cy: Optional[np.ndarray] = None
    r2: Optional[np.ndarray] = None
    costmap: Optional[np.ndarray] = None
    map_x0: float = 0.0
    map_y0: float = 0.0
    map_res: float = 1.0

    @property
    def n(self) -> int:
        return MODELS[self.model][0]

    @property
    def m(self) -> int:
        return MODELS[self.model][1]

    @property
    def rollout_steps(self) -> int:
        return self.K * self.T * self.iters

    def replace(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


def _f32(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(F32))


def _weights(vals) -> np.ndarray:
    w = np.zeros(32, dtype=F32)
    for i, v in vals.items() if isinstance(vals, dict) else enumerate(vals):
        w[i] = v
    return w


# --------------------------------------------------------------------------
# c1: double integrator, quadratic goal cost
# --------------------------------------------------------------------------
def c1(K: int = 1024, T: int = 100, seed_offset: int = 0) -> Workload:
    rng = np.random.Generator(np.random.PCG64(2001 + seed_offset))
    x0 = _f32(rng.uniform(-1.0, 1.0, 4))
    q = [10.0, 10.0, 1.0, 1.0]
    w = {}
    for i in range(4):
        w[i] = q[i]
        w[16 + i] = 10.0 * q[i]
    w[8] = w[9] = 0.1
    return Workload(name="c1_double_integrator", model="double_integrator",
                    integrator="euler", cost="quadratic", K=K, T=T, dt=float(F32(0.02)),
                    lam=1.0, sigma=_f32([0.5, 0.5]), seed=1001 + seed_offset, x0=x0,
                    u0=np.zeros((T, 2), F32), w=_weights(w), ref=np.zeros(4, F32))


# --------------------------------------------------------------------------
# c2: kinematic bicycle on a spline path with circular obstacles
# --------------------------------------------------------------------------
def _spline_scene(rng, n_knots=8):
    from scipy.interpolate import CubicSpline
    kx = np.linspace(10.0, 90.0, n_knots)
    ky = rng.uniform(20.0, 80.0, n_knots)
    cs = CubicSpline(kx, ky, bc_type="natural")
    # cs.c[p, i] multiplies (x - kx[i])^(3 - p)
    coef = np.stack([cs.c[3], cs.c[2], cs.c[1], cs.c[0]], axis=1)
    return _f32(kx), _f32(coef)


def _spline_value(knots, coef, x):
    """Value and slope of the piecewise cubic (input preparation only)."""
    kn = knots.astype(np.float64)
    cf = coef.astype(np.float64)
    x = min(max(x, kn[0]), kn[-1])
    i = min(int(np.searchsorted(kn, x, side="right")) - 1, len(cf) - 1)
    d = x - kn[i]
    a, b, c, e = cf[i]
    return a + d * (b + d * (c + d * e)), b + d * (2 * c + 3 * d * e)


def _circles(rng, n, keep_clear, clear_radius=1.0, lo=0.0, hi=100.0, path=None,
             path_clearance=0.5):
    """n circles (centres U[lo, hi]^2, radii U[0.5, 2]) that keep clear of the
    given points and, if `path` (an [N][2] polyline) is given, of a corridor
    of half-width path_clearance around it."""
    cx, cy, r = [], [], []
    while len(cx) < n:
        x, y = rng.uniform(lo, hi, 2)
        rr = rng.uniform(0.5, 2.0)
        if any(math.hypot(x - px, y - py) <= rr + clear_radius for px, py in keep_clear):
            continue
        if path is not None and np.min(np.hypot(path[:, 0] - x, path[:, 1] - y)) <= rr + path_clearance:
            continue
        cx.append(x); cy.append(y); r.append(rr)
    r = np.asarray(r)
    return _f32(cx), _f32(cy), _f32(r * r)


def rasterise(cx, cy, r2, width=512, height=512, x0=0.0, y0=0.0, res=100.0 / 512,
              value=1.0e4) -> np.ndarray:
    """Costmap [height][width]: value where the cell centre lies in a circle."""
    xs = x0 + (np.arange(width) + 0.5) * res
    ys = y0 + (np.arange(height) + 0.5) * res
    gx, gy = np.meshgrid(xs, ys)
    occ = np.zeros((height, width), dtype=bool)
    for a, b, c in zip(cx.astype(np.float64), cy.astype(np.float64), r2.astype(np.float64)):
        occ |= (gx - a) ** 2 + (gy - b) ** 2 <= c
    return np.ascontiguousarray(np.where(occ, value, 0.0).astype(F32))


def c2(variant: str = "circles", K: int = 8192, T: int = 100, iters: int = 10,
       n_obstacles: int = 200, seed_offset: int = 0) -> Workload:
    rng = np.random.Generator(np.random.PCG64(2002 + seed_offset))
    knots, coef = _spline_scene(rng)
    y0, dy0 = _spline_value(knots, coef, 10.0)
    x0 = _f32([10.0, y0, math.atan(dy0), 5.0, 0.0])
    xs = np.linspace(10.0, 90.0, 4001)
    path = np.array([[x, _spline_value(knots, coef, x)[0]] for x in xs])
    cx, cy, r2 = _circles(rng, n_obstacles, [(float(x0[0]), float(x0[1]))], path=path)
    w = _weights([1.0, 1.0, 0.5, 5.0, 0.1, 0.1, 1.0e4, 10.0])
    wl = Workload(name=f"c2_bicycle_{variant}", model="bicycle", integrator="rk4",
                  cost="path_circles" if variant == "circles" else "path_costmap",
                  K=K, T=T, dt=float(F32(0.02)), lam=0.5, sigma=_f32([1.0, 0.3]),
                  seed=1002 + seed_offset, x0=x0, u0=np.zeros((T, 2), F32), w=w,
                  iters=iters, wheelbase=2.5, knots=knots, coef=coef)
    if variant == "circles":
        wl.cx, wl.cy, wl.r2 = cx, cy, r2
    else:
        wl.costmap = rasterise(cx, cy, r2)
        wl.map_x0, wl.map_y0, wl.map_res = 0.0, 0.0, 100.0 / 512
    return wl


# --------------------------------------------------------------------------
# c3: quadrotor hover at a waypoint
# --------------------------------------------------------------------------
def c3(K: int = 65536, T: int = 200, seed_offset: int = 0) -> Workload:
    rng = np.random.Generator(np.random.PCG64(2003 + seed_offset))
    p0 = rng.uniform(-1.0, 1.0, 3)
    x0 = np.zeros(13)
    x0[0:3] = p0
    x0[3] = 1.0
    g = 9.81
    u0 = np.tile(np.array([g * 1.0, 0.0, 0.0, 0.0]), (T, 1))
    ref = [0.0, 0.0, 1.0, 1.0, 0.0, 0.0, 0.0, g * 1.0, 0.0, 0.0, 0.0]
    w = _weights([10.0, 1.0, 0.1, 10.0, 0.1, 100.0, 5.0, 10.0])
    return Workload(name="c3_quadrotor", model="quadrotor", integrator="rk4",
                    cost="hover", K=K, T=T, dt=float(F32(0.01)), lam=0.1,
                    sigma=_f32([0.2, 0.2, 0.2, 0.2]), seed=1003 + seed_offset,
                    x0=_f32(x0), u0=_f32(u0), w=w, mass=1.0,
                    inertia=(0.01, 0.01, 0.02), gravity=g, ref=_f32(ref))


# --------------------------------------------------------------------------
# c5: bicycle with an MLP residual, tracking a time-indexed reference
# --------------------------------------------------------------------------
def mlp_weights(rng, hidden=64, n_in=7, n_out=5) -> np.ndarray:
    W1 = rng.normal(0.0, 1.0 / math.sqrt(n_in), (hidden, n_in))
    W2 = rng.normal(0.0, 1.0 / math.sqrt(hidden), (hidden, hidden))
    W3 = rng.normal(0.0, 1.0 / math.sqrt(hidden), (n_out, hidden))
    parts = [W1.ravel(), np.zeros(hidden), W2.ravel(), np.zeros(hidden), W3.ravel(),
             np.zeros(n_out)]
    return _f32(np.concatenate(parts))


def c5(K: int = 8192, T: int = 100, hidden: int = 64, seed_offset: int = 0) -> Workload:
    rng = np.random.Generator(np.random.PCG64(2005 + seed_offset))
    knots, coef = _spline_scene(rng)
    dt = float(F32(0.02))
    ref = np.zeros((T + 1, 5))
    for t in range(T + 1):
        x = 10.0 + 5.0 * dt * t
        y, dy = _spline_value(knots, coef, x)
        ref[t] = [x, y, math.atan(dy), 5.0, 0.0]
    x0 = _f32(ref[0])
    w = _weights({0: 1.0, 1: 1.0, 2: 1.0, 3: 0.5, 4: 0.1, 8: 0.1, 9: 0.1, 16: 10.0})
    wl = Workload(name="c5_bicycle_mlp", model="bicycle_mlp", integrator="rk4",
                  cost="track", K=K, T=T, dt=dt, lam=0.5, sigma=_f32([1.0, 0.3]),
                  seed=1005 + seed_offset, x0=x0, u0=np.zeros((T, 2), F32), w=w,
                  wheelbase=2.5, mlp=mlp_weights(rng, hidden), mlp_hidden=hidden,
                  ref=_f32(ref))
    return wl


def c5_uref(T: int = 100, seed_offset: int = 0) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(3005 + seed_offset))
    return _f32(rng.normal(0.0, 0.1, (T, 2)))


# --------------------------------------------------------------------------
# c4: many independent bicycle instances (batched)
# --------------------------------------------------------------------------
def c4(n_instances: int = 256, k_choices=(1024, 2048, 4096, 8192, 16384),
       t_choices=(50, 100, 150, 200), seed_offset: int = 0) -> List[Workload]:
    rng = np.random.Generator(np.random.PCG64(2004 + seed_offset))
    out = []
    for i in range(n_instances):
        K = int(rng.choice(k_choices))
        T = int(rng.choice(t_choices))
        n_obs = int(rng.integers(50, 301))
        lam = float(F32(rng.uniform(0.1, 2.0)))
        goal = rng.uniform(10.0, 90.0, 2)
        p0 = rng.uniform(10.0, 90.0, 2)
        yaw = rng.uniform(-math.pi, math.pi)
        x0 = _f32([p0[0], p0[1], yaw, 0.0, 0.0])
        cx, cy, r2 = _circles(rng, n_obs, [tuple(p0), tuple(goal)])
        w = _weights([0.01, 0.1, 0.1, 1.0e4, 10.0])
        out.append(Workload(name=f"c4_instance_{i}", model="bicycle", integrator="rk4",
                            cost="goal_circles", K=K, T=T, dt=float(F32(0.02)), lam=lam,
                            sigma=_f32([1.0, 0.3]), seed=1004 + seed_offset, instance=i,
                            x0=x0, u0=np.zeros((T, 2), F32), w=w, wheelbase=2.5,
                            ref=_f32(goal), cx=cx, cy=cy, r2=r2))
    return out


CONFIGS = {"c1": c1, "c2": c2, "c3": c3, "c5": c5}
