"""ctypes binding of the binary64 MPPI oracle (test infrastructure only).

Functions take a `workloads.Workload` (inputs in binary32) and widen every
input to binary64 before calling the C oracle.  Noise is drawn by the oracle's
own Philox4x32-10 + Box-Muller implementation (the noise definition is written
out in mppi_oracle.c).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libmppi_oracle.so")

MODEL_ID = {"double_integrator": 0, "bicycle": 1, "quadrotor": 2, "bicycle_mlp": 3}
INTEGRATOR_ID = {"euler": 0, "rk4": 1}
COST_ID = {"quadratic": 0, "path_circles": 1, "path_costmap": 2, "hover": 3,
           "track": 4, "goal_circles": 5}

_dp = C.POINTER(C.c_double)


class OrcProblem(C.Structure):
    _fields_ = [
        ("model", C.c_int32), ("integrator", C.c_int32), ("cost", C.c_int32),
        ("K", C.c_int32), ("T", C.c_int32), ("n", C.c_int32), ("m", C.c_int32),
        ("dt", C.c_double), ("lam", C.c_double),
        ("sigma", C.c_float * 8),
        ("seed", C.c_uint64), ("instance", C.c_uint32),
        ("wheelbase", C.c_double), ("mass", C.c_double),
        ("inertia", C.c_double * 3), ("gravity", C.c_double),
        ("mlp_hidden", C.c_int32), ("mlp", _dp),
        ("w", C.c_double * 32),
        ("ref", _dp), ("ref_len", C.c_int32),
        ("nseg", C.c_int32), ("knots", _dp), ("coef", _dp),
        ("ncirc", C.c_int32), ("cx", _dp), ("cy", _dp), ("r2", _dp),
        ("map_w", C.c_int32), ("map_h", C.c_int32),
        ("map_x0", C.c_double), ("map_y0", C.c_double), ("map_res", C.c_double),
        ("map", _dp),
        ("is_beta", C.c_int32), ("gamma", C.c_double), ("cost_cosines", C.c_int32),
        ("sigma_t", C.POINTER(C.c_float)), ("mean_sample", C.c_int32), ("zero_frac", C.c_double),
        ("mlp_bf16", C.c_int32),
    ]


_lib = None


class _opt_f64p:
    """A C-contiguous float64 array argument that may be None (NULL)."""
    _t = np.ctypeslib.ndpointer(np.float64, flags="C")

    @classmethod
    def from_param(cls, obj):
        return None if obj is None else cls._t.from_param(obj)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(_LIB_PATH)
        P = C.POINTER(OrcProblem)
        f32p = np.ctypeslib.ndpointer(np.float32, flags="C")
        f64p = np.ctypeslib.ndpointer(np.float64, flags="C")
        u32p = np.ctypeslib.ndpointer(np.uint32, flags="C")
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C")
        L.orc_philox4x32.argtypes = [u32p, u32p, C.c_int, u32p]
        L.orc_philox_many.argtypes = [C.c_int64, u32p, u32p, u32p]
        L.orc_bm_radius.argtypes = [C.c_uint32]
        L.orc_bm_radius.restype = C.c_float
        L.orc_bm_tables.argtypes = [f32p, f32p, f32p]
        L.orc_noise.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_int32, C.c_int32,
                                C.c_int32, f32p, C.c_int64, f32p]
        L.orc_rollout_costs.argtypes = [P, f64p, f64p, f32p, C.c_int64, f64p, f64p, i32p, f64p]
        # the same entry with raw pointers, for sample ranges of a larger noise array
        Lr = C.CDLL(_LIB_PATH)
        Lr.orc_rollout_costs.argtypes = [P, f64p, f64p, C.c_void_p, C.c_int64, C.c_void_p,
                                         C.c_void_p, C.c_void_p, C.c_void_p]
        L._ranged = Lr
        L.orc_softmin_update.argtypes = [P, f64p, f32p, C.c_int64, f64p, f64p, f64p, f64p]
        L.orc_softmin_update.restype = C.c_int
        L.orc_mppi.argtypes = [P, f64p, f64p, C.c_int32, C.c_uint32, f32p, f64p, f64p, f64p]
        L.orc_mppi.restype = C.c_int
        L.orc_backward.argtypes = [P, f64p, f64p, f32p, f64p, _opt_f64p, _opt_f64p, f64p,
                                   _opt_f64p, f64p, f64p, f64p, _opt_f64p, _opt_f64p]
        L.orc_backward.restype = C.c_int
        L.orc_backward_iters.argtypes = [P, f64p, f64p, C.c_int32, C.c_uint32, f64p, f64p,
                                         _opt_f64p, _opt_f64p, _opt_f64p]
        L.orc_backward_iters.restype = C.c_int
        L.orc_cost_condition.argtypes = [P, f64p, f64p, f32p, C.c_int64, f64p, _dp]
        L.orc_mlp_vjp.argtypes = [P, f64p, f64p, f64p, f64p]
        L.orc_bf16.argtypes = [C.c_double]
        L.orc_bf16.restype = C.c_double
        L.orc_cost_condition.restype = C.c_int
        L.orc_shift.argtypes = [P, f64p, C.c_int32, C.c_int32]
        L.orc_sample.argtypes = [P, C.c_uint32, C.c_int64, f32p]
        L.orc_trajectory.argtypes = [P, f64p, f64p, f64p]
        L.orc_sequence_cost.argtypes = [P, f64p, f64p]
        L.orc_sequence_cost.restype = C.c_double
        L.orc_sequence_cost_injected.argtypes = [P, f64p, f64p, C.c_int32, C.c_int32, C.c_double]
        L.orc_sequence_cost_injected.restype = C.c_double
        L.orc_eval_running_cost.argtypes = [P, f64p, f64p, C.c_int32]
        L.orc_eval_running_cost.restype = C.c_double
        L.orc_eval_terminal_cost.argtypes = [P, f64p]
        L.orc_eval_terminal_cost.restype = C.c_double
        L.orc_eval_deriv.argtypes = [P, f64p, f64p, f64p]
        L.orc_step.argtypes = [P, f64p, f64p]
        L.orc_eval_spline.argtypes = [P, C.c_double, _dp, _dp]
        L.orc_eval_costmap.argtypes = [P, C.c_double, C.c_double]
        L.orc_eval_costmap.restype = C.c_double
        _lib = L
    return _lib


def _d(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


class Problem:
    """An OrcProblem plus the binary64 arrays it points into."""

    def __init__(self, wl, keep_f64: bool = False, **override):
        self.wl = wl
        r32 = (lambda v: float(v)) if keep_f64 else (lambda v: float(np.float32(v)))
        p = OrcProblem()
        p.model = MODEL_ID[wl.model]
        p.integrator = INTEGRATOR_ID[wl.integrator]
        p.cost = COST_ID[wl.cost]
        p.K, p.T, p.n, p.m = wl.K, wl.T, wl.n, wl.m
        p.dt = float(np.float32(wl.dt))
        p.lam = float(override.get("lam", np.float32(wl.lam)))
        for j in range(wl.m):
            p.sigma[j] = float(wl.sigma[j])
        p.seed = wl.seed
        p.instance = wl.instance
        p.wheelbase = r32(wl.wheelbase)
        p.mass = float(np.float32(wl.mass))
        for i in range(3):
            p.inertia[i] = float(np.float32(wl.inertia[i]))
        p.gravity = float(np.float32(wl.gravity))
        p.is_beta = int(getattr(wl, "is_beta", 0))
        p.gamma = float(np.float32(getattr(wl, "gamma", 1.0)))
        p.cost_cosines = int(getattr(wl, "cost_cosines", 0))
        p.mean_sample = int(getattr(wl, "mean_sample", 0))
        p.mlp_bf16 = int(getattr(wl, "mlp_bf16", 0))
        p.zero_frac = float(np.float32(getattr(wl, "zero_frac", 0.0)))
        sig_t = getattr(wl, "sigma_t", None)
        if sig_t is not None:
            st = np.ascontiguousarray(np.asarray(sig_t, np.float32).ravel())
            self._sigma_t = st
            p.sigma_t = st.ctypes.data_as(C.POINTER(C.c_float))
        for i in range(32):
            p.w[i] = float(wl.w[i])
        self._keep = []

        def ptr(a):
            if a is None:
                return None
            a = _d(a).ravel()
            self._keep.append(a)
            return a.ctypes.data_as(_dp)

        if wl.mlp is not None:
            p.mlp_hidden = wl.mlp_hidden
            p.mlp = ptr(wl.mlp)
        if wl.ref is not None:
            p.ref = ptr(wl.ref)
            p.ref_len = int(np.asarray(wl.ref).size)
        if wl.knots is not None:
            p.nseg = len(wl.knots) - 1
            p.knots = ptr(wl.knots)
            p.coef = ptr(wl.coef)
        if wl.cx is not None:
            p.ncirc = len(wl.cx)
            p.cx, p.cy, p.r2 = ptr(wl.cx), ptr(wl.cy), ptr(wl.r2)
        if wl.costmap is not None:
            p.map_h, p.map_w = wl.costmap.shape
            p.map_x0, p.map_y0 = float(np.float32(wl.map_x0)), float(np.float32(wl.map_y0))
            p.map_res = float(np.float32(wl.map_res))
            p.map = ptr(wl.costmap)
        self.p = p

    @property
    def ref(self):
        return C.byref(self.p)


# --------------------------------------------------------------------------
# Noise
# --------------------------------------------------------------------------
def philox(ctrs: np.ndarray, key) -> np.ndarray:
    """Philox4x32-10 blocks for counters ctrs[n][4] under key (k0, k1)."""
    ctrs = np.ascontiguousarray(ctrs, dtype=np.uint32).reshape(-1, 4)
    out = np.empty_like(ctrs)
    lib().orc_philox_many(len(ctrs), ctrs, np.asarray(key, np.uint32), out)
    return out


def bm_tables():
    """(r[j1-1] for j1 in 1..2^24, cos[j2], sin[j2] for j2 in 0..2^24-1)."""
    n = 1 << 24
    r, c, s = (np.empty(n, np.float32) for _ in range(3))
    lib().orc_bm_tables(r, c, s)
    return r, c, s


def noise(seed: int, iteration: int, instance: int, K: int, T: int, m: int,
          sigma) -> np.ndarray:
    """eps[T][m][K] (binary32) of the noise definition."""
    eps = np.empty((T, m, K), np.float32)
    sig = np.zeros(8, np.float32)
    sig[:m] = sigma
    lib().orc_noise(seed, iteration, instance, K, T, m, sig, K, eps)
    return eps


def workload_noise(wl, iteration: int = 0) -> np.ndarray:
    """eps[T][m][K] of an iteration of the workload, with its sampling options
    (per-step sigma, noiseless mean sample)."""
    P = Problem(wl)
    eps = np.empty((wl.T, wl.m, wl.K), np.float32)
    lib().orc_sample(P.ref, iteration, wl.K, eps)
    return eps


# --------------------------------------------------------------------------
# Algorithm 1
# --------------------------------------------------------------------------
def rollout_costs(wl, eps=None, x0=None, u=None, iteration: int = 0, slope=False,
                  **override):
    """(S[K], margin[K], crashes[K]) of the rollout stage, plus the costmap
    slope exposure slope[K] when slope=True."""
    P = Problem(wl, **override)
    if eps is None:
        eps = workload_noise(wl, iteration)
    eps = np.ascontiguousarray(eps, np.float32)
    x0 = _d(wl.x0 if x0 is None else x0)
    u = _d(wl.u0 if u is None else u).ravel()
    S = np.empty(wl.K)
    margin = np.empty(wl.K)
    crashes = np.empty(wl.K, np.int32)
    sl = np.empty(wl.K)
    lib().orc_rollout_costs(P.ref, x0, u, eps, eps.shape[-1], S, margin, crashes, sl)
    if slope:
        return S, margin, crashes, sl
    return S, margin, crashes


def host_threads() -> int:
    """Worker threads for the sample-parallel oracle: the CPUs this process
    may run on, at most 16."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def rollout_costs_parallel(wl, eps, x0=None, u=None, threads=None, **override):
    """S[K] of the rollout stage, the samples split into contiguous ranges
    that run concurrently on `threads` host threads (default host_threads()).
    Each range is the same oracle call on its own samples (the samples are
    independent), so S is bitwise the single-threaded result."""
    import threading
    threads = threads or host_threads()
    eps = np.ascontiguousarray(eps, np.float32)
    K = eps.shape[-1]
    x0 = _d(wl.x0 if x0 is None else x0)
    u = _d(wl.u0 if u is None else u).ravel()
    S = np.empty(K)
    bounds = np.linspace(0, K, min(threads, K) + 1).astype(np.int64)
    L = lib()._ranged
    probs = []
    errors = []

    def work(a, b):
        try:
            P = Problem(wl.replace(K=int(b - a)), **override)
            probs.append(P)
            L.orc_rollout_costs(P.ref, x0, u, eps.ctypes.data + 4 * int(a), K,
                                S.ctypes.data + 8 * int(a), None, None, None)
        except Exception as e:  # noqa: BLE001
            errors.append(e)
    ts = [threading.Thread(target=work, args=(bounds[i], bounds[i + 1]))
          for i in range(len(bounds) - 1) if bounds[i + 1] > bounds[i]]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    if errors:
        raise errors[0]
    return S


def softmin_update(wl, S, eps, u=None, **override):
    """(w[K], U[T][m], stats[4], status) of the weighting and update stage."""
    P = Problem(wl, **override)
    eps = np.ascontiguousarray(eps, np.float32)
    u = _d(wl.u0 if u is None else u).ravel()
    w = np.empty(wl.K)
    U = np.empty(wl.T * wl.m)
    stats = np.empty(4)
    rc = lib().orc_softmin_update(P.ref, _d(S), eps, eps.shape[-1], u, w, U, stats)
    return w, U.reshape(wl.T, wl.m), stats, rc


def mppi(wl, iters=None, iter0: int = 0, u=None, x0=None, **override):
    """Run `iters` warm-started iterations; returns a dict with the final U and
    the last iteration's eps, S, w and stats."""
    P = Problem(wl, **override)
    iters = wl.iters if iters is None else iters
    u = _d(wl.u0 if u is None else u).ravel().copy()
    x0 = _d(wl.x0 if x0 is None else x0)
    eps = np.empty((wl.T, wl.m, wl.K), np.float32)
    S = np.empty(wl.K)
    w = np.empty(wl.K)
    stats = np.empty(4)
    rc = lib().orc_mppi(P.ref, x0, u, iters, iter0, eps, S, w, stats)
    return {"U": u.reshape(wl.T, wl.m), "eps": eps, "S": S, "w": w, "stats": stats,
            "status": rc}


def shift(wl, u, steps: int, fill: str = "hold"):
    """The MPC warm start: u[t] <- u[t + steps], the tail held at the last
    control (fill "hold") or zero ("zero").  Returns a new [T][m] array."""
    P = Problem(wl)
    out = _d(u).ravel().copy()
    lib().orc_shift(P.ref, out, int(steps), {"hold": 0, "zero": 1}[fill])
    return out.reshape(wl.T, wl.m)


def n_grad(wl) -> int:
    """Length of the gradient vector: [MLP blob | Q diag (n) | wheelbase]."""
    H = wl.mlp_hidden if wl.model == "bicycle_mlp" else 0
    nmlp = 7 * H + H + H * H + H + 5 * H + 5 if H else 0
    return nmlp + wl.n + 1


def backward(wl, dL_dU, u=None, x0=None, eps=None, iteration: int = 0, S=None, rel=None):
    """dL/dtheta (layout [MLP blob | Q diag | wheelbase]) of a loss on the
    controls of one iteration, given dL/dU; plus U, S, w of that iteration and
    grad_abs = sum_k rel_k |a_k dJ_k/dtheta| (rel_k = 1 by default).  S
    (optional): costs that form the weights in place of the oracle's own
    rollout costs."""
    P = Problem(wl)
    if eps is None:
        eps = workload_noise(wl, iteration)
    eps = np.ascontiguousarray(eps, np.float32)
    u = _d(wl.u0 if u is None else u).ravel()
    x0 = _d(wl.x0 if x0 is None else x0)
    grad = np.zeros(n_grad(wl))
    grad_abs = np.zeros(n_grad(wl))
    U = np.empty(wl.T * wl.m)
    S_out = np.empty(wl.K)
    w = np.empty(wl.K)
    S_in = None if S is None else _d(S).ravel()
    rel_in = None if rel is None else _d(rel).ravel()
    du = np.empty(wl.T * wl.m)
    du_abs = np.empty(wl.T * wl.m)
    rc = lib().orc_backward(P.ref, x0, u, eps, _d(dL_dU).ravel(), S_in, rel_in, grad, grad_abs, U,
                            S_out, w, du, du_abs)
    if rc == -1:
        raise ValueError("backward needs a bicycle model with RK4 and the track cost")
    return {"grad": grad, "grad_abs": grad_abs, "U": U.reshape(wl.T, wl.m), "S": S_out, "w": w,
            "du": du.reshape(wl.T, wl.m), "du_abs": du_abs.reshape(wl.T, wl.m), "status": rc}


def backward_iters(wl, dL_dU, iters: int, u=None, x0=None, iter0: int = 0):
    """Gradient through `iters` warm-started iterations from u (default
    wl.u0): {"grad": dL/dtheta, "grad_abs", "du0": dL/du0, "U": u_iters,
    "status"} for a loss with dL/du_iters = dL_dU."""
    P = Problem(wl)
    u = _d(wl.u0 if u is None else u).ravel()
    x0 = _d(wl.x0 if x0 is None else x0)
    grad = np.zeros(n_grad(wl))
    grad_abs = np.zeros(n_grad(wl))
    du0 = np.empty(wl.T * wl.m)
    U = np.empty(wl.T * wl.m)
    rc = lib().orc_backward_iters(P.ref, x0, u, int(iters), int(iter0), _d(dL_dU).ravel(), grad,
                                  grad_abs, du0, U)
    if rc == -1:
        raise ValueError("backward needs a bicycle model with RK4 and the track cost")
    return {"grad": grad, "grad_abs": grad_abs, "du0": du0.reshape(wl.T, wl.m),
            "U": U.reshape(wl.T, wl.m), "status": rc}


def cost_condition(wl, eps=None, x0=None, u=None, iteration: int = 0, bf: bool = False):
    """cond[K]: first-order sensitivity of each J_k to a relative perturbation
    of every state component at every step (sum_t,i |dJ_k/dx_t,i| |x_t,i|).
    bf: also cond_bf[K], the same sum over the inputs of the MLP's products
    (z, h1, h2 as consumed; returns (cond, cond_bf))."""
    P = Problem(wl)
    if eps is None:
        eps = workload_noise(wl, iteration)
    eps = np.ascontiguousarray(eps, np.float32)
    cond = np.empty(wl.K)
    cond_bf = np.zeros(wl.K) if bf else None
    rc = lib().orc_cost_condition(P.ref, _d(wl.x0 if x0 is None else x0),
                                  _d(wl.u0 if u is None else u).ravel(), eps, eps.shape[-1], cond,
                                  None if cond_bf is None else cond_bf.ctypes.data_as(_dp))
    if rc == -1:
        raise ValueError("cost_condition needs a bicycle model with RK4 and the track cost")
    return (cond, cond_bf) if bf else cond


def bf16(x):
    """The oracle's bfloat16 rounding (binary32 first, then 8 significand
    bits, ties to even) of each element, as binary64."""
    f = lib().orc_bf16
    a = np.asarray(x, np.float64)
    return np.array([f(float(v)) for v in a.ravel()]).reshape(a.shape)


def with_theta(wl, theta):
    """The workload with its parameters set from a vector in the gradient layout."""
    theta = np.asarray(theta, np.float64)
    H = wl.mlp_hidden if wl.model == "bicycle_mlp" else 0
    nmlp = 7 * H + H + H * H + H + 5 * H + 5 if H else 0
    w = wl.w.astype(np.float64).copy()
    w[:wl.n] = theta[nmlp:nmlp + wl.n]
    return wl.replace(mlp=theta[:nmlp].copy() if H else wl.mlp, w=w,
                      wheelbase=float(theta[nmlp + wl.n]))


def theta_of(wl):
    parts = [np.asarray(wl.mlp, np.float64)] if wl.model == "bicycle_mlp" else []
    parts += [wl.w[:wl.n].astype(np.float64), [float(np.float32(wl.wheelbase))]]
    return np.concatenate(parts)


def loss_and_controls(wl, u_ref, theta=None, iteration: int = 0, iters: int = 1, u0=None):
    """(L, U) with L = |U - u_ref|^2 after `iters` warm-started iterations
    from u0 (default wl.u0) at parameters theta (binary64 throughout: theta
    and u0 are not rounded to binary32)."""
    w2 = wl if theta is None else with_theta(wl, theta)
    P = Problem(w2, keep_f64=True)
    u = _d(w2.u0 if u0 is None else u0).ravel().copy()
    eps = np.empty((w2.T, w2.m, w2.K), np.float32)
    S = np.empty(w2.K)
    w = np.empty(w2.K)
    stats = np.empty(4)
    lib().orc_mppi(P.ref, _d(w2.x0), u, int(iters), iteration, eps, S, w, stats)
    U = u.reshape(w2.T, w2.m)
    return float(np.sum((U - u_ref) ** 2)), U


# --------------------------------------------------------------------------
# Single-point evaluations (model and cost unit tests)
# --------------------------------------------------------------------------
def step(wl, x, v):
    P = Problem(wl)
    x = _d(x).copy()
    lib().orc_step(P.ref, x, _d(v))
    return x


def mlp_vjp(wl, z, cg):
    """(dz[7], dtheta_mlp) of the MLP residual g at input z for dJ/dg = cg."""
    P = Problem(wl)
    H = wl.mlp_hidden
    dz = np.zeros(7)
    dm = np.zeros(14 * H + H * H + 5)
    lib().orc_mlp_vjp(P.ref, _d(z), _d(cg), dz, dm)
    return dz, dm


def deriv(wl, x, v):
    P = Problem(wl)
    d = np.empty(wl.n)
    lib().orc_eval_deriv(P.ref, _d(x), _d(v), d)
    return d


def trajectory(wl, v_seq, x0=None):
    P = Problem(wl)
    xs = np.empty((wl.T + 1, wl.n))
    lib().orc_trajectory(P.ref, _d(wl.x0 if x0 is None else x0), _d(v_seq).ravel(), xs)
    return xs


def sequence_cost(wl, v_seq, x0=None, **override):
    P = Problem(wl, **override)
    return lib().orc_sequence_cost(P.ref, _d(wl.x0 if x0 is None else x0),
                                   _d(v_seq).ravel())


def sequence_cost_injected(wl, v_seq, s: int, i: int, delta: float, x0=None):
    """Cost of one control sequence with delta added to component i of the
    state after step s (1 <= s <= T) before that state's cost is charged."""
    P = Problem(wl)
    return lib().orc_sequence_cost_injected(P.ref, _d(wl.x0 if x0 is None else x0),
                                            _d(v_seq).ravel(), int(s), int(i), float(delta))


def running_cost(wl, x, v, t=0):
    P = Problem(wl)
    return lib().orc_eval_running_cost(P.ref, _d(x), _d(v), t)


def terminal_cost(wl, x):
    P = Problem(wl)
    return lib().orc_eval_terminal_cost(P.ref, _d(x))


def spline(wl, px):
    P = Problem(wl)
    y, dy = C.c_double(), C.c_double()
    lib().orc_eval_spline(P.ref, float(px), C.byref(y), C.byref(dy))
    return y.value, dy.value


def costmap(wl, px, py):
    P = Problem(wl)
    return lib().orc_eval_costmap(P.ref, float(px), float(py))


__all__ = ["philox", "bm_tables", "noise", "workload_noise", "rollout_costs",
           "softmin_update", "mppi", "step", "deriv", "trajectory", "sequence_cost",
           "running_cost", "terminal_cost", "spline", "costmap", "Problem", "n_grad",
           "backward", "with_theta", "theta_of", "loss_and_controls",
           "cost_condition", "shift", "backward_iters", "sequence_cost_injected",
           "rollout_costs_parallel", "host_threads", "bf16", "mlp_vjp"]
