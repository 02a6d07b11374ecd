"""Python face of libmppi.so: a `Controller` that owns one MPPI context.

PyTorch supplies the device memory (the workspace and the x0 / u / U buffers)
and the HIP stream (torch's current stream); the arithmetic of every step of
the iteration runs in libmppi.so's kernels.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _abi
from ._abi import check, lib


def _fptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_float))


class Controller:
    """One MPPI problem instance on one GPU.

    `problem` is any object with the fields of a workload description
    (model, integrator, cost, K, T, dt, lam, sigma, seed, instance, x0, u0,
    w and the model / cost arrays).
    """

    def __init__(self, problem, device: str | torch.device = "cuda", debug: bool = False,
                 accurate_trig: bool = False, rollout: str = "auto",
                 stream: torch.cuda.Stream | None = None):
        self.device = torch.device(device)
        self.problem = problem
        n, m = int(np.asarray(problem.x0).size), int(np.asarray(problem.sigma).size)
        self.n, self.m, self.K, self.T = n, m, int(problem.K), int(problem.T)
        cfg = _abi.Config()
        cfg.abi_version = _abi.ABI_VERSION
        cfg.dynamics = _abi.DYNAMICS[problem.model]
        cfg.integrator = _abi.INTEGRATORS[problem.integrator]
        cfg.cost = _abi.COSTS[problem.cost]
        cfg.num_samples, cfg.horizon = self.K, self.T
        cfg.state_dim, cfg.control_dim = n, m
        cfg.dt = float(np.float32(problem.dt))
        cfg.lam = float(np.float32(problem.lam))
        for j in range(m):
            cfg.sigma[j] = float(problem.sigma[j])
        cfg.seed = int(problem.seed)
        cfg.instance = int(getattr(problem, "instance", 0))
        cfg.flags = ((_abi.F_DEBUG if debug else 0) | (_abi.F_ACCURATE_TRIG if accurate_trig else 0)
                     | {"auto": 0, "lane": _abi.F_ROLLOUT_LANE, "quad": _abi.F_ROLLOUT_QUAD}[rollout])
        self.cfg = cfg
        self.params, self._keep = self._params(problem)
        L = lib()
        nbytes = L.mppi_workspace_bytes(C.byref(cfg), C.byref(self.params))
        if nbytes == 0:
            raise _abi.MPPIError(_abi.MPPI_EINVAL, L.mppi_last_error().decode())
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        ctx = C.c_void_p()
        check(L.mppi_create(C.byref(cfg), C.byref(self.params), self.workspace.data_ptr(),
                            nbytes, self.stream.cuda_stream, C.byref(ctx)))
        self.ctx = ctx
        self.U = torch.empty((self.T, m), dtype=torch.float32, device=self.device)
        self.set_state(problem.x0)
        self.set_controls(problem.u0)

    # -- parameters ---------------------------------------------------------
    @staticmethod
    def _params(pb):
        p = _abi.Params()
        keep = []

        def arr(a):
            a = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
            keep.append(a)
            return _fptr(a)

        p.wheelbase = float(getattr(pb, "wheelbase", 0.0))
        p.mass = float(getattr(pb, "mass", 0.0))
        for i, v in enumerate(getattr(pb, "inertia", (0.0, 0.0, 0.0))):
            p.inertia[i] = float(v)
        p.gravity = float(getattr(pb, "gravity", 0.0))
        w = np.asarray(pb.w, np.float32)
        for i in range(32):
            p.w[i] = float(w[i])
        if getattr(pb, "mlp", None) is not None:
            p.mlp_hidden = int(pb.mlp_hidden)
            p.mlp = arr(pb.mlp)
        if getattr(pb, "ref", None) is not None:
            p.ref = arr(pb.ref)
            p.ref_len = int(np.asarray(pb.ref).size)
        if getattr(pb, "knots", None) is not None:
            p.num_segments = len(pb.knots) - 1
            p.knots = arr(pb.knots)
            p.coef = arr(pb.coef)
        if getattr(pb, "cx", None) is not None:
            p.num_circles = len(pb.cx)
            p.cx, p.cy, p.r2 = arr(pb.cx), arr(pb.cy), arr(pb.r2)
        if getattr(pb, "costmap", None) is not None:
            p.map_h, p.map_w = pb.costmap.shape
            p.map_x0, p.map_y0 = float(pb.map_x0), float(pb.map_y0)
            p.map_res = float(pb.map_res)
            p.costmap = arr(pb.costmap)
        return p, keep

    def _dev(self, a, shape) -> torch.Tensor:
        t = torch.as_tensor(np.asarray(a, np.float32) if not torch.is_tensor(a) else a)
        t = t.to(device=self.device, dtype=torch.float32).contiguous().reshape(shape)
        self._hold = t  # alive until the enqueued copy has run (stream order)
        return t

    # -- state --------------------------------------------------------------
    def set_state(self, x0) -> None:
        t = self._dev(x0, (self.n,))
        check(lib().mppi_set_state(self.ctx, t.data_ptr()))
        self._x0 = t

    def set_controls(self, u) -> None:
        t = self._dev(u, (self.T, self.m))
        check(lib().mppi_set_controls(self.ctx, t.data_ptr()))
        self._u = t

    def set_iteration(self, iteration: int) -> None:
        check(lib().mppi_set_iteration(self.ctx, int(iteration)))

    # -- the iteration ------------------------------------------------------
    def sample(self) -> None:
        check(lib().mppi_sample(self.ctx))

    def rollout(self) -> None:
        check(lib().mppi_rollout(self.ctx))

    def set_costs(self, S) -> None:
        t = self._dev(S, (self.K,))
        check(lib().mppi_set_costs(self.ctx, t.data_ptr()))
        self._S = t

    def update(self) -> None:
        check(lib().mppi_update(self.ctx))

    def iterate(self, num_iters: int = 1) -> None:
        check(lib().mppi_iterate(self.ctx, int(num_iters)))

    def controls(self) -> torch.Tensor:
        check(lib().mppi_get_controls(self.ctx, self.U.data_ptr()))
        return self.U

    # -- inspection ---------------------------------------------------------
    def noise(self) -> torch.Tensor:
        out = torch.empty((self.T, self.m, self.K), dtype=torch.float32, device=self.device)
        check(lib().mppi_get_debug(self.ctx, _abi.DEBUG_NOISE, out.data_ptr()))
        return out

    def costs(self) -> torch.Tensor:
        out = torch.empty(self.K, dtype=torch.float32, device=self.device)
        check(lib().mppi_get_debug(self.ctx, _abi.DEBUG_COSTS, out.data_ptr()))
        return out

    def weights(self) -> torch.Tensor:
        out = torch.empty(self.K, dtype=torch.float32, device=self.device)
        check(lib().mppi_get_debug(self.ctx, _abi.DEBUG_WEIGHTS, out.data_ptr()))
        return out

    def crashes(self) -> torch.Tensor:
        out = torch.empty(self.K, dtype=torch.int32, device=self.device)
        check(lib().mppi_get_debug(self.ctx, _abi.DEBUG_CRASHES, out.data_ptr()))
        return out

    def stats(self) -> dict:
        raw = torch.empty(8, dtype=torch.float32, device=self.device)
        check(lib().mppi_get_debug(self.ctx, _abi.DEBUG_STATS, raw.data_ptr()))
        self.stream.synchronize()
        f = raw.cpu().numpy()
        i = f.view(np.int32)
        return {"rho": float(f[0]), "eta": float(f[1]), "free_energy": float(f[2]),
                "ess": float(f[3]), "status": int(i[4]), "iteration": int(i[5])}

    def close(self) -> None:
        if getattr(self, "ctx", None):
            self.stream.synchronize()
            lib().mppi_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def noise(seed: int, iteration: int, instance: int, K: int, T: int, m: int, sigma,
          device="cuda") -> torch.Tensor:
    """eps[T][m][K] of the noise definition, drawn on the GPU."""
    sig = np.zeros(_abi.MAX_CONTROL, np.float32)
    sig[:m] = np.asarray(sigma, np.float32)
    out = torch.empty((T, m, K), dtype=torch.float32, device=device)
    st = torch.cuda.current_stream(out.device)
    check(lib().mppi_noise(seed, iteration, instance, K, T, m, _fptr(sig), out.data_ptr(), K,
                           st.cuda_stream))
    return out


def noise_tables(device="cuda"):
    """(r, cos, sin) Box-Muller factors for every possible input, on the GPU."""
    n = 1 << 24
    r, c, s = (torch.empty(n, dtype=torch.float32, device=device) for _ in range(3))
    st = torch.cuda.current_stream(r.device)
    check(lib().mppi_noise_tables(r.data_ptr(), c.data_ptr(), s.data_ptr(), st.cuda_stream))
    return r, c, s
