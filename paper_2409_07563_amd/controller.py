"""Python face of libmppi.so: a `Controller` that owns one MPPI context.

PyTorch supplies the device memory (the workspace and the x0 / u / U buffers)
and a HIP stream; the arithmetic of every step of the iteration runs in
libmppi.so's kernels.  The controller works on a stream of its own (default
priority) so that `iterate` can replay a captured hipGraph; every call first
orders that stream after torch's current stream, and every tensor it returns
is ordered back onto torch's current stream, so callers can ignore streams.

A list of problems makes a batch context: all instances advance together,
one launch per phase.  Per-instance arrays are then packed in instance order
(`offsets(kind)` gives the split points) and `split(t, kind)` unpacks them.
"""
from __future__ import annotations

import ctypes as C
from typing import Sequence

import numpy as np
import torch

from . import _abi
from ._abi import check, lib


def _fptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_float))


def _config(pb, debug: bool, accurate_trig: bool, rollout: str,
            requires_grad: bool = False) -> _abi.Config:
    n, m = int(np.asarray(pb.x0).size), int(np.asarray(pb.sigma).size)
    cfg = _abi.Config()
    cfg.abi_version = _abi.ABI_VERSION
    cfg.dynamics = _abi.DYNAMICS[pb.model]
    cfg.integrator = _abi.INTEGRATORS[pb.integrator]
    cfg.cost = _abi.COSTS[pb.cost]
    cfg.num_samples, cfg.horizon = int(pb.K), int(pb.T)
    cfg.state_dim, cfg.control_dim = n, m
    cfg.dt = float(np.float32(pb.dt))
    cfg.lam = float(np.float32(pb.lam))
    for j in range(m):
        cfg.sigma[j] = float(pb.sigma[j])
    cfg.seed = int(pb.seed)
    cfg.instance = int(getattr(pb, "instance", 0))
    cfg.flags = ((_abi.F_DEBUG if debug else 0) | (_abi.F_ACCURATE_TRIG if accurate_trig else 0)
                 | {"auto": 0, "lane": _abi.F_ROLLOUT_LANE, "quad": _abi.F_ROLLOUT_QUAD}[rollout]
                 | (_abi.F_REQUIRES_GRAD if requires_grad else 0)
                 | (_abi.F_IMPORTANCE_SAMPLING if getattr(pb, "is_beta", 0) else 0)
                 | (_abi.F_MEAN_SAMPLE if getattr(pb, "mean_sample", 0) else 0)
                 | (_abi.F_BF16_MLP if getattr(pb, "mlp_bf16", 0) else 0)
                 | _abi.F_STEP_SIZE)
    cfg.zero_mean_fraction = float(np.float32(getattr(pb, "zero_frac", 0.0)))
    # always explicit (gamma = 1 is Algorithm 1): the instances of a batch
    # share their flags but not their step sizes
    cfg.step_size = float(np.float32(getattr(pb, "gamma", 1.0)))
    return cfg


def _params(pb, keep: list, checkpoint_every: int = 0, tape_len: int = 0) -> _abi.Params:
    p = _abi.Params()
    p.checkpoint_every = int(checkpoint_every)
    p.tape_len = int(tape_len)
    p.cost_cosines = int(getattr(pb, "cost_cosines", 0))
    sig_t = getattr(pb, "sigma_t", None)

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
    if sig_t is not None:
        p.sigma_t = arr(sig_t)
    return p


class Controller:
    """One MPPI problem instance, or a batch of them, on one GPU.

    `problem` is a workload description (model, integrator, cost, K, T, dt,
    lam, sigma, seed, instance, x0, u0, w and the model / cost arrays) or a
    sequence of them (a batch sharing model, integrator and cost kind).

    requires_grad: keep what `backward` needs (state checkpoints every
    `checkpoint_every` steps and the controls of the rollout) and a tape of
    `tape_len` updates for `backward_iters`.

    static_workspace: run on the library's own per-GPU workspace
    (mppi_create_static: no device allocation for the context; one such
    controller per GPU at a time; single instances only).
    """

    def __init__(self, problem, device: str | torch.device = "cuda", debug: bool = False,
                 accurate_trig: bool = False, rollout: str = "auto",
                 stream: torch.cuda.Stream | None = None, requires_grad: bool = False,
                 checkpoint_every: int = 10, tape_len: int = 16,
                 static_workspace: bool = False):
        self.device = torch.device(device)
        self.requires_grad = bool(requires_grad)
        self.batch = isinstance(problem, (list, tuple))
        probs: Sequence = list(problem) if self.batch else [problem]
        self.problems = probs
        self.n_inst = len(probs)
        pb = probs[0]
        self.n, self.m = int(np.asarray(pb.x0).size), int(np.asarray(pb.sigma).size)
        self.K, self.T = int(pb.K), int(pb.T)
        self._keep: list = []
        cfgs = (_abi.Config * self.n_inst)(
            *[_config(q, debug, accurate_trig, rollout, requires_grad) for q in probs])
        params = (_abi.Params * self.n_inst)(
            *[_params(q, self._keep, checkpoint_every if requires_grad else 0,
                      tape_len if requires_grad else 0) for q in probs])
        self.cfg, self._cfgs, self._params = cfgs[0], cfgs, params
        L = lib()
        if self.batch:
            nbytes = L.mppi_batch_workspace_bytes(cfgs, params, self.n_inst)
        else:
            nbytes = L.mppi_workspace_bytes(C.byref(cfgs[0]), C.byref(params[0]))
        if nbytes == 0:
            raise _abi.MPPIError(_abi.MPPI_EINVAL, L.mppi_last_error().decode())
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        self._enter()
        ctx = C.c_void_p()
        if static_workspace:
            if self.batch:
                raise ValueError("static_workspace is for single instances")
            self.workspace = None
            with torch.cuda.device(self.device):
                check(L.mppi_create_static(C.byref(cfgs[0]), C.byref(params[0]),
                                           self.stream.cuda_stream, C.byref(ctx)))
        else:
            with torch.cuda.stream(self.stream):
                self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            if self.batch:
                check(L.mppi_create_batch(cfgs, params, self.n_inst, self.workspace.data_ptr(),
                                          nbytes, self.stream.cuda_stream, C.byref(ctx)))
            else:
                check(L.mppi_create(C.byref(cfgs[0]), C.byref(params[0]),
                                    self.workspace.data_ptr(), nbytes, self.stream.cuda_stream,
                                    C.byref(ctx)))
        self.ctx = ctx
        self._off = {k: self._offsets(k) for k in (_abi.PACKED_STATE, _abi.PACKED_CONTROLS,
                                                   _abi.PACKED_SAMPLES, _abi.PACKED_NOISE)}
        self.set_state(np.concatenate([np.asarray(q.x0, np.float32).ravel() for q in probs]))
        self.set_controls(np.concatenate([np.asarray(q.u0, np.float32).ravel() for q in probs]))

    # -- streams ------------------------------------------------------------
    def _enter(self):
        """Order the library's stream after torch's current stream."""
        self.stream.wait_stream(torch.cuda.current_stream(self.device))

    def _leave(self, t: torch.Tensor) -> torch.Tensor:
        """Order torch's current stream after the library's work on t."""
        cur = torch.cuda.current_stream(self.device)
        cur.wait_stream(self.stream)
        t.record_stream(cur)
        return t

    def _empty(self, shape, dtype=torch.float32) -> torch.Tensor:
        with torch.cuda.stream(self.stream):
            return torch.empty(shape, dtype=dtype, device=self.device)

    def _dev(self, a, n: int) -> torch.Tensor:
        self._enter()
        t = torch.as_tensor(np.asarray(a, np.float32) if not torch.is_tensor(a) else a)
        with torch.cuda.stream(self.stream):
            t = t.to(device=self.device, dtype=torch.float32).contiguous().reshape(n)
        return t

    # -- packing ------------------------------------------------------------
    def _offsets(self, kind: int) -> np.ndarray:
        off = (C.c_int64 * (self.n_inst + 1))()
        check(lib().mppi_offsets(self.ctx, kind, off))
        return np.array(off[:], dtype=np.int64)

    def offsets(self, kind: int) -> np.ndarray:
        return self._off[kind]

    def split(self, t, kind: int):
        """Per-instance views of a packed array."""
        off = self._off[kind]
        return [t[off[i]:off[i + 1]] for i in range(self.n_inst)]

    # -- state --------------------------------------------------------------
    def set_state(self, x0) -> None:
        t = self._dev(x0, int(self._off[_abi.PACKED_STATE][-1]))
        check(lib().mppi_set_state(self.ctx, t.data_ptr()))
        self._x0 = t  # alive until the enqueued copy has run (stream order)

    def set_controls(self, u) -> None:
        t = self._dev(u, int(self._off[_abi.PACKED_CONTROLS][-1]))
        check(lib().mppi_set_controls(self.ctx, t.data_ptr()))
        self._u = t

    def set_iteration(self, iteration: int) -> None:
        self._enter()
        check(lib().mppi_set_iteration(self.ctx, int(iteration)))

    def shift(self, steps: int, fill: str = "hold") -> None:
        """MPC warm start: u[t] <- u[t + steps]; the tail holds the last
        control ("hold") or becomes zero ("zero")."""
        self._enter()
        check(lib().mppi_shift(self.ctx, int(steps),
                               {"hold": _abi.SHIFT_HOLD, "zero": _abi.SHIFT_ZERO}[fill]))

    # -- the iteration ------------------------------------------------------
    def sample(self) -> None:
        self._enter()
        check(lib().mppi_sample(self.ctx))

    def rollout(self) -> None:
        self._enter()
        check(lib().mppi_rollout(self.ctx))

    def set_costs(self, S) -> None:
        t = self._dev(S, int(self._off[_abi.PACKED_SAMPLES][-1]))
        check(lib().mppi_set_costs(self.ctx, t.data_ptr()))
        self._S = t

    def update(self) -> None:
        self._enter()
        check(lib().mppi_update(self.ctx))

    def iterate(self, num_iters: int = 1) -> None:
        self._enter()
        check(lib().mppi_iterate(self.ctx, int(num_iters)))

    def controls(self) -> torch.Tensor:
        """U: [T, m] for one instance, packed [sum T*m] for a batch."""
        n = int(self._off[_abi.PACKED_CONTROLS][-1])
        U = self._empty(n)
        check(lib().mppi_get_controls(self.ctx, U.data_ptr()))
        return self._leave(U if self.batch else U.reshape(self.T, self.m))

    # -- launch shapes ------------------------------------------------------
    def tuning(self) -> dict:
        t = _abi.Tuning()
        check(lib().mppi_get_tuning(self.ctx, C.byref(t)))
        return t.as_dict()

    def set_tuning(self, **shape) -> None:
        """Change launch shapes (lanes_per_sample, rollout_block, batch_tile,
        noise_calls, rollout_form, cost_waves, update_form, batch_form,
        adjoint_tiles); the others keep their values."""
        t = _abi.Tuning()
        check(lib().mppi_get_tuning(self.ctx, C.byref(t)))
        for k, v in shape.items():
            if k not in t.as_dict():
                raise KeyError(k)
            setattr(t, k, int(v))
        self._enter()
        check(lib().mppi_set_tuning(self.ctx, C.byref(t)))

    def autotune(self, reps: int = 10, cache: str | None = None) -> dict:
        """Time the candidate launch shapes on this context and apply the
        fastest.  With a cache file, a stored choice for the same key (device
        architecture, dynamics, integrator, cost, K bucket, horizon, batch
        size) is applied without timing, and a new choice is stored."""
        from . import autotune as _at
        key = _at.key(self)
        if cache is not None:
            hit = _at.load(cache).get(key)
            if hit is not None:
                self.set_tuning(**hit["tuning"])
                return {"key": key, "tuning": self.tuning(), "cached": True}
        buf = C.create_string_buffer(8192)
        self._enter()
        check(lib().mppi_autotune(self.ctx, int(reps), buf, len(buf)))
        result = {"key": key, "tuning": self.tuning(), "cached": False,
                  "timings": _at.parse_report(buf.value.decode())}
        if cache is not None:
            _at.store(cache, key, result)
        return result

    # -- differentiation ----------------------------------------------------
    def theta_len(self) -> int:
        n = lib().mppi_theta_len(self.ctx)
        if n == 0:
            raise _abi.MPPIError(_abi.MPPI_ESTATE, lib().mppi_last_error().decode())
        return int(n)

    def theta(self) -> torch.Tensor:
        """theta of the problem as created: [MLP blob | Q diag | wheelbase] (CPU)."""
        pb = self.problems[0]
        parts = [np.asarray(pb.mlp, np.float32).ravel()] if pb.model == "bicycle_mlp" else []
        parts += [np.asarray(pb.w, np.float32)[:self.n], np.float32([pb.wheelbase])]
        return torch.from_numpy(np.concatenate(parts))

    def set_theta(self, theta) -> None:
        """Replace the MLP weights, the Q diagonal and the wheelbase (waits for
        the upload)."""
        t = theta.detach().to("cpu", torch.float32) if torch.is_tensor(theta) else \
            torch.as_tensor(np.asarray(theta, np.float32))
        a = np.ascontiguousarray(t.numpy().ravel(), np.float32)
        if a.size != self.theta_len():
            raise ValueError(f"theta has {a.size} entries, the context needs {self.theta_len()}")
        self._enter()
        check(lib().mppi_set_theta(self.ctx, _fptr(a)))

    def backward(self, dL_dU) -> torch.Tensor:
        """dL/dtheta of a loss on the controls of the last update."""
        g = self._dev(dL_dU, self.T * self.m)
        out = self._empty(self.theta_len())
        check(lib().mppi_backward(self.ctx, g.data_ptr(), out.data_ptr()))
        self._g = g
        return self._leave(out)

    def backward_iters(self, dL_dU):
        """(dL/dtheta, dL/du0) through every update since the tape started
        (the last set_state / set_controls / set_theta / shift)."""
        g = self._dev(dL_dU, self.T * self.m)
        out = self._empty(self.theta_len())
        du0 = self._empty(self.T * self.m)
        check(lib().mppi_backward_iters(self.ctx, g.data_ptr(), out.data_ptr(), du0.data_ptr()))
        self._g = g
        return self._leave(out), self._leave(du0).reshape(self.T, self.m)

    # -- inspection ---------------------------------------------------------
    def noise(self) -> torch.Tensor:
        n = int(self._off[_abi.PACKED_NOISE][-1])
        out = self._empty(n)
        check(lib().mppi_get_debug(self.ctx, _abi.DEBUG_NOISE, out.data_ptr()))
        return self._leave(out if self.batch else out.reshape(self.T, self.m, self.K))

    def costs(self) -> torch.Tensor:
        out = self._empty(int(self._off[_abi.PACKED_SAMPLES][-1]))
        check(lib().mppi_get_debug(self.ctx, _abi.DEBUG_COSTS, out.data_ptr()))
        return self._leave(out)

    def weights(self) -> torch.Tensor:
        out = self._empty(int(self._off[_abi.PACKED_SAMPLES][-1]))
        check(lib().mppi_get_debug(self.ctx, _abi.DEBUG_WEIGHTS, out.data_ptr()))
        return self._leave(out)

    def crashes(self) -> torch.Tensor:
        out = self._empty(int(self._off[_abi.PACKED_SAMPLES][-1]), dtype=torch.int32)
        check(lib().mppi_get_debug(self.ctx, _abi.DEBUG_CRASHES, out.data_ptr()))
        return self._leave(out)

    def stats(self):
        """dict (one instance) or list of dicts (batch): rho, eta, free energy,
        effective sample size, status word, iteration word."""
        raw = self._empty(8 * self.n_inst)
        check(lib().mppi_get_debug(self.ctx, _abi.DEBUG_STATS, raw.data_ptr()))
        self.stream.synchronize()
        f = raw.cpu().numpy().reshape(self.n_inst, 8)
        i = f.view(np.int32)
        out = [{"rho": float(f[q, 0]), "eta": float(f[q, 1]), "free_energy": float(f[q, 2]),
                "ess": float(f[q, 3]), "status": int(i[q, 4]), "iteration": int(i[q, 5])}
               for q in range(self.n_inst)]
        return out if self.batch else out[0]

    def synchronize(self) -> None:
        self.stream.synchronize()

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
    """eps[T][m][K] of the noise definition, drawn on the GPU (torch's current
    stream)."""
    sig = np.zeros(_abi.MAX_CONTROL, np.float32)
    sig[:m] = np.asarray(sigma, np.float32)
    out = torch.empty((T, m, K), dtype=torch.float32, device=device)
    st = torch.cuda.current_stream(out.device)
    check(lib().mppi_noise(seed, iteration, instance, K, T, m, _fptr(sig), out.data_ptr(), K,
                           st.cuda_stream))
    return out


def noise_tables(device="cuda"):
    """(r, cos, sin) Box-Muller factors for every possible input, on the GPU
    (torch's current stream)."""
    n = 1 << 24
    r, c, s = (torch.empty(n, dtype=torch.float32, device=device) for _ in range(3))
    st = torch.cuda.current_stream(r.device)
    check(lib().mppi_noise_tables(r.data_ptr(), c.data_ptr(), s.data_ptr(), st.cuda_stream))
    return r, c, s
