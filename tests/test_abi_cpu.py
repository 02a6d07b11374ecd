"""The C ABI without a GPU: the library loads, exports every function that
include/mppi.h declares, and rejects invalid configurations synchronously
(mppi_workspace_bytes validates without touching the device)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def abi():
    from paper_2409_07563_amd import _abi
    _abi.lib()
    return _abi


def header_functions():
    text = open(os.path.join(ROOT, "include", "mppi.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mppi_[a-z_]+)\s*\(", text)))


def test_every_declared_function_is_exported(abi):
    names = header_functions()
    assert len(names) >= 17, names
    L = abi.lib()
    for n in names:
        assert hasattr(L, n), n
        assert n in abi.EXPORTS, f"{n} missing from the binding"
    assert sorted(abi.EXPORTS) == names  # and the binding declares nothing else


def test_ceilings_library_exports_its_header():
    """The measurement library (include/mppi_ceilings.h) loads without a GPU
    and exports exactly what its header declares."""
    from paper_2409_07563_amd import ceilings
    text = open(os.path.join(ROOT, "include", "mppi_ceilings.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = sorted(set(re.findall(r"\b(mppi_[a-z_]+)\s*\(", text)))
    L = ceilings.lib()
    for n in names:
        assert hasattr(L, n), n
    assert sorted(ceilings.EXPORTS) == names
    # invalid arguments are refused before any device call
    us, ops = C.c_double(), C.c_double()
    assert L.mppi_ceiling_valu(7, 1, 1, 1, None, None, C.byref(us), C.byref(ops)) == -1
    assert L.mppi_ceiling_chain(0, 1, None, None, None, C.byref(us)) == -1
    assert L.mppi_ceiling_chain(257, 1, None, None, None, C.byref(us)) == -1
    assert L.mppi_ceiling_graph(0, 1, 1, None, C.byref(us)) == -1


def test_struct_sizes_match_the_header(abi):
    # sizes of the C structs as laid out by the host compiler
    assert C.sizeof(abi.Config) == 96
    assert C.sizeof(abi.Params) == 288
    assert C.sizeof(abi.Tuning) == 36


def _bytes(abi, wl, grad=False, ckpt=0, **cfg_override):
    from paper_2409_07563_amd import controller
    cfg = controller._config(wl, False, False, "auto", grad)
    for k, v in cfg_override.items():
        setattr(cfg, k, v)
    keep = []
    params = controller._params(wl, keep, ckpt)
    n = abi.lib().mppi_workspace_bytes(C.byref(cfg), C.byref(params))
    return n, abi.lib().mppi_last_error().decode()


def test_workspace_size_for_valid_configs(abi):
    for wl in (W.c1(), W.c2("circles", K=8192), W.c2("costmap"), W.c3(K=4096, T=50)):
        n, msg = _bytes(abi, wl)
        ldk = (wl.K + 63) // 64 * 64
        eps_bytes = 4 * wl.T * wl.m * ldk
        assert n >= 2 * eps_bytes, (wl.name, n, msg)
        # two noise buffers, the split form's trajectories (at most 16 words
        # per step and sample) and a few MiB of tables
        assert n < 2 * eps_bytes + 4 * wl.T * 16 * ldk + (8 << 20)
    # above 64 MiB of noise a single context keeps one noise buffer: one more
    # step of horizon past the threshold drops the second buffer
    on, _ = _bytes(abi, W.c2("circles", K=8192, T=1024))   # 64 MiB per buffer
    off, _ = _bytes(abi, W.c2("circles", K=8192, T=1025))
    assert 0 < off < on - (60 << 20), (on, off)


@pytest.mark.parametrize("override,needle", [
    ({"abi_version": 99}, "abi_version"), ({"num_samples": 0}, "num_samples"),
    ({"horizon": 0}, "horizon"), ({"lam": 0.0}, "lambda"), ({"lam": float("nan")}, "lambda"),
    ({"dt": -1.0}, "dt"), ({"state_dim": 3}, "dims"), ({"dynamics": 9}, "dynamics"),
    ({"cost": 3}, "not defined"), ({"num_samples": (1 << 20) + 1}, "num_samples")])
def test_invalid_configs_rejected(abi, override, needle):
    n, msg = _bytes(abi, W.c2("circles", K=256, T=10), **override)
    assert n == 0 and needle in msg, msg


def test_batch_workspace_and_mismatch(abi):
    from paper_2409_07563_amd import controller
    insts = W.c4(n_instances=5)
    keep = []
    cfgs = (abi.Config * 5)(*[controller._config(w, False, False, "auto") for w in insts])
    params = (abi.Params * 5)(*[controller._params(w, keep) for w in insts])
    n = abi.lib().mppi_batch_workspace_bytes(cfgs, params, 5)
    eps = sum(4 * w.T * w.m * ((w.K + 63) // 64 * 64) for w in insts)
    # a single context also reserves the split rollout form's trajectory
    # buffer ([T][5][ldk] for the bicycle) and a second noise buffer, which a
    # batch does not have
    traj = sum(4 * w.T * 5 * ((w.K + 63) // 64 * 64) for w in insts)
    singles = sum(_bytes(abi, w)[0] for w in insts)
    assert n > 0 and eps <= n and n >= 0.9 * (singles - traj - eps) and n < singles
    assert abi.lib().mppi_batch_workspace_bytes(cfgs, params, 0) == 0


def test_invalid_params_rejected(abi):
    wl = W.c2("circles", K=256, T=10)
    wl.knots = wl.knots[::-1].copy()
    n, msg = _bytes(abi, wl)
    assert n == 0 and "knots" in msg
    wl = W.c3(K=64, T=4)
    wl.mass = 0.0
    n, msg = _bytes(abi, wl)
    assert n == 0 and "mass" in msg
    n, msg = _bytes(abi, W.c1(K=64, T=4).replace(ref=None))
    assert n == 0 and "ref" in msg


def test_mlp_and_grad_configs(abi):
    wl = W.c5(K=8192, T=100)
    n, msg = _bytes(abi, wl)
    assert n > 0, msg
    ng, msg = _bytes(abi, wl, grad=True)
    # checkpoints (T / c = 10 segments x 7 x K floats) and one partial gradient
    # per 16 samples
    assert ng > n + 4 * 7 * 10 * 8192 + 4 * (8192 // 16) * 5003, msg
    assert _bytes(abi, wl.replace(model="bicycle", mlp=None, mlp_hidden=0), grad=True)[0] > 0
    for bad, needle in ((wl.replace(mlp_hidden=48), "hidden"),
                        (wl.replace(mlp=None), "weight blob"),
                        (wl.replace(cost="path_circles"), "not built"),
                        (wl.replace(wheelbase=0.0), "wheelbase")):
        n, msg = _bytes(abi, bad)
        assert n == 0 and needle in msg, msg
    n, msg = _bytes(abi, wl, grad=True, ckpt=65)
    assert n == 0 and "checkpoint" in msg
    n, msg = _bytes(abi, W.c1(K=64, T=4), grad=True)
    assert n == 0 and "REQUIRES_GRAD" in msg
    n, msg = _bytes(abi, wl, grad=True, integrator=0)
    assert n == 0 and "REQUIRES_GRAD" in msg
