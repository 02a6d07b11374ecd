"""Launch shapes and the autotuner on the GPU: every shape gives the results
the oracle accepts, shapes that only regroup lanes give bitwise the same
results, and the autotuner's choice is applied and cached."""
import sys

import numpy as np
import pytest

import workloads as W
from tests import parity

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _announce(request):
    print(f"\n[gpu-case] {request.node.nodeid}", file=sys.stderr, flush=True)
    yield


@pytest.fixture(scope="module")
def mppi():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_2409_07563_amd as M
    M.lib()
    return M


def _np(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def test_noise_calls_do_not_change_the_noise(mppi):
    wl = W.c2("circles", K=1000, T=37)
    c = mppi.Controller(wl)
    ref = None
    for calls in (1, 2, 4):
        c.set_tuning(noise_calls=calls)
        c.sample()
        eps = _np(c.noise())
        if ref is None:
            ref = eps
        assert np.array_equal(eps.view(np.uint32), ref.view(np.uint32))
    c.close()


def test_rollout_shapes(mppi, oracle_lib):
    wl = W.c2("circles", K=1500, T=60, iters=1)
    c = mppi.Controller(wl)
    c.sample()
    eps = _np(c.noise())
    S_or, margin, _ = oracle_lib.rollout_costs(wl, eps)
    by_lanes = {}
    for lanes in (1, 4, 8, 16):
        for block in (64, 128, 256):
            c.set_tuning(lanes_per_sample=lanes, rollout_block=block)
            c.rollout()
            S = _np(c.costs())
            parity.assert_costs_close(S.astype(np.float64), S_or, margin,
                                      name=f"lanes {lanes} block {block}")
            if lanes in by_lanes:  # the workgroup size only regroups lanes
                assert np.array_equal(S.view(np.uint32), by_lanes[lanes].view(np.uint32))
            by_lanes[lanes] = S
    c.close()


def test_batch_tiles_bitwise(mppi):
    insts = [w.replace(K=w.K // 8, T=min(w.T, 60), u0=np.zeros((min(w.T, 60), 2), np.float32))
             for w in W.c4(n_instances=5)]
    c = mppi.Controller(insts)
    ref = None
    for tile in (64, 128, 256):
        c.set_tuning(batch_tile=tile)
        c.set_controls(np.concatenate([w.u0.ravel() for w in insts]))
        c.set_iteration(0)
        c.iterate(2)
        out = (_np(c.costs()), _np(c.controls()))
        if ref is None:
            ref = out
        for a, b in zip(out, ref):
            assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), tile
    c.close()


def test_autotune_single_and_cache(mppi, tmp_path):
    wl = W.c2("circles", K=4096, T=50, iters=1)
    cache = str(tmp_path / "tune.json")
    c = mppi.Controller(wl)
    r = c.autotune(reps=3, cache=cache)
    assert not r["cached"] and r["timings"]
    phases = {t["phase"] for t in r["timings"]}
    assert {"sample", "rollout", "chosen"} <= phases
    chosen = [t for t in r["timings"] if t["phase"] == "chosen"][0]
    assert chosen["lanes"] == r["tuning"]["lanes_per_sample"]
    # the chosen rollout is the fastest one timed
    rolls = [t for t in r["timings"] if t["phase"] == "rollout"]
    best = min(rolls, key=lambda t: t["us"])
    assert (best["lanes"], best["block"]) == (chosen["lanes"], chosen["block"])
    c.iterate(1)  # still runs after tuning (graph captured with the new shape)
    c.close()
    c2 = mppi.Controller(wl)
    r2 = c2.autotune(reps=3, cache=cache)
    assert r2["cached"] and r2["tuning"] == r["tuning"]
    c2.close()


def test_autotune_batch_and_mlp(mppi):
    insts = [w.replace(K=w.K // 8) for w in W.c4(n_instances=4)]
    c = mppi.Controller(insts)
    r = c.autotune(reps=2)
    assert r["tuning"]["batch_tile"] in (64, 128, 256)
    c.iterate(1)
    c.close()
    c = mppi.Controller(W.c5(K=512, T=20, hidden=16))
    r = c.autotune(reps=2)
    assert r["tuning"]["lanes_per_sample"] == 16
    c.close()
    c = mppi.Controller(W.c5(K=512, T=20, hidden=64))
    r = c.autotune(reps=2)
    assert r["tuning"]["rollout_block"] in (64, 128, 256)
    c.close()


@pytest.mark.parametrize("H", [32, 64])
def test_split_mlp_tile_is_bitwise_the_single_wave_tile(mppi, H):
    """The MLP of a tile split over 2 or 4 waves accumulates in the same order
    as the one-wave form: the costs are bitwise equal, with and without
    checkpoints."""
    wl = W.c5(K=777, T=30, hidden=H)
    out = []
    for block in ((64, 128) if H == 32 else (64, 128, 256)):
        for grad in (False, True):
            c = mppi.Controller(wl, requires_grad=grad)
            c.set_tuning(rollout_block=block)
            c.sample()
            c.rollout()
            out.append(_np(c.costs()))
            c.close()
    for o in out[1:]:
        assert np.array_equal(o.view(np.uint32), out[0].view(np.uint32))


def test_invalid_shapes_rejected(mppi):
    from paper_2409_07563_amd import MPPIError
    c = mppi.Controller(W.c1(K=256, T=10))
    for bad in ({"rollout_block": 96}, {"batch_tile": 32}, {"noise_calls": 3},
                {"lanes_per_sample": 2}, {"lanes_per_sample": 32}):
        with pytest.raises(MPPIError):
            c.set_tuning(**bad)
    with pytest.raises(MPPIError, match="lanes per sample exist"):
        c.set_tuning(lanes_per_sample=8)  # no grouped kernel for the double integrator
    c.close()
    c = mppi.Controller(W.c5(K=64, T=10, hidden=16))
    with pytest.raises(MPPIError, match="16 lanes"):
        c.set_tuning(lanes_per_sample=1)
    with pytest.raises(MPPIError, match="16 lanes"):
        c.set_tuning(rollout_block=256)  # no split form for H = 16
    c.close()
