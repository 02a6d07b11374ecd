"""The segment-parallel reverse pass of mppi_backward (tuning adjoint_tiles)
against the binary64 oracle and against the per-tile sweep, through the C ABI.

With few samples of nonzero weight the checkpoint segments are swept in
parallel, in units of at most 5 steps (a segment of c steps splits into
ceil(c / 5) units; units of a ragged last segment may be empty): each unit's
costate map (the product of its step Jacobians, formed in forward mode
through the RK4 stages and the MLP, plus its running costs' share) chains the
costate from the terminal cost to every unit's end, and each unit's sweep
runs on the forward the map kernel kept for it.  Mathematically the gradient
is the per-tile sweep's; in binary32 the chained costate rounds differently,
so both are held to the oracle at the gradient bound of tests/test_gpu_grad.py
(1e-4 of sum_k |a_k dJ_k/dtheta| per parameter; at T = 100 widened per
sample by its conditioning), and to each other at the same bound.  Cases:
every hidden width (and the plain bicycle), one-wave and split sweeps, ragged
last segments, one-step segments, a single segment, many tiles (up to 128,
and beyond the row budget of 1280 / units, where the per-tile sweep runs),
the accurate trigonometry, the full horizon, the reverse pass through several
iterations (dL/du columns written per unit), the mode's threshold (above it
the per-tile sweep runs, bitwise), and the BF16 mode."""
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


def _wl(H, K, T, lam, **kw):
    wl = W.c5(K=K, T=T, hidden=H if H else 16).replace(lam=lam, **kw)
    if H == 0:
        wl = wl.replace(model="bicycle", mlp=None, mlp_hidden=0)
    return wl


def _close(g, ref, gabs, name):
    scale = 1e-4 * gabs
    tol = scale + 1e-3 * scale.max()
    err = np.abs(g - ref)
    bad = np.flatnonzero(err > tol)
    assert bad.size == 0, (f"{name}: {bad.size} of {g.size} entries off, first {bad[:5]}: "
                           f"got {g[bad[:5]]} want {ref[bad[:5]]} "
                           f"worst ratio {(err / tol).max():.3g}")


def _both(mppi, wl, ce, block=None, accurate=False, tiles=128):
    """One iteration in gradient mode; the gradient by the segment-parallel
    pass (adjoint_tiles = tiles) and by the per-tile sweep (0) on the same
    buffers."""
    c = mppi.Controller(wl, requires_grad=True, checkpoint_every=ce, accurate_trig=accurate)
    if block:
        c.set_tuning(rollout_block=block)
    c.sample()
    c.rollout()
    c.update()
    U = _np(c.controls()).astype(np.float64)
    G = (2.0 * (U - W.c5_uref(T=wl.T))).astype(np.float32)
    c.set_tuning(adjoint_tiles=tiles)
    g_par = _np(c.backward(G)).astype(np.float64)
    g_par2 = _np(c.backward(G)).astype(np.float64)
    c.set_tuning(adjoint_tiles=0)
    g_seq = _np(c.backward(G)).astype(np.float64)
    S = _np(c.costs()).astype(np.float64)
    eps = _np(c.noise())
    c.close()
    assert np.array_equal(g_par, g_par2)  # reproducible
    return g_par, g_seq, G, S, eps


@pytest.mark.parametrize("H,K,T,ce,lam,block", [
    (64, 1024, 40, 10, 50.0, 256), (64, 1024, 40, 10, 0.5, 64), (64, 1000, 40, 10, 50.0, 128),
    (16, 700, 33, 10, 50.0, None), (32, 256, 20, 7, 5.0, 128), (32, 256, 20, 7, 5.0, 64),
    (64, 100, 23, 1, 50.0, 256), (64, 333, 50, 64, 0.5, 256), (64, 333, 50, 13, 50.0, 64),
    (0, 1000, 50, 10, 0.5, None), (0, 1000, 50, 10, 50.0, None), (0, 37, 9, 4, 50.0, None),
    (64, 2048, 20, 10, 50.0, 256), (16, 1024, 40, 1, 50.0, None), (32, 500, 31, 5, 0.5, 128)])
def test_segment_parallel_vs_oracle_and_sweep(mppi, oracle_lib, H, K, T, ce, lam, block):
    wl = _wl(H, K, T, lam)
    g_par, g_seq, G, S, eps = _both(mppi, wl, ce, block)
    ref = oracle_lib.backward(wl, G.astype(np.float64), eps=eps, S=S)
    name = f"H={H} K={K} T={T} c={ce} lambda={lam} block={block}"
    _close(g_par, ref["grad"], ref["grad_abs"], "segment-parallel " + name)
    _close(g_seq, ref["grad"], ref["grad_abs"], "per-tile " + name)
    _close(g_par, g_seq, ref["grad_abs"], "segment-parallel against per-tile " + name)


@pytest.mark.parametrize("ce,lam", [(64, 50.0), (10, 50.0), (10, 5.0)])
def test_segment_parallel_full_horizon(mppi, oracle_lib, ce, lam):
    """T = 100 (the differentiable workload's horizon): part of the samples
    follow chaotic trajectories there, so each sample's share of the bound
    is widened by its own conditioning, as in the full-size gradient test of
    tests/test_gpu_grad.py; c = 64 gives 26 units (the second segment's last
    five empty) and prefixes of up to 60 rebuilt steps."""
    wl = _wl(64, 700, 100, lam)
    g_par, g_seq, G, S, eps = _both(mppi, wl, ce, 256)
    S_or = oracle_lib.rollout_costs(wl, eps)[0]
    cond = oracle_lib.cost_condition(wl, eps)
    rel = np.maximum(1e-4, parity.COND_ULPS * 2.0 ** -24 * cond / np.maximum(np.abs(S_or), 1.0))
    ref = oracle_lib.backward(wl, G.astype(np.float64), eps=eps, S=S, rel=rel)
    name = f"T=100 c={ce} lambda={lam}"
    # grad_abs already carries each sample's relative bound
    _close(g_seq, ref["grad"], 1e4 * ref["grad_abs"], "per-tile " + name)
    _close(g_par, ref["grad"], 1e4 * ref["grad_abs"], "segment-parallel " + name)
    _close(g_par, g_seq, 1e4 * ref["grad_abs"], "segment-parallel against per-tile " + name)


def test_segment_parallel_accurate_trig(mppi, oracle_lib):
    wl = _wl(16, 512, 40, 50.0)
    g_par, g_seq, G, S, eps = _both(mppi, wl, 10, accurate=True)
    ref = oracle_lib.backward(wl, G.astype(np.float64), eps=eps, S=S)
    _close(g_par, ref["grad"], ref["grad_abs"], "accurate trig")
    _close(g_par, g_seq, ref["grad_abs"], "accurate trig against per-tile")


def test_mode_threshold(mppi):
    """Above adjoint_tiles tiles of nonzero weight the per-tile sweep runs:
    the gradient is bitwise the one of adjoint_tiles = 0."""
    wl = _wl(64, 1024, 30, 50.0)  # about 1000 samples of nonzero weight
    g1, g0, *_ = _both(mppi, wl, 10, tiles=1)
    assert np.array_equal(g1, g0)


def test_split_sweep_bitwise_in_segment_mode(mppi):
    """In the segment-parallel mode too the split sweeps accumulate in the
    one-wave sweep's order: bitwise equal gradients."""
    wl = _wl(64, 600, 25, 50.0)
    grads = [_both(mppi, wl, 7, block)[0] for block in (64, 128, 256)]
    for g in grads[1:]:
        assert np.array_equal(grads[0], g)


@pytest.mark.parametrize("H,K,T,ce,lam", [(64, 512, 25, 10, 50.0), (64, 1024, 40, 10, 0.5),
                                         (16, 300, 30, 7, 50.0), (32, 256, 20, 6, 5.0)])
def test_bf16_segment_parallel_vs_oracle_and_sweep(mppi, oracle_lib, H, K, T, ce, lam):
    """The BF16 mode: the rebuild on the bfloat16 products, the tangents
    through the rounded weights (the roundings of the layer inputs taken as
    the identity, as the oracle's bfloat16 option differentiates); split and
    one-wave sweeps bitwise equal."""
    wl = _wl(H, K, T, lam).replace(mlp_bf16=1)
    runs = [_both(mppi, wl, ce, block) for block in ((64, 4 * H) if H >= 32 else (64,))]
    g_par, g_seq, G, S, eps = runs[0]
    ref = oracle_lib.backward(wl, G.astype(np.float64), eps=eps, S=S)
    name = f"bf16 H={H} K={K} T={T} c={ce} lambda={lam}"
    _close(g_par, ref["grad"], ref["grad_abs"], "segment-parallel " + name)
    _close(g_par, g_seq, ref["grad_abs"], "segment-parallel against per-tile " + name)
    for r in runs[1:]:
        assert np.array_equal(r[0], g_par) and np.array_equal(r[1], g_seq)


def test_segment_parallel_through_iterations(mppi, oracle_lib):
    """mppi_backward_iters in the segment-parallel mode: each reverse pass
    writes its dL/du columns segment by segment; gradient and dL/du0 against
    the oracle chained over the recorded iterations."""
    from tests.test_gpu_mpc_grad import _chain, _staged
    wl = _wl(64, 700, 30, 50.0, is_beta=1, gamma=0.8)
    wl = wl.replace(u0=np.random.default_rng(4).normal(0, 0.2, (30, 2)).astype(np.float32))
    ctl, rec = _staged(mppi, wl, 3)
    ctl.set_controls(wl.u0)
    ctl.set_iteration(0)
    ctl.iterate(3)
    U = _np(ctl.controls()).astype(np.float64)
    G = 2.0 * (U - W.c5_uref(T=30))
    ctl.set_tuning(adjoint_tiles=128)
    g, du0 = (_np(x).astype(np.float64) for x in ctl.backward_iters(G.astype(np.float32)))
    ctl.set_tuning(adjoint_tiles=0)
    gs, du0s = (_np(x).astype(np.float64) for x in ctl.backward_iters(G.astype(np.float32)))
    ctl.close()
    grad, gabs, G0, dabs = _chain(oracle_lib, wl, rec, G)
    _close(g, grad, gabs, "iterations, segment-parallel")
    _close(gs, grad, gabs, "iterations, per-tile")
    dtol = 1e-4 * (np.abs(G) + dabs) + 1e-7 * (np.abs(G) + dabs).max()
    assert np.all(np.abs(du0 - G0) <= dtol), np.abs(du0 - G0).max() / dtol.max()
    assert np.all(np.abs(du0s - G0) <= dtol), np.abs(du0s - G0).max() / dtol.max()


def test_adjoint_tiles_bounds(mppi):
    from paper_2409_07563_amd import MPPIError
    c = mppi.Controller(_wl(16, 64, 10, 50.0), requires_grad=True)
    assert c.tuning()["adjoint_tiles"] == 64
    for bad in (-1, 129):
        with pytest.raises(MPPIError) as e:
            c.set_tuning(adjoint_tiles=bad)
        assert e.value.status == -1  # MPPI_EINVAL
    c.set_tuning(adjoint_tiles=128)
    c.set_tuning(adjoint_tiles=0)
    c.close()
