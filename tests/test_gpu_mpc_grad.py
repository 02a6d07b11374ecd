"""GPU parity of the MPC warm-start shift and of the gradient through several
warm-started iterations (the tape of gradient mode and mppi_backward_iters),
through the C ABI, against the oracle.

The reverse pass is checked in two ways.  In isolation: the oracle's
single-iteration adjoint is chained by hand over the GPU's own iterations
(its u_i, noise and costs), dL/du_i = dL/du_{i+1} + sum_k a_k dJ_k/du_i, so the
bound is the one of tests/test_gpu_grad.py (1e-4 of the sum of |terms|).  End
to end: against the oracle's binary64 chain from u0, at a temperature where
the weights are spread (the GPU's binary32 iterations drift from the oracle's,
which the wider bound covers).
"""
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


# ---------------------------------------------------------------------------
# shift
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("steps", [0, 1, 5, 37, 50])
@pytest.mark.parametrize("fill", ["hold", "zero"])
def test_shift_single(mppi, oracle_lib, steps, fill):
    wl = W.c2("circles", K=64, T=37, iters=1)
    u = np.random.default_rng(steps).normal(size=(37, 2)).astype(np.float32)
    ctl = mppi.Controller(wl)
    ctl.set_controls(u)
    ctl.shift(steps, fill)
    U = _np(ctl.controls())
    ctl.close()
    assert np.array_equal(U.astype(np.float64), oracle_lib.shift(wl, u, steps, fill))


def test_shift_batch(mppi, oracle_lib):
    insts = [wl.replace(K=min(wl.K, 256)) for wl in W.c4(n_instances=5)]
    ctl = mppi.Controller(insts)
    us = [np.random.default_rng(i).normal(size=(wl.T, 2)).astype(np.float32)
          for i, wl in enumerate(insts)]
    ctl.set_controls(np.concatenate([u.ravel() for u in us]))
    ctl.shift(7, "zero")
    U = ctl.split(_np(ctl.controls()), 1)
    ctl.close()
    for i, wl in enumerate(insts):
        assert np.array_equal(U[i].reshape(wl.T, 2).astype(np.float64),
                              oracle_lib.shift(wl, us[i], 7, "zero"))


def test_shift_inside_an_mpc_loop(mppi, oracle_lib):
    """Iterate, shift by one, iterate from the shifted sequence: each call
    matches the oracle from the same nominal sequence."""
    wl = W.c2("circles", K=2000, T=60, iters=1)
    ctl = mppi.Controller(wl)
    u = wl.u0.astype(np.float64)
    for call in range(3):
        ctl.set_iteration(call)
        ctl.iterate(1)
        o = oracle_lib.mppi(wl, iters=1, iter0=call, u=u)
        U = _np(ctl.controls())
        parity.assert_end_to_end(oracle_lib, wl, U, _np(ctl.costs()), o["eps"], o["S"],
                                 f"call {call}", u=u)
        ctl.shift(1)
        u = oracle_lib.shift(wl, U.astype(np.float64), 1)
        assert np.array_equal(_np(ctl.controls()).astype(np.float64), u)
    ctl.close()


# ---------------------------------------------------------------------------
# the gradient through several iterations
# ---------------------------------------------------------------------------
def _c5(K, T, H, **kw):
    wl = W.c5(K=K, T=T, hidden=H if H else 16, **kw)
    if H == 0:
        wl = wl.replace(model="bicycle", mlp=None, mlp_hidden=0)
    return wl


def _staged(mppi, wl, iters, block=None):
    """Run `iters` staged iterations in gradient mode, keeping each one's u,
    noise and costs."""
    ctl = mppi.Controller(wl, requires_grad=True)
    if block:
        ctl.set_tuning(rollout_block=block)
    rec = []
    for _ in range(iters):
        u = _np(ctl.controls()).astype(np.float64)
        ctl.sample()
        ctl.rollout()
        rec.append((u, _np(ctl.noise()), _np(ctl.costs()).astype(np.float64)))
        ctl.update()
    return ctl, rec


def _chain(oracle_lib, wl, rec, G):
    grad = np.zeros(oracle_lib.n_grad(wl))
    gabs = np.zeros_like(grad)
    dabs = np.zeros((wl.T, wl.m))
    for u, eps, S in reversed(rec):
        r = oracle_lib.backward(wl, G, u=u, eps=eps, S=S)
        grad += r["grad"]
        gabs += r["grad_abs"]
        dabs += r["du_abs"]
        G = G + r["du"]
    return grad, gabs, G, dabs


@pytest.mark.parametrize("H,iters,lam,is_beta,gamma,block", [
    (64, 1, 50.0, 0, 1.0, 256), (64, 3, 50.0, 0, 1.0, 256), (64, 2, 5.0, 1, 0.6, 64),
    (16, 3, 50.0, 1, 0.8, None), (0, 4, 20.0, 0, 1.0, None), (32, 2, 50.0, 0, 1.0, 128)])
def test_backward_iters_vs_chained_oracle(mppi, oracle_lib, H, iters, lam, is_beta, gamma, block):
    wl = _c5(700, 30, H).replace(lam=lam, is_beta=is_beta, gamma=gamma)
    wl = wl.replace(u0=np.random.default_rng(H + iters).normal(0, 0.2, (30, 2)).astype(np.float32))
    uref = W.c5_uref(T=30)
    ctl, rec = _staged(mppi, wl, iters, block)
    ctl.set_controls(wl.u0)       # the tape restarts: run again through iterate()
    ctl.set_iteration(0)
    ctl.iterate(iters)
    U = _np(ctl.controls()).astype(np.float64)
    G = 2.0 * (U - uref)
    g, du0 = ctl.backward_iters(G.astype(np.float32))
    g, du0 = _np(g).astype(np.float64), _np(du0).astype(np.float64)
    ctl.close()
    grad, gabs, G0, dabs = _chain(oracle_lib, wl, rec, G)
    tol = 1e-4 * gabs + 1e-3 * 1e-4 * gabs.max()
    bad = np.flatnonzero(np.abs(g - grad) > tol)
    assert bad.size == 0, (f"grad: {bad.size} off, first {bad[:5]}: gpu {g[bad[:5]]} "
                           f"oracle {grad[bad[:5]]}")
    dtol = 1e-4 * (np.abs(G) + dabs) + 1e-7 * (np.abs(G) + dabs).max()
    assert np.all(np.abs(du0 - G0) <= dtol), np.abs(du0 - G0).max() / dtol.max()


def test_one_taped_iteration_is_the_single_backward(mppi):
    wl = _c5(512, 25, 64).replace(lam=50.0)
    uref = W.c5_uref(T=25)
    ctl = mppi.Controller(wl, requires_grad=True)
    ctl.iterate(1)
    U = ctl.controls()
    G = 2.0 * (U - __import__("torch").as_tensor(uref, device=U.device, dtype=U.dtype))
    a = _np(ctl.backward(G))
    b, du0 = ctl.backward_iters(G)
    assert np.array_equal(a.view(np.uint32), _np(b).view(np.uint32))
    ctl.close()


def test_last_iteration_in_place_or_rebuilt(mppi):
    """The reverse pass takes the last update from the buffers when they still
    hold it and rebuilds it otherwise (a second reverse pass, or a rollout
    after the update): the gradients agree bitwise."""
    from paper_2409_07563_amd import _abi
    wl = _c5(600, 24, 32).replace(lam=50.0)
    uref = W.c5_uref(T=24)
    ctl = mppi.Controller(wl, requires_grad=True)
    ctl.iterate(3)
    U = _np(ctl.controls())
    G = (2.0 * (U - uref)).astype(np.float32)
    first = [_np(x) for x in ctl.backward_iters(G)]      # last update in place
    again = [_np(x) for x in ctl.backward_iters(G)]      # all three rebuilt
    ctl.close()
    other = mppi.Controller(wl, requires_grad=True)
    other.iterate(3)
    other.rollout()                                      # costs of the new controls
    with pytest.raises(_abi.MPPIError):
        other.backward(G)
    rebuilt = [_np(x) for x in other.backward_iters(G)]
    other.close()
    for a, b, c in zip(first, again, rebuilt):
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
        assert np.array_equal(a.view(np.uint32), c.view(np.uint32))


def test_backward_iters_end_to_end(mppi, oracle_lib):
    wl = _c5(1024, 30, 64).replace(lam=50.0)
    uref = W.c5_uref(T=30)
    ctl = mppi.Controller(wl, requires_grad=True)
    ctl.iterate(3)
    U = _np(ctl.controls()).astype(np.float64)
    g, du0 = ctl.backward_iters((2.0 * (U - uref)).astype(np.float32))
    g, du0 = _np(g).astype(np.float64), _np(du0).astype(np.float64)
    ctl.close()
    _, U_or = oracle_lib.loss_and_controls(wl, uref, iters=3)
    r = oracle_lib.backward_iters(wl, 2.0 * (U_or - uref), 3)
    # three iterations end to end, against the oracle's own three iterations
    parity.assert_controls_close(U, U_or, parity.flat_tol(wl, U_or), "U after 3 iterations")
    scale = r["grad_abs"]
    assert np.all(np.abs(g - r["grad"]) <= 1e-3 * scale + 1e-3 * scale.max()), \
        np.max(np.abs(g - r["grad"]) / (1e-3 * scale + 1e-3 * scale.max()))
    assert np.allclose(du0, r["du0"], rtol=1e-3, atol=1e-3 * np.abs(r["du0"]).max())


def test_tape_rules(mppi):
    from paper_2409_07563_amd import _abi
    wl = _c5(128, 10, 16)
    ctl = mppi.Controller(wl, requires_grad=True, tape_len=2)
    G = np.zeros((10, 2), np.float32)
    with pytest.raises(_abi.MPPIError):
        ctl.backward_iters(G)          # no update yet
    ctl.iterate(3)
    with pytest.raises(_abi.MPPIError):
        ctl.backward_iters(G)          # three updates, two slots
    ctl.set_controls(np.zeros((10, 2), np.float32))
    ctl.iterate(2)
    ctl.backward_iters(G)              # the tape started over
    ctl.sample()
    ctl.set_costs(np.ones(128, np.float32))
    ctl.update()
    with pytest.raises(_abi.MPPIError):
        ctl.backward_iters(G)          # an update on external costs
    ctl.shift(1)
    ctl.iterate(1)
    ctl.backward_iters(G)
    ctl.close()


def test_autograd_through_iterations(mppi):
    import torch
    wl = _c5(512, 20, 16).replace(lam=50.0)
    uref = torch.as_tensor(W.c5_uref(T=20), device="cuda")
    c = mppi.Controller(wl, requires_grad=True)
    theta = c.theta().cuda().requires_grad_(True)
    u0 = torch.zeros(20, 2, device="cuda", requires_grad=True)
    U = mppi.mppi_steps(theta, u0, c, 3)
    ((U - uref) ** 2).sum().backward()
    # the same through the staged API
    ref = mppi.Controller(wl, requires_grad=True)
    ref.iterate(3)
    U2 = ref.controls()
    assert torch.equal(U.detach(), U2)
    g2, du2 = ref.backward_iters(2.0 * (U2 - uref))
    assert torch.equal(theta.grad, g2) and torch.equal(u0.grad, du2)
    c.close()
    ref.close()
