"""GPU parity of the two update options against the oracle, through the C ABI:
the importance-sampling term of the weights (beta = 1, section "MPPI-Generic's
MPPI Implementation", Eq. information_theoretic_weighting) and the step size
gamma of the dynamic mirror-descent update (section "Comparisons to
sampling-efficient algorithms").

The term lambda (v - u/2)' Sigma^-1 u vanishes at u = 0, so every case starts
from seeded nonzero controls.  Each rollout kernel that adds the term (one lane
per sample, 4 / 8 / 16 lanes per sample, the 16-sample tiles of the MLP
dynamics with one, two or four waves, the batched kernel) is run; the
tolerances are those of tests/parity.py, with the controls' bound scaled by
gamma.
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


def _warm(wl, seed, scale):
    u0 = np.random.default_rng(seed).normal(0.0, scale, (wl.T, wl.m)).astype(np.float32)
    return wl.replace(u0=u0)


def _cases():
    return {
        "c1": (_warm(W.c1(K=1000, T=60), 1, 0.5), None, None),
        "c3": (_warm(W.c3(K=700, T=40), 2, 0.3), None, None),
        "c2_lanes1": (_warm(W.c2("circles", K=1500, T=100, iters=1), 3, 0.5), 1, None),
        "c2_lanes4": (_warm(W.c2("circles", K=1500, T=100, iters=1), 3, 0.5), 4, None),
        "c2_lanes8": (_warm(W.c2("circles", K=1500, T=97, iters=1), 3, 0.5), 8, None),
        "c2_lanes16": (_warm(W.c2("circles", K=1500, T=93, iters=1), 3, 0.5), 16, None),
        "c5_h64_1wave": (_warm(W.c5(K=600, T=40, hidden=64), 4, 0.3), None, 64),
        "c5_h64_2waves": (_warm(W.c5(K=600, T=40, hidden=64), 4, 0.3), None, 128),
        "c5_h64_4waves": (_warm(W.c5(K=600, T=40, hidden=64), 4, 0.3), None, 256),
        "c5_h16": (_warm(W.c5(K=333, T=33, hidden=16), 5, 0.3), None, 64),
    }


CASES = _cases()


def _one_iteration(mppi, wl, lanes, block, requires_grad=False):
    ctl = mppi.Controller(wl, requires_grad=requires_grad)
    if lanes is not None:
        ctl.set_tuning(lanes_per_sample=lanes)
    if block is not None:
        ctl.set_tuning(rollout_block=block)
    ctl.sample()
    ctl.rollout()
    S = _np(ctl.costs()).astype(np.float64)
    eps = _np(ctl.noise())
    ctl.update()
    U = _np(ctl.controls())
    st = ctl.stats()
    ctl.close()
    return S, eps, U, st


@pytest.mark.parametrize("gamma", [1.0, 0.4])
@pytest.mark.parametrize("name", list(CASES))
def test_importance_sampling_and_step_size(mppi, oracle_lib, name, gamma):
    base, lanes, block = CASES[name]
    wl = base.replace(is_beta=1, gamma=gamma)
    S, eps, U, st = _one_iteration(mppi, wl, lanes, block)
    assert np.array_equal(eps.view(np.uint32), oracle_lib.workload_noise(wl).view(np.uint32))
    S_or, margin, _ = oracle_lib.rollout_costs(wl, eps=eps)
    cond = oracle_lib.cost_condition(wl, eps) if wl.model == "bicycle_mlp" else None
    parity.assert_costs_close(S, S_or, margin, f"{name} costs", cond=cond)
    # the term is really there: the costs differ from the plain ones
    S_plain, _, _ = oracle_lib.rollout_costs(wl.replace(is_beta=0), eps=eps)
    assert np.abs(S_or - S_plain).max() > parity.REL * np.abs(S_or).max()
    w_or, U_or, stats_or, rc = oracle_lib.softmin_update(wl, S_or, eps)
    assert rc == 0 and st["status"] == 0
    parity.assert_end_to_end(oracle_lib, wl, U, S, eps, S_or, f"{name} controls")


def test_zero_step_size_keeps_the_controls(mppi):
    wl = _warm(W.c2("circles", K=512, T=50, iters=1), 6, 0.5).replace(gamma=0.0, is_beta=1)
    S, eps, U, st = _one_iteration(mppi, wl, None, None)
    assert st["status"] == 0 and np.isfinite(S).all()
    assert np.array_equal(U.view(np.uint32), wl.u0.view(np.uint32))


def test_unit_step_size_is_bitwise_algorithm1(mppi):
    # gamma = 1 takes exactly the path of the plain update
    wl = W.c2("circles", K=1024, T=40, iters=1)
    a = _one_iteration(mppi, wl, None, None)
    b = _one_iteration(mppi, wl.replace(gamma=1.0), None, None)
    assert np.array_equal(a[2].view(np.uint32), b[2].view(np.uint32))


def test_warm_started_iterations_with_options(mppi, oracle_lib):
    """Three iterations from u = 0: the term switches on from the second."""
    wl = W.c2("circles", K=2000, T=100, iters=3).replace(is_beta=1, gamma=0.7)
    ctl = mppi.Controller(wl)
    u = wl.u0.astype(np.float64)
    for i in range(wl.iters):
        o = oracle_lib.mppi(wl, iters=1, iter0=i, u=u)
        ctl.set_controls(u.astype(np.float32))
        ctl.set_iteration(i)
        ctl.iterate(1)
        U = _np(ctl.controls())
        S = _np(ctl.costs())
        margin = oracle_lib.rollout_costs(wl, eps=o["eps"], u=u)[1]
        parity.assert_costs_close(S, o["S"], margin, f"iteration {i} costs")
        parity.assert_end_to_end(oracle_lib, wl, U, S, o["eps"], o["S"], f"iteration {i}", u=u)
        u = o["U"]
    ctl.close()


def test_batch_with_options(mppi, oracle_lib):
    insts = []
    for i, wl in enumerate(W.c4(n_instances=6)):
        K = min(wl.K, 600) - (i % 3) * 17
        insts.append(_warm(wl.replace(K=K), 10 + i, 0.4).replace(
            is_beta=1, gamma=(1.0, 0.5, 0.25)[i % 3]))
    ctl = mppi.Controller(insts)
    ctl.sample()
    ctl.rollout()
    S = ctl.split(_np(ctl.costs()), 2)
    eps = ctl.split(_np(ctl.noise()), 3)
    ctl.update()
    U = ctl.split(_np(ctl.controls()), 1)
    ctl.close()
    for i, wl in enumerate(insts):
        e = eps[i].reshape(wl.T, wl.m, -1)[:, :, :wl.K]
        S_or, margin, _ = oracle_lib.rollout_costs(wl, eps=e)
        parity.assert_costs_close(S[i], S_or, margin, f"instance {i}")
        parity.assert_end_to_end(oracle_lib, wl, U[i].reshape(wl.T, wl.m), S[i],
                                 np.ascontiguousarray(e), S_or, f"instance {i}")


@pytest.mark.parametrize("H,lam,gamma", [(64, 50.0, 0.5), (16, 5.0, 1.0), (0, 50.0, 0.3)])
def test_backward_with_options(mppi, oracle_lib, H, lam, gamma):
    wl = W.c5(K=700, T=30, hidden=H if H else 16).replace(lam=lam)
    if H == 0:
        wl = wl.replace(model="bicycle", mlp=None, mlp_hidden=0)
    wl = _warm(wl, 20 + H, 0.3).replace(is_beta=1, gamma=gamma)
    uref = W.c5_uref(T=30)
    c = mppi.Controller(wl, requires_grad=True)
    c.sample()
    c.rollout()
    c.update()
    U = _np(c.controls()).astype(np.float64)
    G = (2.0 * (U - uref)).astype(np.float32)
    g = _np(c.backward(G)).astype(np.float64)
    S = _np(c.costs()).astype(np.float64)
    eps = _np(c.noise())
    ref = oracle_lib.backward(wl, G.astype(np.float64), eps=eps, S=S)
    scale = 1e-4 * ref["grad_abs"]
    tol = scale + 1e-3 * scale.max()
    err = np.abs(g - ref["grad"])
    bad = np.flatnonzero(err > tol)
    assert bad.size == 0, (f"{bad.size} entries off, first {bad[:5]}: gpu {g[bad[:5]]} "
                           f"oracle {ref['grad'][bad[:5]]}")
    assert np.abs(ref["grad"]).max() > 0
    c.close()
