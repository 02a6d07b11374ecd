"""The captured iteration sequence: mppi_iterate(I), replayed from a
hipGraph, must give bitwise what I single iterations give, leave the last
iteration's noise and costs visible, and keep the iteration word across
replays and staged calls."""
import sys

import numpy as np
import pytest

import workloads as W

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


def _bits(a):
    return np.ascontiguousarray(a).view(np.uint32)


@pytest.mark.parametrize("I", [1, 2, 5, 10])
def test_sequence_equals_single_iterations(mppi, oracle_lib, I):
    wl = W.c2("circles", K=3000, T=50, iters=I)
    seq = mppi.Controller(wl)
    seq.iterate(I)
    one = mppi.Controller(wl)
    for _ in range(I):
        one.iterate(1)
    for name in ("controls", "costs", "noise", "weights"):
        a, b = _np(getattr(seq, name)()), _np(getattr(one, name)())
        assert np.array_equal(_bits(a), _bits(b)), name
    assert seq.stats()["iteration"] == one.stats()["iteration"] == I
    # the visible noise is the last iteration's, by the noise definition
    eps = _np(seq.noise())
    assert np.array_equal(_bits(eps), _bits(oracle_lib.workload_noise(wl, iteration=I - 1)))
    # a replay continues the iteration count
    seq.iterate(I)
    assert seq.stats()["iteration"] == 2 * I
    eps = _np(seq.noise())
    assert np.array_equal(_bits(eps), _bits(oracle_lib.workload_noise(wl, iteration=2 * I - 1)))
    seq.close()
    one.close()


def test_staged_calls_after_a_sequence(mppi, oracle_lib):
    wl = W.c2("circles", K=1000, T=30)
    c = mppi.Controller(wl)
    c.iterate(4)
    c.sample()
    eps = _np(c.noise())
    assert np.array_equal(_bits(eps), _bits(oracle_lib.workload_noise(wl, iteration=4)))
    c.rollout()
    c.update()
    assert c.stats()["iteration"] == 5
    c.iterate(3)
    assert c.stats()["iteration"] == 8
    c.close()


def test_backward_after_a_sequence(mppi):
    # the adjoint differentiates the last iteration of the sequence
    import torch
    wl = W.c5(K=300, T=20, hidden=16).replace(lam=50.0)
    uref = torch.as_tensor(W.c5_uref(T=20), device="cuda")
    a = mppi.Controller(wl, requires_grad=True)
    a.iterate(2)
    ga = a.backward(2.0 * (a.controls() - uref))
    b = mppi.Controller(wl, requires_grad=True)
    b.iterate(1)
    b.iterate(1)
    gb = b.backward(2.0 * (b.controls() - uref))
    assert torch.equal(ga, gb)
    a.close()
    b.close()
