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


def _with_options(wl, seed):
    rng = np.random.default_rng(seed)
    sig_t = (np.asarray(wl.sigma, np.float64)[None, :]
             * rng.uniform(0.5, 1.5, (wl.T, wl.m))).astype(np.float32)
    return wl.replace(sigma_t=sig_t, mean_sample=1, zero_frac=0.1, is_beta=1, gamma=0.8)


# the next iteration's noise is drawn by the update of the one before, into a
# second buffer: every rollout kernel reads the right buffer, per-step
# deviations and the mean sample included
SEQ_CASES = {
    "c3": (lambda: W.c3(K=700, T=40), {}),
    "c2_lanes1": (lambda: W.c2("circles", K=1100, T=60), dict(lanes_per_sample=1)),
    "c2_lanes8": (lambda: W.c2("circles", K=1100, T=61), dict(lanes_per_sample=8)),
    "c2_lanes16_costmap": (lambda: W.c2("costmap", K=1100, T=59), dict(lanes_per_sample=16)),
    "c1_euler_lane": (lambda: W.c1(K=700, T=45).replace(integrator="euler"), {}),
    "c2_split": (lambda: W.c2("circles", K=1100, T=60),
                 dict(rollout_form=1, lanes_per_sample=4, cost_waves=8)),
    "c5_mlp": (lambda: W.c5(K=500, T=30, hidden=64), dict(rollout_block=128)),
}


@pytest.mark.parametrize("name", list(SEQ_CASES))
def test_sequence_with_sampling_options(mppi, oracle_lib, name):
    make, shape = SEQ_CASES[name]
    wl = _with_options(make(), sum(map(ord, name)))
    outs = []
    for split_calls in (False, True):
        c = mppi.Controller(wl)
        if shape:
            c.set_tuning(**shape)
        if split_calls:
            for _ in range(3):
                c.iterate(1)
        else:
            c.iterate(3)
        outs.append([_np(getattr(c, n)()) for n in ("controls", "costs", "noise")])
        assert c.stats()["iteration"] == 3
        c.close()
    for a, b in zip(*outs):
        assert np.array_equal(_bits(a), _bits(b))
    eps = oracle_lib.workload_noise(wl, iteration=2)
    assert np.array_equal(_bits(outs[0][2]), _bits(eps))


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


AHEAD_CASES = {
    "c2": (lambda: W.c2("circles", K=1500, T=40), {}),
    "c2_two_pass": (lambda: W.c2("circles", K=1500, T=40), dict(update_form=0)),
    "c3_chunked": (lambda: W.c3(K=20000, T=20), {}),
    "c5_grad": (lambda: W.c5(K=400, T=20, hidden=16).replace(lam=50.0), dict(grad=True)),
}


@pytest.mark.parametrize("name", list(AHEAD_CASES))
def test_noise_drawn_ahead_across_calls(mppi, oracle_lib, name):
    """An MPC loop (new state, one iteration, shift by one step) reads the noise
    that the previous call's last update drew ahead; forcing a fresh draw in
    every call (set_iteration to the same word) gives bitwise the same
    controls, costs and noise, and the noise is the oracle's."""
    make, shape = AHEAD_CASES[name]
    wl = make()
    shape = dict(shape)
    grad = shape.pop("grad", False)
    rng = np.random.default_rng(5)
    states = [wl.x0 + rng.normal(0.0, 0.05, wl.x0.shape).astype(np.float32) for _ in range(4)]
    runs = []
    for fresh in (False, True):
        c = mppi.Controller(wl, requires_grad=grad)
        if shape:
            c.set_tuning(**shape)
        out = []
        for i, x in enumerate(states):
            c.set_state(x)
            if fresh:
                c.set_iteration(i)
            c.iterate(1)
            out.append([_np(getattr(c, n)()) for n in ("controls", "costs", "noise")])
            c.shift(1)
        assert c.stats()["iteration"] == len(states)
        c.close()
        runs.append(out)
    for a, b in zip(*runs):
        for x, y in zip(a, b):
            assert np.array_equal(_bits(x), _bits(y))
    for i, step in enumerate(runs[0]):
        assert np.array_equal(_bits(step[2]), _bits(oracle_lib.workload_noise(wl, iteration=i)))


def test_noise_drawn_ahead_is_dropped_by_a_new_word(mppi, oracle_lib):
    wl = W.c2("circles", K=1000, T=30)
    c = mppi.Controller(wl)
    c.iterate(2)
    c.set_iteration(7)
    c.iterate(1)
    assert np.array_equal(_bits(_np(c.noise())), _bits(oracle_lib.workload_noise(wl, iteration=7)))
    # a staged update steps the word: the next sequence draws afresh
    c.sample()
    c.rollout()
    c.update()
    c.iterate(2)
    assert c.stats()["iteration"] == 11
    assert np.array_equal(_bits(_np(c.noise())), _bits(oracle_lib.workload_noise(wl, iteration=10)))
    c.close()
