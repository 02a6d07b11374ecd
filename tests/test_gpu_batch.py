"""Batched MPPI (many independent instances in one launch per phase) against
the oracle and against single-instance contexts, through the C ABI."""
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


def small_batch(n=12, kmax=700):
    """Heterogeneous instances of the c4 recipe, K capped so that the oracle
    is quick; K, T, lambda, obstacles and goals all differ."""
    out = []
    for wl in W.c4(n_instances=n):
        K = min(wl.K, kmax) - (wl.instance % 3) * 17   # ragged sizes
        out.append(wl.replace(K=K))
    return out


def test_batch_against_oracle(mppi, oracle_lib):
    insts = small_batch()
    ctl = mppi.Controller(insts, debug=True)
    ctl.sample()
    ctl.rollout()
    S = ctl.split(_np(ctl.costs()), 2)
    eps = ctl.split(_np(ctl.noise()), 3)
    crashes = ctl.split(_np(ctl.crashes()), 2)
    ctl.update()
    U = ctl.split(_np(ctl.controls()), 1)
    stats = ctl.stats()
    ctl.close()
    for i, wl in enumerate(insts):
        e_or = oracle_lib.workload_noise(wl)
        assert np.array_equal(eps[i].view(np.uint32), e_or.ravel().view(np.uint32)), i
        S_or, margin, cr_or = oracle_lib.rollout_costs(wl, eps=e_or)
        parity.assert_costs_close(S[i], S_or, margin, f"instance {i}")
        sure = margin >= parity.AMBIGUOUS_MARGIN
        assert np.array_equal(crashes[i][sure], cr_or[sure])
        parity.assert_end_to_end(oracle_lib, wl, U[i].reshape(wl.T, 2), S[i], e_or, S_or,
                                 f"instance {i}")
        assert stats[i]["status"] == 0 and stats[i]["iteration"] == 1


def test_batch_equals_single_contexts_bitwise(mppi):
    """The batch runs the same lane body and the same reduction order as a
    single-instance context with one lane per sample and the two-pass update:
    results are identical."""
    insts = small_batch(n=6)
    ctl = mppi.Controller(insts)
    ctl.iterate(3)
    U = ctl.split(_np(ctl.controls()), 1)
    S = ctl.split(_np(ctl.costs()), 2)
    ctl.close()
    for i, wl in enumerate(insts):
        one = mppi.Controller(wl, rollout="lane")
        one.set_tuning(update_form=0)
        one.iterate(3)
        u1 = _np(one.controls()).ravel()
        s1 = _np(one.costs())
        one.close()
        assert np.array_equal(U[i].view(np.uint32), u1.view(np.uint32)), i
        assert np.array_equal(S[i].view(np.uint32), s1.view(np.uint32)), i


def test_batch_full_size_sampled(mppi, oracle_lib):
    """All 256 instances of the c4 recipe in one context, in the benchmark's
    launch configuration: every status OK; the instance with the most
    rollout steps checked in full (every cost, and its controls end to end);
    a sample of other instances / samples recomputed by the oracle."""
    insts = W.c4()
    ctl = mppi.Controller(insts)
    ctl.sample()
    ctl.rollout()
    S = ctl.split(_np(ctl.costs()), 2)
    big = int(np.argmax([w.K * w.T for w in insts]))
    eps_big = ctl.split(_np(ctl.noise()), 3)[big]
    ctl.update()
    stats = ctl.stats()
    U = ctl.split(_np(ctl.controls()), 1)
    ctl.close()
    assert all(s["status"] == 0 for s in stats)
    wl = insts[big]
    e_or = oracle_lib.workload_noise(wl)
    assert np.array_equal(eps_big.view(np.uint32), e_or.ravel().view(np.uint32))
    S_or = oracle_lib.rollout_costs_parallel(wl, e_or)
    margin = oracle_lib.rollout_costs(wl, eps=e_or)[1]
    parity.assert_costs_close(S[big], S_or, margin, f"instance {big} (K {wl.K}, T {wl.T})")
    parity.assert_end_to_end(oracle_lib, wl, U[big].reshape(wl.T, 2), S[big], e_or, S_or,
                             f"full-size instance {big}")
    rng = np.random.default_rng(4)
    for i in rng.choice(len(insts), 6, replace=False):
        wl = insts[i]
        idx = rng.choice(wl.K, 48, replace=False)
        eps = oracle_lib.workload_noise(wl)[:, :, idx]
        S_or, margin, _ = oracle_lib.rollout_costs(wl.replace(K=len(idx)), eps=eps)
        parity.assert_costs_close(S[i][idx], S_or, margin, f"instance {i}")


def test_batch_sequence_and_single_calls_agree(mppi, oracle_lib):
    """A 3-iteration sequence, 3 single-iteration calls, and single iterations
    each after a set_iteration to the same word: controls, costs and noise
    are bitwise equal, and the visible noise is the oracle's for the last
    word."""
    insts = small_batch(n=7, kmax=600)
    rng = np.random.default_rng(4)
    insts = [w.replace(sigma_t=(np.asarray(w.sigma)[None, :] * rng.uniform(
        0.5, 1.5, (w.T, w.m))).astype(np.float32), mean_sample=1) for w in insts]
    outs = []
    for mode in ("sequence", "calls", "fresh"):
        ctl = mppi.Controller(insts)
        if mode == "sequence":
            ctl.iterate(3)
        else:
            for i in range(3):
                if mode == "fresh":
                    ctl.set_iteration(i)
                ctl.iterate(1)
        outs.append([_np(ctl.controls()), _np(ctl.costs()), _np(ctl.noise())])
        assert all(s["iteration"] == 3 for s in ctl.stats())
        ctl.close()
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    eps = np.split(outs[0][2], np.cumsum([w.T * w.m * w.K for w in insts])[:-1])
    for i, wl in enumerate(insts):
        e_or = oracle_lib.workload_noise(wl, iteration=2)
        assert np.array_equal(eps[i].view(np.uint32), e_or.ravel().view(np.uint32)), i


@pytest.mark.parametrize("n", [2, 5, 9])
def test_iteration_equals_staged_phases(mppi, n):
    """mppi_iterate (the captured sequence), the staged calls and the
    sequence with 64-sample tiles give bitwise the same controls and costs."""
    insts = small_batch(n=n, kmax=900)
    outs = []
    for mode in ("iterate", "staged", "tile64"):
        ctl = mppi.Controller(insts)
        if mode == "tile64":
            ctl.set_tuning(batch_tile=64)
        for _ in range(2):
            if mode == "staged":
                ctl.sample()
                ctl.rollout()
                ctl.update()
            else:
                ctl.iterate(1)
        outs.append([_np(ctl.controls()), _np(ctl.costs())])
        ctl.close()
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
