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


# ---- the one-launch form: one launch per iteration -------------------------
ONE_LAUNCH = dict(batch_form=1, batch_tile=256, update_form=0)


def _run_batch(mppi, insts, iters, one_launch, debug=False, calls=1):
    ctl = mppi.Controller(insts, debug=debug)
    if one_launch:
        ctl.set_tuning(**ONE_LAUNCH)
    for _ in range(calls):
        ctl.iterate(iters)
    out = {"U": _np(ctl.controls()).copy(), "S": _np(ctl.costs()).copy(),
           "eps": _np(ctl.noise()).copy(), "stats": ctl.stats()}
    if debug:
        out["crashes"] = _np(ctl.crashes()).copy()
    out["U_split"] = ctl.split(out["U"], 1)
    ctl.close()
    return out


def _same(a, b, name):
    assert a.shape == b.shape, name
    assert np.array_equal(np.ascontiguousarray(a).view(np.uint32),
                          np.ascontiguousarray(b).view(np.uint32)), name


def _close_controls(insts, a, b, name):
    """The one-launch update sums the same terms as the per-phase one in
    another order (tile partials rescaled to the instance's minimum): each
    instance's controls agree within the flat bound 1e-4 max(|U|, sigma)."""
    for i, wl in enumerate(insts):
        Ua, Ub = a["U_split"][i].astype(np.float64), b["U_split"][i].astype(np.float64)
        scale = max(np.abs(Ua).max(), float(np.max(wl.sigma)))
        err = np.abs(Ua - Ub).max()
        assert err <= parity.REL * scale, f"{name} instance {i}: {err:.3g} vs {parity.REL * scale:.3g}"


@pytest.mark.parametrize("iters,calls", [(1, 1), (3, 1), (2, 3)])
def test_one_launch_matches_phases(mppi, iters, calls):
    """One launch per iteration draws bitwise the per-phase
    launches' noise and costs (and crash counts) and gives their controls and
    statistics up to the rounding order of the update's sums, over several
    iterations and repeated calls (graph replays).  After the first iteration
    the warm starts differ by that rounding, so costs are compared at the
    first iteration only."""
    insts = small_batch(n=12)
    a = _run_batch(mppi, insts, iters, False, debug=True, calls=calls)
    b = _run_batch(mppi, insts, iters, True, debug=True, calls=calls)
    if iters * calls == 1:
        for k in ("S", "eps", "crashes"):
            _same(a[k], b[k], k)
    else:
        _same(a["eps"], b["eps"], "eps")
    _close_controls(insts, a, b, f"{iters}x{calls}")
    for sa, sb in zip(a["stats"], b["stats"]):
        assert sb["status"] == 0 and sb["iteration"] == sa["iteration"] == iters * calls
        if iters * calls == 1:
            assert sb["rho"] == sa["rho"]
            assert sb["eta"] == pytest.approx(sa["eta"], rel=1e-5)
            assert sb["ess"] == pytest.approx(sa["ess"], rel=1e-4)


def test_one_launch_against_oracle(mppi, oracle_lib):
    """The one-launch iteration end to end against the oracle, for every
    instance of a small heterogeneous batch (costs, crash counts, controls)."""
    insts = small_batch(n=10)
    ctl = mppi.Controller(insts, debug=True)
    ctl.set_tuning(**ONE_LAUNCH)
    ctl.iterate(1)
    S = ctl.split(_np(ctl.costs()), 2)
    eps = ctl.split(_np(ctl.noise()), 3)
    crashes = ctl.split(_np(ctl.crashes()), 2)
    U = ctl.split(_np(ctl.controls()), 1)
    stats = ctl.stats()
    ctl.close()
    for i, wl in enumerate(insts):
        e_or = oracle_lib.workload_noise(wl)
        assert np.array_equal(eps[i].view(np.uint32), e_or.ravel().view(np.uint32)), i
        S_or, margin, cr_or = oracle_lib.rollout_costs(wl, eps=e_or)
        parity.assert_costs_close(S[i], S_or, margin, f"one-launch instance {i}")
        sure = margin >= parity.AMBIGUOUS_MARGIN
        assert np.array_equal(crashes[i][sure], cr_or[sure])
        parity.assert_end_to_end(oracle_lib, wl, U[i].reshape(wl.T, 2), S[i], e_or, S_or,
                                 f"one-launch instance {i}")
        assert stats[i]["status"] == 0 and stats[i]["iteration"] == 1


def test_one_launch_options(mppi, oracle_lib):
    """Sampling and update options in the one-launch form (the importance
    term and step size, samples drawn around zero, the mean sample, a
    per-step noise deviation table): noise and costs bitwise as the per-phase
    launches, controls against the oracle end to end."""
    insts = []
    for i, wl in enumerate(small_batch(n=8)):
        u0 = np.random.default_rng(40 + i).normal(0.0, 0.4, (wl.T, 2)).astype(np.float32)
        wl = wl.replace(u0=u0, is_beta=1, gamma=(1.0, 0.5)[i % 2], zero_frac=0.2, mean_sample=1)
        sig = np.linspace(0.6, 1.4, wl.T)[:, None] * wl.sigma[None, :]
        insts.append(wl.replace(sigma_t=sig.astype(np.float32)))
    a = _run_batch(mppi, insts, 1, False)
    b = _run_batch(mppi, insts, 1, True)
    for k in ("S", "eps"):
        _same(a[k], b[k], k)
    _close_controls(insts, a, b, "options")
    S = np.split(b["S"], np.cumsum([w.K for w in insts])[:-1])
    for i, wl in enumerate(insts):
        e_or = oracle_lib.workload_noise(wl)
        S_or, _, _ = oracle_lib.rollout_costs(wl, eps=e_or)
        parity.assert_end_to_end(oracle_lib, wl, b["U_split"][i].reshape(wl.T, 2), S[i], e_or,
                                 S_or, f"one-launch options instance {i}")


def test_one_launch_full_size(mppi, oracle_lib):
    """All 256 instances of the c4 recipe: two one-launch iterations against two
    per-phase iterations (noise bitwise, controls within the flat bound), every
    status OK, and the instance with the most rollout steps against the oracle
    end to end at its second iteration, from the GPU's own warm start."""
    insts = W.c4()
    a = _run_batch(mppi, insts, 2, False)
    b = _run_batch(mppi, insts, 2, True)
    _same(a["eps"], b["eps"], "eps")
    _close_controls(insts, a, b, "c4")
    assert all(s["status"] == 0 and s["iteration"] == 2 for s in b["stats"])
    ctl = mppi.Controller(insts)
    ctl.set_tuning(**ONE_LAUNCH)
    ctl.iterate(1)
    u1 = ctl.split(_np(ctl.controls()), 1)
    ctl.iterate(1)
    S = ctl.split(_np(ctl.costs()), 2)
    U = ctl.split(_np(ctl.controls()), 1)
    ctl.close()
    big = int(np.argmax([w.K * w.T for w in insts]))
    wl = insts[big]
    u = u1[big].reshape(wl.T, 2).astype(np.float64)
    o = oracle_lib.mppi(wl, iters=1, iter0=1, u=u)
    parity.assert_costs_close(S[big], o["S"], oracle_lib.rollout_costs(wl, eps=o["eps"], u=u)[1],
                              "one-launch c4 largest instance")
    parity.assert_end_to_end(oracle_lib, wl, U[big].reshape(wl.T, 2), S[big], o["eps"], o["S"],
                             "one-launch c4 largest instance", u=u)


def test_one_launch_form_refusals(mppi):
    from paper_2409_07563_amd import MPPIError
    one = mppi.Controller(W.c2("circles", K=256, T=10, iters=1))
    with pytest.raises(MPPIError) as e:
        one.set_tuning(batch_form=1)
    assert e.value.status == -5
    one.close()
    ctl = mppi.Controller(small_batch(n=3))
    with pytest.raises(MPPIError) as e:
        ctl.set_tuning(batch_form=1, batch_tile=128, update_form=0)
    assert e.value.status == -5
    with pytest.raises(MPPIError) as e:
        ctl.set_tuning(batch_form=2)
    assert e.value.status == -1
    ctl.close()
    # an instance past the one-launch form's 65536 samples
    big = small_batch(n=2)
    big[1] = big[1].replace(K=70000)
    ctl = mppi.Controller(big)
    with pytest.raises(MPPIError) as e:
        ctl.set_tuning(**ONE_LAUNCH)
    assert e.value.status == -5
    ctl.close()
