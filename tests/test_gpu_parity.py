"""GPU parity of the HIP path against the binary64 oracle, through the C ABI.

Every case runs the library on seeded synthetic inputs and compares it with
the oracle on the same inputs and the same counter-based noise; the bar and
the tolerances are stated in tests/parity.py.
"""
import sys

import numpy as np
import pytest

import workloads as W
from tests import parity

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _announce(request):
    # name the case before any kernel runs, so a lost run still says which
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
# (a1) noise: bit-exact
# ---------------------------------------------------------------------------
def test_noise_transform_tables_bitexact(mppi, oracle_lib):
    r, c, s = (_np(t) for t in mppi.noise_tables())
    ro, co, so = oracle_lib.bm_tables()
    for name, a, b in (("radius", r, ro), ("cos", c, co), ("sin", s, so)):
        diff = np.flatnonzero(a.view(np.uint32) != b.view(np.uint32))
        assert diff.size == 0, f"{name}: {diff.size} inputs differ, first {diff[:4]}"


@pytest.mark.parametrize("seed,it,inst,K,T,m", [
    (1001, 0, 0, 1024, 100, 2), (1002, 3, 0, 1000, 37, 2), (7, 1, 5, 65, 3, 4),
    (2**64 - 1, 2**32 - 1, 2**32 - 1, 1, 1, 1), (1003, 0, 0, 4096, 50, 4), (9, 2, 0, 333, 7, 3)])
def test_noise_bitexact(mppi, oracle_lib, seed, it, inst, K, T, m):
    sigma = np.linspace(0.2, 1.3, m).astype(np.float32)
    g = _np(mppi.noise(seed, it, inst, K, T, m, sigma))
    o = oracle_lib.noise(seed, it, inst, K, T, m, sigma)
    assert np.array_equal(g.view(np.uint32), o.view(np.uint32))


# ---------------------------------------------------------------------------
# workloads at oracle-friendly sizes (several tiles and a ragged tail)
# ---------------------------------------------------------------------------
def _graded(wl):
    """The rasterised obstacles blurred into a map of many distinct values."""
    m = wl.costmap.astype(np.float64)
    for _ in range(3):
        m = 0.25 * (np.roll(m, 1, 0) + np.roll(m, -1, 0) + np.roll(m, 1, 1) + np.roll(m, -1, 1))
    return wl.replace(costmap=np.ascontiguousarray(m.astype(np.float32)))


def _cases():
    c4 = W.c4(n_instances=2)[1].replace(K=700, T=60, u0=np.zeros((60, 2), np.float32))
    return {
        "c1": W.c1(K=1024, T=100),
        "c1_ragged": W.c1(K=1000, T=37),
        "c2_circles": W.c2("circles", K=2000, T=100, iters=1),
        "c2_costmap": W.c2("costmap", K=2000, T=100, iters=1),
        # a graded map (many distinct values): read from memory, not the LDS bitmap
        "c2_costmap_graded": _graded(W.c2("costmap", K=1500, T=80, iters=1)),
        "c3": W.c3(K=1500, T=60),
        "c4_instance": c4,
        "di_rk4": W.c1(K=300, T=50).replace(integrator="rk4"),
        "bicycle_quadratic": W.c2("circles", K=129, T=20).replace(
            cost="quadratic", w=W._weights({0: 1, 1: 1, 2: 2, 3: 0.5, 4: 0.1, 8: 0.1, 9: 0.2,
                                              16: 3, 17: 3, 18: 3, 19: 3, 20: 3}),
            ref=np.array([20, 30, 0.5, 4, 0], np.float32)),
        "c5_track_no_mlp": W.c5(K=512, T=50).replace(model="bicycle", mlp=None, mlp_hidden=0),
    }


CASES = _cases()
# the same workloads at a higher temperature: the update then averages over
# hundreds of samples (ESS >> 1) instead of one
TEMPERED = {f"{n}_lam_x{f}": CASES[n].replace(lam=float(np.float32(CASES[n].lam * f)))
            for n, f in (("c1", 100), ("c3", 1000), ("c2_circles", 100))}


def _run_one_iteration(mppi, wl, debug=True, accurate_trig=False, rollout="auto", lanes=None):
    ctl = mppi.Controller(wl, debug=debug and wl.cost in ("path_circles", "goal_circles"),
                          accurate_trig=accurate_trig, rollout=rollout)
    if lanes is not None:
        ctl.set_tuning(lanes_per_sample=lanes)
    ctl.sample()
    ctl.rollout()
    S = _np(ctl.costs())
    eps = _np(ctl.noise())
    crashes = _np(ctl.crashes()) if ctl.cfg.flags & 1 else None
    ctl.update()
    U = _np(ctl.controls())
    stats = ctl.stats()
    w = _np(ctl.weights())
    ctl.close()
    return dict(S=S, eps=eps, U=U, stats=stats, w=w, crashes=crashes)


TRIG = [False, True]


@pytest.mark.parametrize("accurate", TRIG, ids=["hw_trig", "lib_trig"])
@pytest.mark.parametrize("name", list(CASES))
def test_rollout_costs_parity(mppi, oracle_lib, name, accurate):
    wl = CASES[name]
    g = _run_one_iteration(mppi, wl, accurate_trig=accurate)
    eps_or = oracle_lib.workload_noise(wl)
    assert np.array_equal(g["eps"].view(np.uint32), eps_or.view(np.uint32))
    S_or, margin, crashes, slope = oracle_lib.rollout_costs(wl, eps=eps_or, slope=True)
    parity.assert_costs_close(g["S"], S_or, margin, name,
                              slope=slope if wl.cost == "path_costmap" else None)
    if g["crashes"] is not None:
        sure = margin >= parity.AMBIGUOUS_MARGIN
        assert np.array_equal(g["crashes"][sure], crashes[sure])
        assert crashes.sum() > 0 or name.startswith("c4")


BICYCLE_CASES = [n for n, w in CASES.items() if w.model == "bicycle"]


@pytest.mark.parametrize("lanes", [1, 4, 8, 16])
@pytest.mark.parametrize("name", BICYCLE_CASES)
def test_rollout_variants_parity(mppi, oracle_lib, name, lanes):
    """Every rollout kernel of the bicycle (one lane per sample, and 4, 8 or
    16 lanes per sample) against the oracle, costs and crash counts."""
    wl = CASES[name]
    rollout = f"lanes{lanes}"
    g = _run_one_iteration(mppi, wl, lanes=lanes)
    eps_or = oracle_lib.workload_noise(wl)
    S_or, margin, crashes, slope = oracle_lib.rollout_costs(wl, eps=eps_or, slope=True)
    parity.assert_costs_close(g["S"], S_or, margin, f"{name}/{rollout}",
                              slope=slope if wl.cost == "path_costmap" else None)
    if g["crashes"] is not None:
        sure = margin >= parity.AMBIGUOUS_MARGIN
        assert np.array_equal(g["crashes"][sure], crashes[sure])
    parity.assert_end_to_end(oracle_lib, wl, g["U"], g["S"], eps_or, S_or, f"{name}/{rollout}")


@pytest.mark.parametrize("lanes", [4, 8, 16])
@pytest.mark.parametrize("K,T", [(1, 1), (3, 5), (17, 6), (64, 7), (65, 4), (33, 23)])
def test_grouped_rollout_ragged_shapes(mppi, oracle_lib, K, T, lanes):
    """Several lanes per sample: partial groups in the last wave, horizons
    that are not a multiple of the unrolled four steps or of the L-step cost
    groups."""
    wl = W.c2("circles", K=K, T=T, iters=1)
    g = _run_one_iteration(mppi, wl, lanes=lanes)
    S_or, margin, crashes = oracle_lib.rollout_costs(wl, eps=oracle_lib.workload_noise(wl))
    parity.assert_costs_close(g["S"], S_or, margin, f"lanes {lanes} K{K} T{T}")
    sure = margin >= parity.AMBIGUOUS_MARGIN
    assert np.array_equal(g["crashes"][sure], crashes[sure])


@pytest.mark.parametrize("name", ["c1", "c2_circles", "c3", "c1_ragged"])
def test_update_parity_on_oracle_costs(mppi, oracle_lib, name):
    """(a3)-(a6) in isolation: both sides weight the same binary32 costs."""
    wl = CASES[name]
    eps = oracle_lib.workload_noise(wl)
    S_or, _, _ = oracle_lib.rollout_costs(wl, eps=eps)
    S32 = S_or.astype(np.float32)
    ctl = mppi.Controller(wl)
    ctl.sample()
    ctl.set_costs(S32)
    ctl.update()
    U = _np(ctl.controls())
    st = ctl.stats()
    w = _np(ctl.weights())
    ctl.close()
    w_or, U_or, stats_or, rc = oracle_lib.softmin_update(wl, S32.astype(np.float64), eps)
    assert rc == 0 and st["status"] == 0
    scale = max(np.abs(U_or).max(), np.abs(wl.sigma).max())
    parity.assert_controls_close(U, U_or, parity.REL * scale, name)
    assert st["rho"] == pytest.approx(stats_or[0], rel=1e-7)
    assert st["eta"] == pytest.approx(stats_or[1], rel=1e-4)
    assert st["ess"] == pytest.approx(stats_or[3], rel=1e-4)
    assert st["free_energy"] == pytest.approx(stats_or[2], rel=1e-4, abs=1e-4)
    assert abs(w.astype(np.float64).sum() - 1.0) < 1e-5
    assert np.allclose(w, w_or, rtol=1e-4, atol=1e-7)


@pytest.mark.parametrize("accurate", TRIG, ids=["hw_trig", "lib_trig"])
@pytest.mark.parametrize("name", list(CASES) + list(TEMPERED))
def test_iteration_end_to_end(mppi, oracle_lib, name, accurate):
    wl = CASES[name] if name in CASES else TEMPERED[name]
    g = _run_one_iteration(mppi, wl, accurate_trig=accurate)
    o = oracle_lib.mppi(wl, iters=1)
    assert np.array_equal(g["eps"].view(np.uint32), o["eps"].view(np.uint32))
    parity.assert_end_to_end(oracle_lib, wl, g["U"], g["S"], o["eps"], o["S"], name)
    if name in TEMPERED:
        # the update averages over many samples here, not just the argmin
        assert g["stats"]["ess"] > 50, g["stats"]["ess"]
    assert g["stats"]["iteration"] == 1


def test_c2_full_size_ten_iterations(mppi, oracle_lib):
    """The benchmark workload (K 8192, T 100, 10 warm-started iterations):
    every iteration checked from the oracle's own warm start (the GPU is
    handed the oracle's u and iteration word)."""
    wl = W.c2("circles")
    ctl = mppi.Controller(wl)
    u = wl.u0.astype(np.float64)
    for i in range(wl.iters):
        o = oracle_lib.mppi(wl, iters=1, iter0=i, u=u)
        ctl.set_controls(u.astype(np.float32))
        ctl.set_iteration(i)
        ctl.iterate(1)
        U = _np(ctl.controls())
        S = _np(ctl.costs())
        parity.assert_costs_close(S, o["S"], oracle_lib.rollout_costs(
            wl, eps=o["eps"], u=u)[1], f"iteration {i} costs")
        parity.assert_end_to_end(oracle_lib, wl, U, S, o["eps"], o["S"], f"iteration {i}", u=u)
        u = o["U"]
    ctl.close()


@pytest.mark.parametrize("lam_scale", [1.0, 100.0], ids=["lam", "lam_x100"])
def test_c3_full_size(mppi, oracle_lib, lam_scale):
    """Quadrotor at the full K 65536, T 200, in the benchmark's launch
    configuration: every cost against the oracle's (which rolls the samples
    out on all host cores), and the controls end to end, at the workload's
    temperature and at 100 times it (ESS >> 1)."""
    wl = W.c3()
    wl = wl.replace(lam=float(np.float32(wl.lam * lam_scale)))
    ctl = mppi.Controller(wl)
    ctl.sample()
    ctl.rollout()
    S = _np(ctl.costs())
    eps = _np(ctl.noise())
    ctl.update()
    st = ctl.stats()
    U = _np(ctl.controls())
    ctl.close()
    assert np.isfinite(S).all() and st["status"] == 0
    e_or = oracle_lib.workload_noise(wl)
    assert np.array_equal(eps.view(np.uint32), e_or.view(np.uint32))
    S_or = oracle_lib.rollout_costs_parallel(wl, e_or)
    parity.assert_costs_close(S, S_or, None, "c3 full size")
    parity.assert_end_to_end(oracle_lib, wl, U, S, e_or, S_or, f"c3 full size x{lam_scale:g}")


def test_deterministic_bitwise(mppi):
    wl = W.c2("circles", K=4096, T=100, iters=3)
    outs = []
    for _ in range(2):
        ctl = mppi.Controller(wl)
        ctl.iterate(3)
        outs.append((_np(ctl.controls()).copy(), _np(ctl.costs()).copy()))
        ctl.close()
    assert np.array_equal(outs[0][0].view(np.uint32), outs[1][0].view(np.uint32))
    assert np.array_equal(outs[0][1].view(np.uint32), outs[1][1].view(np.uint32))


def test_nonfinite_costs(mppi, oracle_lib):
    wl = W.c1(K=300, T=20)
    u0 = np.random.default_rng(1).normal(0, 0.2, (wl.T, 2)).astype(np.float32)
    wl = wl.replace(u0=u0)
    ctl = mppi.Controller(wl)
    ctl.sample()
    ctl.set_costs(np.full(wl.K, np.inf, np.float32))
    ctl.update()
    assert np.array_equal(_np(ctl.controls()), u0)
    assert ctl.stats()["status"] == -6
    # some non-finite: they get zero weight
    eps = oracle_lib.workload_noise(wl, iteration=1)
    S = np.linspace(10.0, 20.0, wl.K).astype(np.float32)
    S[::3] = np.nan
    S[1::7] = np.inf
    ctl.set_controls(u0)
    ctl.sample()
    ctl.set_costs(S)
    ctl.update()
    U = _np(ctl.controls())
    w = _np(ctl.weights())
    assert ctl.stats()["status"] == 0
    assert np.all(w[::3] == 0) and np.all(w[1::7] == 0)
    S_or = np.where(np.isfinite(S), S, np.inf).astype(np.float64)
    w_or, U_or, _, rc = oracle_lib.softmin_update(wl, S_or, eps)
    parity.assert_controls_close(U, U_or, 1e-4 * max(np.abs(U_or).max(), 0.5), "partial nonfinite")
    ctl.close()


def test_single_sample_and_single_step(mppi, oracle_lib):
    for wl in (W.c1(K=1, T=1), W.c2("circles", K=1, T=5, iters=1), W.c3(K=2, T=1)):
        g = _run_one_iteration(mppi, wl)
        o = oracle_lib.mppi(wl, iters=1)
        parity.assert_end_to_end(oracle_lib, wl, g["U"], g["S"], o["eps"], o["S"], wl.name)
        if wl.K == 1:
            assert g["w"][0] == 1.0


def test_api_state_errors(mppi):
    from paper_2409_07563_amd import MPPIError
    wl = W.c1(K=64, T=4)
    ctl = mppi.Controller(wl)
    with pytest.raises(MPPIError):
        ctl.iterate(0)
    ctl2 = mppi.Controller(wl)
    ctl2.close()
    ctl.close()
