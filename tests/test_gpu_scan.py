"""The time-parallel (scan) rollout form of the bicycle with RK4, against the
binary64 oracle through the C ABI: each sample's horizon is spread over the 16
lanes of a DPP row (or the 32 of two rows), the speed, steer, yaw and position
as prefix sums over time, then every step's running cost in parallel.  Checked as every other
rollout kernel is (tests/parity.py): costs, crash counts, the controls end to
end, horizons that fill every compiled chunk length, the sampling and update
options, and the benchmark workload over ten warm-started iterations from a
captured graph (with the next iteration's noise drawn in the same launch)."""
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


SCAN = dict(rollout_form=2, lanes_per_sample=16)


def _graded(wl):
    m = wl.costmap.astype(np.float64)
    for _ in range(3):
        m = 0.25 * (np.roll(m, 1, 0) + np.roll(m, -1, 0) + np.roll(m, 1, 1) + np.roll(m, -1, 1))
    return wl.replace(costmap=np.ascontiguousarray(m.astype(np.float32)))


def _cases():
    c4 = W.c4(n_instances=2)[1].replace(K=700, T=60, u0=np.zeros((60, 2), np.float32))
    return {
        "c2_circles": W.c2("circles", K=2000, T=100, iters=1),
        "c2_costmap": W.c2("costmap", K=2000, T=100, iters=1),
        "c2_costmap_graded": _graded(W.c2("costmap", K=1500, T=80, iters=1)),
        "c4_instance": c4,
        "c4_instance_T200": W.c4(n_instances=3)[2].replace(
            K=500, T=200, u0=np.zeros((200, 2), np.float32)),
        "bicycle_quadratic": W.c2("circles", K=129, T=20).replace(
            cost="quadratic", w=W._weights({0: 1, 1: 1, 2: 2, 3: 0.5, 4: 0.1, 8: 0.1, 9: 0.2,
                                              16: 3, 17: 3, 18: 3, 19: 3, 20: 3}),
            ref=np.array([20, 30, 0.5, 4, 0], np.float32)),
        "c5_track_no_mlp": W.c5(K=512, T=50).replace(model="bicycle", mlp=None, mlp_hidden=0),
        "c2_circles_lam_x100": W.c2("circles", K=2000, T=100, iters=1).replace(lam=50.0),
    }


CASES = _cases()


def _one(mppi, wl, block=256, accurate=False, debug=True, lanes=16):
    ctl = mppi.Controller(wl, debug=debug and wl.cost in ("path_circles", "goal_circles"),
                          accurate_trig=accurate)
    ctl.set_tuning(rollout_block=block, **dict(SCAN, lanes_per_sample=lanes))
    ctl.sample()
    ctl.rollout()
    S = _np(ctl.costs())
    eps = _np(ctl.noise())
    crashes = _np(ctl.crashes()) if ctl.cfg.flags & 1 else None
    ctl.update()
    U = _np(ctl.controls())
    st = ctl.stats()
    ctl.close()
    return dict(S=S, eps=eps, U=U, crashes=crashes, stats=st)


@pytest.mark.parametrize("lanes", [16, 32])
@pytest.mark.parametrize("accurate", [False, True], ids=["hw_trig", "lib_trig"])
@pytest.mark.parametrize("name", list(CASES))
def test_scan_rollout_parity(mppi, oracle_lib, name, accurate, lanes):
    wl = CASES[name]
    g = _one(mppi, wl, accurate=accurate, lanes=lanes)
    eps_or = oracle_lib.workload_noise(wl)
    assert np.array_equal(g["eps"].view(np.uint32), eps_or.view(np.uint32))
    S_or, margin, crashes, slope = oracle_lib.rollout_costs(wl, eps=eps_or, slope=True)
    parity.assert_costs_close(g["S"], S_or, margin, f"scan {name}",
                              slope=slope if wl.cost == "path_costmap" else None)
    if g["crashes"] is not None:
        sure = margin >= parity.AMBIGUOUS_MARGIN
        assert np.array_equal(g["crashes"][sure], crashes[sure])
    parity.assert_end_to_end(oracle_lib, wl, g["U"], g["S"], eps_or, S_or, f"scan {name}")
    if name.endswith("lam_x100"):
        assert g["stats"]["ess"] > 50


# every compiled chunk length (16 lanes: C = 4, 7, 10, 13, 16; 32 lanes:
# C = 4, 8) with full, partial and empty lanes, single samples and partial
# rows and groups of the last wave
@pytest.mark.parametrize("lanes", [16, 32])
@pytest.mark.parametrize("K,T", [(1, 1), (3, 5), (17, 6), (64, 7), (65, 4), (33, 23), (5, 64),
                                 (7, 65), (9, 112), (3, 113), (2, 160), (4, 161), (6, 208),
                                 (11, 209), (5, 256), (1, 250), (2, 128), (3, 129)])
@pytest.mark.parametrize("block", [64, 256])
def test_scan_ragged_shapes(mppi, oracle_lib, K, T, block, lanes):
    wl = W.c2("circles", K=K, T=T, iters=1)
    g = _one(mppi, wl, block=block, lanes=lanes)
    S_or, margin, crashes = oracle_lib.rollout_costs(wl, eps=oracle_lib.workload_noise(wl))
    parity.assert_costs_close(g["S"], S_or, margin, f"scan K{K} T{T} block {block} lanes {lanes}")
    sure = margin >= parity.AMBIGUOUS_MARGIN
    assert np.array_equal(g["crashes"][sure], crashes[sure])


@pytest.mark.parametrize("lanes", [16, 32])
@pytest.mark.parametrize("opt", ["is_gamma", "zero_mean", "mean_sample", "sigma_t"])
def test_scan_sampling_and_update_options(mppi, oracle_lib, opt, lanes):
    wl = W.c2("circles", K=1500, T=93, iters=1)
    u0 = np.random.default_rng(3).normal(0.0, 0.5, (wl.T, wl.m)).astype(np.float32)
    wl = wl.replace(u0=u0)
    if opt == "is_gamma":
        wl = wl.replace(is_beta=1, gamma=0.4)
    elif opt == "zero_mean":
        wl = wl.replace(zero_frac=0.25)
    elif opt == "mean_sample":
        wl = wl.replace(mean_sample=1)
    else:
        sig = np.linspace(0.5, 1.5, wl.T)[:, None] * wl.sigma[None, :]
        wl = wl.replace(sigma_t=sig.astype(np.float32))
    g = _one(mppi, wl, lanes=lanes)
    eps_or = oracle_lib.workload_noise(wl)
    assert np.array_equal(g["eps"].view(np.uint32), eps_or.view(np.uint32))
    S_or, margin, _ = oracle_lib.rollout_costs(wl, eps=eps_or)
    parity.assert_costs_close(g["S"], S_or, margin, f"scan {opt}")
    parity.assert_end_to_end(oracle_lib, wl, g["U"], g["S"], eps_or, S_or, f"scan {opt}")


@pytest.mark.parametrize("lanes", [16, 32])
def test_scan_full_size_ten_iterations(mppi, oracle_lib, lanes):
    """The benchmark workload (K 8192, T 100) in the scan form: ten iterations
    replayed from the captured graph equal ten single iterations bitwise, and
    every iteration matches the oracle from the oracle's own warm start."""
    wl = W.c2("circles")
    tune = dict(SCAN, lanes_per_sample=lanes)
    seq = mppi.Controller(wl)
    seq.set_tuning(**tune)
    seq.iterate(wl.iters)
    U_seq, S_seq = _np(seq.controls()), _np(seq.costs())
    seq.close()
    ctl = mppi.Controller(wl)
    ctl.set_tuning(**tune)
    u = wl.u0.astype(np.float64)
    U_one = S_one = None
    for i in range(wl.iters):
        o = oracle_lib.mppi(wl, iters=1, iter0=i, u=u)
        ctl.set_controls(u.astype(np.float32))
        ctl.set_iteration(i)
        ctl.iterate(1)
        U = _np(ctl.controls())
        S = _np(ctl.costs())
        parity.assert_costs_close(S, o["S"], oracle_lib.rollout_costs(
            wl, eps=o["eps"], u=u)[1], f"scan iteration {i} costs")
        parity.assert_end_to_end(oracle_lib, wl, U, S, o["eps"], o["S"], f"scan iteration {i}",
                                 u=u)
        u = o["U"]
    ctl.close()
    # the graph sequence against single iterations on the GPU's own warm start
    one = mppi.Controller(wl)
    one.set_tuning(**tune)
    for _ in range(wl.iters):
        one.iterate(1)
    U_one, S_one = _np(one.controls()), _np(one.costs())
    one.close()
    assert np.array_equal(U_seq.view(np.uint32), U_one.view(np.uint32))
    assert np.array_equal(S_seq.view(np.uint32), S_one.view(np.uint32))


def test_scan_form_refusals(mppi):
    from paper_2409_07563_amd import MPPIError
    for wl in (W.c3(K=64, T=10), W.c1(K=64, T=10), W.c2("circles", K=64, T=257, iters=1)):
        ctl = mppi.Controller(wl)
        with pytest.raises(MPPIError) as e:
            ctl.set_tuning(**SCAN)
        assert e.value.status == -5  # MPPI_EUNSUPPORTED
        ctl.close()
    ctl = mppi.Controller(W.c2("circles", K=64, T=10, iters=1))
    with pytest.raises(MPPIError) as e:
        ctl.set_tuning(rollout_form=2, lanes_per_sample=8)
    assert e.value.status == -1  # MPPI_EINVAL
    ctl.close()
