"""GPU parity of the split rollout form (section "Split Kernel Description":
a dynamics kernel that writes the trajectories, then a cost kernel that is
parallel over time) and of the cost-complexity load (nested cosines scaled by
zero, Results section), through the C ABI, against the oracle.

Every dynamics / integrator / cost combination that has the split form is
run with one and with several cost waves per 64 samples (one workgroup, or
chunks of 16 waves added by a second kernel; ragged horizons, more waves than
steps), with the four-lane dynamics kernel where it exists; the
tolerances are those of tests/parity.py.  The cost load must leave every cost
bitwise unchanged (it adds +0) in each rollout kernel.
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


def _cases():
    c4 = W.c4(n_instances=2)[1].replace(K=700, T=60, u0=np.zeros((60, 2), np.float32))
    return {
        "c1": W.c1(K=1000, T=37),
        "di_rk4": W.c1(K=300, T=50).replace(integrator="rk4"),
        "c2_circles": W.c2("circles", K=2000, T=100, iters=1),
        "c2_costmap": W.c2("costmap", K=1500, T=100, iters=1),
        "c2_circles_euler": W.c2("circles", K=333, T=41, iters=1).replace(integrator="euler"),
        "c3": W.c3(K=1500, T=60),
        "goal_circles": c4,
        "track": W.c5(K=512, T=50).replace(model="bicycle", mlp=None, mlp_hidden=0),
        "short": W.c2("circles", K=65, T=5, iters=1),
    }


CASES = _cases()
QUAD = {n for n, w in CASES.items() if w.model == "bicycle" and w.integrator == "rk4"}
PARAMS = [(n, lanes, waves) for n in CASES for lanes in ((1, 4) if n in QUAD else (1,))
          for waves in (1, 4, 16, 64)]


def _run(mppi, wl, shape, debug=False):
    ctl = mppi.Controller(wl, debug=debug)
    ctl.set_tuning(**shape)
    ctl.sample()
    ctl.rollout()
    S = _np(ctl.costs()).astype(np.float64)
    eps = _np(ctl.noise())
    crashes = _np(ctl.crashes()) if debug else None
    ctl.update()
    U = _np(ctl.controls())
    st = ctl.stats()
    ctl.close()
    return S, eps, crashes, U, st


@pytest.mark.parametrize("name,lanes,waves", PARAMS)
def test_split_form_parity(mppi, oracle_lib, name, lanes, waves):
    wl = CASES[name]
    debug = wl.cost in ("path_circles", "goal_circles")
    shape = dict(rollout_form=1, lanes_per_sample=lanes, cost_waves=waves, rollout_block=128)
    S, eps, crashes, U, st = _run(mppi, wl, shape, debug=debug)
    assert np.array_equal(eps.view(np.uint32), oracle_lib.workload_noise(wl).view(np.uint32))
    S_or, margin, cr_or, slope = oracle_lib.rollout_costs(wl, eps=eps, slope=True)
    parity.assert_costs_close(S, S_or, margin, f"{name} split lanes={lanes} waves={waves}",
                              slope=slope if wl.cost == "path_costmap" else None)
    if debug:
        sure = margin >= parity.AMBIGUOUS_MARGIN
        assert np.array_equal(crashes[sure], cr_or[sure])
    parity.assert_end_to_end(oracle_lib, wl, U, S, eps, S_or, f"{name} split")
    assert st["status"] == 0


def test_split_form_ten_iterations_in_graph(mppi, oracle_lib):
    """The benchmark workload (K 8192, T 100) through iterate() (the captured
    graph) in the split form, every iteration from the oracle's warm start."""
    wl = W.c2("circles")
    ctl = mppi.Controller(wl)
    ctl.set_tuning(rollout_form=1, lanes_per_sample=4, cost_waves=8)
    u = wl.u0.astype(np.float64)
    for i in range(wl.iters):
        o = oracle_lib.mppi(wl, iters=1, iter0=i, u=u)
        ctl.set_controls(u.astype(np.float32))
        ctl.set_iteration(i)
        ctl.iterate(1)
        U = _np(ctl.controls())
        parity.assert_end_to_end(oracle_lib, wl, U, _np(ctl.costs()), o["eps"], o["S"],
                                 f"iteration {i}", u=u)
        u = o["U"]
    ctl.close()


def test_split_form_with_importance_sampling(mppi, oracle_lib):
    wl = W.c2("circles", K=1000, T=60, iters=1)
    wl = wl.replace(u0=np.random.default_rng(8).normal(0, 0.5, (60, 2)).astype(np.float32),
                    is_beta=1, gamma=0.5)
    S, eps, _, U, st = _run(mppi, wl, dict(rollout_form=1, lanes_per_sample=1, cost_waves=8))
    S_or, margin, _ = oracle_lib.rollout_costs(wl, eps=eps)
    parity.assert_costs_close(S, S_or, margin, "split + IS")
    parity.assert_end_to_end(oracle_lib, wl, U, S, eps, S_or, "split + IS")


# every rollout kernel: lane, grouped (4, 8, 16), split (1 and 4 lanes), the
# MLP tiles (1 and 4 waves), the batched kernel
KERNELS = [
    ("c2_circles", dict(lanes_per_sample=1)),
    ("c2_circles", dict(lanes_per_sample=4)),
    ("c2_circles", dict(lanes_per_sample=8)),
    ("c2_circles", dict(lanes_per_sample=16)),
    ("c2_circles", dict(rollout_form=1, lanes_per_sample=1, cost_waves=4)),
    ("c2_costmap", dict(rollout_form=1, lanes_per_sample=4, cost_waves=16)),
    ("c3", dict(lanes_per_sample=1)),
    ("mlp", dict(rollout_block=64)),
    ("mlp", dict(rollout_block=256)),
]


@pytest.mark.parametrize("name,shape", KERNELS)
def test_cost_load_leaves_costs_bitwise_unchanged(mppi, name, shape):
    if name == "mlp":
        wl = W.c5(K=300, T=30, hidden=64)
    else:
        wl = CASES[name].replace(K=500, T=40, u0=np.zeros((40, CASES[name].m), np.float32))
    a = _run(mppi, wl, shape)
    b = _run(mppi, wl.replace(cost_cosines=25), shape)
    assert np.array_equal(a[0], b[0])
    assert np.array_equal(a[3].view(np.uint32), b[3].view(np.uint32))


def test_cost_load_in_a_batch(mppi):
    insts = [wl.replace(K=min(wl.K, 500)) for wl in W.c4(n_instances=3)]
    outs = []
    for cos in (0, 25):
        ctl = mppi.Controller([wl.replace(cost_cosines=cos) for wl in insts])
        ctl.sample()
        ctl.rollout()
        outs.append(_np(ctl.costs()))
        ctl.close()
    assert np.array_equal(outs[0], outs[1])


def test_split_form_refused_where_it_does_not_exist(mppi):
    from paper_2409_07563_amd import _abi
    for ctl in (mppi.Controller(W.c5(K=128, T=10, hidden=16)),
                mppi.Controller([W.c2("circles", K=128, T=10), W.c2("circles", K=64, T=12)]),
                mppi.Controller(W.c5(K=128, T=10, hidden=16).replace(
                    model="bicycle", mlp=None, mlp_hidden=0), requires_grad=True)):
        with pytest.raises(_abi.MPPIError):
            ctl.set_tuning(rollout_form=1, lanes_per_sample=1)
        ctl.close()
    ctl = mppi.Controller(W.c3(K=128, T=10))
    with pytest.raises(_abi.MPPIError):
        ctl.set_tuning(rollout_form=1, lanes_per_sample=4)  # no quad form for the quadrotor
    with pytest.raises(_abi.MPPIError):
        ctl.set_tuning(rollout_form=1, cost_waves=3)
    ctl.close()


def test_autotuner_considers_both_forms(mppi, oracle_lib):
    """With a heavy cost (200 nested cosines per step) the tuner times the
    fused, split and (the bicycle with RK4) scan forms; whichever it keeps,
    the costs stay at parity."""
    wl = W.c2("circles", K=2048, T=100, iters=1).replace(cost_cosines=200)
    ctl = mppi.Controller(wl)
    res = ctl.autotune(reps=3)
    forms = {r.get("form") for r in res["timings"] if r["phase"] == "rollout"}
    assert forms == {0, 1, 2}
    ctl.sample()
    ctl.rollout()
    S = _np(ctl.costs()).astype(np.float64)
    eps = _np(ctl.noise())
    ctl.close()
    S_or, margin, _ = oracle_lib.rollout_costs(wl, eps=eps)
    parity.assert_costs_close(S, S_or, margin, f"after autotune {res['tuning']}")
