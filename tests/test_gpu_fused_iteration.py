"""The one-launch form of a single context (batch_form = 1 on a single
double-integrator context with forward Euler and the quadratic cost): the
whole iteration in one time-parallel launch (noise drawn by the lanes that
use it, the linear model's states as two row scans, tile partials of the
softmin and of the weighted noise rows, the last workgroup's combination),
against the binary64 oracle through the C ABI.  The noise is bitwise the
noise kernel's; costs at the 1e-4 bound; controls end to end (exact
propagation, first order and the flat 1e-4 bound); statistics; every
compiled chunk length with full, partial and empty lanes; the sampling and
update options; ten warm-started iterations from a captured graph; and the
per-phase form on the same context."""
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


FUSED = dict(batch_form=1)


def _one(mppi, wl, iters=1):
    ctl = mppi.Controller(wl)
    ctl.set_tuning(**FUSED)
    ctl.iterate(iters)
    out = dict(S=_np(ctl.costs()).astype(np.float64), eps=_np(ctl.noise()),
               U=_np(ctl.controls()), stats=ctl.stats())
    ctl.close()
    return out


def _check(oracle_lib, wl, g, name, u=None, iteration=0):
    o = oracle_lib.mppi(wl, iters=1, iter0=iteration,
                        u=None if u is None else np.asarray(u, np.float64))
    assert np.array_equal(g["eps"].view(np.uint32), o["eps"].view(np.uint32)), name
    S_or, _, _ = oracle_lib.rollout_costs(wl, eps=o["eps"], u=u, iteration=iteration)
    parity.assert_costs_close(g["S"], S_or, name=name)
    parity.assert_end_to_end(oracle_lib, wl, g["U"], g["S"], o["eps"], S_or, name, u=u)
    w_or, _, stats_or, rc = oracle_lib.softmin_update(wl, g["S"], o["eps"],
                                                     u=wl.u0 if u is None else u)
    assert rc == 0 and g["stats"]["status"] == 0
    assert g["stats"]["rho"] == pytest.approx(stats_or[0], rel=1e-7)
    assert g["stats"]["eta"] == pytest.approx(stats_or[1], rel=1e-4)
    assert g["stats"]["ess"] == pytest.approx(stats_or[3], rel=1e-4)
    assert g["stats"]["free_energy"] == pytest.approx(stats_or[2], rel=1e-4, abs=1e-4)
    return o


@pytest.mark.parametrize("lam", [1.0, 100.0], ids=["c1", "c1_tempered"])
def test_fused_c1_iteration(mppi, oracle_lib, lam):
    wl = W.c1().replace(lam=lam)
    g = _one(mppi, wl)
    _check(oracle_lib, wl, g, f"fused c1 lambda={lam}")
    assert g["stats"]["iteration"] == 1
    if lam > 1.0:
        assert g["stats"]["ess"] > 50


# every chunk length C = 2 ceil(T / 32) (2 .. 16) with full, partial and
# empty lanes; one sample, a partial last tile, the most samples (4096)
@pytest.mark.parametrize("K,T", [(1, 1), (1, 2), (15, 31), (16, 32), (17, 33), (100, 64),
                                 (1000, 65), (333, 96), (64, 100), (129, 127), (50, 160),
                                 (257, 161), (31, 200), (4096, 224), (7, 255), (20, 256)])
def test_fused_shapes(mppi, oracle_lib, K, T):
    wl = W.c1(K=K, T=T).replace(lam=10.0)
    g = _one(mppi, wl)
    _check(oracle_lib, wl, g, f"fused K{K} T{T}")


@pytest.mark.parametrize("opt", ["is_gamma", "zero_mean", "mean_sample", "sigma_t", "cosines"])
def test_fused_options(mppi, oracle_lib, opt):
    wl = W.c1(K=1000, T=93).replace(lam=10.0)
    u0 = np.random.default_rng(3).normal(0.0, 0.5, (wl.T, wl.m)).astype(np.float32)
    wl = wl.replace(u0=u0)
    if opt == "is_gamma":
        wl = wl.replace(is_beta=1, gamma=0.4)
    elif opt == "zero_mean":
        wl = wl.replace(zero_frac=0.25)
    elif opt == "mean_sample":
        wl = wl.replace(mean_sample=1)
    elif opt == "sigma_t":
        sig = np.linspace(0.5, 1.5, wl.T)[:, None] * wl.sigma[None, :]
        wl = wl.replace(sigma_t=sig.astype(np.float32))
    else:
        wl = wl.replace(cost_cosines=3)
    g = _one(mppi, wl)
    _check(oracle_lib, wl, g, f"fused {opt}")


def test_fused_ten_iterations_from_graph(mppi, oracle_lib):
    """Ten warm-started iterations replayed from the captured graph equal ten
    single iterations bitwise, and every iteration matches the oracle from
    the GPU's own warm start."""
    wl = W.c1()
    seq = mppi.Controller(wl)
    seq.set_tuning(**FUSED)
    seq.iterate(10)
    U_seq, S_seq = _np(seq.controls()), _np(seq.costs())
    assert seq.stats()["iteration"] == 10
    seq.close()
    ctl = mppi.Controller(wl)
    ctl.set_tuning(**FUSED)
    u = wl.u0.astype(np.float64)
    for i in range(10):
        ctl.iterate(1)
        g = dict(S=_np(ctl.costs()).astype(np.float64), eps=_np(ctl.noise()),
                 U=_np(ctl.controls()), stats=ctl.stats())
        _check(oracle_lib, wl, g, f"fused iteration {i}", u=u, iteration=i)
        u = g["U"].astype(np.float64)
    assert np.array_equal(U_seq.view(np.uint32), g["U"].view(np.uint32))
    assert np.array_equal(S_seq.view(np.uint32), g["S"].astype(np.float32).view(np.uint32))
    ctl.close()


def test_fused_and_per_phase_forms_on_one_context(mppi, oracle_lib):
    """Switching forms on a live context: the per-phase form's iterations
    (noise drawn ahead into the second buffer) and the one-launch form's
    continue one iteration sequence, each iteration on its own noise."""
    wl = W.c1(K=512, T=50).replace(lam=10.0)
    ctl = mppi.Controller(wl)
    u = wl.u0.astype(np.float64)
    for i, form in enumerate([0, 0, 1, 1, 0, 1]):
        ctl.set_tuning(batch_form=form)
        ctl.iterate(1)
        g = dict(S=_np(ctl.costs()).astype(np.float64), eps=_np(ctl.noise()),
                 U=_np(ctl.controls()), stats=ctl.stats())
        _check(oracle_lib, wl, g, f"form {form} iteration {i}", u=u, iteration=i)
        assert g["stats"]["iteration"] == i + 1
        u = g["U"].astype(np.float64)
    ctl.close()


def test_fused_autotune_and_refusals(mppi):
    from paper_2409_07563_amd import MPPIError
    ctl = mppi.Controller(W.c1())
    rep = ctl.autotune(reps=3)
    assert any(t["phase"] == "iteration" and t["batch"] == 1 for t in rep["timings"])
    ctl.close()
    for wl in (W.c2("circles", K=64, T=10, iters=1), W.c1(K=4097, T=10),
               W.c1(K=64, T=257), W.c1(K=64, T=10).replace(integrator="rk4")):
        ctl = mppi.Controller(wl)
        with pytest.raises(MPPIError) as e:
            ctl.set_tuning(**FUSED)
        assert e.value.status == -5  # MPPI_EUNSUPPORTED
        ctl.close()
    # staged phases on a context in the one-launch form still run per phase
    wl = W.c1(K=64, T=10)
    ctl = mppi.Controller(wl)
    ctl.set_tuning(**FUSED)
    ctl.sample()
    ctl.rollout()
    ctl.update()
    assert ctl.stats()["iteration"] == 1
    ctl.close()
