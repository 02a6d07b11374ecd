"""The MLP's bfloat16 mode (MPPI_F_BF16_MLP: the three products on
v_mfma_f32_16x16x32_bf16 with bfloat16 operands and binary32 accumulation)
against the oracle's bfloat16 option, which rounds the weights and the
products' inputs at the same points, through the C ABI.

Costs: the bounds of tests/parity.py (assert_costs_close_bf16): every sample
within the binary32 bound plus the first-order effect of rounding decisions
going the other way, at most 1 % of the samples needing that allowance, and
the GPU's median deviation a small fraction of the roundings' own effect.
Gradient: the adjoint differentiates the bfloat16 forward with the roundings
taken as the identity, as the oracle's option does, so the binary32 mode's
gradient bound applies unchanged; central differences of the GPU's own
bfloat16 forward check it independently of the oracle.  The binary32 mode
stays the 1e-4 gate (tests/test_gpu_grad.py)."""
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


def _c5(K, T, H=64, **kw):
    return W.c5(K=K, T=T, hidden=H).replace(mlp_bf16=1, **kw)


def _costs(mppi, wl, **kw):
    c = mppi.Controller(wl, **kw)
    c.sample()
    c.rollout()
    S = _np(c.costs()).astype(np.float64)
    eps = _np(c.noise())
    c.close()
    return S, eps


def _oracle(oracle_lib, wl, eps, u=None):
    S_bf = oracle_lib.rollout_costs_parallel(wl, eps, u=u)
    S_fp = oracle_lib.rollout_costs_parallel(wl.replace(mlp_bf16=0), eps, u=u)
    cond, cond_bf = oracle_lib.cost_condition(wl, eps, u=u, bf=True)
    return S_bf, S_fp, cond, cond_bf


@pytest.mark.parametrize("H,K,T", [(64, 2048, 1), (64, 1000, 60), (16, 777, 40), (32, 300, 25),
                                   (64, 37, 13), (64, 1, 5), (64, 1024, 100)])
def test_bf16_rollout_costs(mppi, oracle_lib, H, K, T):
    wl = _c5(K, T, H)
    S, eps = _costs(mppi, wl)
    assert np.array_equal(eps.view(np.uint32), oracle_lib.workload_noise(wl).view(np.uint32))
    S_bf, S_fp, cond, cond_bf = _oracle(oracle_lib, wl, eps)
    parity.assert_costs_close_bf16(S, S_bf, S_fp, cond, cond_bf, f"bf16 H={H} K={K} T={T}")


def test_bf16_full_size_sampled(mppi, oracle_lib):
    """K 8192, T 100, H 64 (the differentiable workload) in the launch shape
    the benchmark uses, checked on 512 samples drawn across the whole range
    (the samples are independent: each is the oracle's own rollout of its
    noise column)."""
    wl = _c5(8192, 100)
    c = mppi.Controller(wl)
    c.autotune(reps=2)
    c.sample()
    c.rollout()
    S = _np(c.costs()).astype(np.float64)
    eps = _np(c.noise())
    c.close()
    idx = np.sort(np.random.default_rng(9).choice(wl.K, 512, replace=False))
    sub = wl.replace(K=len(idx))
    e = np.ascontiguousarray(eps[:, :, idx])
    S_bf, S_fp, cond, cond_bf = _oracle(oracle_lib, sub, e)
    parity.assert_costs_close_bf16(S[idx], S_bf, S_fp, cond, cond_bf, "bf16 full size (sampled)")


def test_bf16_iterations_end_to_end(mppi, oracle_lib):
    wl = _c5(2048, 60)
    c = mppi.Controller(wl)
    u = wl.u0.astype(np.float64)
    for it in range(3):
        c.sample()
        c.rollout()
        c.update()
        eps = _np(c.noise())
        S = _np(c.costs()).astype(np.float64)
        U = _np(c.controls())
        S_bf, S_fp, cond, cond_bf = _oracle(oracle_lib, wl, eps, u=u)
        parity.assert_costs_close_bf16(S, S_bf, S_fp, cond, cond_bf, f"bf16 iteration {it}")
        parity.assert_end_to_end(oracle_lib, wl, U, S, eps, S_bf, f"bf16 iteration {it}", u=u)
        u = U.astype(np.float64)
    c.close()


def test_bf16_graph_iterations_equal_staged(mppi):
    wl = _c5(1000, 30)
    a = mppi.Controller(wl)
    a.iterate(3)
    b = mppi.Controller(wl)
    for _ in range(3):
        b.sample()
        b.rollout()
        b.update()
    assert np.array_equal(_np(a.controls()).view(np.uint32), _np(b.controls()).view(np.uint32))
    a.close()
    b.close()


def test_bf16_differs_from_binary32_mode(mppi):
    # the flag reaches the kernels: the two modes differ by the roundings
    wl = _c5(512, 20)
    S16, _ = _costs(mppi, wl)
    S32, _ = _costs(mppi, wl.replace(mlp_bf16=0))
    rel = np.abs(S16 - S32) / np.maximum(np.abs(S32), 1.0)
    assert np.median(rel) > 1e-5 and rel.max() < 0.1


# ---------------------------------------------------------------------------
# adjoint
# ---------------------------------------------------------------------------
def _assert_grad_close(g, ref, name=""):
    scale = 1e-4 * ref["grad_abs"]
    tol = scale + 1e-3 * scale.max()
    err = np.abs(g - ref["grad"])
    bad = np.flatnonzero(err > tol)
    assert bad.size == 0, (f"{name}: {bad.size} of {g.size} entries off, first {bad[:5]}: "
                           f"gpu {g[bad[:5]]} oracle {ref['grad'][bad[:5]]} "
                           f"worst ratio {(err / tol).max():.3g}")


@pytest.mark.parametrize("H,K,T,ce,lam", [
    (64, 1024, 40, 10, 50.0), (64, 1024, 40, 10, 0.5), (16, 700, 33, 10, 50.0),
    (32, 256, 20, 7, 5.0), (64, 333, 50, 64, 50.0), (64, 100, 23, 1, 50.0)])
def test_bf16_backward_vs_oracle(mppi, oracle_lib, H, K, T, ce, lam):
    wl = _c5(K, T, H, lam=lam)
    uref = W.c5_uref(T=T)
    c = mppi.Controller(wl, requires_grad=True, checkpoint_every=ce)
    c.sample()
    c.rollout()
    c.update()
    U = _np(c.controls()).astype(np.float64)
    G = (2.0 * (U - uref)).astype(np.float32)
    g = _np(c.backward(G)).astype(np.float64)
    S = _np(c.costs()).astype(np.float64)
    eps = _np(c.noise())
    c.close()
    ref = oracle_lib.backward(wl, G.astype(np.float64), eps=eps, S=S)
    _assert_grad_close(g, ref, name=f"bf16 H={H} K={K} T={T} c={ce} lambda={lam}")
    # and the binary64 model's gradient is measurably another one
    ref64 = oracle_lib.backward(wl.replace(mlp_bf16=0), G.astype(np.float64), eps=eps, S=S)
    assert np.abs(g - ref64["grad"]).max() > np.abs(g - ref["grad"]).max()


def test_bf16_gradient_against_gpu_finite_differences(mppi):
    # central differences of the GPU's bfloat16 forward for the wheelbase and
    # the Q diagonal.  The forward rounds the states it feeds the MLP, so it
    # is piecewise smooth in the wheelbase; a step of 1e-2 relative crosses
    # many rounding boundaries over the samples and the quotient follows the
    # straight-through derivative.  Bound as in the binary32 mode's check.
    wl = _c5(2048, 40, 16, lam=50.0)
    uref = W.c5_uref(T=40)
    c = mppi.Controller(wl, requires_grad=True)
    th = c.theta().numpy().astype(np.float64)

    def loss(theta):
        c.set_theta(theta.astype(np.float32))
        c.set_controls(wl.u0)
        c.set_iteration(0)
        c.sample()
        c.rollout()
        c.update()
        U = _np(c.controls()).astype(np.float64)
        return float(((U - uref) ** 2).sum()), U

    L0, U0 = loss(th)
    g = _np(c.backward((2.0 * (U0 - uref)).astype(np.float32))).astype(np.float64)
    idx = list(range(th.size - 6, th.size))
    fd = []
    for i in idx:
        h = 1e-2 * max(1.0, abs(th[i]))
        tp, tm = th.copy(), th.copy()
        tp[i] += h
        tm[i] -= h
        fd.append((loss(tp)[0] - loss(tm)[0]) / (2 * h))
    fd = np.array(fd)
    assert np.all(np.abs(g[idx] - fd) <= 1e-2 * np.abs(fd).max() + 1e-3 * np.abs(fd)), (g[idx], fd)
    c.close()


def test_bf16_set_theta(mppi, oracle_lib):
    wl = _c5(400, 30, 16)
    c = mppi.Controller(wl, requires_grad=True)
    th = oracle_lib.theta_of(wl)
    rng = np.random.default_rng(5)
    th2 = th + 0.05 * rng.normal(size=th.size) * np.abs(th).clip(0.1)
    th2[-1] = 2.2
    th2 = th2.astype(np.float32)
    c.set_theta(th2)
    c.sample()
    c.rollout()
    S = _np(c.costs()).astype(np.float64)
    eps = _np(c.noise())
    c.close()
    wl2 = oracle_lib.with_theta(wl, th2.astype(np.float64))
    S_bf, S_fp, cond, cond_bf = _oracle(oracle_lib, wl2, eps)
    parity.assert_costs_close_bf16(S, S_bf, S_fp, cond, cond_bf, "bf16 after set_theta")


@pytest.mark.parametrize("H,block", [(64, 128), (64, 256), (32, 128)])
def test_bf16_split_forms_are_bitwise_the_single_wave_form(mppi, H, block):
    """The MLP split over 2 or 4 waves (h2 tiles exchanged, the output formed
    over every K-block in order) computes every product as the one-wave
    kernel does: costs, controls and gradients bitwise equal."""
    wl = _c5(1000, 30, H, lam=50.0)
    uref = W.c5_uref(T=30)
    out = []
    for b in (64, block):
        c = mppi.Controller(wl, requires_grad=True, checkpoint_every=7)
        c.set_tuning(rollout_block=b)
        c.sample()
        c.rollout()
        c.update()
        U = _np(c.controls())
        G = (2.0 * (U.astype(np.float64) - uref)).astype(np.float32)
        g = _np(c.backward(G))
        out.append((_np(c.costs()), U, g))
        c.close()
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    # and the plain (non-gradient) split forward too
    S = []
    for b in (64, block):
        c = mppi.Controller(wl)
        c.set_tuning(rollout_block=b)
        c.sample()
        c.rollout()
        S.append(_np(c.costs()))
        c.close()
    assert np.array_equal(S[0].view(np.uint32), S[1].view(np.uint32))


def test_bf16_refusals(mppi):
    from paper_2409_07563_amd import MPPIError
    with pytest.raises(MPPIError) as e:
        mppi.Controller(W.c2("circles", K=64, T=10, iters=1).replace(mlp_bf16=1))
    assert e.value.status == -1  # MPPI_EINVAL
