"""Pins for the oracle's gradient of a loss on the updated controls.

The adjoint (a reverse sweep through the softmin Jacobian, the RK4 stages and
the MLP residual) is checked against central finite differences of the
oracle's own forward iteration, which runs through entirely separate code
(the rollout, the update and the loss are re-evaluated at perturbed
parameters).  Central differences with step h have truncation error O(h^2);
a first-layer weight that multiplies a position of tens of metres sits where
the loss is strongly curved, so the difference quotients at h and h/2 are
combined by Richardson extrapolation (error O(h^4)).
"""
import numpy as np
import pytest

import workloads as W
from oracle import oracle as O


def _central(wl, uref, theta, i, h):
    tp = theta.copy()
    tp[i] += h
    tm = theta.copy()
    tm[i] -= h
    return (O.loss_and_controls(wl, uref, tp)[0] - O.loss_and_controls(wl, uref, tm)[0]) / (2 * h)


def _fd(wl, uref, theta, i, h):
    return (4.0 * _central(wl, uref, theta, i, h / 2) - _central(wl, uref, theta, i, h)) / 3.0


def _check(wl, uref, idx, rtol=2e-5):
    L0, U0 = O.loss_and_controls(wl, uref)
    r = O.backward(wl, 2.0 * (U0 - uref))
    assert r["status"] == 0
    np.testing.assert_allclose(r["U"], U0, rtol=0, atol=1e-12)
    theta = O.theta_of(wl)
    scale = np.max(np.abs(r["grad"]))
    for i in idx:
        h = 1e-3 * max(1.0, abs(theta[i]))
        fd = _fd(wl, uref, theta, i, h)
        assert abs(r["grad"][i] - fd) <= rtol * max(abs(fd), 1e-3 * scale), (i, r["grad"][i], fd)
    return r


def test_adjoint_vs_fd_bicycle_mlp():
    wl = W.c5(K=64, T=20, hidden=16)
    uref = W.c5_uref(T=20)
    n = O.n_grad(wl)
    rng = np.random.default_rng(1)
    H = 16
    nmlp = 7 * H + H + H * H + H + 5 * H + 5
    # a few entries of every parameter block, every Q entry and the wheelbase
    blocks = [(0, 7 * H), (7 * H, 8 * H), (8 * H, 8 * H + H * H), (8 * H + H * H, 9 * H + H * H),
              (9 * H + H * H, 14 * H + H * H), (14 * H + H * H, nmlp)]
    idx = [int(rng.integers(a, b)) for a, b in blocks for _ in range(3)]
    idx += list(range(nmlp, n))
    _check(wl, uref, idx)


def test_adjoint_vs_fd_plain_bicycle():
    wl = W.c5(K=48, T=15, hidden=16).replace(model="bicycle", mlp=None, mlp_hidden=0)
    uref = W.c5_uref(T=15)
    r = _check(wl, uref, range(O.n_grad(wl)))
    assert O.n_grad(wl) == 6
    assert np.all(np.isfinite(r["grad"]))


@pytest.mark.parametrize("gamma", [0.6, 1.0])
def test_adjoint_vs_fd_with_importance_sampling_and_step_size(gamma):
    """The importance-sampling term does not depend on theta but reweights the
    samples; the step size scales U - u and with it the gradient."""
    wl = W.c5(K=48, T=15, hidden=8)
    wl.u0 = np.random.default_rng(9).normal(0, 0.3, (wl.T, wl.m)).astype(np.float32)
    wl = wl.replace(is_beta=1, gamma=gamma)
    uref = W.c5_uref(T=15)
    rng = np.random.default_rng(4)
    n = O.n_grad(wl)
    idx = sorted(set(int(i) for i in rng.integers(0, n - 6, 8))) + list(range(n - 6, n))
    _check(wl, uref, idx)


def test_adjoint_linear_in_loss_gradient():
    wl = W.c5(K=32, T=10, hidden=8)
    rng = np.random.default_rng(2)
    G1, G2 = rng.normal(size=(2, 10, 2))
    g1 = O.backward(wl, G1)["grad"]
    g2 = O.backward(wl, G2)["grad"]
    g12 = O.backward(wl, 0.5 * G1 - 2.0 * G2)["grad"]
    np.testing.assert_allclose(g12, 0.5 * g1 - 2.0 * g2, rtol=1e-10, atol=1e-12 * np.abs(g1).max())


def test_adjoint_zero_when_loss_ignores_controls():
    wl = W.c5(K=16, T=8, hidden=8)
    r = O.backward(wl, np.zeros((8, 2)))
    assert np.all(r["grad"] == 0.0)


def test_adjoint_single_sample_has_no_gradient():
    # with K = 1 the weight is 1 whatever the cost: U = u + eps_0
    wl = W.c5(K=1, T=8, hidden=8)
    r = O.backward(wl, np.ones((8, 2)))
    assert np.all(r["grad"] == 0.0)


def test_adjoint_rejects_other_models():
    with pytest.raises(ValueError):
        O.backward(W.c1(K=8, T=4), np.zeros((4, 2)))


# ---------------------------------------------------------------------------
# the dependence on the nominal sequence, and several warm-started iterations
# ---------------------------------------------------------------------------
def _central_u(wl, uref, u0, idx, h, iters):
    up = u0.copy()
    up.flat[idx] += h
    um = u0.copy()
    um.flat[idx] -= h
    Lp = O.loss_and_controls(wl, uref, iters=iters, u0=up)[0]
    Lm = O.loss_and_controls(wl, uref, iters=iters, u0=um)[0]
    return (Lp - Lm) / (2 * h)


def _fd_u(wl, uref, u0, idx, h, iters):
    return (4.0 * _central_u(wl, uref, u0, idx, h / 2, iters)
            - _central_u(wl, uref, u0, idx, h, iters)) / 3.0


def _fd_theta(wl, uref, theta, i, h, iters):
    def c(hh):
        tp = theta.copy()
        tp[i] += hh
        tm = theta.copy()
        tm[i] -= hh
        return (O.loss_and_controls(wl, uref, tp, iters=iters)[0]
                - O.loss_and_controls(wl, uref, tm, iters=iters)[0]) / (2 * hh)
    return (4.0 * c(h / 2) - c(h)) / 3.0


@pytest.mark.parametrize("model,is_beta", [("bicycle_mlp", 0), ("bicycle", 1)])
def test_control_gradient_vs_fd(model, is_beta):
    """dL/du = G + sum_k a_k dJ_k/du for one iteration (the costs depend on u
    through v = u + eps, and directly through the importance-sampling term)."""
    wl = W.c5(K=40, T=12, hidden=8)
    if model == "bicycle":
        wl = wl.replace(model="bicycle", mlp=None, mlp_hidden=0)
    u0 = np.random.default_rng(3).normal(0, 0.3, (wl.T, wl.m))
    wl = wl.replace(u0=u0.astype(np.float32), is_beta=is_beta, gamma=0.8)
    u0 = wl.u0.astype(np.float64)
    uref = W.c5_uref(T=wl.T)
    L0, U0 = O.loss_and_controls(wl, uref, u0=u0)
    G = 2.0 * (U0 - uref)
    r = O.backward(wl, G)
    dLdu = G + r["du"]
    scale = np.abs(dLdu).max()
    for idx in range(0, wl.T * wl.m, 3):
        fd = _fd_u(wl, uref, u0, idx, 1e-3, 1)
        assert abs(dLdu.flat[idx] - fd) <= 2e-5 * max(abs(fd), 1e-3 * scale), (idx, dLdu.flat[idx], fd)


@pytest.mark.parametrize("iters,is_beta,gamma", [(2, 0, 1.0), (3, 1, 0.7)])
def test_multi_iteration_gradient_vs_fd(iters, is_beta, gamma):
    """Through several warm-started iterations both theta and u0 matter at
    every iteration; each is checked against Richardson-extrapolated central
    differences of the oracle's own I-iteration forward."""
    wl = W.c5(K=48, T=12, hidden=8).replace(lam=20.0)
    u0 = np.random.default_rng(5).normal(0, 0.2, (wl.T, wl.m)).astype(np.float32)
    wl = wl.replace(u0=u0, is_beta=is_beta, gamma=gamma)
    uref = W.c5_uref(T=wl.T)
    L0, U0 = O.loss_and_controls(wl, uref, iters=iters)
    r = O.backward_iters(wl, 2.0 * (U0 - uref), iters)
    assert r["status"] == 0
    np.testing.assert_allclose(r["U"], U0, rtol=0, atol=1e-12)
    theta = O.theta_of(wl)
    n = O.n_grad(wl)
    rng = np.random.default_rng(6)
    idx = sorted(set(int(i) for i in rng.integers(0, n - 6, 6))) + list(range(n - 6, n))
    scale = np.abs(r["grad"]).max()
    for i in idx:
        h = 1e-3 * max(1.0, abs(theta[i]))
        fd = _fd_theta(wl, uref, theta, i, h, iters)
        assert abs(r["grad"][i] - fd) <= 2e-5 * max(abs(fd), 1e-3 * scale), (i, r["grad"][i], fd)
    su = np.abs(r["du0"]).max()
    for j in range(1, wl.T * wl.m, 5):
        fd = _fd_u(wl, uref, wl.u0.astype(np.float64), j, 1e-3, iters)
        assert abs(r["du0"].flat[j] - fd) <= 2e-5 * max(abs(fd), 1e-3 * su), (j, r["du0"].flat[j], fd)


def test_one_iteration_of_the_chain_is_the_single_backward():
    wl = W.c5(K=32, T=10, hidden=8)
    uref = W.c5_uref(T=10)
    L0, U0 = O.loss_and_controls(wl, uref)
    G = 2.0 * (U0 - uref)
    a = O.backward(wl, G)
    b = O.backward_iters(wl, G, 1)
    assert np.array_equal(a["grad"], b["grad"])
    assert np.array_equal(G + a["du"], b["du0"])


def test_gradient_with_sampling_options_vs_fd():
    """Per-step sigma (in the importance term's derivative) and the noiseless
    mean sample through two iterations."""
    wl = W.c5(K=40, T=10, hidden=8).replace(lam=20.0)
    sig_t = np.random.default_rng(8).uniform(0.5, 1.2, (10, 2)).astype(np.float32)
    u0 = np.random.default_rng(9).normal(0, 0.2, (10, 2)).astype(np.float32)
    wl = wl.replace(u0=u0, sigma_t=sig_t, mean_sample=1, is_beta=1, gamma=0.9)
    uref = W.c5_uref(T=10)
    L0, U0 = O.loss_and_controls(wl, uref, iters=2)
    r = O.backward_iters(wl, 2.0 * (U0 - uref), 2)
    theta = O.theta_of(wl)
    n = O.n_grad(wl)
    scale = np.abs(r["grad"]).max()
    for i in list(range(0, n - 6, 37)) + list(range(n - 6, n)):
        h = 1e-3 * max(1.0, abs(theta[i]))
        fd = _fd_theta(wl, uref, theta, i, h, 2)
        assert abs(r["grad"][i] - fd) <= 2e-5 * max(abs(fd), 1e-3 * scale), (i, r["grad"][i], fd)
    su = np.abs(r["du0"]).max()
    for j in range(0, 20, 3):
        fd = _fd_u(wl, uref, u0.astype(np.float64), j, 1e-3, 2)
        assert abs(r["du0"].flat[j] - fd) <= 2e-5 * max(abs(fd), 1e-3 * su), (j, r["du0"].flat[j], fd)


def test_backward_refuses_zero_mean_samples():
    wl = W.c5(K=16, T=5, hidden=8).replace(zero_frac=0.5)
    with pytest.raises(ValueError):
        O.backward(wl, np.zeros((5, 2)))
