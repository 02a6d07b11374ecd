"""Pins of the oracle's update options: the importance-sampling term
(section "MPPI-Generic's MPPI Implementation", Eqs. info_theory_weighting and
information_theoretic_weighting, beta in {0, 1}) and the step size gamma of
the dynamic mirror-descent update (section "Comparisons to sampling-efficient
algorithms").

The importance-sampling weight is p(V)/s(V|theta) with p the zero-mean and s
the u-mean Gaussian of covariance diag(sigma^2); the tests evaluate it from
the Gaussian densities themselves (scipy's log-pdf, mpmath's pdf), not from
the closed form the oracle uses.  The cost inflation of the cost-complexity
experiment (Results section: nested cosines scaled by zero) must leave every
cost unchanged.
"""
import numpy as np
import pytest
from scipy.stats import norm

import workloads as W


def _lam32(wl):
    return float(np.float32(wl.lam))


def _log_ratio(wl, eps):
    """ln p(V^k)/s(V^k|u) for every sample, from Gaussian log-densities."""
    u = wl.u0.astype(np.float64)[:, :, None]
    v = u + eps.astype(np.float64)
    sg = wl.sigma.astype(np.float64)[None, :, None]
    return (norm.logpdf(v, 0.0, sg) - norm.logpdf(v, u, sg)).sum(axis=(0, 1))


def _with_controls(wl, seed, scale):
    wl.u0 = np.random.default_rng(seed).normal(0, scale, (wl.T, wl.m)).astype(np.float32)
    return wl


def test_is_term_is_minus_lambda_log_density_ratio(oracle_lib):
    wl = _with_controls(W.c2(K=512, T=40, iters=1), 5, 0.4)
    eps = oracle_lib.workload_noise(wl)
    S0, _, _ = oracle_lib.rollout_costs(wl, eps=eps)
    S1, _, _ = oracle_lib.rollout_costs(wl.replace(is_beta=1), eps=eps)
    I = _log_ratio(wl, eps)
    scale = np.abs(S0) + np.abs(_lam32(wl) * I)
    assert np.all(np.abs((S1 - S0) - (-_lam32(wl) * I)) <= 1e-12 * scale)


def test_is_term_vanishes_at_zero_mean(oracle_lib):
    wl = W.c2(K=256, T=30, iters=1)
    assert not wl.u0.any()
    eps = oracle_lib.workload_noise(wl)
    S0, _, _ = oracle_lib.rollout_costs(wl, eps=eps)
    S1, _, _ = oracle_lib.rollout_costs(wl.replace(is_beta=1), eps=eps)
    assert np.array_equal(S0, S1)


def test_is_weights_are_the_reweighted_softmin(oracle_lib):
    """w_k is proportional to exp(-J_k/lambda) p(V^k)/s(V^k)."""
    wl = _with_controls(W.c1(K=300, T=25), 11, 0.3)
    eps = oracle_lib.workload_noise(wl)
    J, _, _ = oracle_lib.rollout_costs(wl, eps=eps)
    wis = wl.replace(is_beta=1)
    S, _, _ = oracle_lib.rollout_costs(wis, eps=eps)
    w, U, stats, rc = oracle_lib.softmin_update(wis, S, eps)
    logq = -J / _lam32(wl) + _log_ratio(wl, eps)
    ref = np.exp(logq - logq.max())
    ref /= ref.sum()
    assert rc == 0
    cond = 64 * np.finfo(float).eps * np.abs(logq).max()
    assert np.allclose(w, ref, rtol=1e-10 + cond, atol=1e-300)


def _mp_options(wl, eps, gamma):
    """Algorithm 1 with the importance-sampling weight and the step size, in
    50-digit mpmath for the Euler double integrator and the quadratic cost:
    rollout, cost after each step, terminal cost; weight exp(-J/lambda) times
    the product of Gaussian densities p/s; U = (1-gamma) u + gamma E_w[v]."""
    import mpmath as mp
    mp.mp.dps = 50
    T, m, K = eps.shape
    dt = mp.mpf(float(np.float32(wl.dt)))
    cw = [mp.mpf(float(v)) for v in wl.w]
    goal = [mp.mpf(float(v)) for v in wl.ref]
    sg = [mp.mpf(float(v)) for v in wl.sigma]
    lam = mp.mpf(_lam32(wl))
    g = mp.mpf(float(np.float32(gamma)))
    u = [[mp.mpf(float(wl.u0[t, j])) for j in range(m)] for t in range(T)]
    q, V = [], []
    for k in range(K):
        x = [mp.mpf(float(c)) for c in wl.x0]
        J = mp.mpf(0)
        ratio = mp.mpf(1)
        vs = []
        for t in range(T):
            v = [u[t][j] + mp.mpf(float(eps[t, j, k])) for j in range(m)]
            vs.append(v)
            for j in range(m):
                ratio *= mp.npdf(v[j], 0, sg[j]) / mp.npdf(v[j], u[t][j], sg[j])
            x = [x[0] + dt * x[2], x[1] + dt * x[3], x[2] + dt * v[0], x[3] + dt * v[1]]
            J += sum(cw[i] * (x[i] - goal[i]) ** 2 for i in range(4))
            J += sum(cw[8 + j] * v[j] ** 2 for j in range(m))
        J += sum(cw[16 + i] * (x[i] - goal[i]) ** 2 for i in range(4))
        q.append(mp.e ** (-J / lam) * ratio)
        V.append(vs)
    tot = sum(q)
    w = [a / tot for a in q]
    U = [[(1 - g) * u[t][j] + g * sum(w[k] * V[k][t][j] for k in range(K))
          for j in range(m)] for t in range(T)]
    return w, U


@pytest.mark.parametrize("K,T,lam,gamma", [(1, 1, 1.0, 0.5), (2, 1, 1.0, 0.25),
                                           (3, 2, 2.0, 1.0), (4, 2, 30.0, 0.7),
                                           (3, 3, 0.5, 0.0)])
def test_tiny_problems_against_mpmath_brute_force(oracle_lib, K, T, lam, gamma):
    wl = _with_controls(W.c1(K=K, T=T), 100 + K * T, 0.5)
    wl.lam = lam
    wl = wl.replace(is_beta=1, gamma=gamma)
    eps = oracle_lib.workload_noise(wl)
    S, _, _ = oracle_lib.rollout_costs(wl, eps=eps)
    w, U, stats, rc = oracle_lib.softmin_update(wl, S, eps)
    w_mp, U_mp = _mp_options(wl, eps, gamma)
    assert rc == 0
    cond = 1e-12 + 64 * np.finfo(float).eps * np.abs(S).max() / _lam32(wl)
    assert np.allclose(w, [float(v) for v in w_mp], rtol=cond, atol=1e-300)
    assert np.allclose(U, np.array([[float(v) for v in row] for row in U_mp]),
                       rtol=cond, atol=cond)


def test_step_size_scales_the_correction(oracle_lib):
    wl = _with_controls(W.c2(K=1024, T=40, iters=1), 7, 0.2)
    eps = oracle_lib.workload_noise(wl)
    S, _, _ = oracle_lib.rollout_costs(wl, eps=eps)
    u = wl.u0.astype(np.float64)
    w1, U1, _, _ = oracle_lib.softmin_update(wl, S, eps)
    w0, U0, _, _ = oracle_lib.softmin_update(wl.replace(gamma=0.0), S, eps)
    assert np.array_equal(U0, u)
    for g in (0.125, 0.5, 2.0):           # powers of two: exact scaling
        wg, Ug, _, _ = oracle_lib.softmin_update(wl.replace(gamma=g), S, eps)
        assert np.array_equal(wg, w1)
        assert np.allclose(Ug - u, g * (U1 - u), rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("make", [lambda: W.c2("circles", K=64, T=30, iters=1),
                                  lambda: W.c3(K=32, T=20), lambda: W.c1(K=50, T=10)])
def test_cost_inflation_adds_exactly_zero(oracle_lib, make):
    wl = make()
    eps = oracle_lib.workload_noise(wl)
    S0, m0, c0 = oracle_lib.rollout_costs(wl, eps=eps)
    S1, m1, c1 = oracle_lib.rollout_costs(wl.replace(cost_cosines=40), eps=eps)
    assert np.array_equal(S0, S1) and np.array_equal(c0, c1)


def test_shift_worked_example(oracle_lib):
    """The warm start of an MPC step (section "Beginner": the nominal
    sequence moves forward by the optimisation stride), worked by hand."""
    wl = W.c1(K=4, T=3)
    u = np.array([[1.0, 2.0], [3.0, 4.0], [5.0, 6.0]])
    assert np.array_equal(oracle_lib.shift(wl, u, 1), [[3, 4], [5, 6], [5, 6]])
    assert np.array_equal(oracle_lib.shift(wl, u, 1, "zero"), [[3, 4], [5, 6], [0, 0]])
    assert np.array_equal(oracle_lib.shift(wl, u, 2), [[5, 6], [5, 6], [5, 6]])
    assert np.array_equal(oracle_lib.shift(wl, u, 0), u)
    assert np.array_equal(oracle_lib.shift(wl, u, 7, "zero"), np.zeros((3, 2)))


def test_shift_composes(oracle_lib):
    wl = W.c2("circles", K=8, T=37, iters=1)
    u = np.random.default_rng(2).normal(size=(37, 2))
    for fill in ("hold", "zero"):
        for a, b in ((1, 1), (3, 5), (20, 20), (0, 9)):
            two = oracle_lib.shift(wl, oracle_lib.shift(wl, u, a, fill), b, fill)
            assert np.array_equal(two, oracle_lib.shift(wl, u, a + b, fill))


# ---------------------------------------------------------------------------
# sampling options (section "Sampling Distributions")
# ---------------------------------------------------------------------------
def test_noiseless_mean_sample(oracle_lib):
    wl = _with_controls(W.c2("circles", K=200, T=30, iters=1), 12, 0.4)
    plain = oracle_lib.workload_noise(wl)
    wm = wl.replace(mean_sample=1)
    eps = oracle_lib.workload_noise(wm)
    assert np.all(eps[:, :, 0].view(np.uint32) == 0)           # +0.0 exactly
    assert np.array_equal(eps[:, :, 1:], plain[:, :, 1:])
    S, _, _ = oracle_lib.rollout_costs(wm, eps=eps)
    assert S[0] == oracle_lib.sequence_cost(wl, wl.u0)


def test_zero_mean_samples(oracle_lib):
    wl = _with_controls(W.c2("circles", K=300, T=30, iters=1), 13, 0.4)
    wz = wl.replace(zero_frac=0.25, gamma=0.6)
    eps = oracle_lib.workload_noise(wz)
    S, _, _ = oracle_lib.rollout_costs(wz, eps=eps)
    S_u, _, _ = oracle_lib.rollout_costs(wl, eps=eps)
    S_0, _, _ = oracle_lib.rollout_costs(wl, eps=eps, u=np.zeros((30, 2)))
    n_plain = 300 - 75
    assert np.array_equal(S[:n_plain], S_u[:n_plain])
    assert np.array_equal(S[n_plain:], S_0[n_plain:])
    w, U, _, rc = oracle_lib.softmin_update(wz, S, eps)
    # the mirror-descent form over the samples' controls v_k
    u = wl.u0.astype(np.float64)
    v = eps.astype(np.float64).copy()
    v[:, :, :n_plain] += u[:, :, None]
    U_ref = (1 - np.float32(0.6)) * u + np.float32(0.6) * np.tensordot(v, w, axes=([2], [0]))
    assert rc == 0 and np.allclose(U, U_ref, rtol=1e-13, atol=1e-13)


def test_all_samples_around_zero_forget_u(oracle_lib):
    """With every sample drawn around zero (and gamma = 1, no importance
    term) the update is sum_k w_k eps_k, whatever u was."""
    wl = W.c1(K=64, T=12).replace(zero_frac=1.0)
    a = oracle_lib.mppi(_with_controls(wl, 1, 0.5), iters=1)
    b = oracle_lib.mppi(_with_controls(wl, 2, 0.5), iters=1)
    assert np.array_equal(a["S"], b["S"])
    assert np.allclose(a["U"], b["U"], rtol=0, atol=1e-14)


def test_time_varying_sigma(oracle_lib):
    wl = _with_controls(W.c2("circles", K=100, T=25, iters=1), 14, 0.3)
    z = oracle_lib.noise(wl.seed, 0, wl.instance, wl.K, wl.T, wl.m, np.ones(2, np.float32))
    sig_t = np.random.default_rng(4).uniform(0.2, 1.5, (25, 2)).astype(np.float32)
    ws = wl.replace(sigma_t=sig_t)
    eps = oracle_lib.workload_noise(ws)
    assert np.array_equal(eps, (sig_t[:, :, None] * z).astype(np.float32))
    const = wl.replace(sigma_t=np.tile(wl.sigma, (25, 1)))
    assert np.array_equal(oracle_lib.workload_noise(const), oracle_lib.workload_noise(wl))
    # the importance term against per-step Gaussian log-densities
    S0, _, _ = oracle_lib.rollout_costs(ws, eps=eps)
    S1, _, _ = oracle_lib.rollout_costs(ws.replace(is_beta=1), eps=eps)
    u = ws.u0.astype(np.float64)[:, :, None]
    v = u + eps.astype(np.float64)
    sg = sig_t.astype(np.float64)[:, :, None]
    I = (norm.logpdf(v, 0.0, sg) - norm.logpdf(v, u, sg)).sum(axis=(0, 1))
    scale = np.abs(S0) + np.abs(_lam32(ws) * I)
    assert np.all(np.abs((S1 - S0) + _lam32(ws) * I) <= 1e-12 * scale)
