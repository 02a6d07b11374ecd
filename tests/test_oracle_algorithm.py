"""Pins of the oracle's Algorithm 1 (rollout costs, softmin weights, update).

Each test checks the oracle against a result that the mathematics fixes
independently of the oracle's code: the exact quadratic form of the Euler
double integrator, a 50-digit mpmath brute force of Algorithm 1, the
invariances of the update rule Eq. (mppi_update_rule), its temperature
limits, the free-energy identity (Section II-B) and the Gaussian optimal
density Eq. (optimal_distribution) in the linear-quadratic case.
"""
import math

import numpy as np
import pytest

import workloads as W


def di_matrices(T, dt):
    """Stacked Euler double-integrator maps: X = Phi x0 + Gam V with
    X = (x_1..x_T), V = (v_0..v_{T-1}); x_{t+1} = A x_t + B v_t."""
    A = np.eye(4)
    A[0, 2] = A[1, 3] = dt
    B = np.zeros((4, 2))
    B[2, 0] = B[3, 1] = dt
    Phi = np.zeros((4 * T, 4))
    Gam = np.zeros((4 * T, 2 * T))
    Ak = np.eye(4)
    for t in range(T):
        Ak = A @ Ak
        Phi[4 * t:4 * t + 4] = Ak
        for s in range(t + 1):
            Gam[4 * t:4 * t + 4, 2 * s:2 * s + 2] = np.linalg.matrix_power(A, t - s) @ B
    return Phi, Gam


def di_quadratic_form(wl):
    """S(eps) = c + g.eps + 1/2 eps' H eps for the c1 problem: running cost
    on x_1..x_T and v_0..v_{T-1}, terminal cost on x_T."""
    T, dt = wl.T, float(np.float32(wl.dt))
    Phi, Gam = di_matrices(T, dt)
    w = wl.w.astype(np.float64)
    q, r, qf = w[0:4], w[8:10], w[16:20]
    Qbar = np.kron(np.eye(T), np.diag(q))
    Qbar[-4:, -4:] += np.diag(qf)
    Rbar = np.kron(np.eye(T), np.diag(r))
    x0 = wl.x0.astype(np.float64)
    u = wl.u0.astype(np.float64).ravel()
    goal = np.tile(wl.ref.astype(np.float64), T)
    # S(V) = (Phi x0 + Gam V - goal)' Qbar (...) + V' Rbar V,  V = u + eps
    d0 = Phi @ x0 + Gam @ u - goal
    H = 2.0 * (Gam.T @ Qbar @ Gam + Rbar)
    g = 2.0 * (Gam.T @ Qbar @ d0 + Rbar @ u)
    c = d0 @ Qbar @ d0 + u @ Rbar @ u
    return c, g, H


def eps_flat(eps):
    """[T][m][K] -> [K][T*m] (time-major per sample)."""
    T, m, K = eps.shape
    return eps.transpose(2, 0, 1).reshape(K, T * m).astype(np.float64)


def test_double_integrator_costs_are_the_exact_quadratic_form(oracle_lib):
    wl = W.c1(K=256, T=30)
    wl.u0 = np.random.default_rng(3).normal(0, 0.3, (wl.T, 2)).astype(np.float32)
    eps = oracle_lib.workload_noise(wl)
    S, _, _ = oracle_lib.rollout_costs(wl, eps=eps)
    c, g, H = di_quadratic_form(wl)
    E = eps_flat(eps)
    S_ref = c + E @ g + 0.5 * np.einsum("ki,ij,kj->k", E, H, E)
    assert np.allclose(S, S_ref, rtol=1e-12, atol=0)


def test_zero_noise_gives_uniform_weights_and_unchanged_controls(oracle_lib):
    wl = W.c2(K=64, T=40, iters=1)
    wl.sigma = np.zeros(2, np.float32)
    res = oracle_lib.mppi(wl, iters=1)
    assert np.all(res["S"] == res["S"][0])
    assert np.allclose(res["w"], 1.0 / wl.K, rtol=1e-15)
    assert np.array_equal(res["U"], wl.u0.astype(np.float64))
    # every rollout is the deterministic integration of u
    xs = oracle_lib.trajectory(wl, wl.u0)
    assert res["S"][0] == pytest.approx(oracle_lib.sequence_cost(wl, wl.u0), rel=1e-15)
    assert np.isfinite(xs).all()


def _mp_algorithm1(wl, eps, lam):
    """Algorithm 1 for the Euler double integrator with the quadratic cost,
    evaluated with 50-digit mpmath (independent pure-Python transcription of
    the loops: rollout, cost after each step, terminal cost, min, eta, w,
    U = u + sum w eps)."""
    import mpmath as mp
    mp.mp.dps = 50
    T, m, K = eps.shape
    dt = mp.mpf(float(np.float32(wl.dt)))
    w = [mp.mpf(float(v)) for v in wl.w]
    goal = [mp.mpf(float(v)) for v in wl.ref]
    S = []
    for k in range(K):
        x = [mp.mpf(float(v)) for v in wl.x0]
        J = mp.mpf(0)
        for t in range(T):
            v = [mp.mpf(float(wl.u0[t, j])) + mp.mpf(float(eps[t, j, k])) for j in range(m)]
            x = [x[0] + dt * x[2], x[1] + dt * x[3], x[2] + dt * v[0], x[3] + dt * v[1]]
            J += sum(w[i] * (x[i] - goal[i]) ** 2 for i in range(4))
            J += sum(w[8 + j] * v[j] ** 2 for j in range(m))
        J += sum(w[16 + i] * (x[i] - goal[i]) ** 2 for i in range(4))
        S.append(J)
    rho = min(S)
    lam = mp.mpf(float(np.float32(lam)))  # inputs are binary32 values
    e = [mp.e ** (-(s - rho) / lam) for s in S]
    eta = sum(e)
    wk = [v / eta for v in e]
    U = [[mp.mpf(float(wl.u0[t, j])) + sum(wk[k] * mp.mpf(float(eps[t, j, k])) for k in range(K))
          for j in range(m)] for t in range(T)]
    return S, wk, U


@pytest.mark.parametrize("K,T,lam", [(1, 1, 1.0), (2, 1, 1.0), (3, 2, 1.0), (3, 2, 30.0),
                                     (2, 2, 0.05)])
def test_tiny_problems_against_mpmath_brute_force(oracle_lib, K, T, lam):
    wl = W.c1(K=K, T=T)
    wl.lam = lam
    eps = oracle_lib.workload_noise(wl)
    S, _, _ = oracle_lib.rollout_costs(wl, eps=eps)
    w, U, stats, rc = oracle_lib.softmin_update(wl, S, eps)
    S_mp, w_mp, U_mp = _mp_algorithm1(wl, eps, lam)
    assert rc == 0
    assert np.allclose(S, [float(v) for v in S_mp], rtol=1e-13, atol=0)
    # the softmin amplifies a relative error d in S by |S| d / lambda in w
    cond = 1e-12 + 64 * np.finfo(float).eps * np.abs(S).max() / lam
    assert np.allclose(w, [float(v) for v in w_mp], rtol=cond, atol=1e-300)
    assert np.allclose(U, np.array([[float(v) for v in row] for row in U_mp]),
                       rtol=cond, atol=cond)


def test_single_sample_update_is_its_noise(oracle_lib):
    wl = W.c2(K=1, T=20, iters=1)
    eps = oracle_lib.workload_noise(wl)
    S, _, _ = oracle_lib.rollout_costs(wl, eps=eps)
    w, U, stats, rc = oracle_lib.softmin_update(wl, S, eps)
    assert w[0] == 1.0 and stats[1] == 1.0
    assert np.array_equal(U, wl.u0 + eps[:, :, 0].astype(np.float64))


@pytest.fixture(scope="module")
def c2_small(oracle_lib):
    wl = W.c2(K=2048, T=50, iters=1)
    eps = oracle_lib.workload_noise(wl)
    S, margin, crashes = oracle_lib.rollout_costs(wl, eps=eps)
    return wl, eps, S


def test_weights_normalised_and_bounded(oracle_lib, c2_small):
    wl, eps, S = c2_small
    w, U, stats, rc = oracle_lib.softmin_update(wl, S, eps)
    rho, eta = stats[0], stats[1]
    assert rho == S.min()
    assert abs(w.sum() - 1.0) < 1e-14
    assert 1.0 <= eta <= wl.K
    assert w.max() == pytest.approx(1.0 / eta, rel=1e-15)
    assert np.all(w >= 0)


def test_update_invariant_to_cost_shift(oracle_lib, c2_small):
    wl, eps, S = c2_small
    w0, U0, _, _ = oracle_lib.softmin_update(wl, S, eps)
    w1, U1, _, _ = oracle_lib.softmin_update(wl, S + 1.0e3, eps)
    assert np.allclose(w0, w1, rtol=1e-12, atol=1e-300)
    assert np.abs(U0 - U1).max() < 1e-12 * np.abs(eps).max()


def test_temperature_limits(oracle_lib, c2_small):
    wl, eps, S = c2_small
    # lambda -> inf: plain average of the noise
    _, U, _, _ = oracle_lib.softmin_update(wl, S, eps, lam=1.0e8)
    mean_eps = eps.astype(np.float64).mean(axis=2)
    assert np.allclose(U, wl.u0 + mean_eps, rtol=1e-6, atol=1e-6)
    # lambda -> 0 with a clear minimum: the argmin sample's noise
    order = np.argsort(S)
    assert S[order[1]] - S[order[0]] > 1e-3
    _, U, _, _ = oracle_lib.softmin_update(wl, S, eps, lam=1.0e-6)
    assert np.array_equal(U, wl.u0 + eps[:, :, order[0]].astype(np.float64))


def test_free_energy_gibbs_identity(oracle_lib, c2_small):
    """F = -lambda ln((1/K) sum exp(-S/lambda)) equals sum w S + lambda sum w
    ln(K w) for the empirical Gibbs weights (Section II-B: the free-energy bound
    is tight at the optimal density)."""
    wl, eps, S = c2_small
    for lam in (0.5, 20.0):
        w, U, stats, _ = oracle_lib.softmin_update(wl, S, eps, lam=lam)
        nz = w > 0
        rhs = np.sum(w * S) + lam * np.sum(w[nz] * np.log(wl.K * w[nz]))
        assert stats[2] == pytest.approx(rhs, rel=1e-10)
        # and equals the direct log-mean-exp evaluation done with mpmath
        import mpmath as mp
        mp.mp.dps = 40
        lam32 = float(np.float32(lam))
        F = -lam32 * mp.log(sum(mp.e ** (-mp.mpf(s) / lam32) for s in S) / wl.K)
        assert stats[2] == pytest.approx(float(F), rel=1e-12)


def test_all_nonfinite_costs_keep_controls(oracle_lib):
    wl = W.c1(K=8, T=3)
    eps = oracle_lib.workload_noise(wl)
    S = np.full(8, np.inf)
    w, U, stats, rc = oracle_lib.softmin_update(wl, S, eps)
    assert rc == -6 and np.all(w == 0) and np.array_equal(U, wl.u0.astype(np.float64))
    S = np.linspace(1, 8, 8)
    S[3] = np.inf
    w, U, stats, rc = oracle_lib.softmin_update(wl, S, eps)
    assert rc == 0 and w[3] == 0 and abs(w.sum() - 1) < 1e-14


@pytest.mark.slow
def test_linear_quadratic_large_K_limit(oracle_lib):
    """With p = N(0, Sbar) and S quadratic, the optimal density Eq.
    (optimal_distribution) is Gaussian with precision Sbar^-1 + H/lambda and
    mean -(Sbar^-1 + H/lambda)^-1 g / lambda; the MPPI update tends to u plus
    that mean.  Checked statistically at large K."""
    wl = W.c1(K=1 << 17, T=4)
    lam = 40.0
    eps = oracle_lib.workload_noise(wl)
    S, _, _ = oracle_lib.rollout_costs(wl, eps=eps)
    w, U, stats, _ = oracle_lib.softmin_update(wl, S, eps, lam=lam)
    c, g, H = di_quadratic_form(wl)
    sig2 = np.tile(wl.sigma.astype(np.float64) ** 2, wl.T)
    P = np.diag(1.0 / sig2) + H / lam
    mu = -np.linalg.solve(P, g) / lam
    ess = stats[3]
    assert ess > 100
    sd = np.sqrt(np.diag(np.linalg.inv(P)) / ess)
    dev = (U.ravel() - wl.u0.ravel() - mu) / sd
    assert np.abs(dev).max() < 5.0, dev
