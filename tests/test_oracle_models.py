"""Pins of the oracle's dynamics and cost pieces.

Each piece is checked against an independent evaluation: scipy's ODE
integrator, rotation and interpolation routines, a torch float64 MLP forward,
or a closed-form motion (circular arc, free fall, hover equilibrium).
"""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

import workloads as W


def _rk4_vs_ode(oracle_lib, wl, x0, v, T):
    wl = wl.replace(T=T)
    v_seq = np.tile(np.asarray(v, np.float64), (T, 1))
    xs = oracle_lib.trajectory(wl, v_seq, x0=x0)
    f = lambda t, x: oracle_lib.deriv(wl, x, v)  # noqa: E731
    sol = solve_ivp(f, (0.0, T * float(np.float32(wl.dt))), np.asarray(x0, np.float64),
                    rtol=1e-12, atol=1e-12, method="DOP853")
    return xs[-1], sol.y[:, -1]


def test_bicycle_circular_arc_closed_form(oracle_lib):
    wl = W.c2(K=1, T=100)
    L = 2.5
    psi0, s, delta = 0.3, 4.0, 0.2
    x0 = np.array([10.0, 20.0, psi0, s, delta])
    xs = oracle_lib.trajectory(wl, np.zeros((wl.T, 2)), x0=x0)
    dt = float(np.float32(wl.dt))
    om = s * math.tan(delta) / L
    t = np.arange(wl.T + 1) * dt
    px = 10.0 + s / om * (np.sin(psi0 + om * t) - math.sin(psi0))
    py = 20.0 - s / om * (np.cos(psi0 + om * t) - math.cos(psi0))
    assert np.abs(xs[:, 0] - px).max() < 1e-9
    assert np.abs(xs[:, 1] - py).max() < 1e-9
    assert np.allclose(xs[:, 2], psi0 + om * t, atol=1e-12)


def test_bicycle_rk4_order_four(oracle_lib):
    wl = W.c2(K=1, T=50)
    x0 = [10.0, 30.0, 0.4, 3.0, 0.1]
    v = [0.7, -0.2]
    errs = []
    for scale in (1, 2, 4):
        w2 = wl.replace(dt=float(np.float32(wl.dt)) / scale)
        xT, ref = _rk4_vs_ode(oracle_lib, w2, x0, v, 50 * scale)
        errs.append(np.abs(xT - ref).max())
    assert errs[0] < 1e-7
    for a, b in zip(errs, errs[1:]):
        assert 12.0 < a / b < 20.0, errs  # 2^4 = 16


def _quat_xyzw(q):
    return np.array([q[1], q[2], q[3], q[0]])


def test_quadrotor_derivative_against_scipy_rotation(oracle_lib):
    from scipy.spatial.transform import Rotation as R
    wl = W.c3(K=1, T=10)
    rng = np.random.default_rng(11)
    for _ in range(5):
        q = rng.normal(size=4)
        q /= np.linalg.norm(q)
        x = np.concatenate([rng.normal(size=3), q, rng.normal(size=3), rng.normal(size=3)])
        v = rng.normal(size=4) + np.array([9.81, 0, 0, 0])
        d = oracle_lib.deriv(wl, x, v)
        Rm = R.from_quat(_quat_xyzw(q)).as_matrix()
        assert np.allclose(d[7:10], Rm @ np.array([0, 0, v[0]]) / 1.0 - [0, 0, 9.81], atol=1e-12)
        assert np.allclose(d[0:3], x[7:10])
        # body-frame angular velocity: q(h) = q (x) exp(omega h)
        om = x[10:13]
        h = 1e-6
        qh = (R.from_quat(_quat_xyzw(q)) * R.from_rotvec(om * h)).as_quat()
        qh = np.array([qh[3], qh[0], qh[1], qh[2]])
        if np.dot(qh, q) < 0:
            qh = -qh
        assert np.allclose(d[3:7], (qh - q) / h, atol=1e-5)
        # Euler's equations J w' = tau - w x J w
        J = np.array([0.01, 0.01, 0.02])
        assert np.allclose(J * d[10:13], v[1:4] - np.cross(om, J * om), atol=1e-10)


def test_quadrotor_hover_is_an_equilibrium_with_zero_cost(oracle_lib):
    wl = W.c3(K=1, T=50)
    x0 = np.zeros(13)
    x0[2] = 1.0
    x0[3] = 1.0
    u = np.tile([9.81, 0.0, 0.0, 0.0], (wl.T, 1)).astype(np.float32).astype(np.float64)
    g32 = float(np.float32(9.81))
    u[:, 0] = g32  # thrust equal to m g in the binary32 value the model uses
    xs = oracle_lib.trajectory(wl, u, x0=x0)
    assert np.abs(xs - x0).max() < 1e-12
    assert oracle_lib.sequence_cost(wl, u, x0=x0) < 1e-20
    # attitude cost has the quaternion double cover: q and -q cost the same
    x1 = x0.copy()
    x1[3:7] = [0.6, 0.8, 0.0, 0.0]
    x2 = x1.copy()
    x2[3:7] *= -1
    assert oracle_lib.running_cost(wl, x1, u[0]) == oracle_lib.running_cost(wl, x2, u[0])


def test_quadrotor_free_fall_and_torque_free_spin(oracle_lib):
    wl = W.c3(K=1, T=100)
    dt = float(np.float32(wl.dt))
    g = float(np.float32(9.81))
    x0 = np.zeros(13)
    x0[3] = 1.0
    xs = oracle_lib.trajectory(wl, np.zeros((wl.T, 4)), x0=x0)
    t = np.arange(wl.T + 1) * dt
    assert np.allclose(xs[:, 2], -0.5 * g * t * t, atol=1e-11)  # RK4 exact on a quadratic
    assert np.allclose(xs[:, 9], -g * t, atol=1e-11)
    # spin about the z principal axis: q(t) = (cos(w t/2), 0, 0, sin(w t/2))
    x0[12] = 2.0
    xs = oracle_lib.trajectory(wl, np.zeros((wl.T, 4)), x0=x0)
    assert np.allclose(xs[:, 3], np.cos(t), atol=1e-9)
    assert np.allclose(xs[:, 6], np.sin(t), atol=1e-9)
    # generic torque-free tumble: kinetic energy and |J w| conserved
    x0[10:13] = [3.0, -1.0, 2.0]
    xs = oracle_lib.trajectory(wl, np.zeros((wl.T, 4)), x0=x0)
    J = np.array([0.01, 0.01, 0.02])
    E = 0.5 * (xs[:, 10:13] ** 2 * J).sum(1)
    Lm = np.linalg.norm(xs[:, 10:13] * J, axis=1)
    assert np.abs(E / E[0] - 1).max() < 1e-8
    assert np.abs(Lm / Lm[0] - 1).max() < 1e-8
    assert np.abs(np.linalg.norm(xs[:, 3:7], axis=1) - 1.0).max() < 1e-14


def test_spline_against_scipy_ppoly(oracle_lib):
    from scipy.interpolate import PPoly
    wl = W.c2(K=1, T=1)
    c = wl.coef.astype(np.float64)
    pp = PPoly(np.stack([c[:, 3], c[:, 2], c[:, 1], c[:, 0]]), wl.knots.astype(np.float64))
    for x in np.concatenate([np.linspace(10.0, 90.0, 977), [10.0, 90.0, 21.4285717]]):
        y, dy = oracle_lib.spline(wl, x)
        assert y == pytest.approx(pp(x), rel=1e-13, abs=1e-12)
        assert dy == pytest.approx(pp(x, 1), rel=1e-12, abs=1e-12)
    # clamped outside the knot range
    assert oracle_lib.spline(wl, -5.0)[0] == pytest.approx(pp(10.0), rel=1e-13)
    assert oracle_lib.spline(wl, 150.0)[1] == pytest.approx(pp(90.0, 1), rel=1e-12)


def test_costmap_against_scipy_grid_interpolator(oracle_lib):
    from scipy.interpolate import RegularGridInterpolator
    wl = W.c2("costmap", K=1, T=1)
    H, Wd = wl.costmap.shape
    res = float(np.float32(wl.map_res))
    xs = (np.arange(Wd) + 0.5) * res
    ys = (np.arange(H) + 0.5) * res
    rgi = RegularGridInterpolator((ys, xs), wl.costmap.astype(np.float64), method="linear")
    rng = np.random.default_rng(5)
    pts = rng.uniform(-3.0, 103.0, (4000, 2))
    for px, py in pts:
        qx = min(max(px, xs[0]), xs[-1])
        qy = min(max(py, ys[0]), ys[-1])
        ref = float(rgi([[qy, qx]])[0])
        assert oracle_lib.costmap(wl, px, py) == pytest.approx(ref, rel=1e-9, abs=1e-7)


def test_crash_indicator_against_distance_check(oracle_lib):
    wl = W.c2(K=256, T=100, iters=1)
    eps = oracle_lib.workload_noise(wl)
    S, margin, crashes = oracle_lib.rollout_costs(wl, eps=eps)
    r = np.sqrt(wl.r2.astype(np.float64))
    assert crashes.sum() > 0
    for k in range(wl.K):
        v = wl.u0.astype(np.float64) + eps[:, :, k].astype(np.float64)
        xs = oracle_lib.trajectory(wl, v)
        d = np.hypot(xs[1:, 0, None] - wl.cx.astype(np.float64),
                     xs[1:, 1, None] - wl.cy.astype(np.float64))
        if margin[k] > 1e-9:
            assert crashes[k] == np.count_nonzero((d <= r).any(axis=1)), k


def test_path_cost_special_cases(oracle_lib):
    wl = W.c2(K=1, T=1)
    wl.cx = wl.cx[:0]; wl.cy = wl.cy[:0]; wl.r2 = wl.r2[:0]
    for px in (12.0, 33.3, 71.0):
        y, dy = oracle_lib.spline(wl, px)
        x = np.array([px, y, math.atan(dy), 5.0, 0.3])
        assert oracle_lib.running_cost(wl, x, [0.0, 0.0]) == pytest.approx(0.0, abs=1e-24)
        x[1] += 0.7  # lateral offset along y only
        assert oracle_lib.running_cost(wl, x, [0.0, 0.0]) == pytest.approx(0.49, rel=1e-12)
        assert oracle_lib.terminal_cost(wl, x) == pytest.approx(4.9, rel=1e-12)
        x[1] -= 0.7
        assert oracle_lib.running_cost(wl, x, [2.0, -1.0]) == pytest.approx(0.1 * 4 + 0.1 * 1)


def test_track_cost_is_time_indexed_on_post_step_state(oracle_lib):
    wl = W.c5(K=1, T=10)
    ref = wl.ref.astype(np.float64).reshape(wl.T + 1, 5)
    for t in (0, 4, 9):
        assert oracle_lib.running_cost(wl, ref[t + 1], [0.0, 0.0], t) == 0.0
        assert oracle_lib.running_cost(wl, ref[t], [0.0, 0.0], t) > 0.0
    assert oracle_lib.terminal_cost(wl, ref[wl.T]) == 0.0


def test_mlp_residual_against_torch(oracle_lib):
    import torch
    wl = W.c5(K=1, T=1)
    H = wl.mlp_hidden
    p = torch.tensor(wl.mlp.astype(np.float64))
    o = 0
    def take(n, shape):
        nonlocal o
        t = p[o:o + n].reshape(shape)
        o += n
        return t
    W1 = take(H * 7, (H, 7)); b1 = take(H, (H,)); W2 = take(H * H, (H, H)); b2 = take(H, (H,))
    W3 = take(5 * H, (5, H)); b3 = take(5, (5,))
    plain = wl.replace(model="bicycle", mlp=None, mlp_hidden=0)
    rng = np.random.default_rng(2)
    dt = float(np.float32(wl.dt))
    for _ in range(4):
        x = np.array([10.0, 40.0, 0.2, 5.0, 0.05]) + rng.normal(0, 0.5, 5)
        v = rng.normal(0, 1.0, 2)
        z = torch.tensor(np.concatenate([x, v]))
        g = W3 @ torch.tanh(W2 @ torch.tanh(W1 @ z + b1) + b2) + b3
        diff = oracle_lib.step(wl, x, v) - oracle_lib.step(plain, x, v)
        assert np.allclose(diff, dt * g.numpy(), rtol=1e-12, atol=1e-14)


def test_quadratic_cost_zero_at_goal(oracle_lib):
    wl = W.c1(K=1, T=1)
    assert oracle_lib.running_cost(wl, np.zeros(4), [0.0, 0.0]) == 0.0
    assert oracle_lib.running_cost(wl, [1.0, 0, 0, 0], [0.0, 0.0]) == 10.0
    assert oracle_lib.running_cost(wl, [0.0, 0, 0, 0], [1.0, 2.0]) == pytest.approx(0.5)
    assert oracle_lib.terminal_cost(wl, [0.0, 0, 1.0, 0]) == pytest.approx(10.0)


def test_hover_cost_terms_one_at_a_time(oracle_lib):
    wl = W.c3(K=1, T=1)
    g32 = float(np.float32(9.81))
    base = np.zeros(13); base[2] = 1.0; base[3] = 1.0
    u = np.array([g32, 0.0, 0.0, 0.0])
    rc = lambda x, v=u: oracle_lib.running_cost(wl, x, v)  # noqa: E731
    assert rc(base) == 0.0
    x = base.copy(); x[0] = 0.5; x[2] = 2.0
    assert rc(x) == pytest.approx(10.0 * (0.25 + 1.0))           # position
    assert oracle_lib.terminal_cost(wl, x) == pytest.approx(100.0 * 1.25)
    x = base.copy(); x[7:10] = [1.0, 2.0, -2.0]
    assert rc(x) == pytest.approx(1.0 * 9.0)                     # velocity
    x = base.copy(); x[10:13] = [1.0, 0.0, 3.0]
    assert rc(x) == pytest.approx(0.1 * 10.0)                    # body rates
    x = base.copy(); x[3:7] = [math.cos(math.pi / 4), math.sin(math.pi / 4), 0, 0]
    assert rc(x) == pytest.approx(10.0 * 0.5)                    # 90 deg tilt
    assert rc(base, u + np.array([1.0, 0.5, 0.0, -0.5])) == pytest.approx(0.1 * 1.5)
    x = base.copy(); x[1] = -6.5; x[2] = 1.0
    assert rc(x) == pytest.approx(10.0 * 6.5 ** 2 + 100.0 * 1.5 ** 2)  # box penalty


def test_goal_cost_terms(oracle_lib):
    wl = W.c4(n_instances=1)[0]
    gx, gy = (float(v) for v in wl.ref)
    x = np.array([gx + 3.0, gy - 4.0, 0.0, 1.0, 0.0])
    wl.cx = np.array([500.0], np.float32); wl.cy = np.array([500.0], np.float32)
    wl.r2 = np.array([1.0], np.float32)
    assert oracle_lib.running_cost(wl, x, [1.0, 2.0]) == pytest.approx(0.01 * 25 + 0.1 + 0.4)
    assert oracle_lib.terminal_cost(wl, x) == pytest.approx(10.0 * 0.01 * 25)
    wl.cx[0], wl.cy[0] = x[0] + 0.5, x[1]
    assert oracle_lib.running_cost(wl, x, [0.0, 0.0]) == pytest.approx(0.25 + 1.0e4)
