"""Shared parity helpers: run a workload through the GPU library and through
the oracle on the same seeded noise, and the tolerances of the comparison.

Tolerances (the target is 1e-4 relative in binary32):
  * noise: bit-exact (same counter-based definition on both sides);
  * rollout costs J: |J_gpu - J_or| <= 1e-4 max(|J_or|, 1) for every sample
    whose crash decisions are not within binary32 reach of flipping (their
    smallest relative margin |d^2 - r^2| / r^2 is >= AMBIGUOUS_MARGIN); for the
    costmap cost the bound adds the forward error of evaluating the map at a
    binary32 position, POS_EPS * sum_t |grad M(p_t)|_1, where POS_EPS =
    2^-24 * 100 m is half an ulp at the scene's coordinate scale (a 0/1e4
    map rasterised at 0.2 m has slopes of 5e4 per metre, so one rounding of a
    position moves a step's cost by ~0.3);
  * rollout costs of ill-conditioned trajectories (the MLP residual dynamics,
    whose saturated random network drives the steering towards the tan
    singularity over a long horizon): the bound adds COND_ULPS * 2^-24 *
    cond_k, where cond_k = sum_t,i |dJ_k/dx_t,i| |x_t,i| (from the oracle's
    adjoint) is the first-order change of J_k when every state component is
    rounded once per step; a binary32 step rounds each component a few times
    (RK4 stages, the MLP's sums), COND_ULPS = 32 covers that with margin;
  * chaotic samples: where nudging every noise input of the oracle by one
    binary32 ulp (up, or down: a 6e-8 relative change) already moves a cost
    by more than CHAOS_REL = 1e-2 relative, the amplification exceeds 1e5
    and a first-order bound no longer describes what the GPU's own rounding
    does (the MLP residual dynamics can diverge there): no single value is
    the right one.  Such samples are exempt from the cost comparison (a GPU
    cost must still not be NaN) and must be rare; where controls are
    compared with the oracle's, they must also carry negligible weight
    (below 1e-6 in all), so the controls' bound is unchanged (`chaotic`);
  * controls: |U_gpu - U_or| <= 1e-4 max(|U_or|_inf, |sigma|_inf) plus the
    change that the allowed cost deviation can cause through the softmin:
    sum_k |dU/dJ_k| 1e-4 max(|J_k|, 1), dU_t/dJ_k = -(gamma w_k/lambda)(eps_k,t -
    sum_i w_i eps_i,t), gamma the step size (all computed from the oracle's own
    values).
"""
import numpy as np

REL = 1e-4
AMBIGUOUS_MARGIN = 1e-3
POS_EPS = 2.0 ** -24 * 100.0
COND_ULPS = 32.0
CHAOS_REL = 1e-2


def cost_tol(S_or, cond=None):
    tol = REL * np.maximum(np.abs(S_or), 1.0)
    if cond is not None:
        tol = tol + COND_ULPS * 2.0 ** -24 * cond
    return tol


def controls_tol(wl, S_or, w_or, eps, lam=None, cond=None):
    lam = float(np.float32(wl.lam if lam is None else lam))
    E = eps.astype(np.float64)                        # [T][m][K]
    mean = np.tensordot(E, w_or, axes=([2], [0]))     # sum_i w_i eps_i  [T][m]
    gamma = abs(float(np.float32(getattr(wl, "gamma", 1.0))))  # U - u = gamma sum w eps
    dU = (gamma * w_or / lam) * np.abs(E - mean[:, :, None])  # |dU_t / dJ_k|  [T][m][K]
    prop = np.tensordot(dU, cost_tol(S_or, cond), axes=([2], [0]))
    scale = max(np.abs(wl.u0).max(), np.abs(wl.sigma).max())
    return REL * scale + prop


def chaotic(oracle_lib, wl, eps, S_or, u=None):
    """Samples whose oracle cost moves by more than CHAOS_REL relative when
    every noise input moves by one binary32 ulp (either direction)."""
    tol = CHAOS_REL * np.maximum(np.abs(S_or), 1.0)
    out = np.zeros(np.shape(S_or), bool)
    for direction in (np.inf, -np.inf):
        e = np.nextafter(np.asarray(eps, np.float32), np.float32(direction))
        S = oracle_lib.rollout_costs(wl, e, u=u)[0]
        out |= ~(np.abs(S - S_or) <= tol)
    return out


def assert_costs_close(S_gpu, S_or, margin=None, name="", slope=None, cond=None, skip=None):
    S_gpu = np.asarray(S_gpu, np.float64)
    tol = cost_tol(S_or, cond) if slope is None else cost_tol(S_or, cond) + POS_EPS * slope
    ok = np.abs(S_gpu - S_or) <= tol
    if margin is not None:
        ok |= margin < AMBIGUOUS_MARGIN
    if skip is not None:
        assert not np.isnan(S_gpu[skip]).any(), name
        ok |= skip
    bad = np.flatnonzero(~ok)
    assert bad.size == 0, (
        f"{name}: {bad.size} costs off; first {bad[:5]}: gpu {S_gpu[bad[:5]]} "
        f"oracle {S_or[bad[:5]]} rel {(np.abs(S_gpu - S_or) / np.maximum(np.abs(S_or), 1))[bad[:5]]}")


def assert_controls_close(U_gpu, U_or, tol, name=""):
    U_gpu = np.asarray(U_gpu, np.float64)
    err = np.abs(U_gpu - U_or)
    bad = err > tol
    assert not bad.any(), (f"{name}: {bad.sum()} controls off, max err {err.max():.3g}, "
                           f"worst ratio {(err / tol).max():.3g}")
