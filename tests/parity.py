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
  * controls, end to end (Algorithm 1, Eq. mppi_update_rule): the GPU's
    controls are compared with the oracle's on the same noise, the softmin
    propagating the GPU's *measured* cost deviations dJ_k = J_gpu,k - J_or,k
    (which the cost checks bound separately):
      - exact propagation: |U_gpu - U_or(J_gpu)| <= 1e-4 max(|U_or|_inf,
        |sigma|_inf), U_or(J_gpu) being the oracle's binary64 update fed with
        the GPU's binary32 costs;
      - first order: |U_gpu - U_or - sum_k dU/dJ_k dJ_k| <= the same bound
        plus |R|, R = U_or(J_gpu) - U_or - sum_k dU/dJ_k dJ_k the remainder
        of the linearisation (reported; negligible wherever dJ_k / lambda
        is small), dU_t/dJ_k = -(gamma w_k / lambda)(d_k,t - sum_i w_i d_i,t)
        with d_k = v_k - u;
      - flat: |U_gpu - U_or| <= 1e-4 max(|U_or|_inf, |sigma|_inf) outright,
        asserted for every workload except the MLP residual dynamics (whose
        long-horizon trajectories are ill-conditioned: there the first two
        checks carry the claim).
  * update alone (both sides weight the same binary32 costs): the flat bound.
  * the MLP's bfloat16 mode (products on bfloat16 operands, binary32
    accumulation) against the oracle's bfloat16 option, which rounds the same
    operands at the same points (binary64 -> binary32 -> bfloat16, nearest
    even).  The binary32 arithmetic between the roundings differs, so a
    rounding decision can go the other way where an operand lies within
    binary32 reach of a tie; the operand then moves by one bfloat16 unit in
    the last place, at most 2^-7 of its size.  Bounds (assert_costs_close_bf16):
      - every sample: |J_gpu - J_bf| <= cost_tol(J_bf, cond) + 2^-7 cond_bf,
        cond_bf = sum over the rounded operands o of |dJ/do| |o| (from the
        oracle's adjoint): the first-order change if every decision flipped;
      - at most BF_FLIP_FRAC of the samples may need the second term (the
        rest meet the binary32 bound outright);
      - the GPU takes the oracle's decisions, not merely some rounding: the
        median |J_gpu - J_bf| is at most BF_SAME_ROUNDING of the median
        |J_bf - J_fp64| (the whole effect of the roundings; a kernel that
        truncated, or skipped a rounding, would sit near 1).
"""
import numpy as np

REL = 1e-4
# A sample whose smallest relative crash margin |d^2 - r^2| / r^2 is below
# this is "ambiguous": a binary32 trajectory may take the other crash
# decision there (|d^2 - r^2| / r^2 ~ 2 |d - r| / r, so a position error e
# flips only decisions of margin below 2 e / r).  Tests report the fraction
# of samples it excludes.
AMBIGUOUS_MARGIN = 1e-5
POS_EPS = 2.0 ** -24 * 100.0
COND_ULPS = 32.0
CHAOS_REL = 1e-2


def cost_tol(S_or, cond=None):
    tol = REL * np.maximum(np.abs(S_or), 1.0)
    if cond is not None:
        tol = tol + COND_ULPS * 2.0 ** -24 * cond
    return tol


def n_plain(wl):
    """Samples drawn around u (the rest are drawn around zero)."""
    nz = int(np.floor(float(np.float32(getattr(wl, "zero_frac", 0.0))) * wl.K))
    nz = min(nz, wl.K - (1 if getattr(wl, "mean_sample", 0) else 0))
    return wl.K - max(nz, 0)


def sigma_max(wl):
    s = float(np.abs(np.asarray(wl.sigma, np.float64)).max())
    sig_t = getattr(wl, "sigma_t", None)
    if sig_t is not None:
        s = max(s, float(np.abs(np.asarray(sig_t, np.float64)).max()))
    return s


def flat_tol(wl, U_or):
    """1e-4 max(|U_or|_inf, |sigma|_inf)."""
    return REL * max(float(np.abs(U_or).max()), sigma_max(wl))


def _finite(S):
    S = np.asarray(S, np.float64)
    return np.where(np.isfinite(S), S, np.inf)


E2E_LOG = []  # (name, flat ratio, first-order residual ratio, remainder ratio, max |dJ|/lambda)


def assert_end_to_end(oracle_lib, wl, U_gpu, S_gpu, eps, S_or, name="", u=None, flat=None,
                      lam=None):
    """Controls of one iteration against the oracle's, the softmin carrying
    the GPU's measured cost deviations (see the module docstring).  eps: the
    iteration's noise [T][m][K]; S_or: the oracle's costs on it; u: the
    nominal controls the iteration started from (default wl.u0).  flat
    (default: every workload without the MLP residual dynamics, whose long
    horizons are ill-conditioned) also asserts the flat bound outright."""
    if flat is None:
        flat = wl.model != "bicycle_mlp"
    over = {} if lam is None else {"lam": lam}
    u = np.asarray(wl.u0 if u is None else u, np.float64).reshape(wl.T, wl.m)
    S_or = _finite(S_or)
    S_g = _finite(S_gpu)
    w_or, U_or, _, rc_or = oracle_lib.softmin_update(wl, S_or, eps, u=u, **over)
    w_g, U_g, _, rc_g = oracle_lib.softmin_update(wl, S_g, eps, u=u, **over)
    assert rc_or == 0 and rc_g == 0, f"{name}: all costs non-finite"
    U_gpu = np.asarray(U_gpu, np.float64).reshape(wl.T, wl.m)
    bound = flat_tol(wl, U_or)
    # first-order propagation of the measured deviations through the softmin
    lam_v = float(np.float32(wl.lam if lam is None else lam))
    gamma = float(np.float32(getattr(wl, "gamma", 1.0)))
    dev = eps.astype(np.float64).copy()                 # d_k = v_k - u  [T][m][K]
    dev[:, :, n_plain(wl):] -= u[:, :, None]
    mean = np.tensordot(dev, w_or, axes=([2], [0]))     # sum_i w_i d_i
    both = np.isfinite(S_or) & np.isfinite(S_g)
    dJ = np.where(both, S_g - np.where(both, S_or, 0.0), 0.0)
    coef = -(gamma / lam_v) * w_or * dJ                 # [K]
    J1 = np.tensordot(dev, coef, axes=([2], [0])) - mean * coef.sum()
    R = U_g - U_or - J1
    exact_err = np.abs(U_gpu - U_g)
    fo_err = np.abs(U_gpu - U_or - J1)
    flat_err = np.abs(U_gpu - U_or)
    rec = (name, float(flat_err.max() / bound), float(fo_err.max() / bound),
           float(np.abs(R).max() / bound),
           float(np.abs(dJ[w_or > 0]).max() / lam_v) if (w_or > 0).any() else 0.0)
    E2E_LOG.append(rec)
    import sys
    print(f"[e2e] {name}: |U-U_or|/bound {rec[1]:.3g}, first-order residual {rec[2]:.3g}, "
          f"remainder {rec[3]:.3g}, max |dJ|/lambda (weighted samples) {rec[4]:.3g}",
          file=sys.stderr, flush=True)
    assert (exact_err <= bound).all(), (
        f"{name}: U differs from the oracle's update of the GPU's costs by {exact_err.max():.3g} "
        f"(bound {bound:.3g})")
    assert (fo_err <= bound + np.abs(R)).all(), (
        f"{name}: first-order residual {fo_err.max():.3g} (bound {bound:.3g} + remainder)")
    if flat:
        assert (flat_err <= bound).all(), (
            f"{name}: |U - U_or| = {flat_err.max():.3g} above the flat bound {bound:.3g}")
    return rec


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


BF_ULP = 2.0 ** -7
BF_FLIP_FRAC = 0.01
BF_SAME_ROUNDING = 0.1


def assert_costs_close_bf16(S_gpu, S_bf, S_fp, cond, cond_bf, name=""):
    """The bfloat16 mode's costs against the oracle's bfloat16 option (S_bf)
    and its binary64 model (S_fp); cond, cond_bf from cost_condition(bf=True).
    Returns (fraction of samples beyond the binary32 bound, median ratio)."""
    S_gpu = np.asarray(S_gpu, np.float64)
    d = np.abs(S_gpu - S_bf)
    tol = cost_tol(S_bf, cond)
    outer = tol + BF_ULP * cond_bf
    bad = np.flatnonzero(~(d <= outer))
    assert bad.size == 0, (
        f"{name}: {bad.size} costs beyond the bfloat16 bound; first {bad[:5]}: gpu "
        f"{S_gpu[bad[:5]]} oracle {S_bf[bad[:5]]} bound {outer[bad[:5]]}")
    flipped = float(np.mean(d > tol))
    assert flipped <= BF_FLIP_FRAC, f"{name}: {flipped:.4f} of the samples beyond the binary32 bound"
    effect = float(np.median(np.abs(S_bf - S_fp)))
    ratio = float(np.median(d)) / effect if effect > 0 else 0.0
    assert ratio <= BF_SAME_ROUNDING, (
        f"{name}: median |J_gpu - J_bf| is {ratio:.3g} of the roundings' median effect")
    import sys
    print(f"[bf16] {name}: beyond binary32 bound {flipped:.4f}, worst |d|/bound "
          f"{float(np.max(d / outer)):.3g}, median |d| / median rounding effect {ratio:.3g}",
          file=sys.stderr, flush=True)
    return flipped, ratio


def assert_controls_close(U_gpu, U_or, tol, name=""):
    U_gpu = np.asarray(U_gpu, np.float64)
    err = np.abs(U_gpu - U_or)
    bad = err > tol
    assert not bad.any(), (f"{name}: {bad.sum()} controls off, max err {err.max():.3g}, "
                           f"worst ratio {(err / tol).max():.3g}")
