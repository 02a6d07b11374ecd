"""CPU checks of the parity helpers the GPU tests rely on (tests/parity.py).

The end-to-end control check propagates measured cost deviations through the
softmin with the Jacobian dU_t/dJ_k = -(gamma w_k / lambda)(d_k,t -
sum_i w_i d_i,t).  Here that Jacobian is compared with central differences of
the oracle's own update, and the check itself is exercised on synthetic
"GPU" results built from the oracle: an exact propagation passes, a control
moved by twice the bound fails.
"""
import numpy as np
import pytest

import workloads as W
from oracle import oracle as O
from tests import parity


def _first_order(wl, S, eps, dJ, u=None):
    u = np.asarray(wl.u0 if u is None else u, np.float64)
    w, U, _, _ = O.softmin_update(wl, S, eps, u=u)
    lam = float(np.float32(wl.lam))
    gamma = float(np.float32(getattr(wl, "gamma", 1.0)))
    dev = eps.astype(np.float64).copy()
    dev[:, :, parity.n_plain(wl):] -= u[:, :, None]
    mean = np.tensordot(dev, w, axes=([2], [0]))
    coef = -(gamma / lam) * w * dJ
    return np.tensordot(dev, coef, axes=([2], [0])) - mean * coef.sum()


@pytest.mark.parametrize("options", [False, True])
def test_softmin_jacobian_matches_central_differences(options):
    wl = W.c2("circles", K=200, T=10, iters=1).replace(lam=5.0)
    if options:
        rng = np.random.default_rng(3)
        wl = wl.replace(u0=rng.normal(0, 0.3, (10, 2)).astype(np.float32), zero_frac=0.25,
                        gamma=0.6)
    eps = O.workload_noise(wl)
    S = O.rollout_costs(wl, eps=eps)[0]
    rng = np.random.default_rng(0)
    direction = rng.normal(size=wl.K)
    h = 1e-4
    Up = O.softmin_update(wl, S + h * direction, eps)[1]
    Um = O.softmin_update(wl, S - h * direction, eps)[1]
    fd = (Up - Um) / (2 * h)
    lin = _first_order(wl, S, eps, direction)
    np.testing.assert_allclose(lin, fd, rtol=1e-6, atol=1e-9 * np.abs(fd).max())


def test_end_to_end_check_accepts_exact_propagation_and_rejects_offsets():
    wl = W.c1(K=500, T=20)
    eps = O.workload_noise(wl)
    S_or = O.rollout_costs(wl, eps=eps)[0]
    rng = np.random.default_rng(1)
    S_gpu = (S_or * (1 + 1e-6 * rng.normal(size=wl.K))).astype(np.float32)
    U_gpu = O.softmin_update(wl, S_gpu.astype(np.float64), eps)[1]
    rec = parity.assert_end_to_end(O, wl, U_gpu, S_gpu, eps, S_or, "exact")
    assert rec[2] < 1.0 and rec[3] < 1.0
    U_or = O.softmin_update(wl, S_or, eps)[1]
    bad = U_gpu.copy()
    bad[3, 1] += 2.0 * parity.flat_tol(wl, U_or)
    with pytest.raises(AssertionError):
        parity.assert_end_to_end(O, wl, bad, S_gpu, eps, S_or, "offset")


def test_bf16_cost_check_accepts_the_oracle_and_rejects_other_roundings(oracle_lib):
    """The bfloat16 cost check on results of the oracle itself: its own
    bfloat16 option (plus a binary32-sized jitter) passes; the binary64 model,
    the weights rounded but not the activations, and a costs shifted past the
    outer bound fail."""
    wl = W.c5(K=200, T=20, hidden=16).replace(mlp_bf16=1)
    eps = oracle_lib.workload_noise(wl)
    S_bf = oracle_lib.rollout_costs(wl, eps)[0]
    S_fp = oracle_lib.rollout_costs(wl.replace(mlp_bf16=0), eps)[0]
    cond, cond_bf = oracle_lib.cost_condition(wl, eps, bf=True)
    assert (cond_bf > 0).all()
    jitter = 1.0 + 2.0 ** -22 * np.random.default_rng(1).standard_normal(wl.K)
    parity.assert_costs_close_bf16(S_bf * jitter, S_bf, S_fp, cond, cond_bf, "oracle")
    with pytest.raises(AssertionError):
        parity.assert_costs_close_bf16(S_fp, S_bf, S_fp, cond, cond_bf, "binary64 model")
    wr = wl.replace(mlp=oracle_lib.bf16(wl.mlp).astype(np.float32), mlp_bf16=0)
    S_wr = oracle_lib.rollout_costs(wr, eps)[0]
    with pytest.raises(AssertionError):
        parity.assert_costs_close_bf16(S_wr, S_bf, S_fp, cond, cond_bf, "weights only")
    S_off = S_bf.copy()
    S_off[7] += 2.0 * (parity.cost_tol(S_bf, cond) + parity.BF_ULP * cond_bf)[7]
    with pytest.raises(AssertionError):
        parity.assert_costs_close_bf16(S_off, S_bf, S_fp, cond, cond_bf, "one sample off")
