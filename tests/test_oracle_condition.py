"""Pin for the oracle's cost-condition number (orc_cost_condition).

cond_k = sum_{s=1..T} sum_i |dJ_k/dx_{s,i}| |x_{s,i}| is the first-order
change of a sample's cost J_k when every state component of its trajectory is
moved by one unit of its own size; the parity bounds of ill-conditioned
rollouts scale with it.  The oracle forms dJ_k/dx_s with its adjoint sweep.
Here every one of those sensitivities is recomputed independently, by central
differences of the forward rollout with a perturbation injected into x_s
(orc_sequence_cost_injected, which shares only the forward step and cost
with the rest of the oracle), and combined into the same sum.  A dropped
running-cost term, a wrong index in the costate recursion or a missing MLP
Jacobian changes the sum well beyond the bound.
"""
import numpy as np
import pytest

import workloads as W
from oracle import oracle as O


def _dJ_dx(wl, v_seq, s, i, x_si):
    h = 1e-5 * max(1.0, abs(x_si))

    def central(hh):
        return (O.sequence_cost_injected(wl, v_seq, s, i, hh)
                - O.sequence_cost_injected(wl, v_seq, s, i, -hh)) / (2.0 * hh)
    # Richardson: error O(h^4)
    return (4.0 * central(h / 2) - central(h)) / 3.0


def _cond_fd(wl, eps, k):
    u = wl.u0.astype(np.float64)
    v_seq = u + eps[:, :, k].astype(np.float64)
    xs = O.trajectory(wl, v_seq)
    total = 0.0
    terms = np.zeros((wl.T, wl.n))
    for s in range(1, wl.T + 1):
        for i in range(wl.n):
            g = _dJ_dx(wl, v_seq, s, i, xs[s, i])
            terms[s - 1, i] = abs(g) * abs(xs[s, i])
    total = terms.sum()
    return total, terms


@pytest.mark.parametrize("model,T", [("bicycle_mlp", 12), ("bicycle_mlp", 40), ("bicycle", 30)])
def test_cost_condition_matches_injected_differences(model, T):
    wl = W.c5(K=3, T=T, hidden=16)
    if model == "bicycle":
        wl = wl.replace(model="bicycle", mlp=None, mlp_hidden=0)
    eps = O.workload_noise(wl)
    cond = O.cost_condition(wl, eps=eps)
    assert cond.shape == (wl.K,) and np.all(cond > 0)
    for k in range(wl.K):
        fd, terms = _cond_fd(wl, eps, k)
        assert abs(cond[k] - fd) <= 1e-6 * fd, (k, cond[k], fd)
        # the sum is not dominated by one term: many sensitivities are pinned
        assert np.count_nonzero(terms > 1e-3 * terms.max()) >= wl.T


def test_injection_at_zero_is_the_plain_cost():
    wl = W.c5(K=2, T=15, hidden=16)
    eps = O.workload_noise(wl)
    v_seq = wl.u0.astype(np.float64) + eps[:, :, 1].astype(np.float64)
    base = O.sequence_cost(wl, v_seq)
    for s in (1, 7, 15):
        assert O.sequence_cost_injected(wl, v_seq, s, 2, 0.0) == base


def test_condition_of_a_terminal_only_cost_is_the_terminal_gradient():
    # With no running state cost (Q = 0 in l, only phi), the last step's
    # term is |dphi/dx_T| |x_T| = sum_i 2 w16 Q_i |x_T,i - r_T,i| |x_T,i|, a closed
    # form; the earlier steps add the propagated terms on top.
    wl = W.c5(K=1, T=1, hidden=16).replace(model="bicycle", mlp=None, mlp_hidden=0)
    w = wl.w.astype(np.float64).copy()
    eps = O.workload_noise(wl)
    v_seq = wl.u0.astype(np.float64) + eps[:, :, 0].astype(np.float64)
    xT = O.trajectory(wl, v_seq)[1]
    rT = wl.ref.reshape(wl.T + 1, wl.n)[1].astype(np.float64)
    q = w[:wl.n]
    # l and phi both act on x_1 here: d/dx (l + phi) = 2 (1 + w16) Q (x - r)
    expect = np.sum(2.0 * (1.0 + w[16]) * q * np.abs(xT - rT) * np.abs(xT))
    cond = O.cost_condition(wl, eps=eps)
    assert cond[0] == pytest.approx(expect, rel=1e-12)
