"""Pins for the oracle's bfloat16 option of the MLP residual dynamics.

In that option the MLP's three products take bfloat16 operands: the weights
and each product's input (z = (x, v), h1, h2) are rounded to binary32 and then
to the nearest bfloat16, ties to even; biases, sums and tanh stay binary64;
the backward pass takes the roundings as the identity (straight-through).
Every piece is checked against torch on the CPU, whose float32 -> bfloat16
conversion rounds to nearest-even:
  * the rounding itself, on random values of every scale, constructed ties
    (both parities), values one unit either side of a tie, subnormals, signed
    zeros, the overflow threshold, infinities and NaN;
  * one step of the dynamics against the residual evaluated in float64 from
    torch-rounded operands;
  * the backward of the residual against torch autograd through a
    straight-through rounding (x + (round(x) - x).detach());
  * the bfloat16 sensitivity sum cond_bf of a one-step rollout against torch
    autograd, the derivatives taken with respect to the rounded operands.
A plausible slip (rounding before tanh instead of after, leaving z or the
weights unrounded, truncating instead of rounding, the unrounded activations
in the weight gradients) fails one of them.
"""
import numpy as np
import pytest
import torch

import workloads as W


def _tbf(a):
    """torch's nearest-even bfloat16 of float32(a), as float64."""
    t = torch.tensor(np.asarray(a, np.float64).astype(np.float32))
    return t.to(torch.bfloat16).to(torch.float64).numpy()


def _bits(u32):
    with np.errstate(invalid="ignore"):
        return np.asarray(u32, np.uint32).view(np.float32).astype(np.float64)


def test_bf16_rounding_against_torch(oracle_lib):
    rng = np.random.default_rng(7)
    vals = [rng.normal(0.0, 1.0, 2000) * 10.0 ** rng.integers(-35, 36, 2000)]
    # ties: the low 16 bits exactly half of the kept unit, kept value even and odd
    kept = rng.integers(0, 2 ** 15, 500, dtype=np.uint32) << np.uint32(16)
    for low in (0x8000, 0x7FFF, 0x8001, 0x0000, 0xFFFF):
        for parity in (0, 1):
            b = (kept | (np.uint32(parity) << np.uint32(16))) | np.uint32(low)
            vals.append(_bits(b))
            vals.append(-_bits(b))
    vals.append(_bits(np.arange(1, 70000, 97, dtype=np.uint32)))  # subnormals
    big = np.float32(3.3961e38)  # near the halfway point above bfloat16's largest finite
    vals.append(np.array([0.0, -0.0, np.inf, -np.inf, float(np.finfo(np.float32).max),
                          float(big), float(np.nextafter(big, np.float32(0))), 1.0, -1.0]))
    x = np.concatenate(vals)
    got = oracle_lib.bf16(x)
    want = _tbf(x)
    assert np.array_equal(np.isnan(got), np.isnan(want))
    ok = ~np.isnan(want)
    assert np.array_equal(got[ok], want[ok])
    assert np.array_equal(np.signbit(got[ok]), np.signbit(want[ok]))
    assert np.isnan(oracle_lib.bf16([np.nan]))[0]
    # binary64 inputs go through binary32 first
    d = rng.normal(0.0, 3.0, 500)
    assert np.array_equal(oracle_lib.bf16(d), _tbf(d.astype(np.float32)))


def _blocks(wl):
    H = wl.mlp_hidden
    p = np.asarray(wl.mlp, np.float64)
    o = 0
    out = []
    for n, shape in ((H * 7, (H, 7)), (H, (H,)), (H * H, (H, H)), (H, (H,)), (5 * H, (5, H)),
                     (5, (5,))):
        out.append(p[o:o + n].reshape(shape))
        o += n
    return out


@pytest.mark.parametrize("hidden", [16, 64])
def test_mlp_residual_bf16_against_torch(oracle_lib, hidden):
    wl = W.c5(K=1, T=1, hidden=hidden).replace(mlp_bf16=1)
    W1, b1, W2, b2, W3, b3 = _blocks(wl)
    W1r, W2r, W3r = _tbf(W1), _tbf(W2), _tbf(W3)
    plain = wl.replace(model="bicycle", mlp=None, mlp_hidden=0)
    full = wl.replace(mlp_bf16=0)
    rng = np.random.default_rng(2)
    dt = float(np.float32(wl.dt))
    for _ in range(6):
        x = np.array([10.0, 40.0, 0.2, 5.0, 0.05]) + rng.normal(0, 0.5, 5)
        v = rng.normal(0, 1.0, 2)
        z = _tbf(np.concatenate([x, v]))
        h1 = _tbf(np.tanh(W1r @ z + b1))
        h2 = _tbf(np.tanh(W2r @ h1 + b2))
        g = W3r @ h2 + b3
        diff = oracle_lib.step(wl, x, v) - oracle_lib.step(plain, x, v)
        np.testing.assert_allclose(diff, dt * g, rtol=1e-12, atol=1e-14)
        # the option changes the result (by the roundings, not more)
        d64 = oracle_lib.step(full, x, v) - oracle_lib.step(plain, x, v)
        assert np.abs(diff - d64).max() > 0.0
        assert np.abs(diff - d64).max() < 0.1 * np.abs(d64).max()


def _ste(t):
    r = t.detach().to(torch.float32).to(torch.bfloat16).to(torch.float64)
    return t + (r - t).detach()


@pytest.mark.parametrize("bf", [0, 1], ids=["binary64", "bf16"])
def test_mlp_vjp_against_torch_autograd(oracle_lib, bf):
    wl = W.c5(K=1, T=1, hidden=16).replace(mlp_bf16=bf)
    rnd = _ste if bf else (lambda t: t)
    rng = np.random.default_rng(11)
    for _ in range(4):
        x = np.array([10.0, 40.0, 0.2, 5.0, 0.05]) + rng.normal(0, 0.5, 5)
        z = np.concatenate([x, rng.normal(0, 1.0, 2)])
        cg = rng.normal(0, 1.0, 5)
        p = torch.tensor(np.asarray(wl.mlp, np.float64), requires_grad=True)
        zt = torch.tensor(z, requires_grad=True)
        H = wl.mlp_hidden
        o = [0]

        def take(n, shape):
            t = p[o[0]:o[0] + n].reshape(shape)
            o[0] += n
            return t
        W1 = take(H * 7, (H, 7)); b1 = take(H, (H,)); W2 = take(H * H, (H, H))
        b2 = take(H, (H,)); W3 = take(5 * H, (5, H)); b3 = take(5, (5,))
        h1 = torch.tanh(rnd(W1) @ rnd(zt) + b1)
        h2 = torch.tanh(rnd(W2) @ rnd(h1) + b2)
        g = rnd(W3) @ rnd(h2) + b3
        (g * torch.tensor(cg)).sum().backward()
        dz, dm = oracle_lib.mlp_vjp(wl, z, cg)
        np.testing.assert_allclose(dz, zt.grad.numpy(), rtol=1e-11, atol=1e-13)
        np.testing.assert_allclose(dm, p.grad.numpy(), rtol=1e-11, atol=1e-13)


def test_bf16_sensitivity_one_step_against_torch(oracle_lib):
    """cond_bf of a one-step rollout: sum over the rounded product inputs o of
    |dJ/do| |o|, J = l(x1, v0) + phi(x1) with x1 = bicycle step + dt g."""
    wl = W.c5(K=5, T=1, hidden=16).replace(mlp_bf16=1)
    W1, b1, W2, b2, W3, b3 = _blocks(wl)
    W1r, W2r, W3r = (torch.tensor(_tbf(a)) for a in (W1, W2, W3))
    b1, b2, b3 = (torch.tensor(a) for a in (b1, b2, b3))
    plain = wl.replace(model="bicycle", mlp=None, mlp_hidden=0)
    eps = oracle_lib.workload_noise(wl)
    cond, cond_bf = oracle_lib.cost_condition(wl, eps=eps, bf=True)
    Q = torch.tensor(np.asarray(wl.w[:5], np.float64))
    term = float(wl.w[16])
    ref1 = torch.tensor(np.asarray(wl.ref, np.float64)[1])
    dt = float(np.float32(wl.dt))
    x0 = np.asarray(wl.x0, np.float64)
    for k in range(wl.K):
        v = np.asarray(wl.u0[0], np.float64) + eps[0, :, k].astype(np.float64)
        # the rounded operands as the products consume them; the derivatives
        # pass the later roundings straight through, as the oracle's do
        z = torch.tensor(_tbf(np.concatenate([x0, v])), requires_grad=True)
        h1 = _ste(torch.tanh(W1r @ z + b1))
        h1.retain_grad()
        h2 = _ste(torch.tanh(W2r @ h1 + b2))
        h2.retain_grad()
        g = W3r @ h2 + b3
        x1 = torch.tensor(oracle_lib.step(plain, x0, v)) + dt * g
        dev = x1 - ref1
        J = (1.0 + term) * (Q * dev * dev).sum()
        # the control term does not depend on the operands; the value check
        # ties the torch cost to the oracle's
        x1n = x1.detach().numpy()
        J_or = oracle_lib.running_cost(wl, x1n, v, 0) + oracle_lib.terminal_cost(wl, x1n)
        ctrl = oracle_lib.running_cost(wl, np.asarray(wl.ref, np.float64)[1], v, 0)
        assert abs(J.item() + ctrl - J_or) <= 1e-9 * max(1.0, abs(J_or))
        J.backward()
        want = sum((t.grad.abs() * t.detach().abs()).sum().item() for t in (z, h1, h2))
        assert cond_bf[k] == pytest.approx(want, rel=1e-10, abs=1e-14)
