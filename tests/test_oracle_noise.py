"""Pins of the oracle's noise generator (Philox4x32-10 + Box-Muller).

The paper draws eps ~ N(0, Sigma) (Algorithm 1) without naming a generator;
the noise definition used here is written out in oracle/mppi_oracle.c.  These
tests pin the oracle's implementation to things other than itself:
  * the raw Philox4x32-10 stream against PyTorch's independent C++
    implementation (ATen/core/PhiloxRNGEngine.h), compiled here with g++;
  * the binary32 -2 ln u1 / sincos(2 pi u2) recipe against libm (numpy,
    binary64) over every one of the 2^24 possible inputs;
  * the distribution of the produced numbers (moments, KS test, correlation).
"""
import os
import subprocess
import tempfile

import numpy as np
import pytest
import torch

DRIVER = r"""
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdio>
#include <cstdlib>
int main(int argc, char** argv) {
  // args: seed counter0 counter1 counter2 counter3 (decimal)
  unsigned long long seed = strtoull(argv[1], 0, 10);
  unsigned long long c[4];
  for (int i = 0; i < 4; ++i) c[i] = strtoull(argv[2 + i], 0, 10);
  at::philox_engine e(seed, c[2] | (c[3] << 32), c[0] | (c[1] << 32));
  for (int i = 0; i < 4; ++i) printf("%u\n", e());
  return 0;
}
"""


@pytest.fixture(scope="module")
def torch_philox(tmp_path_factory):
    inc = os.path.join(os.path.dirname(torch.__file__), "include")
    d = tmp_path_factory.mktemp("philox")
    src = d / "drv.cpp"
    src.write_text(DRIVER)
    exe = d / "drv"
    subprocess.run(["g++", "-O1", "-std=c++17", f"-I{inc}", str(src), "-o", str(exe)],
                   check=True)

    def run(seed, ctr):
        out = subprocess.run([str(exe), str(seed)] + [str(int(c)) for c in ctr],
                             check=True, capture_output=True, text=True).stdout
        return np.array([int(v) for v in out.split()], dtype=np.uint32)
    return run


def test_philox_matches_pytorch_engine(oracle_lib, torch_philox):
    rng = np.random.default_rng(7)
    cases = [(0, [0, 0, 0, 0]), (1002, [0, 0, 0, 0]), (1002, [1, 2, 3, 4]),
             ((1 << 64) - 1, [0xFFFFFFFF] * 4)]
    for _ in range(12):
        seed = int(rng.integers(0, 1 << 63))
        cases.append((seed, [int(v) for v in rng.integers(0, 1 << 32, 4)]))
    for seed, ctr in cases:
        key = [seed & 0xFFFFFFFF, seed >> 32]
        ours = oracle_lib.philox(np.array(ctr, np.uint32), key)[0]
        ref = torch_philox(seed, ctr)
        assert np.array_equal(ours, ref), (seed, ctr, ours, ref)


@pytest.fixture(scope="module")
def tables(oracle_lib):
    return oracle_lib.bm_tables()


def test_radius_recipe_vs_libm_all_inputs(tables):
    r = tables[0].astype(np.float64)
    j1 = np.arange(1, (1 << 24) + 1, dtype=np.float64)
    exact = np.sqrt(-2.0 * np.log(j1 * 2.0 ** -24))
    assert r[-1] == 0.0 and exact[-1] == 0.0
    rel = np.abs(r[:-1] - exact[:-1]) / exact[:-1]
    # a few binary32 ulps (2^-24 relative each) over all 2^24 inputs
    assert rel.max() < 2.0 ** -21, rel.max()
    assert np.isfinite(r).all() and (np.diff(r) <= 0).all()  # monotone in u1


def test_angle_recipe_vs_libm_all_inputs(tables):
    c = tables[1].astype(np.float64)
    s = tables[2].astype(np.float64)
    a = 2.0 * np.pi * np.arange(1 << 24, dtype=np.float64) * 2.0 ** -24
    assert np.abs(c - np.cos(a)).max() < 2.0 ** -22
    assert np.abs(s - np.sin(a)).max() < 2.0 ** -22
    assert c[0] == 1.0 and s[0] == 0.0


def test_noise_layout_matches_definition(oracle_lib, tables):
    """eps[t][j][k] = sigma_j * z(n = t m + j) with the counter layout
    (n // 4, k, iter, instance); composed here from the separately pinned
    Philox blocks and transform tables."""
    seed, it, inst, K, T, m = 0x1234567890ABCDEF, 5, 3, 37, 7, 2
    sigma = np.array([1.0, 0.3], np.float32)
    eps = oracle_lib.noise(seed, it, inst, K, T, m, sigma)
    r_t, c_t, s_t = tables
    key = [seed & 0xFFFFFFFF, seed >> 32]
    for k in range(K):
        for t in range(T):
            for j in range(m):
                n = t * m + j
                x = oracle_lib.philox(np.array([n // 4, k, it, inst], np.uint32), key)[0]
                p = (n % 4) // 2
                a, b = int(x[2 * p]), int(x[2 * p + 1])
                r = r_t[(a >> 8)]  # table index j1 - 1
                trig = s_t if n % 2 else c_t
                z = np.float32(r * trig[b >> 8])
                assert eps[t, j, k] == np.float32(sigma[j] * z)


def test_noise_distribution(oracle_lib):
    from scipy import stats
    eps = oracle_lib.noise(1002, 0, 0, 4096, 64, 4, np.ones(4, np.float32))
    z = eps.astype(np.float64).ravel()
    N = z.size
    assert abs(z.mean()) < 5.0 / np.sqrt(N)
    assert abs(z.var() - 1.0) < 5.0 * np.sqrt(2.0 / N)
    assert abs(stats.skew(z)) < 5.0 * np.sqrt(6.0 / N)
    assert abs(stats.kurtosis(z)) < 5.0 * np.sqrt(24.0 / N)
    assert stats.kstest(z[:200000], "norm").pvalue > 1e-4
    # neighbouring samples, neighbouring time steps and the two members of a
    # Box-Muller pair are uncorrelated
    lim = 5.0 / np.sqrt(eps.shape[0] * eps.shape[2])
    for a, b in [(eps[:, 0, :-1], eps[:, 0, 1:]), (eps[:-1, 1, :], eps[1:, 1, :]),
                 (eps[:, 0, :], eps[:, 1, :]), (eps[:, 1, :], eps[:, 2, :])]:
        assert abs(np.corrcoef(a.ravel(), b.ravel())[0, 1]) < lim


def test_noise_iteration_and_instance_streams_differ(oracle_lib):
    a = oracle_lib.noise(1, 0, 0, 64, 4, 2, np.ones(2, np.float32))
    b = oracle_lib.noise(1, 1, 0, 64, 4, 2, np.ones(2, np.float32))
    c = oracle_lib.noise(1, 0, 1, 64, 4, 2, np.ones(2, np.float32))
    assert not np.array_equal(a, b) and not np.array_equal(a, c)
    # prefix property: K and T only select a window of one stream
    d = oracle_lib.noise(1, 0, 0, 32, 3, 2, np.ones(2, np.float32))
    assert np.array_equal(d, a[:3, :, :32])
