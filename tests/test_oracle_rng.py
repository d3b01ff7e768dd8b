"""Pins of the oracle's random-number stream (Sec. III-A: dw ~ N(0, I dt), v ~ N(0, R)).

Philox4x32-10 is pinned to an independent implementation, rocRAND's
`philox4x32_10` engine (a library routine, compiled here as host code); the
uniform map is pinned to its exact definition; the normals to N(0, 1) by
moments and a Kolmogorov-Smirnov test; the Euler-Maruyama step to the exact
moments of the EM recursion on an Ornstein-Uhlenbeck process.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

HERE = os.path.dirname(os.path.abspath(__file__))
REF_SRC = os.path.join(HERE, "golden", "rocrand_philox_ref.hip")

CASES = [
    ((0, 0), (0, 0, 0, 0)),
    ((0xFFFFFFFF, 0xFFFFFFFF), (0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF)),
    ((7, 9), (100, 5, 2, 1)),
    ((0, 0), (104831, 999999, 2, 1)),
    ((0x12345678, 0x9ABCDEF0 ^ 63), (17, 123456, 1, 3)),
    ((5, 0), (3, 42, 0, 31)),
]


@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND reference")
    exe = str(tmp_path_factory.mktemp("rr") / "rocrand_philox_ref")
    subprocess.run([hipcc, "-O1", "-x", "hip", "--offload-arch=gfx950", REF_SRC, "-o", exe], check=True,
                   capture_output=True)
    return exe


def test_philox_matches_rocrand(orc, rocrand_ref):
    for key, ctr in CASES:
        out = subprocess.run([rocrand_ref, *[str(v) for v in key], *[str(v) for v in ctr]], check=True,
                             capture_output=True, text=True).stdout.split()
        ref = np.array([int(v) for v in out], dtype=np.uint32)
        got = orc.philox(ctr, key)
        assert np.array_equal(got, ref), (key, ctr, got, ref)


def test_uniform_exact_map(orc):
    assert orc.uniform(0) == 2.0 ** -24
    assert orc.uniform(0xFFFFFFFF) == 1.0 - 2.0 ** -24
    rng = np.random.default_rng(0)
    for x in rng.integers(0, 2 ** 32, size=2000, dtype=np.uint64):
        u = orc.uniform(int(x))
        assert u == (2 * (int(x) >> 9) + 1) / 2.0 ** 24
        assert float(np.float32(u)) == u        # exactly representable in FP32
        assert 0.0 < u < 1.0


def test_normals_are_standard(orc):
    # theta = 0, h = 1, one step: X_1 = normal #0 of counter (0, path, DIFF, 0)
    n = 200_000
    z = orc.em_ou(0.0, 1.0, 0.0, 1.0, 1, n, 12345)
    assert abs(z.mean()) < 5 / np.sqrt(n)
    assert abs(z.var() - 1.0) < 5 * np.sqrt(2.0 / n)
    assert stats.kstest(z, "norm").pvalue > 1e-4
    # the four normals of one call are uncorrelated
    zz = np.array([orc.normals4((0, p, 2, 0), (3, 4)) for p in range(20000)])
    c = np.corrcoef(zz.T)
    assert np.all(np.abs(c - np.eye(4)) < 5 / np.sqrt(20000))


@pytest.mark.parametrize("theta,h,n", [(0.5, 0.1, 20), (0.2, 1.0, 7), (1.5, 0.5, 3)])
def test_em_ou_moments(orc, theta, h, n):
    """EM on dX = -theta X dt + s dW: X_n = a X_{n-1} + s sqrt(h) xi, a = 1 - theta h, so
    E X_n = a^n x0 and Var X_n = s^2 h (1 - a^(2n)) / (1 - a^2) exactly."""
    s, x0, paths = 0.7, 2.0, 200_000
    x = orc.em_ou(theta, s, x0, h, n, paths, 777)
    a = 1.0 - theta * h
    mean = a ** n * x0
    var = s * s * h * (1 - a ** (2 * n)) / (1 - a * a)
    assert abs(x.mean() - mean) < 5 * np.sqrt(var / paths)
    assert abs(x.var() - var) < 5 * var * np.sqrt(2.0 / paths)


def test_em_ou_weak_limit(orc):
    """As h -> 0 the EM moments approach the exact OU law with O(h) error."""
    theta, s, x0, t = 0.5, 1.0, 2.0, 2.0
    exact_var = s * s * (1 - np.exp(-2 * theta * t)) / (2 * theta)
    errs = []
    for h in (0.2, 0.1):
        n = int(round(t / h))
        a = 1.0 - theta * h
        var_em = s * s * h * (1 - a ** (2 * n)) / (1 - a * a)
        errs.append(abs(var_em - exact_var))
        x = orc.em_ou(theta, s, x0, h, n, 100_000, 99)
        assert abs(x.var() - var_em) < 5 * var_em * np.sqrt(2.0 / 100_000)
        assert abs(x.mean() - x0 * np.exp(-theta * t)) < 2 * theta * h * x0 + 5 * np.sqrt(var_em / 100_000)
    assert 1.6 < errs[0] / errs[1] < 2.4
