"""Pins of the oracle's virtual population (Sec. II-A, Sec. IV-B parameter sampling).

Parameters are lognormal with median = nominal and the given CV. A draw is kept
iff the basal steady state exists; at G* = 6 mmol/L that is exactly EGP0 > F01,
so the first-attempt acceptance rate has the closed form Phi(ln(EGP0/F01) /
(s sqrt 2)), s = sqrt(ln(1 + CV^2)), and the other 13 parameters stay exactly
lognormal.
"""
import numpy as np
from scipy import stats

from paper_2202_13927_amd import workloads as W

N = 40_000


def _pop(orc, **kw):
    t = W.with_(W.base_trial(), n_patients=N, **kw)
    return t, orc.sample_population(t)


def test_lognormal_moments(orc):
    t, p = _pop(orc)
    s = np.sqrt(np.log(1 + 0.2 ** 2))
    assert abs(s - 0.198042) < 1e-6
    nom = np.array(W.NOMINAL)
    for j, name in enumerate(W.PARAM_NAMES):
        if name in ("EGP0", "F01"):
            continue
        z = np.log(p[:, j] / nom[j])
        assert abs(z.mean()) < 5 * s / np.sqrt(N), name
        assert abs(z.std() - s) < 5 * s / np.sqrt(2 * N), name
        assert stats.kstest(z / s, "norm").pvalue > 1e-4, name


def test_acceptance_rate_closed_form(orc):
    t, p = _pop(orc)
    s = np.sqrt(np.log(1 + 0.2 ** 2))
    pacc = stats.norm.cdf(np.log(W.NOMINAL[0] / W.NOMINAL[1]) / (s * np.sqrt(2)))
    first = np.mean(p[:, 17] == 1)
    assert abs(first - pacc) < 5 * np.sqrt(pacc * (1 - pacc) / N)
    assert np.all(p[:, 0] > p[:, 1])              # kept draws have EGP0 > F01
    assert np.all(p[:, 15] > 0) and np.all(p[:, 16] > 0)
    assert np.all(p[:, 18] == 0)


def test_min_basal_flag(orc):
    t, p = _pop(orc, pop_flags=1)
    ok = p[:, 18] == 0
    assert ok.mean() > 0.99
    assert np.all(p[ok, 15] >= 400.0 / 60.0)


def test_exhausted_resample_falls_back_to_nominal(orc):
    nom = list(W.NOMINAL)
    nom[1] = nom[0] * 1.5          # F01 > EGP0: no basal state exists for any draw
    t = W.with_(W.base_trial(), n_patients=5, nominal=nom, cv=1e-9)
    p = orc.sample_population(t)
    assert np.all(p[:, 18] == 4)
    assert np.allclose(p[:, :15], nom, rtol=0, atol=0)
    assert np.all(p[:, 17] == 32)


def test_patient_ranges_are_independent(orc):
    t = W.with_(W.base_trial(), n_patients=64)
    full = orc.sample_population(t)
    part = orc.sample_population(t, first=17, count=9)
    assert np.array_equal(full[17:26], part)
    t2 = W.with_(t, arm_id=3)
    assert not np.array_equal(orc.sample_population(t2)[:, :15], full[:, :15])
