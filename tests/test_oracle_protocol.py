"""Pins of the oracle's Northern-European protocol (Sec. II-B, Tables I and II).

Each check compares the oracle with what the paper's tables fix, independent of the
arrangement the oracle draws: every season holds the weeks of Table I (top) and every week
the days of Table I (bottom), so a year has fixed totals of week and day types; the meal
plan of each day type gives the meal count and, with no size noise, carbohydrate amounts
that are Table II's grams per kg times the body weight; the shuffles put each week and day
type in each position with the probability its count fixes (chi-square); the size noise
has the stated relative SD and the onsets stay within the jitter.
"""
import numpy as np
import pytest

from paper_2202_13927_amd import workloads as W

SEASON_WEEKS = {0: (6, 4, 3), 1: (6, 6, 1), 2: (7, 3, 3), 3: (9, 3, 1)}   # standard, active, vacation
WEEK_DAYS = {0: (4, 1, 1, 1), 1: (3, 3, 1, 0), 2: (5, 0, 0, 2)}          # standard, active, movie, late
G_PER_KG = {"large": 1.29, "medium": 0.86, "small": 0.57, "snack": 0.29}


def _trial(**kw):
    return W.with_(W.base_trial(), **{"proto": W.PROTO_NORDIC, "meal_cv": 0.0, "jitter": 0, "n_days": 364,
                                      "noise_seed": 9, **kw})


def _year(orc, t, patient):
    return np.array([orc.nordic_day(t, patient, d) for d in range(364)])


def test_year_follows_table1(orc):
    t = _trial()
    for patient in (0, 1, 17, 999):
        y = _year(orc, t, patient)
        assert np.array_equal(y[:, 0], np.repeat(np.arange(4), 91))
        weeks = y[::7, 1]
        assert np.all(y[:, 1].reshape(52, 7) == weeks[:, None])            # one type per week
        for s in range(4):
            counts = np.bincount(weeks[13 * s:13 * (s + 1)], minlength=3)
            assert tuple(counts) == SEASON_WEEKS[s], (patient, s, counts)
        for w in range(52):
            counts = np.bincount(y[7 * w:7 * (w + 1), 2], minlength=4)
            assert tuple(counts) == WEEK_DAYS[weeks[w]], (patient, w)
        # yearly totals fixed by the tables: 28/16/8 weeks, 200/76/44/44 days
        assert tuple(np.bincount(weeks, minlength=3)) == (28, 16, 8)
        assert tuple(np.bincount(y[:, 2], minlength=4)) == (200, 76, 44, 44)
    # the arrangement is the patient's own and the seed's
    assert not np.array_equal(_year(orc, t, 0), _year(orc, t, 1))
    assert not np.array_equal(_year(orc, t, 0), _year(orc, _trial(noise_seed=10), 0))


def test_meals_follow_table2(orc):
    """No size noise and no jitter: every meal is a Table II size times the body weight, at
    the planned clock time, and the day's meal count is 4 (+1 on a movie night, +2 on a
    late night)."""
    t = _trial(n_patients=5)
    bw = orc.sample_population(t)[:, 14]
    plan_times = {420, 600, 720, 900, 1080, 1260, 1350}
    for patient in range(5):
        y = _year(orc, t, patient)
        for d in range(0, 364, 3):
            season, wtype, dtype = y[d]
            m = orc.day_meals(t, patient, d)
            assert len(m) == 4 + (dtype >= 2) + (dtype == 3)
            minutes = m[:, 0] * 5
            assert set(minutes) <= plan_times and np.all(np.diff(minutes) > 0)
            cold, vac = season in (0, 3), wtype == 2
            expect = {420: "medium" if vac else "small", 720: "large" if vac else "medium",
                      1080: "large" if (cold or vac) else "medium", 600: "snack", 900: "snack", 1260: "snack",
                      1350: "snack"}
            assert (900 in minutes) == cold and (600 in minutes) == (not cold)
            for mi, g in zip(minutes, m[:, 1]):
                assert g == pytest.approx(G_PER_KG[expect[int(mi)]] * bw[patient], rel=1e-12)
            assert np.allclose(m[:, 2], m[:, 1] * (1000.0 / 180.16) / 5.0, rtol=1e-12)
    # Table II's grams for a 70 kg patient
    for name, grams in (("large", 90), ("medium", 60), ("small", 40), ("snack", 20)):
        assert abs(G_PER_KG[name] * 70.0 - grams) < 0.5


def test_arrangements_are_uniform(orc):
    """Fisher-Yates gives every position the type's share: in winter a week is a vacation week
    with probability 3/13, in a standard week a day is the late night with probability 1/7
    (chi-square over positions, 99.9 % points)."""
    t = _trial()
    n = 6000
    vac = np.zeros(13)
    late = np.zeros(7)
    n_std_weeks = 0
    for patient in range(n):
        for wk in range(13):
            s, wt, _ = orc.nordic_day(t, patient, 7 * wk)
            vac[wk] += wt == 2
            if wk == 0 and wt == 0:
                n_std_weeks += 1
                for dd in range(7):
                    late[dd] += orc.nordic_day(t, patient, dd)[2] == 3
    e = n * 3 / 13
    assert ((vac - e) ** 2 / (e * (1 - 3 / 13))).sum() < 34.5     # 12 dof
    e = n_std_weeks / 7
    assert ((late - e) ** 2 / (e * (1 - 1 / 7))).sum() < 22.5      # 6 dof


def test_meal_noise_and_jitter(orc):
    t = _trial(n_patients=400, meal_cv=0.1, jitter=30)
    bw = orc.sample_population(t)[:, 14]
    ratio = []
    for patient in range(400):
        for d in (0, 91, 182, 273):
            m = orc.day_meals(t, patient, d)
            size = "medium" if orc.nordic_day(t, patient, d)[1] == 2 else "small"   # breakfast
            ratio.append(m[0, 1] / (G_PER_KG[size] * bw[patient]))
            assert np.all(m[:, 0] >= 0) and np.all(np.diff(m[:, 0]) > 0)   # time order kept
    r = np.array(ratio)
    assert abs(r.mean() - 1.0) < 4 * 0.1 / np.sqrt(len(r))
    assert r.std() == pytest.approx(0.1, rel=0.1)
    # onsets: breakfast at 07:00 +- 30 min, i.e. samples 78..90 (the interval containing the minute)
    kb = np.array([orc.day_meals(t, p, 5)[0, 0] for p in range(400)])
    assert kb.min() >= (420 - 30) // 5 and kb.max() <= (420 + 30) // 5
    assert len(np.unique(kb)) > 8
