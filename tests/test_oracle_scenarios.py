"""Pins of the oracle's scenario setting (Sec. IV-E: trial B, the basal rate underestimated
by 50 %): the controller works with basal_scale u_b in place of u_b.

With all PID gains zero the PID law reduces to its baseline, so the closed loop must equal
the open-loop controller at u_rel = basal_scale, and the delivered insulin has the closed
form basal_scale u_b K Ts; with the gains on, trial B delivers less insulin in total."""
import numpy as np
import pytest

from paper_2202_13927_amd import workloads as W


def _trial(**kw):
    return W.with_(W.c1_fp64_pid(), **{"n_patients": 40, "n_days": 3, **kw})


def test_zero_gain_pid_is_scaled_open_loop(orc):
    for scale in (1.0, 0.5, 1.7):
        pid = orc.simulate(_trial(kp=0.0, ki=0.0, kd=0.0, basal_scale=scale), threads=4)
        opn = orc.simulate(_trial(ctrl_kind=W.CTRL_OPEN, u_rel=scale), threads=4)
        for k in ("bins", "events", "sum_g", "min_g", "argmin_k"):
            assert np.array_equal(pid[k], opn[k]), (scale, k)
        ub = pid["params"][:, 15]
        assert np.allclose(pid["sum_u"], scale * ub * pid["K"] * 5.0, rtol=1e-12)


def test_open_loop_scale_multiplies_the_rate(orc):
    a = orc.simulate(_trial(ctrl_kind=W.CTRL_OPEN, u_rel=1.0, basal_scale=0.5), threads=4)
    b = orc.simulate(_trial(ctrl_kind=W.CTRL_OPEN, u_rel=0.5), threads=4)
    for k in ("bins", "sum_g", "sum_u"):
        assert np.array_equal(a[k], b[k]), k


def test_underestimated_basal_delivers_less(orc):
    a = orc.simulate(_trial(), threads=4)
    b = orc.simulate(_trial(basal_scale=0.5), threads=4)
    assert b["sum_u"].sum() < a["sum_u"].sum()
    assert b["sum_g"].sum() > a["sum_g"].sum()          # less insulin, higher glucose
    with pytest.raises(Exception):
        orc.simulate(_trial(basal_scale=0.0), threads=4)
