"""CPU-side checks of the C ABI: the library loads, exports every symbol the header
declares, reports sizes, and rejects invalid arguments before any device work."""
import ctypes as C
import os
import re

import pytest

from paper_2202_13927_amd import vct, workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    txt = open(os.path.join(ROOT, "include", "vct.h")).read()
    return sorted(set(re.findall(r"\b(vct_[a-z_]+)\s*\(", txt)))


def test_header_and_binding_agree():
    assert header_symbols() == sorted(vct.EXPORTS)


def test_library_exports_every_symbol():
    L = vct.lib()
    for name in header_symbols():
        assert hasattr(L, name), name
    assert vct.vct_abi_version() == 1


def test_sizes():
    assert vct.vct_population_bytes(1000) == 1000 * 19 * 8
    assert vct.vct_metrics_bytes(1000) == 64000
    assert vct.vct_traj_bytes(8, 7, 5) == 3 * 8 * 2016 * 8
    assert vct.vct_traj_bytes(0, 7, 5) == 0
    assert vct.vct_population_bytes(0) == 0


def _fake_pop():
    return C.c_void_p(0)


@pytest.mark.parametrize("field,value", [("n_patients", 0), ("cv", -0.1), ("ag", 1.5), ("tau_cgm", 0.0),
                                         ("g_target", -1.0), ("flags", 8)])
def test_create_population_rejects(field, value):
    d = vct.population_desc(W.base_trial())
    setattr(d, field, value)
    with pytest.raises(vct.VctError) as e:
        vct.vct_create_population(d, 1 << 20)
    assert e.value.code == vct.VCT_EINVAL
    assert vct.vct_last_error() != ""


def test_create_population_rejects_bad_nominal():
    d = vct.population_desc(W.base_trial())
    d.nominal[3] = 0.0
    with pytest.raises(vct.VctError):
        vct.vct_create_population(d, 1 << 20)
    with pytest.raises(vct.VctError):
        vct.vct_create_population(vct.population_desc(W.base_trial()), None)


def test_read_metrics_rejects():
    with pytest.raises(vct.VctError) as e:
        vct.vct_read_metrics(None, 10, 100)
    assert e.value.code == vct.VCT_EINVAL
    with pytest.raises(vct.VctError):
        vct.vct_read_metrics(1 << 20, 0, 100)
    with pytest.raises(vct.VctError):
        vct.vct_read_metrics(1 << 20, 10, 0)
