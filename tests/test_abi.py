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
    assert vct.vct_abi_version() == 5


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


def test_mlp_sizes_and_rejects():
    assert vct.vct_mlp_blob_bytes() == vct.VCT_MLP_BLOB_BYTES
    P = vct.VCT_MLP_PARAMS
    assert vct.vct_mlp_train_bytes(100) == 0 and vct.vct_mlp_train_bytes(0) == 0
    assert vct.vct_mlp_train_bytes(64) >= 16 * P + 4
    assert vct.vct_mlp_train_bytes(4096) >= 16 * P + 4096 // 64 * 4 * P
    fake = 1 << 20
    bad = [
        lambda: vct.vct_mlp_init(1, None, fake),
        lambda: vct.vct_mlp_init(1, fake + 8, fake),                        # misaligned training buffer
        lambda: vct.vct_mlp_normalize(fake, 0, 0.0, fake, fake),
        lambda: vct.vct_mlp_normalize(fake, 10, 0.5, fake, fake),
        lambda: vct.vct_mlp_train_step(fake, 100, None, 1, 0, 100, 1e-3, 1, fake, fake),     # batch not x64
        lambda: vct.vct_mlp_train_step(fake, 100, None, 1, -1, 64, 1e-3, 1, fake, fake),
        lambda: vct.vct_mlp_train_step(fake, 100, None, 1, 0, 64, float("nan"), 1, fake, fake),
        lambda: vct.vct_mlp_train_step(fake, 0, None, 1, 0, 64, 1e-3, 1, fake, fake),
        lambda: vct.vct_mlp_forward(fake, 0, fake, fake),
        lambda: vct.vct_mlp_forward(fake, 10, fake + 4, fake),
    ]
    for f in bad:
        with pytest.raises(vct.VctError) as e:
            f()
        assert e.value.code == vct.VCT_EINVAL



def test_create_population_rejects_bad_slice():
    for first, n in ((-1, 10), ((1 << 32) - 5, 10)):
        d = vct.population_desc(W.with_(W.base_trial(), first_patient=first, n_patients=n))
        with pytest.raises(vct.VctError) as e:
            vct.vct_create_population(d, 1 << 20)
        assert e.value.code == vct.VCT_EINVAL
