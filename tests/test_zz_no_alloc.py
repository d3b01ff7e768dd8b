"""The allocation-free reduction (vct_read_metrics_noalloc) against vct_read_metrics.

Both entry points run the same kernels with the same launch shapes, so every field of the
summary must be equal bit for bit. Two calls in a row on the shared static workspace, the
second with fewer patients and samples (what the first leaves behind must not leak into
it); the largest supported sample count; rejection beyond it.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _records(torch, n, K, seed):
    from paper_2202_13927_amd import vct
    rng = np.random.default_rng(seed)
    tir = rng.integers(0, K + 1, n)
    rest = K - tir
    b0 = rng.integers(0, rest + 1)
    bins = np.stack([b0, np.zeros(n, np.int64), tir, rest - b0, np.zeros(n, np.int64)], 1).astype(np.int32)
    parts = {"sum_g": rng.uniform(0, 15 * K, n), "min_g": np.round(rng.uniform(-1, 6, n), 2),
             "sum_u": rng.uniform(0, 1e5, n), "bins": bins.T, "events": rng.integers(0, 50, (3, n)),
             "argmin_k": rng.integers(0, K, n), "status": np.where(rng.random(n) < 0.05, 2, 0)}
    buf = np.zeros(vct.vct_metrics_bytes(n), np.uint8)
    for name, kind, off, rows in vct.METRIC_LAYOUT:
        a = np.ascontiguousarray(parts[name]).astype({"f8": "<f8", "i4": "<i4", "u4": "<u4"}[kind])
        raw = a.reshape(-1).view(np.uint8)
        buf[off * n:off * n + raw.size] = raw
    return torch.from_numpy(buf).cuda()


def _same(a, b):
    da, db = a.as_dict(), b.as_dict()
    assert da.keys() == db.keys()
    for k in da:
        assert np.array_equal(np.asarray(da[k]), np.asarray(db[k])), k


def test_noalloc_equals_read_metrics_twice(dev):
    from paper_2202_13927_amd import vct
    cases = ((1_000_000, 104_832, 1), (4_099, 2_016, 2))
    bufs = [_records(dev, n, K, seed) for n, K, seed in cases]
    got = []
    for (n, K, _), buf in zip(cases, bufs):       # consecutive calls on the static workspace
        print(f"[gpu] noalloc reduction n={n} K={K}", flush=True)
        got.append(vct.vct_read_metrics_noalloc(buf, n, K))
    for (n, K, _), buf, g in zip(cases, bufs, got):
        _same(g, vct.vct_read_metrics(buf, n, K))


def test_noalloc_largest_sample_count(dev):
    from paper_2202_13927_amd import vct
    K = vct.VCT_NOALLOC_MAX_SAMPLES
    print(f"[gpu] noalloc reduction at K={K}", flush=True)
    buf = _records(dev, 70_001, K, 3)
    _same(vct.vct_read_metrics_noalloc(buf, 70_001, K), vct.vct_read_metrics(buf, 70_001, K))
    with pytest.raises(vct.VctError) as e:
        vct.vct_read_metrics_noalloc(buf, 70_001, K + 1)
    assert e.value.code == vct.VCT_EINVAL
