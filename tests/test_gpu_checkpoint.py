"""Checkpoint round trip through the C-ABI (pf_save / pf_load): a filter
restored from a checkpoint continues bit for bit like the one that was
saved; mismatched, truncated or corrupt checkpoints are rejected."""
import numpy as np
import pytest

import workloads as W
from tests.gpu_util import log

pytestmark = pytest.mark.gpu


def _same_record(a, b):
    assert a.keys() == b.keys()
    for k in a:
        assert np.array_equal(np.asarray(a[k]), np.asarray(b[k])), k


def _state(f):
    x, w, t, ln = f.get_state()
    return x.copy(), w.copy(), t, ln


@pytest.mark.parametrize("name,N,radix,dtype", [
    ("lg4dense", 8192, 64, "f32"),
    ("lg4dense", 8192, 8192, "f32"),     # global path: log-weights all zero
    ("ar1", 1024, 2, "f64"),
    ("sv", 16384, 256, "bf16"),          # block path, BF16 storage
])
def test_save_load_continues_bit_exact(name, N, radix, dtype):
    from paper_1812_01502_amd import Filter
    model = {"lg4dense": lambda: W.dense_lg_model(4, 12), "ar1": W.ar1_model, "sv": W.sv_model}[name]()
    _, ys = W.simulate(model, 12, seed=9)
    log(f"[case] checkpoint {name} N={N} r={radix} {dtype}")
    a = Filter(model, N, radix, dtype=dtype, seed=5, history=2)
    for t in range(6):
        a.step(ys[t])
    blob = a.save()
    saved = _state(a)
    rec_a6 = a.estimate()
    for t in range(6, 11):
        a.step(ys[t])
    end_a = _state(a)
    est_a = a.estimate()

    b = Filter(model, N, radix, dtype=dtype, seed=5, history=2)
    b.step(ys[0])                     # some other state first
    b.load(blob)
    got = _state(b)
    for u, v in zip(saved[:2], got[:2]):
        assert np.array_equal(u, v)
    assert got[2] == saved[2] == 6 and got[3] == saved[3]
    _same_record(b.estimate(), rec_a6)
    for t in range(6, 11):
        b.step(ys[t])
    end_b = _state(b)
    for u, v in zip(end_a[:2], end_b[:2]):
        assert np.array_equal(u, v)
    assert end_a[2:] == end_b[2:]
    _same_record(b.estimate(), est_a)
    a.close()
    b.close()


def test_load_rejects_mismatch_and_corruption():
    from paper_1812_01502_amd import Filter, PfError
    model = W.dense_lg_model(4, 12)
    _, ys = W.simulate(model, 3, seed=9)
    a = Filter(model, 4096, 64, seed=1)
    a.step(ys[0])
    blob = a.save()
    other_n = Filter(model, 8192, 64, seed=1)
    other_r = Filter(model, 4096, 4, seed=1)
    other_m = Filter(W.dense_lg_model(4, 13), 4096, 64, seed=1)
    for f in (other_n, other_r, other_m):
        with pytest.raises(PfError):
            f.load(blob)
    with pytest.raises(PfError):
        a.load(blob[:-8])
    bad = bytearray(blob)
    bad[0] ^= 1
    with pytest.raises(PfError):
        a.load(bytes(bad))
    # a different seed is allowed: the state comes back, later draws differ
    c = Filter(model, 4096, 64, seed=2)
    c.load(blob)
    x0, w0, t0, ln0 = a.get_state()
    x1, w1, t1, ln1 = c.get_state()
    assert np.array_equal(x0, x1) and np.array_equal(w0, w1) and (t0, ln0) == (t1, ln1)
    for f in (a, other_n, other_r, other_m, c):
        f.close()
