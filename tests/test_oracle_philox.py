"""Pins of the oracle's Philox4x32-10 and of the stream mapping built on it."""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
from scipy import stats

from oracle import philox

HERE = os.path.dirname(os.path.abspath(__file__))
DUMP_SRC = os.path.join(HERE, "philox_ref", "rocrand_philox_dump.cpp")


@pytest.fixture(scope="module")
def rocrand_dump():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists(
            "/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"):
        pytest.skip("rocRAND headers or hipcc not available")
    d = tempfile.mkdtemp(prefix="philox_ref_")
    exe = os.path.join(d, "dump")
    subprocess.run([hipcc, "--offload-arch=gfx950", "-O1", "-o", exe, DUMP_SRC],
                   check=True, capture_output=True)
    yield exe
    shutil.rmtree(d, ignore_errors=True)


def _run_dump(exe, rows):
    inp = "\n".join(" ".join(str(int(v)) for v in r) for r in rows) + "\n"
    out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True)
    return np.array([[int(w) for w in ln.split()] for ln in out.stdout.strip().splitlines()],
                    dtype=np.uint64)


def test_philox_matches_rocrand(rocrand_dump):
    """Bit-exact agreement with rocRAND's independent Philox4x32-10 on
    random counters/keys and on the counters the filter uses."""
    rng = np.random.Generator(np.random.PCG64(7))
    n = 4000
    c = rng.integers(0, 2 ** 32, size=(n, 4), dtype=np.uint64)
    c[:, 1] &= np.uint64((1 << 30) - 1)     # the dump's offset limit
    k = rng.integers(0, 2 ** 32, size=(n, 2), dtype=np.uint64)
    # stream-shaped counters: (pair, tau, block, stream)
    extra = np.array([[p, tau, b, sid, 101, 0] for p in (0, 1, 2, 511, 2 ** 23 - 1)
                      for tau in (0, 1, 1000) for b in (0, 1, 8) for sid in (0, 4095)],
                     dtype=np.uint64)
    rows = np.concatenate([np.concatenate([c, k], axis=1), extra])
    ref = _run_dump(rocrand_dump, rows)
    # keys differ per row, so evaluate row by row
    out = np.empty_like(ref)
    for i, r in enumerate(rows):
        w = philox.philox4x32_10(r[0], r[1], r[2], r[3], int(r[4]), int(r[5]))
        out[i] = [int(v) for v in w]
    assert np.array_equal(out, ref)


def test_uniforms_on_24bit_grid_and_uniform():
    u = philox.resample_uniforms(seed=11, stream_id=0, tau=3, n=1 << 18)
    assert np.all((u >= 0) & (u < 1))
    assert np.all(u * 2 ** 24 == np.floor(u * 2 ** 24))
    assert stats.kstest(u, "uniform").pvalue > 1e-3
    assert abs(u.mean() - 0.5) < 5 * np.sqrt(1 / 12 / u.size)


def test_normals_moments_and_independence():
    z = philox.normals(seed=5, stream_id=3, tau=7, n=1 << 16, d=5)
    assert z.shape == (1 << 16, 5)
    for j in range(5):
        assert stats.kstest(z[:, j], "norm").pvalue > 1e-3
    c = np.corrcoef(z.T)
    assert np.max(np.abs(c - np.eye(5))) < 5 / np.sqrt(z.shape[0])
    # even/odd particles of a pair are uncorrelated (cosine vs sine branch)
    assert abs(np.corrcoef(z[0::2, 0], z[1::2, 0])[0, 1]) < 5 / np.sqrt(z.shape[0] / 2)


def test_stream_mapping_layout():
    """Block 0 feeds uniforms (w0, w1) and dim-0 normals (w2, w3); block b
    feeds dims 2b-1 and 2b; different tau / stream ids give different draws."""
    seed, sid, tau, n = 9, 2, 4, 16
    w = philox.philox4x32_10(np.arange(n // 2), tau, 0, sid, *philox.seed_key(seed))
    u = philox.resample_uniforms(seed, sid, tau, n)
    assert np.array_equal(u[0::2], (w[0] >> 8).astype(np.float64) / 2 ** 24)
    assert np.array_equal(u[1::2], (w[1] >> 8).astype(np.float64) / 2 ** 24)
    z = philox.normals(seed, sid, tau, n, 4)
    u1 = ((w[2] >> 8).astype(np.float64) + 1) / 2 ** 24
    u2 = (w[3] >> 8).astype(np.float64) / 2 ** 24
    rho = np.sqrt(-2 * np.log(u1))
    assert np.allclose(z[0::2, 0], rho * np.cos(2 * np.pi * u2), rtol=0, atol=1e-15)
    assert np.allclose(z[1::2, 0], rho * np.sin(2 * np.pi * u2), rtol=0, atol=1e-15)
    w1 = philox.philox4x32_10(np.arange(n // 2), tau, 1, sid, *philox.seed_key(seed))
    u1 = ((w1[2] >> 8).astype(np.float64) + 1) / 2 ** 24
    u2 = (w1[3] >> 8).astype(np.float64) / 2 ** 24
    assert np.allclose(z[1::2, 2], np.sqrt(-2 * np.log(u1)) * np.sin(2 * np.pi * u2), atol=1e-15)
    assert philox.n_blocks(1) == 1 and philox.n_blocks(2) == 2
    assert philox.n_blocks(8) == 5 and philox.n_blocks(16) == 9
    assert not np.array_equal(u, philox.resample_uniforms(seed, sid + 1, tau, n))
    assert not np.array_equal(u, philox.resample_uniforms(seed, sid, tau + 1, n))
    # the normal's radius is finite: u1 > 0 always
    assert np.all(np.isfinite(philox.normals(seed, sid, 0, 1 << 12, 2)))
