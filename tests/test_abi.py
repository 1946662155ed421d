"""CPU checks of the C-ABI library: it loads, exports every function that
include/pf.h declares, its ctypes layouts match the C header, and host-side
argument validation reports errors without touching a GPU."""
import ctypes
import os
import re
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pf.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(pf_\w+)\s*\(", src, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_1812_01502_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libpf.so is not built (run __graft_entry__.build())")
    return _lib.load()


def test_exports_every_declared_symbol(lib):
    from paper_1812_01502_amd import _lib
    declared = _declared_functions()
    assert len(declared) >= 14
    assert sorted(_lib.EXPORTS) == declared
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (pf_\w+)$", out, flags=re.M))
    for name in declared:
        assert name in exported, name
        assert hasattr(lib, name)


def test_struct_layouts_match_header():
    """sizeof/offsetof of the public structs from a C compiler equal ctypes'."""
    from paper_1812_01502_amd import _lib as L
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    fields = {
        "pf_model": ("PfModel", ["kind", "d", "A", "Q_chol", "H", "R_chol", "m0", "P0_chol",
                                 "phi", "sigma", "beta"]),
        "pf_config": ("PfConfig", ["n_particles", "radix", "resampler", "state_dtype", "seed",
                                   "stream_id", "history", "keep_ancestors", "full_cycle",
                                   "island", "island_swap", "ess_threshold"]),
        "pf_estimate_t": ("PfEstimate", ["t", "stage", "radix", "valid", "log_normaliser", "ess",
                                         "max_log_weight", "next_offset", "mean", "var"]),
        "pf_info_t": ("PfInfo", ["n_particles", "d", "n_stages", "radices", "global_path",
                                 "state_dtype", "device_bytes", "t", "tile_elems"]),
        "pf_batch_tune_t": ("PfBatchTune", ["class_index", "dim", "model_kind", "pairs_per_thread",
                                            "radix", "chosen", "ms_per_step", "reserved"]),
    }
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(){"]
    for cname, (_, fl) in fields.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f in fl:
            lines.append(f'printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0;}")
    d = tempfile.mkdtemp()
    try:
        src = os.path.join(d, "l.c")
        open(src, "w").write("\n".join(lines))
        exe = os.path.join(d, "l")
        subprocess.run([cc, src, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout
    finally:
        shutil.rmtree(d, ignore_errors=True)
    got = dict(line.split() for line in out.strip().splitlines())
    for cname, (pyname, fl) in fields.items():
        cls = getattr(L, pyname)
        assert int(got[cname]) == ctypes.sizeof(cls), cname
        for f in fl:
            assert int(got[f"{cname}.{f}"]) == getattr(cls, f).offset, (cname, f)


def _model_lg(d=2):
    from paper_1812_01502_amd import _lib as L
    keep = [np.eye(d) for _ in range(5)] + [np.zeros(d)]
    m = L.PfModel()
    m.kind, m.d = L.PF_MODEL_LG, d
    for nm, a in zip(("A", "Q_chol", "H", "R_chol", "P0_chol", "m0"), keep):
        setattr(m, nm, a.ctypes.data_as(L.DPTR))
    return m, keep


def _cfg(n=1024, radix=2, resampler=0, dtype=0):
    from paper_1812_01502_amd import _lib as L
    c = L.PfConfig()
    c.n_particles, c.radix, c.resampler, c.state_dtype, c.seed = n, radix, resampler, dtype, 1
    return c


@pytest.mark.parametrize("case", ["n_not_pow2", "n_one", "radix_3", "radix_1", "dtype_bad",
                                  "resampler_bad", "d_zero", "d_17", "null_matrix",
                                  "not_lower", "neg_diag", "nan_entry", "sv_phi",
                                  "island_3", "island_n", "island_8192", "island_full_cycle",
                                  "ess_negative", "ess_above_one", "ess_bf16", "ess_radix_128",
                                  "ess_island"])
def test_create_rejects_invalid_arguments(lib, case):
    from paper_1812_01502_amd import _lib as L
    m, keep = _model_lg(2)
    c = _cfg()
    if case == "n_not_pow2":
        c.n_particles = 1000
    elif case == "n_one":
        c.n_particles = 1
    elif case == "radix_3":
        c.radix = 3
    elif case == "radix_1":
        c.radix = 1
    elif case == "dtype_bad":
        c.state_dtype = 7
    elif case == "resampler_bad":
        c.resampler = 5
    elif case == "d_zero":
        m.d = 0
    elif case == "d_17":
        m.d = 17
    elif case == "null_matrix":
        m.A = ctypes.cast(None, L.DPTR)
    elif case == "not_lower":
        bad = np.array([[1.0, 0.5], [0.0, 1.0]])
        keep.append(bad)
        m.Q_chol = bad.ctypes.data_as(L.DPTR)
    elif case == "neg_diag":
        bad = np.array([[-1.0, 0.0], [0.0, 1.0]])
        keep.append(bad)
        m.R_chol = bad.ctypes.data_as(L.DPTR)
    elif case == "nan_entry":
        bad = np.array([[np.nan, 0.0], [0.0, 1.0]])
        keep.append(bad)
        m.A = bad.ctypes.data_as(L.DPTR)
    elif case == "sv_phi":
        m = L.PfModel()
        m.kind, m.d, m.phi, m.sigma, m.beta = L.PF_MODEL_SV, 1, 1.0, 0.25, 0.6
    elif case == "island_3":
        c.island = 3
    elif case == "island_n":
        c.island = 1024                 # one island: at least two are needed
    elif case == "island_8192":
        c.n_particles, c.island = 1 << 16, 8192
    elif case == "island_full_cycle":
        c.island, c.full_cycle = 64, 1
    elif case == "ess_negative":
        c.ess_threshold = -0.5
    elif case == "ess_above_one":
        c.ess_threshold = 1.5
    elif case == "ess_bf16":
        c.ess_threshold, c.state_dtype = 0.5, 1
    elif case == "ess_radix_128":
        c.ess_threshold, c.radix = 0.5, 128
    elif case == "ess_island":
        c.ess_threshold, c.island = 0.5, 64
    h = ctypes.c_void_p()
    st = lib.pf_create(ctypes.byref(m), ctypes.byref(c), None, ctypes.byref(h))
    assert st == -1, (case, st, lib.pf_last_error(None))
    assert h.value is None
    assert lib.pf_last_error(None)


def test_unsupported_radix_reported(lib):
    """A stage radix the tile kernels cannot hold is refused before any
    device work (r = 8192 with N = 2^20: two stages of 8192, then 16)."""
    m, keep = _model_lg(2)
    c = _cfg(n=1 << 20, radix=8192)
    h = ctypes.c_void_p()
    st = lib.pf_create(ctypes.byref(m), ctypes.byref(c), None, ctypes.byref(h))
    assert st == -2
    assert b"radix" in lib.pf_last_error(None)


def test_misc_entry_points_without_device(lib):
    assert lib.pf_destroy(None) == 0
    assert lib.pf_status_string(0) == b"ok"
    assert lib.pf_status_string(-5) == b"non-finite value"
    assert lib.pf_step(None, None) == -1
    assert lib.pf_sync(None) == -1
    n = ctypes.c_uint64(0)
    assert lib.pf_save(None, None, 0, ctypes.byref(n)) == -1
    assert lib.pf_load(None, None, 0) == -1


def test_batch_create_rejects_invalid_arguments(lib):
    """Argument checks of pf_batch_create run before any device work."""
    from paper_1812_01502_amd import _lib as L
    m, keep = _model_lg(2)
    h = ctypes.c_void_p()
    ms = (L.PfModel * 2)(m, m)

    def cfgs(**kw):
        arr = (L.PfConfig * 2)()
        for i in range(2):
            arr[i] = _cfg(n=kw.get("n", 4096), radix=kw.get("radix", 4))
            arr[i].state_dtype = kw.get("dtype", 0)
        return arr

    assert lib.pf_batch_create(ms, cfgs(), 0, None, ctypes.byref(h)) == -1
    assert lib.pf_batch_create(ms, cfgs(n=256), 2, None, ctypes.byref(h)) == -1
    assert lib.pf_batch_create(ms, cfgs(radix=128), 2, None, ctypes.byref(h)) == -1
    assert lib.pf_batch_create(ms, cfgs(radix=3), 2, None, ctypes.byref(h)) == -1
    assert lib.pf_batch_create(ms, cfgs(dtype=1), 2, None, ctypes.byref(h)) == -2
    assert b"FP32" in lib.pf_batch_last_error(None)
    arr = cfgs()
    arr[1].island = 64
    assert lib.pf_batch_create(ms, arr, 2, None, ctypes.byref(h)) == -2
    assert b"island" in lib.pf_batch_last_error(None)
    arr = cfgs()
    arr[0].full_cycle = 1
    assert lib.pf_batch_create(ms, arr, 2, None, ctypes.byref(h)) == -2
    bad = (L.PfModel * 2)(m, m)
    bad[1].d = 0
    assert lib.pf_batch_create(bad, cfgs(), 2, None, ctypes.byref(h)) == -1
    assert b"filter 1" in lib.pf_batch_last_error(None)
    assert lib.pf_batch_destroy(None) == 0
    assert lib.pf_batch_step(None, None, None) == -1


class _CountingAllocator:
    """Hands out fake, 256-byte aligned addresses (nothing is dereferenced on
    the host) and records every alloc and free."""

    def __init__(self, misalign=False, fail_after=None):
        self.next = 1 << 40
        self.live = {}
        self.allocs = []
        self.frees = []
        self.misalign = misalign
        self.fail_after = fail_after

    def alloc(self, n):
        if self.fail_after is not None and len(self.allocs) >= self.fail_after:
            return None
        p = self.next + (8 if self.misalign else 0)
        self.next += (n + 4095) & ~4095
        self.live[p] = n
        self.allocs.append((p, n))
        return p

    def free(self, p):
        assert p in self.live, "free of a pointer the allocator did not hand out"
        del self.live[p]
        self.frees.append(p)


@pytest.fixture
def restore_allocator(lib):
    import paper_1812_01502_amd as P
    saved = dict(P._allocator)
    yield P
    P.set_allocator("hip")
    P._allocator.clear()
    P._allocator.update(saved)


def test_set_allocator_argument_checks(lib):
    from paper_1812_01502_amd import _lib as L
    f = L.FREE_FN(lambda p, c: None)
    a = L.ALLOC_FN(lambda n, c: None)
    assert lib.pf_set_allocator(a, L.FREE_FN(), None) == -1       # exactly one NULL
    assert lib.pf_set_allocator(L.ALLOC_FN(), f, None) == -1
    assert lib.pf_set_allocator(L.ALLOC_FN(), L.FREE_FN(), None) == 0


def _batch_args(n_filters=3):
    from paper_1812_01502_amd import _lib as L
    m, keep = _model_lg(2)
    ms = (L.PfModel * n_filters)(*([m] * n_filters))
    cs = (L.PfConfig * n_filters)()
    for i in range(n_filters):
        cs[i] = _cfg(n=4096, radix=4)
    return ms, cs, keep


def test_batch_buffers_come_from_the_installed_allocator(lib, restore_allocator):
    """Every device buffer of a batch comes from the installed callbacks, and
    a create that fails afterwards (here: no GPU, so the first upload fails)
    hands every one of them back through the free callback."""
    P = restore_allocator
    ca = _CountingAllocator()
    P.set_allocator("custom", alloc=ca.alloc, free=ca.free)
    ms, cs, keep = _batch_args()
    h = ctypes.c_void_p()
    st = lib.pf_batch_create(ms, cs, 3, None, ctypes.byref(h))
    assert st != 0 and h.value is None
    assert len(ca.allocs) >= 10                     # the pools and tables of the batch
    assert sorted(ca.frees) == sorted(p for p, _ in ca.allocs)
    assert not ca.live


def test_handle_buffers_come_from_the_installed_allocator(lib, restore_allocator):
    P = restore_allocator
    ca = _CountingAllocator()
    P.set_allocator("custom", alloc=ca.alloc, free=ca.free)
    m, keep = _model_lg(2)
    c = _cfg()
    h = ctypes.c_void_p()
    st = lib.pf_create(ctypes.byref(m), ctypes.byref(c), None, ctypes.byref(h))
    assert st != 0 and h.value is None
    assert len(ca.allocs) >= 1
    assert sorted(ca.frees) == sorted(p for p, _ in ca.allocs) and not ca.live


def test_allocator_failures_are_reported(lib, restore_allocator):
    """A NULL from the allocator is PF_E_OOM; a pointer that is not
    256-byte aligned is PF_E_INVALID and goes back to the allocator."""
    P = restore_allocator
    ms, cs, keep = _batch_args()
    h = ctypes.c_void_p()
    ca = _CountingAllocator(fail_after=4)
    P.set_allocator("custom", alloc=ca.alloc, free=ca.free)
    assert lib.pf_batch_create(ms, cs, 3, None, ctypes.byref(h)) == -3
    assert len(ca.allocs) == 4 and not ca.live
    cm = _CountingAllocator(misalign=True)
    P.set_allocator("custom", alloc=cm.alloc, free=cm.free)
    assert lib.pf_batch_create(ms, cs, 3, None, ctypes.byref(h)) == -1
    assert b"aligned" in lib.pf_batch_last_error(None)
    assert len(cm.allocs) == 1 and not cm.live
    m, keep2 = _model_lg(2)
    c = _cfg()
    assert lib.pf_create(ctypes.byref(m), ctypes.byref(c), None, ctypes.byref(h)) == -1
    assert b"aligned" in lib.pf_last_error(None)
    assert not cm.live
