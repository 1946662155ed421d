"""Butterfly-interaction bootstrap particle filter on MI355X (gfx950).

Python binding over the C-ABI of ``include/pf.h`` (``libpf.so``, hand-written
HIP kernels). This module only marshals arguments: model parameters are
copied into the library, observations go by value (``step``) or as a device
array (``run``), and results come back as NumPy arrays.

Method: Heine, Whiteley, Cemgil, "Parallelising Particle Filters with
Butterfly Interactions" (arXiv 1812.01502): Algorithm 1 with one stage of
augmented resampling (Algorithm 3, eq. ``A matrices`` generalised to radix
r) per time step, the stage rotating with the step.
"""
from __future__ import annotations

import atexit
import ctypes
import weakref

import numpy as np

from . import _lib as L

__all__ = ["Filter", "BatchFilter", "PfError", "load_library", "set_allocator", "DTYPES", "RESAMPLERS"]

DTYPES = {"f32": L.PF_DTYPE_F32, "bf16": L.PF_DTYPE_BF16, "f64": L.PF_DTYPE_F64}
RESAMPLERS = {"multinomial": L.PF_RESAMPLE_MULTINOMIAL, "systematic": L.PF_RESAMPLE_SYSTEMATIC}


# NumPy view of pf_estimate_t
ESTIMATE_DTYPE = np.dtype([("t", np.uint32), ("stage", np.uint32), ("radix", np.uint32),
                           ("valid", np.uint32), ("log_normaliser", np.float64), ("ess", np.float64),
                           ("max_log_weight", np.float64), ("next_offset", np.float64),
                           ("mean", np.float64, (L.PF_MAX_DIM,)), ("var", np.float64, (L.PF_MAX_DIM,))])
assert ESTIMATE_DTYPE.itemsize == ctypes.sizeof(L.PfEstimate)


class PfError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{L.STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def load_library():
    return L.load()


# The device allocator of filters created from now on (pf_set_allocator):
# None until the first filter is created or set_allocator is called.
_allocator = {"kind": None, "fns": None}


def set_allocator(kind: str = "torch", alloc=None, free=None):
    """Choose where the device buffers of filters and batches created from now
    on come from: ``"torch"`` (``torch.cuda``'s caching allocator, on the
    current device and stream), ``"hip"`` (``hipMalloc``/``hipFree`` inside
    the library) or ``"custom"`` with Python callables ``alloc(nbytes) ->
    int device pointer (or None)`` and ``free(ptr)``. Existing filters keep
    the allocator they were created with. The callbacks stay referenced here,
    so they outlive every filter that uses them."""
    lib = L.load()
    if kind == "hip":
        st = lib.pf_set_allocator(L.ALLOC_FN(), L.FREE_FN(), None)
        fns = None
    else:
        if kind == "torch":
            import torch

            def alloc(nbytes):
                return torch.cuda.caching_allocator_alloc(int(nbytes))

            def free(ptr):
                torch.cuda.caching_allocator_delete(int(ptr))
        elif kind != "custom" or alloc is None or free is None:
            raise ValueError("set_allocator: kind is 'torch', 'hip' or 'custom' (with alloc and free)")
        user_alloc, user_free = alloc, free

        def c_alloc(nbytes, _ctx):
            try:
                p = user_alloc(int(nbytes))
            except Exception:   # out of memory: the create reports PF_E_OOM
                return None
            return int(p) if p else None

        def c_free(ptr, _ctx):
            try:
                user_free(int(ptr))
            except Exception as e:  # cannot propagate through the C caller
                import sys
                print(f"paper_1812_01502_amd: allocator free failed: {e}", file=sys.stderr)

        fns = (L.ALLOC_FN(c_alloc), L.FREE_FN(c_free))
        st = lib.pf_set_allocator(fns[0], fns[1], None)
    if st != L.PF_OK:
        raise PfError(st, "pf_set_allocator")
    if _allocator["fns"] is not None:
        # filters created with the previous callbacks may still hold them
        _allocator.setdefault("retired", []).append(_allocator["fns"])
    _allocator.update(kind=kind, fns=fns)


# Live filters and batches: closed at interpreter exit, before torch (whose
# allocator may own their memory) is torn down.
_live = weakref.WeakSet()


def _close_live():
    for obj in list(_live):
        try:
            obj.close()
        except Exception:
            pass


def _default_allocator():
    """First filter of the process: device memory from torch's caching
    allocator when torch has a GPU, else from hipMalloc."""
    if _allocator["kind"] is not None:
        return
    atexit.register(_close_live)   # after torch's import: runs before torch's own exit hooks
    try:
        import torch
        use_torch = torch.cuda.is_available()
    except ImportError:
        use_torch = False
    set_allocator("torch" if use_torch else "hip")


def _dptr(a):
    return a.ctypes.data_as(L.DPTR)


class _VacantModel:
    """Stand-in model of a vacant batch slot (never read by the library)."""
    kind, d, phi, sigma, beta = "sv", 1, 0.5, 1.0, 1.0


_VACANT_MODEL = _VacantModel()


def _pf_model(model, keep: list) -> L.PfModel:
    """``pf_model`` from a model object (arrays kept alive in ``keep``)."""
    m = L.PfModel()
    m.d = int(model.d)
    if model.kind == "lg":
        m.kind = L.PF_MODEL_LG
        for nm in ("A", "Q_chol", "H", "R_chol", "P0_chol"):
            arr = np.ascontiguousarray(np.asarray(getattr(model, nm), dtype=np.float64))
            keep.append(arr)
            setattr(m, nm, _dptr(arr))
        m0 = np.ascontiguousarray(np.asarray(model.m0, dtype=np.float64))
        keep.append(m0)
        m.m0 = _dptr(m0)
    elif model.kind == "sv":
        m.kind = L.PF_MODEL_SV
        m.phi, m.sigma, m.beta = float(model.phi), float(model.sigma), float(model.beta)
    else:
        raise ValueError(f"unknown model kind {model.kind!r}")
    return m


class Filter:
    """One particle filter on the GPU.

    ``model`` needs the attributes ``kind`` ("lg" or "sv"), ``d`` and, for LG,
    ``A, Q_chol, H, R_chol, m0, P0_chol`` (FP64 arrays); for SV ``phi, sigma,
    beta``. ``radix >= n`` selects the global bootstrap filter. ``island = M``
    selects the island filter (AIRPF) with islands of M particles (radix is
    then ignored); ``island_swap`` runs the plain island stages of Algorithm 6
    instead of the no-swap rule of Algorithm 7. ``ess_threshold`` in (0, 1]
    gates the butterfly stages by the effective sample size (Section 1.2)
    with a rotating start (Section 6.4).
    """

    def __init__(self, model, n: int, radix: int, resampler: str = "multinomial",
                 dtype: str = "f32", seed: int = 0, stream_id: int = 0, history: int = 1,
                 keep_ancestors: bool = False, stream: int | None = None, full_cycle: bool = False,
                 island: int = 0, island_swap: bool = False, ess_threshold: float = 0.0):
        self._lib = L.load()
        _default_allocator()
        self.d = int(model.d)
        self.n = int(n)
        self.dtype = dtype
        self._keep = []
        m = _pf_model(model, self._keep)
        c = L.PfConfig()
        c.n_particles = self.n
        c.radix = int(radix)
        c.resampler = RESAMPLERS[resampler]
        c.state_dtype = DTYPES[dtype]
        c.seed = int(seed)
        c.stream_id = int(stream_id)
        c.history = int(history)
        c.keep_ancestors = 1 if keep_ancestors else 0
        c.full_cycle = 1 if full_cycle else 0
        c.island = int(island)
        c.island_swap = 1 if island_swap else 0
        c.ess_threshold = float(ess_threshold)
        h = ctypes.c_void_p()
        st = self._lib.pf_create(ctypes.byref(m), ctypes.byref(c),
                                 ctypes.c_void_p(stream) if stream else None, ctypes.byref(h))
        if st != L.PF_OK:
            raise PfError(st, self._lib.pf_last_error(None).decode())
        self._h = h
        _live.add(self)
        self._x_dtype = {"f32": np.float32, "bf16": np.uint16, "f64": np.float64}[dtype]
        self._w_dtype = np.float64 if dtype == "f64" else np.float32

    # -- plumbing ----------------------------------------------------------
    def _check(self, st, allow_numeric: bool = False):
        if st != L.PF_OK and not (allow_numeric and st == L.PF_E_NUMERIC):
            raise PfError(st, self._lib.pf_last_error(self._h).decode())
        return st

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            self._lib.pf_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- the filter --------------------------------------------------------
    def step(self, y):
        y = np.ascontiguousarray(np.asarray(y, dtype=np.float64).reshape(self.d))
        self._check(self._lib.pf_step(self._h, _dptr(y)))

    def run(self, y_dev_ptr: int, n_steps: int, stride: int | None = None, use_graph: bool = False):
        """``n_steps`` steps reading observations from a device array (pointer
        ``y_dev_ptr``, compute dtype, ``stride`` elements per step)."""
        self._check(self._lib.pf_run(self._h, ctypes.c_void_p(int(y_dev_ptr)), int(n_steps),
                                     int(stride if stride is not None else self.d),
                                     1 if use_graph else 0))

    def sync(self):
        self._check(self._lib.pf_sync(self._h))

    def reset(self):
        self._check(self._lib.pf_reset(self._h))

    @staticmethod
    def _rec(e: L.PfEstimate, d: int) -> dict:
        return dict(t=e.t, stage=e.stage, radix=e.radix, valid=e.valid,
                    log_norm=e.log_normaliser, ess=e.ess, max_ell=e.max_log_weight,
                    offset=e.next_offset, mean=np.array(e.mean[:d]), var=np.array(e.var[:d]))

    def estimate(self, check: bool = True) -> dict:
        """Record of the last step. A numeric failure (the record's ``valid``
        is 0) raises ``PfError`` unless ``check`` is False."""
        e = L.PfEstimate()
        self._check(self._lib.pf_estimate(self._h, ctypes.byref(e)), allow_numeric=not check)
        return self._rec(e, self.d)

    def history(self, n_max: int, check: bool = True) -> list:
        """The last ``n_max`` records, oldest first (as ``estimate``)."""
        buf = (L.PfEstimate * n_max)()
        n = ctypes.c_uint32()
        self._check(self._lib.pf_history(self._h, buf, n_max, ctypes.byref(n)), allow_numeric=not check)
        return [self._rec(buf[i], self.d) for i in range(n.value)]

    def get_state(self):
        """``(x (d, N) in the storage dtype, logW (N,), t, log_norm)``."""
        x = np.empty((self.d, self.n), dtype=self._x_dtype)
        w = np.empty(self.n, dtype=self._w_dtype)
        t = ctypes.c_uint32()
        ln = ctypes.c_double()
        self._check(self._lib.pf_get_state(self._h, x.ctypes.data_as(ctypes.c_void_p),
                                           w.ctypes.data_as(ctypes.c_void_p), ctypes.byref(t),
                                           ctypes.byref(ln)))
        return x, w, t.value, ln.value

    def set_state(self, x, logw=None, t: int = 0, log_norm: float = 0.0):
        x = np.ascontiguousarray(np.asarray(x, dtype=self._x_dtype).reshape(self.d, self.n))
        wp = None
        if logw is not None:
            w = np.ascontiguousarray(np.asarray(logw, dtype=self._w_dtype).reshape(self.n))
            wp = w.ctypes.data_as(ctypes.c_void_p)
        self._check(self._lib.pf_set_state(self._h, x.ctypes.data_as(ctypes.c_void_p), wp,
                                           int(t), float(log_norm)))

    def save(self) -> bytes:
        """Checkpoint of the complete filter state (``pf_save``)."""
        n = ctypes.c_uint64(0)
        self._check(self._lib.pf_save(self._h, None, 0, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        self._check(self._lib.pf_save(self._h, buf, n.value, ctypes.byref(n)))
        return buf.raw

    def load(self, blob: bytes):
        """Restore a checkpoint made by ``save`` (``pf_load``)."""
        self._check(self._lib.pf_load(self._h, blob, len(blob)))

    def ancestors(self) -> np.ndarray:
        a = np.empty(self.n, dtype=np.uint32)
        self._check(self._lib.pf_get_ancestors(self._h, a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))))
        return a

    def info(self) -> dict:
        i = L.PfInfo()
        self._check(self._lib.pf_info(self._h, ctypes.byref(i)))
        S = i.n_stages
        return dict(n=i.n_particles, d=i.d, stages=list(i.radices[:S]),
                    tile_elems=list(i.tile_elems[:S]), global_path=bool(i.global_path),
                    device_bytes=i.device_bytes, t=i.t)


def bf16_to_f32(u16: np.ndarray) -> np.ndarray:
    """BF16 bit patterns (uint16) to FP32."""
    return (np.asarray(u16, dtype=np.uint32) << 16).view(np.float32)


def f32_to_bf16(x: np.ndarray) -> np.ndarray:
    """FP32 to BF16 bit patterns, round to nearest even (finite inputs)."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = u + 0x7FFF + ((u >> 16) & 1)
    return (u >> 16).astype(np.uint16)


class BatchFilter:
    """Many independent filters advanced together (``pf_batch_*``).

    ``models``, ``ns``, ``radices`` (0 = autotune), ``seeds`` and
    ``stream_ids`` are per-filter sequences. Observations of one step are
    packed in filter order (filter i's ``d_i`` values at ``y_offsets[i]``).
    """

    def __init__(self, models, ns, radices, seeds, stream_ids=None, resampler: str = "multinomial",
                 stream: int | None = None):
        self._lib = L.load()
        _default_allocator()
        n = len(models)
        self.n = n
        self.resampler = resampler
        # n = 0 (model None allowed): a vacant slot
        self.ds = [int(m.d) if int(N) > 0 else 0 for m, N in zip(models, ns)]
        self.ns = [int(v) for v in ns]
        self._layout()
        keep = []
        M = (L.PfModel * n)()
        C = (L.PfConfig * n)()
        sids = stream_ids if stream_ids is not None else range(n)
        for i, (m, N, r, sd, sid) in enumerate(zip(models, ns, radices, seeds, sids)):
            M[i] = _pf_model(m if m is not None else _VACANT_MODEL, keep)
            C[i] = self._config(N, r, sd, sid)
        h = ctypes.c_void_p()
        st = self._lib.pf_batch_create(M, C, n, ctypes.c_void_p(stream) if stream else None,
                                       ctypes.byref(h))
        if st != L.PF_OK:
            raise PfError(st, self._lib.pf_batch_last_error(None).decode())
        self._h = h
        _live.add(self)

    def _config(self, N, r, seed, sid):
        c = L.PfConfig()
        c.n_particles = int(N)
        c.radix = int(r)
        c.resampler = RESAMPLERS[self.resampler]
        c.state_dtype = L.PF_DTYPE_F32
        c.seed = int(seed)
        c.stream_id = int(sid)
        c.history = 1
        return c

    def _layout(self):
        """Packed observation offsets of the current slot dimensions."""
        self.y_offsets = np.concatenate([[0], np.cumsum(self.ds)[:-1]]).astype(np.int64)
        self.y_len = int(sum(self.ds))

    def _check(self, st):
        if st != L.PF_OK:
            raise PfError(st, self._lib.pf_batch_last_error(self._h).decode())

    def rebind(self, bindings):
        """Give slots to other filters in one call (``pf_batch_rebind``):
        ``bindings`` is a sequence of ``(slot, model, n, radix, seed,
        stream_id)``; ``n = 0`` leaves the slot vacant. Synchronises, and
        changes the packed observation layout (``y_offsets``, ``y_len``).
        Raises ``PfError`` (PF_E_OOM) if a filter did not fit: that slot is
        then vacant, the others are bound."""
        bindings = list(bindings)
        if not bindings:
            return
        k = len(bindings)
        keep = []
        S = (ctypes.c_uint32 * k)()
        M = (L.PfModel * k)()
        C = (L.PfConfig * k)()
        for i, (f, model, n, radix, seed, sid) in enumerate(bindings):
            S[i] = int(f)
            M[i] = _pf_model(model if model is not None and n > 0 else _VACANT_MODEL, keep)
            C[i] = self._config(n, radix, seed, sid)
        st = self._lib.pf_batch_rebind(self._h, k, S, M, C)
        if st not in (L.PF_OK, L.PF_E_OOM):
            self._check(st)
        for f, model, n, _, _, _ in bindings:
            info = self.info(f)
            self.ns[f] = int(info["n"])
            self.ds[f] = int(info["d"]) if info["n"] > 0 else 0
        self._layout()
        self._check(st)

    def vacate(self, slots):
        """Release the particle memory of ``slots`` (vacant slots never step)."""
        self.rebind([(f, None, 0, 0, 0, 0) for f in slots])

    def estimates_async(self, out: np.ndarray):
        """Enqueue a copy of every record into ``out`` (``ESTIMATE_DTYPE``, n
        records, page-locked memory) on the batch's stream; read it only
        after the stream, or an event recorded after this call, completes."""
        assert out.dtype == ESTIMATE_DTYPE and out.size >= self.n and out.flags.c_contiguous
        self._check(self._lib.pf_batch_estimates_async(self._h, ctypes.c_void_p(out.ctypes.data)))

    def close(self):
        if getattr(self, "_h", None):
            self._lib.pf_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, y_dev_ptr: int, active_dev_ptr: int | None = None):
        self._check(self._lib.pf_batch_step(self._h, ctypes.c_void_p(int(y_dev_ptr)),
                                            ctypes.c_void_p(int(active_dev_ptr)) if active_dev_ptr else None))

    def run(self, y_dev_ptr: int, n_steps: int, stride: int | None = None,
            active_dev_ptr: int | None = None, use_graph: bool = False):
        self._check(self._lib.pf_batch_run(
            self._h, ctypes.c_void_p(int(y_dev_ptr)), int(n_steps),
            int(stride if stride is not None else self.y_len),
            ctypes.c_void_p(int(active_dev_ptr)) if active_dev_ptr else None, 1 if use_graph else 0))

    def sync(self):
        self._check(self._lib.pf_batch_sync(self._h))

    def estimates(self) -> list:
        recs = (L.PfEstimate * self.n)()
        self._check(self._lib.pf_batch_estimates(self._h, recs))
        return [Filter._rec(recs[i], self.ds[i]) for i in range(self.n)]

    def estimates_array(self, out: np.ndarray | None = None) -> np.ndarray:
        """Records of every filter as a NumPy structured array (``ESTIMATE_DTYPE``)."""
        if out is None:
            out = np.empty(self.n, dtype=ESTIMATE_DTYPE)
        self._check(self._lib.pf_batch_estimates(self._h, out.ctypes.data_as(ctypes.POINTER(L.PfEstimate))))
        return out

    def info(self, f: int) -> dict:
        i = L.PfInfo()
        self._check(self._lib.pf_batch_filter_info(self._h, int(f), ctypes.byref(i)))
        return dict(n=i.n_particles, d=i.d, stages=list(i.radices[:i.n_stages]),
                    tile=i.tile_elems[0], t=i.t, device_bytes=i.device_bytes)

    def tuning(self) -> list:
        cnt = ctypes.c_uint32()
        self._check(self._lib.pf_batch_tuning(self._h, None, 0, ctypes.byref(cnt)))
        arr = (L.PfBatchTune * max(cnt.value, 1))()
        self._check(self._lib.pf_batch_tuning(self._h, arr, cnt.value, ctypes.byref(cnt)))
        return [dict(cls=a.class_index, dim=a.dim, model_kind=a.model_kind, ppt=a.pairs_per_thread,
                     radix=a.radix, chosen=bool(a.chosen), ms=a.ms_per_step) for a in arr[:cnt.value]]

    def get_state(self, f: int):
        d, N = self.ds[f], self.ns[f]
        x = np.empty((d, N), dtype=np.float32)
        w = np.empty(N, dtype=np.float32)
        t = ctypes.c_uint32()
        ln = ctypes.c_double()
        self._check(self._lib.pf_batch_get_state(self._h, int(f), x.ctypes.data_as(ctypes.c_void_p),
                                                 w.ctypes.data_as(ctypes.c_void_p), ctypes.byref(t),
                                                 ctypes.byref(ln)))
        return x, w, t.value, ln.value

    def set_state(self, f: int, x, logw=None, t: int = 0, log_norm: float = 0.0):
        d, N = self.ds[f], self.ns[f]
        x = np.ascontiguousarray(np.asarray(x, dtype=np.float32).reshape(d, N))
        wp = None
        if logw is not None:
            w = np.ascontiguousarray(np.asarray(logw, dtype=np.float32).reshape(N))
            wp = w.ctypes.data_as(ctypes.c_void_p)
        self._check(self._lib.pf_batch_set_state(self._h, int(f), x.ctypes.data_as(ctypes.c_void_p), wp,
                                                 int(t), float(log_norm)))

    def reset(self, f: int, seed: int, stream_id: int):
        self._check(self._lib.pf_batch_reset(self._h, int(f), int(seed), int(stream_id)))

