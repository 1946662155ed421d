"""pf_run_noalloc through the C-ABI: the allocation-free variant of pf_run
computes, on caller-owned buffers, the same states, log-weights and
estimate records as a handle (pf_create + pf_run + pf_history) of the same
configuration, bit for bit; it allocates nothing (no allocator callback and
no torch allocation during the calls); two calls in a row, the second on a
smaller filter, each match their handle; an unsupported size is refused with
a message."""
import ctypes

import numpy as np
import pytest

import workloads as W
from tests.gpu_util import log

pytestmark = pytest.mark.gpu


def _args(model, N, radix, dtype, seed, sid):
    import paper_1812_01502_amd as P
    from paper_1812_01502_amd import _lib as L
    keep = []
    m = P._pf_model(model, keep)
    c = L.PfConfig()
    c.n_particles = N
    c.radix = radix
    c.resampler = P.RESAMPLERS["multinomial"]
    c.state_dtype = P.DTYPES[dtype]
    c.seed = seed
    c.stream_id = sid
    c.history = 1
    return m, c, keep


def _one(model, N, radix, T, dtype, seed, sid, counter):
    """The handle's run and the allocation-free run from the same cloud."""
    import torch
    import paper_1812_01502_amd as P
    from paper_1812_01502_amd import _lib as L
    lib = L.load()
    cdt = torch.float64 if dtype == "f64" else torch.float32
    xdt = {"f32": torch.float32, "bf16": torch.int16, "f64": torch.float64}[dtype]
    _, ys = W.simulate(model, T, seed=seed)
    yd = torch.tensor(ys, dtype=cdt, device="cuda").contiguous()
    f = P.Filter(model, N, radix, dtype=dtype, seed=seed, stream_id=sid, history=T)
    x0, w0, t0, _ = f.get_state()
    assert t0 == 0 and np.all(w0 == 0)
    f.run(yd.data_ptr(), T, model.d)
    xh, wh, th, lnh = f.get_state()
    hist = f.history(T)
    f.close()
    x_dev = torch.from_numpy(x0.view(np.int16) if dtype == "bf16" else x0).to("cuda").contiguous()
    assert x_dev.dtype == xdt
    w_dev = torch.zeros(N, dtype=cdt, device="cuda")
    est = torch.zeros(T * ctypes.sizeof(L.PfEstimate), dtype=torch.uint8, device="cuda")
    m, c, keep = _args(model, N, radix, dtype, seed, sid)
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    before = (torch.cuda.memory_allocated(), counter[0])
    with torch.cuda.stream(s):
        st = lib.pf_run_noalloc(ctypes.byref(m), ctypes.byref(c), ctypes.c_void_p(x_dev.data_ptr()),
                                ctypes.c_void_p(w_dev.data_ptr()), ctypes.c_void_p(yd.data_ptr()), T, model.d, 0,
                                ctypes.c_void_p(est.data_ptr()), ctypes.c_void_p(s.cuda_stream))
    s.synchronize()
    assert st == 0, lib.pf_last_error(None)
    assert (torch.cuda.memory_allocated(), counter[0]) == before     # nothing allocated
    xn = x_dev.cpu().numpy()
    if dtype == "bf16":
        xn = xn.view(np.uint16)
    wn = w_dev.cpu().numpy()
    recs = np.frombuffer(est.cpu().numpy().tobytes(), dtype=P.ESTIMATE_DTYPE)
    assert np.array_equal(xn, xh), "states"
    # the handle reports log-weights relative to their maximum
    assert np.array_equal(wn - wn.max(), wh.astype(wn.dtype) - wh.max()) or np.allclose(wn - wn.max(), wh, atol=1e-6)
    for j, h in enumerate(hist):
        r = recs[j]
        assert r["valid"] == 1 and r["t"] == j and r["stage"] == h["stage"]
        assert np.array_equal(r["mean"][:model.d], h["mean"]) and np.array_equal(r["var"][:model.d], h["var"]), j
        assert r["ess"] == h["ess"] and r["log_normaliser"] == h["log_norm"], j
    return recs


def test_noalloc_matches_pf_run_twice_then_smaller():
    import paper_1812_01502_amd as P
    count = [0]

    def alloc(nbytes):
        import torch
        count[0] += 1
        return torch.cuda.caching_allocator_alloc(int(nbytes))

    def free(ptr):
        import torch
        torch.cuda.caching_allocator_delete(int(ptr))

    P.set_allocator("custom", alloc=alloc, free=free)
    try:
        log("[case] noalloc: SV N=2^18 radix 64, 9 steps (two cycles and one stage)")
        _one(W.sv_model(), 1 << 18, 64, 9, "f32", 41, 3, count)
        log("[case] noalloc: second call, smaller: 8-D LG N=2^14 radix 32, 7 steps")
        _one(W.config("c2")["model"], 1 << 14, 32, 7, "f32", 42, 4, count)
        log("[case] noalloc: BF16 states, block path: SV N=2^16 radix 256, 5 steps")
        _one(W.sv_model(), 1 << 16, 256, 5, "bf16", 43, 5, count)
    finally:
        P.set_allocator("torch")


def test_noalloc_refuses_what_it_cannot_hold():
    import paper_1812_01502_amd as P
    from paper_1812_01502_amd import _lib as L
    lib = L.load()
    model = W.random_stable_lg(16, 3)
    m, c, keep = _args(model, 1 << 26, 64, "f32", 1, 0)
    dummy = ctypes.c_void_p(16)    # never dereferenced: the size check fails first
    st = lib.pf_run_noalloc(ctypes.byref(m), ctypes.byref(c), dummy, dummy, dummy, 1, 16, 0, dummy, None)
    assert st == -2 and b"scratch" in lib.pf_last_error(None)
    m2, c2, keep2 = _args(W.sv_model(), 1 << 10, 1 << 10, "f32", 1, 0)
    st = lib.pf_run_noalloc(ctypes.byref(m2), ctypes.byref(c2), dummy, dummy, dummy, 1, 1, 0, dummy, None)
    assert st == -2 and b"global" in lib.pf_last_error(None)
