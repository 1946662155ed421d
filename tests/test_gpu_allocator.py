"""Device memory from torch's caching allocator (pf_set_allocator): the
binding installs it by default; a filter's buffers then show up in torch's
accounting while it lives and go back when it is closed; results are the same
bit for bit as with the library's own hipMalloc."""
import numpy as np
import pytest

import workloads as W
from tests.gpu_util import log

pytestmark = pytest.mark.gpu


def _run(P, model, ys, N, radix):
    import torch
    f = P.Filter(model, N, radix, seed=5, history=8)
    yd = torch.tensor(ys, dtype=torch.float32, device="cuda").contiguous()
    f.run(yd.data_ptr(), len(ys), model.d)
    x, w, t, ln = f.get_state()
    recs = f.history(len(ys))
    info = f.info()
    return f, x, w, ln, recs, info


def test_torch_allocator_holds_filter_memory_and_results_match():
    import torch
    import paper_1812_01502_amd as P
    model = W.config("c2")["model"]
    _, ys = W.simulate(model, 8, seed=2)
    N = 1 << 16
    P.set_allocator("torch")
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    f, x1, w1, ln1, r1, info = _run(P, model, ys, N, 64)
    held = torch.cuda.memory_allocated() - base
    log(f"[allocator] torch holds {held} bytes for a filter of {info['device_bytes']} bytes")
    assert held >= info["device_bytes"]
    f.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == base
    P.set_allocator("hip")
    try:
        g, x2, w2, ln2, r2, _ = _run(P, model, ys, N, 64)
        assert torch.cuda.memory_allocated() == base      # hipMalloc is outside torch's pool
        g.close()
    finally:
        P.set_allocator("torch")
    assert np.array_equal(x1, x2) and np.array_equal(w1, w2) and ln1 == ln2
    for a, b in zip(r1, r2):
        assert np.array_equal(a["mean"], b["mean"]) and a["ess"] == b["ess"]


def test_torch_allocator_batch():
    import torch
    import paper_1812_01502_amd as P
    P.set_allocator("torch")
    models = [W.random_stable_lg(d, 40 + d) for d in (1, 4)]
    y = torch.zeros(sum(m.d for m in models), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    b = P.BatchFilter(models, [4096, 8192], [8, 16], [1, 2])
    assert torch.cuda.memory_allocated() > base
    b.step(y.data_ptr())
    recs = b.estimates()
    assert all(r["valid"] for r in recs)
    b.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == base
