"""Numeric failure detection on the device.

The reduction of every step checks the step's partial sums. A non-finite
observation delivered in device memory (never checked on the host) or
weights with no positive entry make the step a numeric failure: its record
is invalid, it adds nothing to the log-normaliser, and a sticky per-filter
flag keeps every later record invalid until the filter is re-initialised or
given a new state. In a batch only the failing filter is affected: the
others compute exactly what they compute without it. The kernels stay in
bounds on such inputs (every search index is clamped by construction), so
these runs end normally.
"""
import numpy as np
import pytest

import workloads as W
from tests.gpu_util import log

pytestmark = pytest.mark.gpu


def _dev(a, dtype):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda").contiguous()


@pytest.mark.parametrize("radix", [16, 256, 1 << 14], ids=["wave-path", "block-path", "global"])
def test_single_filter_nan_observation_is_flagged(radix):
    import torch
    import paper_1812_01502_amd as P
    model = W.random_stable_lg(4, 7)
    N, T = 1 << 14, 6
    _, ys = W.simulate(model, T, seed=3)
    ys = ys.astype(np.float32)
    bad = ys.copy()
    bad[3, 1] = np.nan
    log(f"[case] NaN device observation at step 3, radix {radix}")
    f = P.Filter(model, N, radix, seed=5, history=T)
    f.run(_dev(bad, torch.float32).data_ptr(), T, model.d)
    with pytest.raises(P.PfError) as ei:
        f.estimate()
    assert ei.value.status == -5
    h = f.history(T, check=False)
    assert [r["valid"] for r in h] == [1, 1, 1, 0, 0, 0], [r["valid"] for r in h]
    assert all(np.isfinite(r["log_norm"]) for r in h)
    assert h[5]["log_norm"] == h[2]["log_norm"]       # nothing added after the failure
    with pytest.raises(P.PfError) as ei:
        f.step(ys[0])
    assert ei.value.status == -5
    # re-initialised, the filter runs as a fresh one
    f.reset()
    g = P.Filter(model, N, radix, seed=5, history=T)
    yd = _dev(ys, torch.float32)
    f.run(yd.data_ptr(), T, model.d)
    g.run(yd.data_ptr(), T, model.d)
    hf, hg = f.history(T), g.history(T)
    assert all(r["valid"] == 1 for r in hf)
    assert [r["log_norm"] for r in hf] == [r["log_norm"] for r in hg]
    f.close()
    g.close()


def test_single_filter_no_positive_weight_is_flagged():
    """An observation so far away that every weight underflows."""
    import torch
    import paper_1812_01502_amd as P
    model = W.random_stable_lg(4, 7)
    N, T = 1 << 14, 4
    ys = np.zeros((T, model.d), dtype=np.float32)
    ys[2, :] = 1e30
    log("[case] observation far outside the cloud at step 2")
    f = P.Filter(model, N, 64, seed=5, history=T)
    f.run(_dev(ys, torch.float32).data_ptr(), T, model.d)
    h = f.history(T, check=False)
    assert [r["valid"] for r in h] == [1, 1, 0, 0], [r["valid"] for r in h]
    f.close()


def test_batch_nan_in_one_filter_leaves_the_others_unaffected():
    import torch
    from paper_1812_01502_amd import BatchFilter
    spec = [(W.random_stable_lg(1, 4001), 2048, 8), (W.random_stable_lg(4, 4002), 4096, 64),
            (W.sv_model(), 4096, 32), (W.random_stable_lg(4, 4003), 2048, 4)]
    models = [m for m, _, _ in spec]
    T = 5
    Y = np.concatenate([W.simulate(m, T, seed=30 + i)[1].reshape(T, -1) for i, m in enumerate(models)],
                       axis=1).astype(np.float32)
    j = 1                                   # the failing filter
    off = sum(m.d for m in models[:j])
    Ybad = Y.copy()
    Ybad[2, off] = np.nan
    log("[case] batch: NaN observation of filter 1 at step 2")

    def run(Yin):
        b = BatchFilter(models, [n for _, n, _ in spec], [r for _, _, r in spec], [100 + i for i in range(4)])
        yd = _dev(Yin, torch.float32)
        valid = []
        for t in range(T):
            b.step(yd[t].data_ptr())
            valid.append([r["valid"] for r in b.estimates()])
        return b, valid

    ref, vref = run(Y)
    bad, vbad = run(Ybad)
    assert all(all(v == 1 for v in row) for row in vref)
    assert [row[j] for row in vbad] == [1, 1, 0, 0, 0]
    for i in range(len(spec)):
        if i == j:
            continue
        assert all(row[i] == 1 for row in vbad)
        a, c = ref.get_state(i), bad.get_state(i)
        assert np.array_equal(a[0], c[0]) and np.array_equal(a[1], c[1]) and a[2:] == c[2:], i
    # a reset slot runs again
    bad.reset(j, seed=101, stream_id=j)
    bad.step(_dev(Y[0], torch.float32).data_ptr())
    assert bad.estimates()[j]["valid"] == 1
    ref.close()
    bad.close()
