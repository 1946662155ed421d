"""ESS-gated stages with a rotating start (Section 1.2, Section 6.4) on the
GPU against the FP64 oracle, through the C-ABI.

* teacher-forced steps for thresholds that run no stage, some stages and
  every stage; three consecutive steps, the later ones from the device's own
  state and rotation (so the rotation is compared as well);
* pf_run equals stepping and its graph replay, bit for bit;
* a checkpoint carries the rotation: the continuation is bit for bit;
* the benchmarked shape (LG-8, N = 2^20, radix 64).
"""
import numpy as np
import pytest

import workloads as W
from oracle.adaptive import AdaptiveOracle
from tests.gpu_util import compare_adaptive_step, log

pytestmark = pytest.mark.gpu

CASES = [
    # label, model, N, radix, theta, T0 (oracle steps before the comparison)
    ("ar1-r2-th0.5", "ar1", 4096, 2, 0.5, 3),
    ("dense4-r4-th0.7", "dense4", 1 << 13, 4, 0.7, 2),
    ("lg8-r64-th0.3", "lg8", 1 << 14, 64, 0.3, 2),
    ("sv-r32-th0.9", "sv", 1 << 15, 32, 0.9, 3),
    ("lg3-r8-th1", "lg3", 4096, 8, 1.0, 2),
    ("lg4-r16-tiny", "lg4", 1 << 13, 16, 1e-6, 2),
    ("ar1-small-r4-th0.7", "ar1", 1024, 4, 0.7, 0),   # 64-thread tiles
]


def _model(name):
    return {"ar1": W.ar1_model(), "dense4": W.dense_lg_model(4, 12), "lg8": W.random_stable_lg(8, 81),
            "sv": W.sv_model(), "lg3": W.random_stable_lg(3, 31), "lg4": W.random_stable_lg(4, 41)}[name]


@pytest.mark.parametrize("label,mname,N,r,theta,T0", CASES, ids=[c[0] for c in CASES])
def test_adaptive_steps_against_oracle(label, mname, N, r, theta, T0):
    from paper_1812_01502_amd import Filter
    model = _model(mname)
    orc = AdaptiveOracle(model, N, r, theta, seed=77, stream_id=3)
    _, ys = W.simulate(model, T0 + 3, seed=55)
    st, _ = orc.run(ys[:T0])
    st.next_stage = 0          # set_state restarts the rotation at stage 0
    log(f"[case] adaptive {label}: N={N} r={r} theta={theta} S={orc.S}")
    flt = Filter(model, N, r, seed=77, stream_id=3, ess_threshold=theta)
    runs = []
    for j in range(3):
        st, info = compare_adaptive_step(flt, orc, st, ys[T0 + j], label=f"{label}/{j}", upload=(j == 0))
        runs.append(info["stages"])
    log(f"   ok stages per step {runs}")
    if theta >= 1.0:
        assert runs == [orc.S] * 3
    if theta < 1e-3:
        assert runs == [0, 0, 0]
    flt.close()


def test_adaptive_run_graph_steps_and_checkpoint():
    import torch
    from paper_1812_01502_amd import Filter
    model = W.random_stable_lg(4, 44)
    N, r, T = 1 << 14, 8, 12
    _, ys = W.simulate(model, T, seed=3)
    yd = torch.tensor(ys, dtype=torch.float32, device="cuda").contiguous()
    log("[case] adaptive pf_run vs steps vs graph vs checkpoint")
    a = Filter(model, N, r, seed=5, ess_threshold=0.6)
    for y in ys:
        a.step(y)
    b = Filter(model, N, r, seed=5, ess_threshold=0.6)
    b.run(yd.data_ptr(), T, model.d)
    s = torch.cuda.Stream()
    c = Filter(model, N, r, seed=5, ess_threshold=0.6, stream=s.cuda_stream)
    with torch.cuda.stream(s):
        c.run(yd.data_ptr(), T, model.d, use_graph=True)
    c.sync()
    d = Filter(model, N, r, seed=5, ess_threshold=0.6)
    d.run(yd.data_ptr(), 5, model.d)
    blob = d.save()
    e = Filter(model, N, r, seed=5, ess_threshold=0.6)
    e.load(blob)
    e.run(yd[5:].data_ptr(), T - 5, model.d)
    sa, sb, sc, se = a.get_state(), b.get_state(), c.get_state(), e.get_state()
    assert np.array_equal(sb[0], sc[0]) and np.array_equal(sb[1], sc[1]) and sb[2:] == sc[2:]
    assert np.array_equal(sa[0], sb[0]) and np.array_equal(sa[1], sb[1]) and sa[2] == sb[2]
    assert np.array_equal(se[0], sb[0]) and np.array_equal(se[1], sb[1]) and se[2:] == sb[2:]
    log(f"   ok last record: stages {b.estimate()['stage']}")
    for f in (a, b, c, d, e):
        f.close()


def test_adaptive_full_size_lg8():
    from oracle.adaptive import AdaptiveState
    from paper_1812_01502_amd import Filter
    model = W.config("c2")["model"]
    N, r = 1 << 20, 64
    orc = AdaptiveOracle(model, N, r, 0.5, seed=21, stream_id=1)
    _, ys = W.simulate(model, 2, seed=4)
    st = orc.init()
    log(f"[case] adaptive full size N={N} r={r}")
    flt = Filter(model, N, r, seed=21, stream_id=1, ess_threshold=0.5)
    st, info = compare_adaptive_step(flt, orc, st, ys[0], label="lg8-2^20")
    log(f"   ok stages={info['stages']} sure={info['sure']:.4f} max_dx={info['max_dx']:.2e}")
    flt.close()
