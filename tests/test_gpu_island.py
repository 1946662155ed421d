"""The island filter (AIRPF, Algorithms 4-7) on the GPU against the FP64
oracle, through the C-ABI.

* teacher-forced steps: device and oracle start from the same state; the
  particle each destination copies, the states, the estimates and the
  log-normaliser agree (where every draw involved clears the margin); the
  output is unweighted; a second step continues from the device's own
  unweighted output (log-weights not read);
* island stages with every stage's uniforms in LDS, one stage's at a time,
  in two launches (more than 1024 islands in LDS: the first ten stages in
  blocks of 1024 islands, then the rest; 2048 and 4096 islands), and with
  the stage arrays in global memory (2^15 and 2^17 islands);
* islands from 2 particles (32768 islands, whose stage arrays live in
  global memory) to 4096 (the block path; islands of 1024 to 4096 whose
  plane spans 8 KB stage each source island in LDS for the mutation, one to
  four pairs per thread), FP64/FP32/BF16 storage,
  multinomial and systematic within-island draws, Algorithms 6 and 7;
* pf_run equals stepping, and its graph replay equals both, bit for bit;
* a checkpoint taken between steps continues bit for bit.
"""
import numpy as np
import pytest

import workloads as W
from oracle import IslandOracle
from tests.gpu_util import compare_island_step, device_x, log

pytestmark = pytest.mark.gpu


def _model(name):
    return {"ar1": W.ar1_model(), "lg8": W.random_stable_lg(8, 81), "dense4": W.dense_lg_model(4, 12),
            "sv": W.sv_model(), "lg3": W.random_stable_lg(3, 31), "lg16": W.random_stable_lg(16, 61),
            "lg4": W.random_stable_lg(4, 41)}[name]


CASES = [
    # label, model, N, M, dtype, resampler, no_swap
    ("ar1-f64-M64", "ar1", 4096, 64, "f64", "multinomial", True),
    ("lg8-f32-M256", "lg8", 1 << 14, 256, "f32", "multinomial", True),
    ("dense4-f32-M16-alg6", "dense4", 1 << 13, 16, "f32", "multinomial", False),
    ("sv-f32-M1024-sys", "sv", 1 << 15, 1024, "f32", "systematic", True),
    ("lg3-bf16-M32", "lg3", 4096, 32, "bf16", "multinomial", True),
    ("lg16-f32-M512", "lg16", 1 << 13, 512, "f32", "multinomial", True),
    ("ar1-f32-M2-many", "ar1", 1 << 16, 2, "f32", "multinomial", True),
    ("lg4-f32-M2048-two", "lg4", 4096, 2048, "f32", "multinomial", True),
    ("lg8-f32-M2048-one-group-tiles", "lg8", 8192, 2048, "f32", "multinomial", True),
    ("sv-f32-M4096", "sv", 1 << 14, 4096, "f32", "multinomial", True),
    ("ar1-f32-M8-m4096", "ar1", 1 << 15, 8, "f32", "multinomial", True),
    ("ar1-f32-M2-m131072", "ar1", 1 << 18, 2, "f32", "multinomial", True),
    ("sv-f32-M16-m2048", "sv", 1 << 15, 16, "f32", "multinomial", True),
    ("ar1-f64-M4-m4096-alg6-sys", "ar1", 1 << 14, 4, "f64", "systematic", False),
    ("lg4-f64-M1024", "lg4", 8192, 1024, "f64", "multinomial", False),
]


@pytest.mark.parametrize("label,mname,N,M,dtype,resampler,no_swap", CASES, ids=[c[0] for c in CASES])
def test_island_step_against_oracle(label, mname, N, M, dtype, resampler, no_swap):
    from paper_1812_01502_amd import Filter
    model = _model(mname)
    seed, sid = 400 + N % 97, 7
    orc = IslandOracle(model, N, M, resampler, seed=seed, stream_id=sid, no_swap=no_swap)
    T0 = 3
    _, ys = W.simulate(model, T0 + 2, seed=90)
    st, _ = orc.run(ys[:T0])
    log(f"[case] island {label}: N={N} M={M} m={N // M} dtype={dtype} t={T0}")
    flt = Filter(model, N, 2, resampler=resampler, dtype=dtype, seed=seed, stream_id=sid,
                 keep_ancestors=True, island=M, island_swap=not no_swap)
    # weighted start (the log-weights are read), then a step from the
    # device's own unweighted output
    rng = np.random.Generator(np.random.PCG64(N + M))
    lw0 = rng.standard_normal(N) * 0.2
    lw0 -= lw0.max()
    r1 = compare_island_step(flt, orc, st.x, lw0, T0, ys[T0], log_norm=st.log_norm, label=label)
    x1, w1, t1, ln1 = flt.get_state()
    r2 = compare_island_step(flt, orc, device_x(flt, x1), np.zeros(N), t1, ys[T0 + 1], log_norm=ln1,
                             label=label + "/own", upload=False)
    log(f"   ok sure={r1['sure']:.4f}/{r2['sure']:.4f} flips={r1['flips']}/{r2['flips']} "
        f"max_dx={r1['max_dx']:.2e}/{r2['max_dx']:.2e}")
    flt.close()


def test_island_run_graph_and_steps_agree():
    import torch
    from paper_1812_01502_amd import Filter
    model = W.random_stable_lg(4, 44)
    N, M, T = 1 << 14, 128, 9
    _, ys = W.simulate(model, T, seed=3)
    yd = torch.tensor(ys, dtype=torch.float32, device="cuda").contiguous()
    log("[case] island pf_run vs steps vs graph")
    a = Filter(model, N, 2, seed=5, island=M)
    for y in ys:
        a.step(y)
    b = Filter(model, N, 2, seed=5, island=M)
    b.run(yd.data_ptr(), T, model.d)
    s = torch.cuda.Stream()
    c = Filter(model, N, 2, seed=5, island=M, stream=s.cuda_stream)
    with torch.cuda.stream(s):
        c.run(yd.data_ptr(), T, model.d, use_graph=True)
    c.sync()
    sa, sb, sc = a.get_state(), b.get_state(), c.get_state()
    ea, eb, ec = a.estimate(), b.estimate(), c.estimate()
    # pf_step passes y by value in FP64 -> rounded to FP32 like the device copy
    assert np.array_equal(sb[0], sc[0]) and sb[2:] == sc[2:]
    assert np.array_equal(sa[0], sb[0]) and sa[2] == sb[2]
    assert abs(sa[3] - sb[3]) <= 1e-9 * max(1.0, abs(sa[3]))
    assert np.array_equal(eb["mean"], ec["mean"]) and ea["stage"] == eb["stage"] == 7
    for f in (a, b, c):
        f.close()


def test_island_checkpoint_continues_bit_exact():
    import torch
    from paper_1812_01502_amd import Filter
    model = W.sv_model()
    N, M = 1 << 15, 512
    _, ys = W.simulate(model, 8, seed=6)
    yd = torch.tensor(ys, dtype=torch.float32, device="cuda").contiguous()
    log("[case] island checkpoint")
    a = Filter(model, N, 2, seed=9, island=M)
    a.run(yd.data_ptr(), 4, 1)
    blob = a.save()
    a.run(yd[4:].data_ptr(), 4, 1)
    b = Filter(model, N, 2, seed=9, island=M)
    b.load(blob)
    b.run(yd[4:].data_ptr(), 4, 1)
    sa, sb = a.get_state(), b.get_state()
    assert np.array_equal(sa[0], sb[0]) and sa[2:] == sb[2:]
    a.close()
    b.close()


def test_island_full_size_lg8_step():
    """The benchmarked shape: LG-8, N = 2^20 in 1024 islands of 1024, one
    teacher-forced step (the oracle's full FP64 step)."""
    from paper_1812_01502_amd import Filter
    model = W.config("c2")["model"]
    N, M = 1 << 20, 1024
    orc = IslandOracle(model, N, M, seed=21, stream_id=1)
    _, ys = W.simulate(model, 2, seed=4)
    st = orc.init()
    log(f"[case] island full size N={N} M={M}")
    flt = Filter(model, N, 2, seed=21, stream_id=1, keep_ancestors=True, island=M)
    r = compare_island_step(flt, orc, st.x, np.zeros(N), 0, ys[0], label="lg8-2^20")
    log(f"   ok sure={r['sure']:.4f} flips={r['flips']} max_dx={r['max_dx']:.2e}")
    flt.close()
