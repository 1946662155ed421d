"""GPU parity of the HIP path against the FP64 oracle (through the C-ABI).

Ancestors: identical wherever the oracle's draw margin exceeds 1e-5 of the
group total. Filter means: within 1e-4 max(|m|, sd). Log-weights, states,
variances, ESS and the log-normaliser within tolerances derived from the
arithmetic precision (tests/gpu_util.py).
"""
import numpy as np
import pytest

import workloads as W
from oracle import ButterflyOracle, kalman
from tests.gpu_util import compare_one_step, log, MARGIN_TOL

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_1812_01502_amd as P
    P.load_library()
    yield


def _filter(model, N, radix, resampler="multinomial", dtype="f32", seed=7, sid=0, history=4):
    from paper_1812_01502_amd import Filter
    return Filter(model, N, radix, resampler=resampler, dtype=dtype, seed=seed, stream_id=sid,
                  history=history, keep_ancestors=True)


MODELS = {
    "ar1": lambda: W.ar1_model(),
    "lg4dense": lambda: W.dense_lg_model(4, 12),
    "lg8": lambda: W.lg8_model(seed=2),
    "lg3stable": lambda: W.random_stable_lg(3, 11),
    "lg2stable": lambda: W.random_stable_lg(2, 13),
    "lg16stable": lambda: W.random_stable_lg(16, 17),
    "sv": lambda: W.sv_model(),
}


def _teacher_forced(model_name, N, radix, resampler, dtype, n_steps=None, seed=7, sid=0,
                    warm=0, obs_seed=5):
    """Run the oracle from its own init; at each of the steps start the
    device from the oracle's (rounded) state and compare one step."""
    model = MODELS[model_name]()
    orc = ButterflyOracle(model, N, radix, resampler, seed=seed, stream_id=sid)
    S = orc.S
    steps = n_steps if n_steps is not None else S + 1
    _, ys = W.simulate(model, warm + steps, seed=obs_seed)
    flt = _filter(model, N, radix, resampler, dtype, seed=seed, sid=sid)
    st = orc.init()
    tot_flips = 0
    for t in range(warm + steps):
        if t >= warm:
            label = f"{model_name} N={N} r={radix} {resampler} {dtype} t={t}"
            log(f"[case] {label}")
            stats = compare_one_step(flt, orc, st.x, st.logw, t, ys[t], st.log_norm, label)
            tot_flips += stats["flips"]
            log(f"   ok flips={stats['flips']} near={stats['near']} dw={stats['max_dw']:.2e} "
                f"dx={stats['max_dx']:.2e} dm={stats['max_dm']:.2e}")
        st, _ = orc.step(st, ys[t], keep=False)
    flt.close()
    return tot_flips


CASES = [
    ("ar1", 1024, 2, "multinomial", "f32"),
    ("ar1", 1024, 2, "systematic", "f32"),
    ("ar1", 1024, 1024, "multinomial", "f32"),
    ("ar1", 1024, 1024, "systematic", "f32"),
    ("ar1", 1024, 2, "multinomial", "f64"),
    ("ar1", 1024, 1024, "multinomial", "f64"),
    ("lg4dense", 4096, 4, "multinomial", "f32"),
    ("lg4dense", 8192, 64, "multinomial", "f32"),
    ("lg3stable", 2048, 8, "systematic", "f32"),
    ("lg8", 16384, 32, "multinomial", "f32"),
    ("lg8", 16384, 64, "multinomial", "f32"),
    ("lg8", 16384, 16384, "multinomial", "f32"),
    ("sv", 16384, 64, "multinomial", "f32"),
    ("sv", 16384, 256, "multinomial", "f32"),
    ("sv", 65536, 1024, "systematic", "f32"),
    ("sv", 16384, 2048, "multinomial", "f32"),
    ("sv", 32768, 4096, "multinomial", "f32"),
    ("sv", 16384, 64, "multinomial", "bf16"),
    ("sv", 4096, 4096, "multinomial", "bf16"),
    ("lg4dense", 4096, 16, "multinomial", "f64"),
    ("ar1", 128, 2, "multinomial", "f32"),
    ("ar1", 128, 128, "multinomial", "f32"),
    ("lg8", 128, 64, "systematic", "f32"),
    # the systematic global draw at every weight-tile size (d = 1: 4096,
    # d = 4: 2048, d = 8: 1024; below 4096 particles: 128) and every dtype
    ("sv", 65536, 65536, "systematic", "f32"),
    ("sv", 16384, 16384, "systematic", "bf16"),
    ("lg4dense", 8192, 8192, "systematic", "f32"),
    ("lg8", 16384, 16384, "systematic", "f32"),
    ("ar1", 1024, 1024, "systematic", "f64"),
    ("ar1", 128, 128, "systematic", "f32"),
    # d = 2 (compiled dimension 2): the wave path and both block-path tiles
    ("lg2stable", 8192, 64, "systematic", "f32"),
    ("lg2stable", 16384, 256, "multinomial", "f32"),
    ("lg2stable", 16384, 1024, "multinomial", "f32"),
    ("lg2stable", 4096, 4096, "systematic", "f32"),
    # d = 16 (the largest compiled dimension): wave path, block path, both
    # global draws
    ("lg16stable", 8192, 64, "multinomial", "f32"),
    ("lg16stable", 8192, 256, "systematic", "f32"),
    ("lg16stable", 4096, 4096, "multinomial", "f32"),
    ("lg16stable", 4096, 4096, "systematic", "f32"),
]


@pytest.mark.parametrize("model_name,N,radix,resampler,dtype", CASES,
                         ids=[f"{c[0]}-N{c[1]}-r{c[2]}-{c[3][:3]}-{c[4]}" for c in CASES])
def test_teacher_forced_step(model_name, N, radix, resampler, dtype):
    """Every stage of the plan (one full cycle and one more step) from an
    oracle trajectory: ancestors, log-weights, states and estimates."""
    _teacher_forced(model_name, N, radix, resampler, dtype, warm=1)


@pytest.mark.parametrize("model_name,dtype", [("ar1", "f32"), ("lg4dense", "f32"), ("sv", "f32"),
                                              ("ar1", "f64"), ("sv", "bf16"), ("lg8", "f32")])
def test_init_matches_oracle(model_name, dtype):
    """Initialisation (Algorithm 1): x_0 = prior(z(tau = 0)), unit weights."""
    from paper_1812_01502_amd import bf16_to_f32
    model = MODELS[model_name]()
    N = 4096
    flt = _filter(model, N, 64, dtype=dtype, seed=123, sid=9)
    x, w, t, ln = flt.get_state()
    orc = ButterflyOracle(model, N, 64, seed=123, stream_id=9)
    x0 = orc.init().x.T
    xg = bf16_to_f32(x).astype(np.float64) if dtype == "bf16" else x.astype(np.float64)
    rtol = {"f64": 1e-12, "f32": 2e-6, "bf16": 8e-3}[dtype]
    assert np.all(np.abs(xg - x0) <= 2e-6 + rtol * np.abs(x0)), float(np.max(np.abs(xg - x0)))
    assert np.all(w == 0) and t == 0 and ln == 0.0
    flt.close()


def test_free_running_fp64_matches_oracle_c1():
    """AR(1), N = 1024, T = 100 in FP64 (the double instantiation of the same
    kernels), radix 2 and the global path: ancestors identical at every step
    and estimates equal to rounding; both filters track the Kalman mean."""
    cfg = W.config("c1")
    model = cfg["model"]
    _, ys = W.simulate(model, cfg["T"], cfg["seed_obs"])
    kf = kalman.kalman_filter(model, ys)
    for radix in cfg["radices"]:
        log(f"[case] c1 fp64 radix={radix}")
        orc = ButterflyOracle(model, cfg["N"], radix, seed=cfg["seed_pf"])
        flt = _filter(model, cfg["N"], radix, dtype="f64", seed=cfg["seed_pf"], history=cfg["T"])
        st = orc.init()
        for t, y in enumerate(ys):
            flt.step(y)
            st, rec = orc.step(st, y, keep=True)
            anc = flt.ancestors().astype(np.int64)
            mism = anc != rec["ancestors"]
            assert not np.any(mism & (rec["margin"] > 1e-12)), (radix, t)
        hist = flt.history(cfg["T"])
        _, recs = ButterflyOracle(model, cfg["N"], radix, seed=cfg["seed_pf"]).run(ys)
        mg = np.array([h["mean"][0] for h in hist])
        mo = np.array([r["mean"][0] for r in recs])
        sd = np.sqrt(np.array([r["var"][0] for r in recs]))
        assert np.all(np.abs(mg - mo) <= 1e-9 * np.maximum(np.abs(mo), sd))
        assert abs(hist[-1]["log_norm"] - recs[-1]["log_norm"]) < 1e-8
        mse = float(np.sum((mg - kf["mean"][:, 0]) ** 2))
        raw = float(np.sum((ys[:, 0] - kf["mean"][:, 0]) ** 2))
        log(f"   MSE vs Kalman {mse:.4f} (raw observations {raw:.2f})")
        assert mse < 0.05 * raw
        flt.close()


@pytest.mark.parametrize("radix", [2, 64])
def test_free_running_fp32_means(radix):
    """AR(1), N = 4096, T = 100 in FP32: per-step means within 1e-4 max(|m|,
    sd) of the oracle until the first tolerated near-tie flip (after which
    the trajectories legitimately differ); flips are counted and reported."""
    model = W.ar1_model()
    N, T = 4096, 100
    _, ys = W.simulate(model, T, seed=1)
    orc = ButterflyOracle(model, N, radix, seed=101)
    flt = _filter(model, N, radix, dtype="f32", seed=101, history=T)
    st = orc.init()
    first_flip = None
    for t, y in enumerate(ys):
        flt.step(y)
        st, rec = orc.step(st, y, keep=True)
        anc = flt.ancestors().astype(np.int64)
        mism = anc != rec["ancestors"]
        if first_flip is None and np.any(mism):
            assert np.all(rec["margin"][mism] <= MARGIN_TOL), (t, "flip beyond the margin")
            first_flip = t
        if first_flip is None:
            e = flt.estimate()
            sd = np.sqrt(rec["var"])
            assert np.all(np.abs(e["mean"] - rec["mean"]) <= 1e-4 * np.maximum(np.abs(rec["mean"]), sd)), t
    log(f"   radix {radix}: first tolerated flip at step {first_flip} of {T}")
    flt.close()


def test_run_device_observations_and_graph_bit_identical():
    """pf_run over a device observation array, with and without HIP-graph
    capture, gives exactly the states and records of the pf_step loop."""
    import torch
    model = W.lg8_model(seed=2)
    N, T = 1 << 15, 12
    _, ys = W.simulate(model, T, seed=2)
    outs = []
    for mode in ("step", "run", "graph"):
        stream = torch.cuda.Stream() if mode == "graph" else None
        from paper_1812_01502_amd import Filter
        flt = Filter(model, N, 64, seed=5, history=T,
                     stream=stream.cuda_stream if stream is not None else None)
        if mode == "step":
            for y in ys:
                flt.step(y)
        else:
            yd = torch.tensor(ys, dtype=torch.float32, device="cuda").contiguous()
            torch.cuda.synchronize()
            flt.run(yd.data_ptr(), T, model.d, use_graph=(mode == "graph"))
            flt.sync()
        x, w, t, ln = flt.get_state()
        outs.append((x, w, t, ln, [h["mean"] for h in flt.history(T)]))
        flt.close()
    for o in outs[1:]:
        assert np.array_equal(o[0], outs[0][0]) and np.array_equal(o[1], outs[0][1])
        assert o[2] == outs[0][2] == T and o[3] == outs[0][3]
        assert all(np.array_equal(a, b) for a, b in zip(o[4], outs[0][4]))


def test_graph_replays_match_eager():
    """A captured graph replayed several times (eager work and syncs between
    replays) matches the eager path at every replay."""
    import torch
    from paper_1812_01502_amd import Filter
    model = W.sv_model()
    N, T = 1 << 14, 8
    _, ys = W.simulate(model, 3 * T, seed=3)
    yd = torch.tensor(ys, dtype=torch.float32, device="cuda").contiguous()
    s = torch.cuda.Stream()
    fg = Filter(model, N, 32, seed=9, history=3 * T, stream=s.cuda_stream)
    fe = Filter(model, N, 32, seed=9, history=3 * T)
    for rep in range(3):
        fg.run(yd[rep * T:].data_ptr(), T, 1, use_graph=True)
        fg.sync()
        for y in ys[rep * T:(rep + 1) * T]:
            fe.step(y)
        _ = torch.ones(1000, device="cuda").sum().item()   # eager work between replays
        xg, wg, tg, lg = fg.get_state()
        xe, we, te, le = fe.get_state()
        assert np.array_equal(xg, xe) and np.array_equal(wg, we) and tg == te and lg == le, rep
    fg.close()
    fe.close()


def test_history_records_and_errors():
    from paper_1812_01502_amd import Filter, PfError
    model = W.ar1_model()
    flt = Filter(model, 1024, 4, seed=1, history=8)
    with pytest.raises(PfError):
        flt.estimate()                    # no step yet
    _, ys = W.simulate(model, 10, seed=4)
    for y in ys:
        flt.step(y)
    h = flt.history(8)
    assert [r["t"] for r in h] == list(range(2, 10))
    assert [r["stage"] for r in h] == [t % 5 for t in range(2, 10)]
    assert all(r["valid"] == 1 and 0 < r["ess"] <= 1 for r in h)
    with pytest.raises(PfError) as ei:
        flt.step([np.nan])
    assert ei.value.status == -5
    flt.step(ys[0])                       # the handle stays usable
    assert flt.estimate()["t"] == 10
    with pytest.raises(PfError):
        flt.ancestors()                   # created without keep_ancestors
    info = flt.info()
    assert info["stages"] == [4] * 5 and not info["global_path"]
    flt.close()


FULL_CASES = [
    ("ar1", 1024, 4, "multinomial", "f32"),       # S = 5
    ("ar1", 1024, 2, "multinomial", "f64"),       # S = 10, FP64
    ("lg4dense", 4096, 8, "systematic", "f32"),   # S = 4, dense model
    ("sv", 16384, 64, "multinomial", "f32"),      # stages 64, 64, 4
    ("sv", 16384, 64, "multinomial", "bf16"),
    ("lg8", 16384, 256, "multinomial", "f32"),    # block-path stages 256, 64
]


@pytest.mark.parametrize("model_name,N,radix,resampler,dtype", FULL_CASES)
def test_full_cycle_step(model_name, N, radix, resampler, dtype):
    """Full augmented resampling per step (all S stages of Algorithm 3),
    teacher-forced against the FP64 oracle at three consecutive steps."""
    from paper_1812_01502_amd import Filter
    from tests.gpu_util import compare_full_cycle_step
    model = MODELS[model_name]()
    orc = ButterflyOracle(model, N, radix, resampler, seed=7, full_cycle=True)
    _, ys = W.simulate(model, 6, seed=5)
    flt = Filter(model, N, radix, resampler=resampler, dtype=dtype, seed=7, history=4, full_cycle=True)
    st = orc.init()
    for t in range(5):
        if t >= 2:
            label = f"full-cycle {model_name} N={N} r={radix} S={orc.S} {resampler} {dtype} t={t}"
            log(f"[case] {label}")
            s = compare_full_cycle_step(flt, orc, st.x, st.logw, t, ys[t], st.log_norm, label)
            log(f"   ok sure={s['sure']:.4f} dw={s['max_dw']:.2e} dx={s['max_dx']:.2e}")
        st, _ = orc.step(st, ys[t], keep=False)
    flt.close()


@pytest.mark.parametrize("case", ["one_tile", "last_particle", "alternate_tiles"])
def test_global_systematic_concentrated_weights(case):
    """The systematic global draw when the weight sits on few particles: one
    weight tile takes nearly every output (its outputs split into several
    items), the last particle takes nearly all (targets near the total), or
    every other tile has no weight (tiles without outputs). Start states
    from the oracle, log-weights set on both sides, one step compared."""
    model = MODELS["sv"]()
    N = 1 << 16
    orc = ButterflyOracle(model, N, N, "systematic", seed=31, stream_id=4)
    flt = _filter(model, N, N, "systematic", "f32", seed=31, sid=4)
    st = orc.init()
    _, ys = W.simulate(model, 2, seed=8)
    rng = np.random.Generator(np.random.PCG64(17))
    logw = np.full(N, -40.0)
    if case == "one_tile":
        logw[3 * 4096:4 * 4096] = rng.normal(0.0, 1.0, 4096)
    elif case == "last_particle":
        logw[-1] = 0.0
        logw[-5:-1] = -3.0
    else:
        tiles = np.arange(N) // 4096
        # weights that underflow to zero against the others (FP64 too)
        logw = np.where(tiles % 2 == 0, rng.normal(0.0, 0.5, N), -1e4)
    label = f"sv N={N} global systematic {case}"
    log(f"[case] {label}")
    s = compare_one_step(flt, orc, st.x, logw, 0, ys[0], 0.0, label)
    log(f"   ok flips={s['flips']} near={s['near']} dw={s['max_dw']:.2e}")
    anc = flt.ancestors().astype(np.int64)
    assert np.all(np.diff(anc) >= 0)  # systematic ancestors do not decrease
    flt.close()
