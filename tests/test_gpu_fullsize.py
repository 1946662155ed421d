"""GPU parity at the full workload sizes, in the launch configuration the
benchmark times (same N, radix, tiles): teacher-forced single steps from
oracle trajectories, every particle compared (ancestors under the margin
rule, log-weights, states, estimates)."""
import numpy as np
import pytest

import workloads as W
from oracle import ButterflyOracle
from tests.gpu_util import compare_one_step, log

pytestmark = pytest.mark.gpu


def _run(cfg_name, N, radix, steps, dtype="f32", resampler="multinomial", seed=11):
    from paper_1812_01502_amd import Filter
    cfg = W.config(cfg_name)
    model = cfg["model"]
    _, ys = W.simulate(model, max(steps) + 1, seed=cfg["seed_obs"])
    orc = ButterflyOracle(model, N, radix, resampler, seed=seed)
    flt = Filter(model, N, radix, resampler=resampler, dtype=dtype, seed=seed, keep_ancestors=True)
    st = orc.init()
    for t in range(max(steps) + 1):
        if t in steps:
            label = f"{cfg_name} N={N} r={radix} {dtype} t={t} stage={t % orc.S}"
            log(f"[case] {label}")
            s = compare_one_step(flt, orc, st.x, st.logw, t, ys[t], st.log_norm, label)
            log(f"   ok flips={s['flips']} near={s['near']} dw={s['max_dw']:.2e} dx={s['max_dx']:.2e} "
                f"dm={s['max_dm']:.2e}")
        if t < max(steps):
            st, _ = orc.step(st, ys[t], keep=False)
    flt.close()


def test_lg8_n2p20_radix64_every_stage():
    """8-D LG, N = 2^20, radix 64 (stages 64, 64, 64, 4): all four stages."""
    _run("c2", 1 << 20, 64, steps=[0, 1, 2, 3, 4])


def test_lg8_n2p20_global():
    """8-D LG, N = 2^20, the global bootstrap filter (r = N)."""
    _run("c2", 1 << 20, 1 << 20, steps=[0, 1])


def test_lg8_n2p20_radix2_wide_stride():
    """Radix 2 at the widest strides of N = 2^20 (stages 17..19)."""
    _run("c2", 1 << 20, 2, steps=[17, 18, 19], seed=3)


def test_sv_n2p24_radix1024():
    """SV, N = 2^24, radix 1024 (stages 1024, 1024, 16): the block path at
    strides 1 and 1024, then the radix-16 stage at stride 2^20."""
    _run("c3", 1 << 24, 1024, steps=[0, 1, 2])


def test_sv_n2p24_radix64_and_bf16():
    """SV, N = 2^24, radix 64 (four stages of 64), FP32 and BF16 states."""
    _run("c3", 1 << 24, 64, steps=[3])
    _run("c3", 1 << 24, 64, steps=[1], dtype="bf16")


def test_sv_n2p24_radix32_first_and_top_stage():
    """SV, N = 2^24, radix 32 (stages 32, 32, 32, 32, 16): the stride-1 stage
    and the radix-16 stage at stride 2^20."""
    _run("c3", 1 << 24, 32, steps=[0, 4])


def test_sv_n2p24_radix256():
    """SV, N = 2^24, radix 256 (stages 256, 256, 256): the block path at
    stride 256."""
    _run("c3", 1 << 24, 256, steps=[1])


def test_sv_n2p24_global_f32_and_bf16():
    """SV, N = 2^24, the global bootstrap filter (r = N), FP32 and BF16
    states."""
    _run("c3", 1 << 24, 1 << 24, steps=[0, 1])
    _run("c3", 1 << 24, 1 << 24, steps=[1], dtype="bf16")


def test_sv_n2p24_global_systematic():
    """SV, N = 2^24, the global filter with systematic resampling: the merge
    draw over the prefix kernel's items, at the benchmarked shape."""
    _run("c3", 1 << 24, 1 << 24, steps=[0, 1], resampler="systematic")


def test_lg8_n2p20_global_systematic():
    """8-D LG, N = 2^20, the global filter with systematic resampling (the
    states gathered from the particle-major copy)."""
    _run("c2", 1 << 20, 1 << 20, steps=[1], resampler="systematic")


def test_sv_n2p24_radix1024_bf16():
    """SV, N = 2^24, radix 1024 with BF16 states: the block path at stride
    1024."""
    _run("c3", 1 << 24, 1024, steps=[1], dtype="bf16")


def test_sv_n2p24_island_m4096():
    """The island filter at its benchmarked shape: SV, N = 2^24 in 4096
    islands of 4096 (within-island launch of 1024-thread tiles, island
    stages in two launches, LDS-staged gather), one teacher-forced step."""
    from oracle import IslandOracle
    from paper_1812_01502_amd import Filter
    from tests.gpu_util import compare_island_step
    cfg = W.config("c3")
    model = cfg["model"]
    N, M = 1 << 24, 4096
    orc = IslandOracle(model, N, M, seed=23, stream_id=2)
    _, ys = W.simulate(model, 2, seed=cfg["seed_obs"])
    st = orc.init()
    log(f"[case] island full size SV N={N} M={M}")
    flt = Filter(model, N, 2, seed=23, stream_id=2, keep_ancestors=True, island=M)
    r = compare_island_step(flt, orc, st.x, np.zeros(N), 0, ys[0], label="sv-2^24-M4096")
    log(f"   ok sure={r['sure']:.4f} flips={r['flips']} max_dx={r['max_dx']:.2e}")
    flt.close()
