"""Helpers of the GPU parity tests: oracle-generated start states and the
one-step comparison of the device path against the FP64 oracle.

Every input of both sides comes from the oracle or the seeded generators:
the device is given the oracle's state (rounded to the device storage
type), never the other way round.
"""
from __future__ import annotations

import sys

import numpy as np

from oracle import ButterflyOracle, State

MARGIN_TOL = 1e-5          # ancestors must match where the draw's margin exceeds this
MEAN_RTOL = 1e-4           # filter means: |dm| <= 1e-4 max(|m|, sd)


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def round_state(x: np.ndarray, logw: np.ndarray, dtype: str):
    """Oracle state (x: (N, d) FP64) in the device's storage precision:
    returns (device x planes (d, N), device logW, oracle x (N, d), oracle logW)
    where the oracle arrays hold exactly the device values in FP64."""
    from paper_1812_01502_amd import bf16_to_f32, f32_to_bf16
    if dtype == "f64":
        xd = np.ascontiguousarray(x.T)
        wd = logw.copy()
        return xd, wd, xd.T.copy(), wd.copy()
    w32 = logw.astype(np.float32)
    if dtype == "f32":
        x32 = np.ascontiguousarray(x.T.astype(np.float32))
        return x32, w32, x32.T.astype(np.float64), w32.astype(np.float64)
    xb = f32_to_bf16(np.ascontiguousarray(x.T.astype(np.float32)))
    return xb, w32, bf16_to_f32(xb).T.astype(np.float64), w32.astype(np.float64)


def device_x(flt, x_raw):
    """Device state planes (d, N) as FP64 (N, d)."""
    from paper_1812_01502_amd import bf16_to_f32
    if flt.dtype == "bf16":
        x_raw = bf16_to_f32(x_raw)
    return x_raw.astype(np.float64).T


def tolerances(dtype: str):
    if dtype == "f64":
        return dict(w_atol=1e-9, x_atol=1e-9, x_rtol=1e-10, mean_rtol=1e-9, var_rtol=1e-8,
                    ess_rtol=1e-10, ln_atol=1e-8)
    if dtype == "f32":
        return dict(w_atol=3e-4, x_atol=5e-5, x_rtol=2e-5, mean_rtol=MEAN_RTOL, var_rtol=2e-3,
                    ess_rtol=2e-4, ln_atol=2e-4)
    # BF16 storage: states carry 8 mantissa bits
    return dict(w_atol=3e-4, x_atol=5e-5, x_rtol=8e-3, mean_rtol=MEAN_RTOL, var_rtol=2e-3,
                ess_rtol=2e-4, ln_atol=2e-4)


def compare_one_step(flt, orc: ButterflyOracle, x_or: np.ndarray, logw_or: np.ndarray, t: int,
                     y, log_norm: float = 0.0, label: str = ""):
    """Start device and oracle from the same state at step t, advance one
    step and compare. Returns a dict of statistics (flips, errors)."""
    dtype = flt.dtype
    tol = tolerances(dtype)
    xd, wd, xo, wo = round_state(x_or, logw_or, dtype)
    flt.set_state(xd, wd, t=t, log_norm=log_norm)
    flt.step(y)
    rec_g = flt.estimate()
    xg_raw, wg, tg, lng = flt.get_state()
    anc_g = flt.ancestors().astype(np.int64)
    st_o, rec_o = orc.step(State(x=xo, logw=wo, t=t, log_norm=log_norm), y, keep=True)
    assert tg == t + 1
    assert rec_g["t"] == t and rec_g["stage"] == rec_o["stage"], (rec_g["t"], rec_g["stage"], rec_o["stage"])
    # ancestors: exact wherever the margin exceeds the tolerance
    anc_o = rec_o["ancestors"]
    mism = anc_g != anc_o
    bad = mism & (rec_o["margin"] > MARGIN_TOL)
    assert not np.any(bad), (label, "ancestor mismatch beyond margin", np.nonzero(bad)[0][:8],
                             anc_g[bad][:8], anc_o[bad][:8], rec_o["margin"][bad][:8])
    # every device ancestor lies in its group
    N = flt.n
    r, R = rec_o["radix"], rec_o["stride"]
    i = np.arange(N)
    assert np.array_equal((anc_g // (r * R), anc_g % R), (i // (r * R), i % R)) or r == N
    # a tolerated flip must still be a valid draw: the target lies within the
    # margin of the device ancestor's own cumulative-weight interval
    if np.any(mism):
        dr = rec_o["draw"]
        idx = np.nonzero(mism)[0]
        qg = (anc_g[idx] // R) % r
        rows = dr["row"][idx]
        hi = dr["cdf"][rows, qg]
        lo = np.where(qg > 0, dr["cdf"][rows, np.maximum(qg - 1, 0)], 0.0)
        tg = dr["target"][idx]
        ok_int = (tg >= lo - MARGIN_TOL) & (tg <= hi + MARGIN_TOL)
        assert np.all(ok_int), (label, "flip outside the ancestor's interval", idx[~ok_int][:8])
    # new log-weights (normalised so that the max is 0)
    dw = np.abs(wg.astype(np.float64) - st_o.logw)
    assert np.max(dw) <= tol["w_atol"], (label, "logw", float(np.max(dw)))
    # propagated states where the ancestor agrees
    xg = device_x(flt, xg_raw)
    ok = ~mism
    err = np.abs(xg[ok] - st_o.x[ok])
    lim = tol["x_atol"] + tol["x_rtol"] * np.abs(st_o.x[ok])
    assert np.all(err <= lim), (label, "x", float(np.max(err - lim)))
    # estimates of the step (R13 for the means)
    sd = np.sqrt(rec_o["var"])
    dm = np.abs(rec_g["mean"] - rec_o["mean"])
    assert np.all(dm <= tol["mean_rtol"] * np.maximum(np.abs(rec_o["mean"]), sd)), (label, "mean", dm, sd)
    dv = np.abs(rec_g["var"] - rec_o["var"])
    assert np.all(dv <= tol["var_rtol"] * rec_o["var"] + 1e-12), (label, "var", dv, rec_o["var"])
    assert abs(rec_g["ess"] - rec_o["ess"]) <= tol["ess_rtol"] * rec_o["ess"], (label, "ess")
    assert abs(lng - rec_o["log_norm"]) <= tol["ln_atol"] * (1 + abs(rec_o["log_norm"] - log_norm)), \
        (label, "log_norm", lng, rec_o["log_norm"])
    return dict(flips=int(mism.sum()), near=int(np.sum(rec_o["margin"] <= MARGIN_TOL)),
                max_dw=float(np.max(dw)), max_dx=float(np.max(err)) if err.size else 0.0,
                max_dm=float(np.max(dm / np.maximum(np.abs(rec_o["mean"]), sd))))


def compare_full_cycle_step(flt, orc: ButterflyOracle, x_or: np.ndarray, logw_or: np.ndarray, t: int,
                            y, log_norm: float = 0.0, label: str = ""):
    """One full-cycle step (all S stages) from the same state on both sides.
    Estimates, log-normaliser and the (equal) new log-weights are compared
    everywhere; states where every draw along the particle's ancestry cleared
    the margin (a flipped draw changes every descendant)."""
    dtype = flt.dtype
    tol = tolerances(dtype)
    xd, wd, xo, wo = round_state(x_or, logw_or, dtype)
    flt.set_state(xd, wd, t=t, log_norm=log_norm)
    flt.step(y)
    rec_g = flt.estimate()
    xg_raw, wg, tg, lng = flt.get_state()
    st_o, rec_o = orc.step(State(x=xo, logw=wo, t=t, log_norm=log_norm), y, keep=True)
    assert tg == t + 1
    assert rec_g["t"] == t and rec_g["stage"] == orc.S == rec_o["stage"], (rec_g["stage"], orc.S)
    # after all stages every weight is the global mean: the normalised
    # log-weights are zero up to rounding
    dw = np.abs(wg.astype(np.float64) - st_o.logw)
    assert np.max(dw) <= tol["w_atol"], (label, "logw", float(np.max(dw)))
    sure = np.ones(flt.n, dtype=bool)
    for anc, margin in rec_o["stages"]:
        sure = (margin > MARGIN_TOL) & sure[anc]
    xg = device_x(flt, xg_raw)
    err = np.abs(xg[sure] - st_o.x[sure])
    lim = tol["x_atol"] + tol["x_rtol"] * np.abs(st_o.x[sure])
    assert np.all(err <= lim), (label, "x", float(np.max(err - lim)))
    assert np.mean(sure) > 0.5, (label, "too few particles with clear draws", float(np.mean(sure)))
    sd = np.sqrt(rec_o["var"])
    dm = np.abs(rec_g["mean"] - rec_o["mean"])
    assert np.all(dm <= tol["mean_rtol"] * np.maximum(np.abs(rec_o["mean"]), sd)), (label, "mean", dm, sd)
    dv = np.abs(rec_g["var"] - rec_o["var"])
    assert np.all(dv <= tol["var_rtol"] * rec_o["var"] + 1e-12), (label, "var", dv, rec_o["var"])
    assert abs(rec_g["ess"] - rec_o["ess"]) <= tol["ess_rtol"] * rec_o["ess"], (label, "ess")
    assert abs(lng - rec_o["log_norm"]) <= tol["ln_atol"] * (1 + abs(rec_o["log_norm"] - log_norm)), \
        (label, "log_norm", lng, rec_o["log_norm"])
    return dict(sure=float(np.mean(sure)), max_dw=float(np.max(dw)),
                max_dx=float(np.max(err)) if err.size else 0.0)


def island_sure(rec_o, M: int):
    """Per destination particle: every draw its value depends on cleared the
    margin (its within-island draw in the source island, and at every island
    stage both draws of the pair that decided where its island's sample came
    from: the no-swap rule looks at both)."""
    stages = rec_o["island_stages"]
    m = rec_o["src"].shape[0]
    sure_isl = np.ones(m, dtype=bool)
    for s, (pick, margin) in enumerate(stages):
        partner = np.arange(m) ^ (1 << s)
        pair_ok = (margin > MARGIN_TOL) & (margin[partner] > MARGIN_TOL)
        sure_isl = pair_ok & sure_isl[pick]
    N = rec_o["origin"].shape[0]
    k = np.arange(N) // M
    j = np.arange(N) % M
    src = rec_o["src"]
    return sure_isl[k] & (rec_o["margin"][src[k] * M + j] > MARGIN_TOL)


def compare_island_step(flt, orc, x_or: np.ndarray, logw_or: np.ndarray, t: int, y,
                        log_norm: float = 0.0, label: str = "", upload: bool = True):
    """One island-filter step from the same state on both sides. Ancestors
    (the particle each destination copies) and states are compared wherever
    every draw they depend on cleared the margin; the ancestors of a
    destination island all lie in one source island; the output is
    unweighted; estimates and the log-normaliser everywhere. With
    ``upload=False`` the device already holds the state (its own previous
    output, whose log-weights are all zero and are then not read)."""
    dtype = flt.dtype
    tol = tolerances(dtype)
    xd, wd, xo, wo = round_state(x_or, logw_or, dtype)
    if upload:
        flt.set_state(xd, wd, t=t, log_norm=log_norm)
    flt.step(y)
    rec_g = flt.estimate()
    xg_raw, wg, tg, lng = flt.get_state()
    anc_g = flt.ancestors().astype(np.int64)
    st_o, rec_o = orc.step(State(x=xo, logw=wo, t=t, log_norm=log_norm), y, keep=True)
    M = orc.M
    assert tg == t + 1
    assert rec_g["t"] == t and rec_g["stage"] == orc.S_I and rec_g["radix"] == M, (rec_g["stage"], orc.S_I)
    assert np.all(wg == 0.0), (label, "island output must be unweighted")
    sure = island_sure(rec_o, M)
    bad = sure & (anc_g != rec_o["origin"])
    assert not np.any(bad), (label, "ancestor mismatch", np.nonzero(bad)[0][:8], anc_g[bad][:8],
                             rec_o["origin"][bad][:8])
    # whole islands are copied: the ancestors of a destination island all
    # come from one source island
    N = flt.n
    src_g = (anc_g // M).reshape(N // M, M)
    assert np.all(src_g == src_g[:, :1]), (label, "an island mixes source islands")
    xg = device_x(flt, xg_raw)
    err = np.abs(xg[sure] - st_o.x[sure])
    lim = tol["x_atol"] + tol["x_rtol"] * np.abs(st_o.x[sure])
    assert np.all(err <= lim), (label, "x", float(np.max(err - lim)))
    assert np.mean(sure) > 0.5, (label, "too few particles with clear draws", float(np.mean(sure)))
    sd = np.sqrt(rec_o["var"])
    dm = np.abs(rec_g["mean"] - rec_o["mean"])
    assert np.all(dm <= tol["mean_rtol"] * np.maximum(np.abs(rec_o["mean"]), sd)), (label, "mean", dm, sd)
    dv = np.abs(rec_g["var"] - rec_o["var"])
    assert np.all(dv <= tol["var_rtol"] * rec_o["var"] + 1e-12), (label, "var", dv, rec_o["var"])
    assert abs(rec_g["ess"] - rec_o["ess"]) <= tol["ess_rtol"] * rec_o["ess"], (label, "ess")
    assert abs(lng - rec_o["log_norm"]) <= tol["ln_atol"] * (1 + abs(rec_o["log_norm"] - log_norm)), \
        (label, "log_norm", lng, rec_o["log_norm"])
    return dict(sure=float(np.mean(sure)), flips=int(np.sum(anc_g != rec_o["origin"])),
                max_dx=float(np.max(err)) if err.size else 0.0)


ESS_TOL = 1e-3   # ESS decisions are compared where the oracle's ESS is this far (relative) from theta


def compare_adaptive_step(flt, orc, st_or, y, label: str = "", upload: bool = True):
    """One step with ESS-gated stages from the same state on both sides
    (``st_or``: an oracle ``AdaptiveState``; with ``upload`` it is set on the
    device, whose rotation then restarts at stage 0, so ``st_or.next_stage``
    must be 0). The number of stages run must agree (the oracle's ESS values
    must clear theta by ESS_TOL); states where every draw along the
    particle's ancestry cleared the margin; the carried log-weights,
    estimates and log-normaliser everywhere. Returns (new oracle state,
    statistics)."""
    from oracle.adaptive import AdaptiveState
    dtype = flt.dtype
    tol = tolerances(dtype)
    xd, wd, xo, wo = round_state(st_or.x, st_or.logw, dtype)
    if upload:
        assert st_or.next_stage == 0
        flt.set_state(xd, wd, t=st_or.t, log_norm=st_or.log_norm)
    flt.step(y)
    rec_g = flt.estimate()
    xg_raw, wg, tg, lng = flt.get_state()
    st0 = AdaptiveState(x=xo, logw=wo, t=st_or.t, log_norm=st_or.log_norm, next_stage=st_or.next_stage)
    st_o, rec_o = orc.step(st0, y, keep=True)
    th = orc.theta
    # every ESS value that decided something (after S stages the step stops anyway)
    decisive = rec_o["ess_trace"][:orc.S] if rec_o["stage"] == orc.S else rec_o["ess_trace"]
    gaps = [abs(e - th) / th for e in decisive]
    assert min(gaps) > ESS_TOL, (label, "an ESS value is too close to theta for a parity case", rec_o["ess_trace"])
    assert tg == st_or.t + 1 and rec_g["t"] == st_or.t
    assert rec_g["stage"] == rec_o["stage"], (label, "stages run", rec_g["stage"], rec_o["stage"], rec_o["ess_trace"])
    dw = np.abs(wg.astype(np.float64) - st_o.logw)
    assert np.max(dw) <= tol["w_atol"], (label, "logw", float(np.max(dw)))
    sure = np.ones(flt.n, dtype=bool)
    for anc, margin in rec_o["stages"]:
        sure = (margin > MARGIN_TOL) & sure[anc]
    xg = device_x(flt, xg_raw)
    err = np.abs(xg[sure] - st_o.x[sure])
    lim = tol["x_atol"] + tol["x_rtol"] * np.abs(st_o.x[sure])
    assert np.all(err <= lim), (label, "x", float(np.max(err - lim)))
    assert np.mean(sure) > 0.5, (label, "too few particles with clear draws", float(np.mean(sure)))
    sd = np.sqrt(rec_o["var"])
    dm = np.abs(rec_g["mean"] - rec_o["mean"])
    assert np.all(dm <= tol["mean_rtol"] * np.maximum(np.abs(rec_o["mean"]), sd)), (label, "mean", dm, sd)
    dv = np.abs(rec_g["var"] - rec_o["var"])
    assert np.all(dv <= tol["var_rtol"] * rec_o["var"] + 1e-12), (label, "var", dv, rec_o["var"])
    assert abs(rec_g["ess"] - rec_o["ess"]) <= tol["ess_rtol"] * rec_o["ess"], (label, "ess")
    assert abs(lng - rec_o["log_norm"]) <= tol["ln_atol"] * (1 + abs(rec_o["log_norm"] - st_or.log_norm)), \
        (label, "log_norm", lng, rec_o["log_norm"])
    # the next step continues from the device's own state and rotation
    nxt = AdaptiveState(x=device_x(flt, xg_raw), logw=wg.astype(np.float64), t=tg, log_norm=lng,
                        next_stage=st_o.next_stage)
    return nxt, dict(stages=int(rec_o["stage"]), sure=float(np.mean(sure)),
                     max_dx=float(np.max(err)) if err.size else 0.0)
