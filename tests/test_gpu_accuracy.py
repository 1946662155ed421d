"""Accuracy of the device filters as filters, and the error of the BF16
state-storage variant against the FP64 oracle, per result.

* BF16 storage, one step: from the oracle's FP64 cloud at several steps of
  a trajectory, the device loads the cloud rounded to its storage type (FP32
  or BF16) and runs one step; the oracle runs the same step from the exact
  cloud. The differences of the step's mean, variance, effective sample size
  and log-normaliser increment are the error that storage rounding adds to
  each result. BF16's must stay within the Monte Carlo error of the filter.
* BF16 storage, free running: device FP32, device BF16 and the FP64 oracle
  over T steps with the same seed and observations; each against the oracle
  and against the exact filter (the grid filter of the SV model).
* The 8-D linear-Gaussian workload at N = 2^20 against the Kalman filter
  (the accuracy measure of the paper's experiments: squared error of the
  filter mean against the exact one, summed over steps), over 16 seeds, with
  the mean effective sample size of each: every radix of the workload with
  one stage per step, the global filter, every stage per step (Algorithm 3),
  ESS-gated stages and the island filter.

Each test prints its table; the asserted bounds are loose (statistical).
"""
import numpy as np
import pytest

import workloads as W
from oracle import ButterflyOracle, State
from oracle.gridfilter import sv_grid_filter
from oracle.kalman import kalman_filter
from tests.gpu_util import log, round_state

pytestmark = pytest.mark.gpu


def _one_step_errors(flt, orc, st, y):
    """Device step from the cloud rounded to the device's storage type,
    oracle step from the exact cloud; errors of the step's results."""
    xd, wd, _, _ = round_state(st.x, st.logw, flt.dtype)
    flt.set_state(xd, wd, t=st.t, log_norm=0.0)
    flt.step(y)
    e = flt.estimate()
    _, ro = orc.step(State(x=st.x, logw=st.logw, t=st.t, log_norm=0.0), y, keep=False)
    sd = float(np.sqrt(ro["var"][0]))
    return dict(mean=abs(e["mean"][0] - ro["mean"][0]) / sd,
                var=abs(e["var"][0] - ro["var"][0]) / ro["var"][0],
                ess=abs(e["ess"] - ro["ess"]) / ro["ess"],
                lam=abs(e["log_norm"] - ro["log_norm"]),
                mc_mean=1.0 / np.sqrt(orc.N * ro["ess"]))


def test_bf16_storage_error_per_result_one_step():
    """SV, N = 2^16, radix 64: the error each result picks up from storing
    the cloud in BF16 (or FP32) for one step, at 8 steps of an oracle
    trajectory."""
    from paper_1812_01502_amd import Filter
    model = W.sv_model()
    N, T = 1 << 16, 64
    _, ys = W.simulate(model, T, seed=3)
    orc = ButterflyOracle(model, N, 64, seed=303)
    st = orc.init()
    rows = {"f32": [], "bf16": []}
    flts = {dt: Filter(model, N, 64, dtype=dt, seed=303) for dt in rows}
    for t in range(T):
        if t % 8 == 7:
            for dt, f in flts.items():
                rows[dt].append(_one_step_errors(f, orc, st, ys[t]))
        st, _ = orc.step(st, ys[t], keep=False)
    for f in flts.values():
        f.close()
    log("[table] one-step error against the FP64 oracle, SV N=2^16 r=64 (max over 8 steps)")
    log("   storage  |dmean|/sd   |dvar|/var   |dESS|/ESS   |dLambda|   MC sd of mean / sd")
    for dt, rs in rows.items():
        mx = {k: max(r[k] for r in rs) for k in rs[0]}
        log(f"   {dt:7s}  {mx['mean']:.2e}    {mx['var']:.2e}    {mx['ess']:.2e}    {mx['lam']:.2e}   "
            f"{mx['mc_mean']:.2e}")
        # storage rounding stays well inside the Monte Carlo error of the mean
        assert mx["mean"] <= 0.1 * min(r["mc_mean"] for r in rs), (dt, mx)
        assert mx["var"] <= 1e-2 and mx["ess"] <= 1e-2 and mx["lam"] <= 1e-2, (dt, mx)


def test_bf16_storage_error_per_result_free_running():
    """SV, N = 2^16, radix 64, T = 200 with the same seed: device FP32,
    device BF16 and the FP64 oracle, each against the oracle and against
    the exact filter (grid filter)."""
    import torch
    from paper_1812_01502_amd import Filter
    model = W.sv_model()
    N, T = 1 << 16, 200
    _, ys = W.simulate(model, T, seed=3)
    exact = sv_grid_filter(model, ys, n_nodes=4096)
    _, ro = ButterflyOracle(model, N, 64, seed=303).run(ys)
    mo = np.array([r["mean"][0] for r in ro])
    vo = np.array([r["var"][0] for r in ro])
    eo = np.array([r["ess"] for r in ro])
    lo = np.array([r["log_norm"] for r in ro])
    res = {"oracle": (mo, vo, eo, lo)}
    yd = torch.tensor(ys, dtype=torch.float32, device="cuda").contiguous()
    for dt in ("f32", "bf16"):
        f = Filter(model, N, 64, dtype=dt, seed=303, history=T)
        f.run(yd.data_ptr(), T, 1)
        h = f.history(T)
        f.close()
        res[dt] = (np.array([r["mean"][0] for r in h]), np.array([r["var"][0] for r in h]),
                   np.array([r["ess"] for r in h]), np.array([r["log_norm"] for r in h]))
    sd = np.sqrt(vo)
    log(f"[table] free-running, SV N=2^16 r=64 T={T}: against the FP64 oracle (max over steps) "
        f"and against the exact filter")
    log("   filter   |dmean|/sd   |dvar|/var   |dESS|/ESS  |dLambda_T|   RMSE(mean - exact)  "
        "Lambda_T - exact")
    for k, (m, v, e, ln) in res.items():
        rmse = float(np.sqrt(np.mean((m - exact["mean"]) ** 2)))
        log(f"   {k:7s}  {np.max(np.abs(m - mo) / sd):.2e}    {np.max(np.abs(v - vo) / vo):.2e}    "
            f"{np.max(np.abs(e - eo) / eo):.2e}    {abs(ln[-1] - lo[-1]):.2e}    {rmse:.4e}          "
            f"{ln[-1] - exact['loglik']:+.3f}")
    rm = {k: float(np.sqrt(np.mean((v[0] - exact["mean"]) ** 2))) for k, v in res.items()}
    # every variant is a filter of the same accuracy: its error against the
    # exact filter stays at the oracle's Monte Carlo level
    for k in ("f32", "bf16"):
        assert rm[k] <= 2.0 * rm["oracle"] + 1e-3, (k, rm)
        assert abs(res[k][3][-1] - exact["loglik"]) <= abs(lo[-1] - exact["loglik"]) + 1.0, k


def test_lg8_accuracy_against_kalman_per_radix():
    """8-D LG, N = 2^20, T = 500: squared error of the filter mean against
    the Kalman mean, summed over steps and components, mean over 16 seeds,
    for radix 2, 4, 32, 64 and the global filter with one stage per step;
    the same radices with every stage per step (Algorithm 3); ESS-gated
    stages; the island filter. Mean and minimum ESS per filter."""
    import torch
    from paper_1812_01502_amd import Filter
    cfg = W.config("c2")
    model = cfg["model"]
    N, T = cfg["N"], cfg["T"]
    _, ys = W.simulate(model, T, seed=cfg["seed_obs"])
    kf = kalman_filter(model, ys)
    raw = float(np.sum((ys - kf["mean"]) ** 2))
    yd = torch.tensor(ys, dtype=torch.float32, device="cuda").contiguous()
    seeds = range(16)
    log(f"[table] LG-8 N=2^20 T={T}, 16 seeds: sum_t |mean - Kalman mean|^2 (raw observations: {raw:.1f})")
    log("   filter                 MSE mean    MSE sd     mean ESS   min ESS    log Z - Kalman (mean, sd)")
    variants = [(f"r={r} one stage", dict(radix=r)) for r in (2, 4, 32, 64)]
    variants += [("global (r=N)", dict(radix=N))]
    variants += [(f"r={r} all stages", dict(radix=r, full_cycle=True)) for r in (2, 32, 64)]
    variants += [("r=64 ESS-gated 0.5", dict(radix=64, ess_threshold=0.5)),
                 ("islands M=1024", dict(radix=2, island=1024))]
    out = {}
    for name, kw in variants:
        mses, ess_mean, ess_min, dlz = [], [], [], []
        for s in seeds:
            kw2 = dict(kw)
            f = Filter(model, N, kw2.pop("radix"), seed=1000 + s, history=T, **kw2)
            f.run(yd.data_ptr(), T, model.d)
            h = f.history(T)
            f.close()
            m = np.array([x["mean"] for x in h])
            e = np.array([x["ess"] for x in h])
            mses.append(float(np.sum((m - kf["mean"]) ** 2)))
            ess_mean.append(float(np.mean(e)))
            ess_min.append(float(np.min(e)))
            dlz.append(h[-1]["log_norm"] - kf["loglik"])
        out[name] = float(np.mean(mses))
        log(f"   {name:21s}  {np.mean(mses):10.4f}  {np.std(mses):9.4f}  {np.mean(ess_mean):9.2e}  "
            f"{np.min(ess_min):9.2e}   {np.mean(dlz):+9.2f} {np.std(dlz):7.2f}")
    assert all(np.isfinite(v) for v in out.values()), out
    # the global filter is close to exact
    assert out["global (r=N)"] < 0.01 * raw, out
