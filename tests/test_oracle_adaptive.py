"""Pins of the ESS-gated butterfly oracle (Section 1.2, rotation of Section 6.4).

* theta = 1 runs every stage every step, starting at stage 0: the full-cycle
  filter (all S stages of Algorithm 3), bit for bit;
* theta <= 1/N never resamples: sequential importance sampling, written out
  here as the plain recursion (propagate every particle, add log g);
* for intermediate theta every step obeys the stop rule (the ESS before each
  executed stage was below theta; after the last one it is at least theta or
  S stages ran) and the rotation (a step starts at the stage after the last
  one executed; steps without resampling leave it unchanged);
* on an AR(1) model the filter means agree with the Kalman filter.
"""
import numpy as np
import pytest

import workloads as W
from oracle import ButterflyOracle, kalman, models, philox
from oracle.adaptive import AdaptiveOracle, ess


@pytest.mark.parametrize("N,r", [(64, 4), (1024, 32), (512, 2)])
def test_theta_one_is_the_full_cycle_filter(N, r):
    model = W.random_stable_lg(2, 5)
    _, ys = W.simulate(model, 7, seed=2)
    a = AdaptiveOracle(model, N, r, 1.0, seed=13, stream_id=4)
    b = ButterflyOracle(model, N, r, seed=13, stream_id=4, full_cycle=True)
    sa, ra = a.run(ys, keep=True)
    sb, rb = b.run(ys, keep=True)
    for x, y in zip(ra, rb):
        assert x["stage"] == a.S and x["stages_run"] == list(range(a.S))
        assert np.array_equal(x["origin"], y["origin"])
        assert np.array_equal(x["mean"], y["mean"]) and x["log_norm"] == y["log_norm"]
    assert np.array_equal(sa.x, sb.x) and np.array_equal(sa.logw, sb.logw)


def test_tiny_theta_is_sequential_importance_sampling():
    model = W.ar1_model()
    N, T = 256, 9
    _, ys = W.simulate(model, T, seed=3)
    orc = AdaptiveOracle(model, N, 4, 0.5 / N, seed=8, stream_id=1)
    st, recs = orc.run(ys)
    # the plain recursion: no particle ever changes its ancestry
    x = models.sample_prior(model, philox.normals(8, 1, 0, N, model.d))
    lw = np.zeros(N)
    ln = 0.0
    for t, y in enumerate(ys):
        lg = models.log_g(model, x, y)
        l = lw + lg
        ln += np.log(np.sum(np.exp(l))) - np.log(np.sum(np.exp(lw)))
        lw = l - l.max()
        x = models.propagate(model, x, philox.normals(8, 1, t + 1, N, model.d))
        assert recs[t]["stage"] == 0
    assert np.allclose(st.x, x, rtol=0, atol=1e-12)
    assert np.allclose(st.logw, lw, rtol=0, atol=1e-9)
    assert abs(st.log_norm - ln) < 1e-9


@pytest.mark.parametrize("theta", [0.3, 0.6, 0.9])
def test_stop_rule_and_rotation(theta):
    model = W.random_stable_lg(3, 17)
    N, r, T = 4096, 4, 25
    _, ys = W.simulate(model, T, seed=11)
    orc = AdaptiveOracle(model, N, r, theta, seed=2)
    st = orc.init()
    nxt = 0
    total = 0
    for y in ys:
        st, rec = orc.step(st, y, keep=True)
        run, tr = rec["stages_run"], rec["ess_trace"]
        assert len(tr) == len(run) + 1 and len(run) <= orc.S
        assert all(e < theta for e in tr[:-1])
        assert tr[-1] >= theta or len(run) == orc.S
        if run:
            assert run == [(nxt + j) % orc.S for j in range(len(run))]
            nxt = (run[-1] + 1) % orc.S
        assert st.next_stage == nxt
        assert abs(ess(rec["logw_new"]) - tr[-1]) < 1e-12
        total += len(run)
    assert 0 < total < T * orc.S


def test_adaptive_filter_against_kalman():
    model = W.ar1_model()
    T = 40
    _, ys = W.simulate(model, T, seed=21)
    kf = kalman.kalman_filter(model, ys)
    orc = AdaptiveOracle(model, 1 << 12, 8, 0.5, seed=5)
    _, recs = orc.run(ys)
    mu = np.array([r["mean"][0] for r in recs])
    sd = np.sqrt(kf["cov"][:, 0, 0])
    assert np.max(np.abs(mu - kf["mean"][:, 0]) / sd) < 0.25
    assert abs(recs[-1]["log_norm"] - kf["loglik"]) < 1.0
