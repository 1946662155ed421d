"""Pins of the island-filter oracle (AIRPF, Algorithms 4-7).

* one island stage with the no-swap rule has the pair law printed in the
  proof of Proposition 7 (appendix D): lower member keeps its sample with
  probability p_l^2 + 2 p_l p_r and takes the partner's with p_r^2;
* the full island resampling (Algorithm 6, and Algorithm 7) leaves every
  input island with expected copies m V_j / sum V (the island analogue of
  Proposition 1), by exact enumeration and by sampling;
* the no-swap rule changes only where a sample sits, never the multiset of
  samples of a pair, and the carried weights are those of Algorithm 6;
* within-island resampling carries the island mean of g (eq. ``out
  weight``) and never leaves the island;
* with one island (M = N) the filter is the plain bootstrap filter, bit for
  bit (Algorithms 1 and 2);
* on a linear-Gaussian model the filter means agree with the Kalman filter
  within Monte Carlo error.
"""
import numpy as np
import pytest

import workloads as W
from oracle import bpf, kalman
from oracle.butterfly import State, group_resample
from oracle.island import (IslandOracle, island_expected_counts, island_resample,
                           island_stage, island_uniforms, pair_outcome_law)


@pytest.mark.parametrize("p_lo", [0.5, 0.3, 0.9, 0.01])
def test_pair_law_is_proposition7(p_lo):
    p_r = 1.0 - p_lo
    law = pair_outcome_law(p_lo, no_swap=True)
    keep_lo = law.get(("lo", "hi"), 0.0) + law.get(("lo", "lo"), 0.0)
    take_lo = law.get(("hi", "hi"), 0.0)       # lower island now holds the upper's sample
    keep_hi = law.get(("lo", "hi"), 0.0) + law.get(("hi", "hi"), 0.0)
    take_hi = law.get(("lo", "lo"), 0.0)       # upper island now holds the lower's sample
    assert abs(keep_lo - (p_lo ** 2 + 2 * p_r * p_lo)) < 1e-15
    assert abs(take_lo - p_r ** 2) < 1e-15
    assert abs(keep_hi - (p_r ** 2 + 2 * p_r * p_lo)) < 1e-15
    assert abs(take_hi - p_lo ** 2) < 1e-15
    assert ("hi", "lo") not in law              # a pure exchange never happens


@pytest.mark.parametrize("a,b", [(1.0, 1.0), (0.3, 0.7), (2.0, 0.05)])
def test_island_stage_draws_follow_proposition7(a, b):
    """The sampling code itself: one pair per (U_lo, U_hi) on a K x K grid of
    uniforms; the outcome frequencies are the Proposition 7 probabilities up
    to the grid resolution."""
    K = 256
    u = (np.arange(K) + 0.5) / K
    Ulo, Uhi = np.meshgrid(u, u, indexing="ij")
    n = K * K
    lv = np.empty(2 * n)
    lv[0::2], lv[1::2] = np.log(a), np.log(b)
    U = np.empty(2 * n)
    U[0::2], U[1::2] = Ulo.ravel(), Uhi.ravel()
    pick, lv_new, _ = island_stage(lv, U, 0, no_swap=True)
    lo_idx = np.arange(0, 2 * n, 2)
    keep_lo = np.mean(pick[lo_idx] == lo_idx)
    take_hi = np.mean(pick[lo_idx + 1] == lo_idx)
    p_l = a / (a + b)
    p_r = 1.0 - p_l
    tol = 2.5 / K
    assert abs(keep_lo - (p_l ** 2 + 2 * p_r * p_l)) < tol
    assert abs(take_hi - p_l ** 2) < tol
    assert np.all(np.abs(lv_new - np.log((a + b) / 2)) < 1e-14)
    # no pure exchange survives
    assert not np.any((pick[lo_idx] == lo_idx + 1) & (pick[lo_idx + 1] == lo_idx))


@pytest.mark.parametrize("no_swap", [True, False])
@pytest.mark.parametrize("V", [[1.0, 2.0], [0.5, 1.5, 0.25, 3.0], [1.0, 1e-3, 2.0, 0.7]])
def test_island_resampling_unbiased_exact(no_swap, V):
    V = np.asarray(V)
    m = V.size
    counts = island_expected_counts(np.log(V), no_swap=no_swap)
    assert np.allclose(counts, m * V / V.sum(), rtol=1e-12, atol=1e-12)
    assert abs(counts.sum() - m) < 1e-12


def test_island_resampling_unbiased_sampled():
    """m = 16 islands, Algorithm 7, over many seeds: mean copies within
    sampling error of m V_j / sum V; every carried weight is the global mean."""
    rng = np.random.Generator(np.random.PCG64(7))
    m = 16
    lv = rng.standard_normal(m)
    V = np.exp(lv)
    reps = 3000
    counts = np.zeros(m)
    for r in range(reps):
        UI = [island_uniforms(r, 5, 1, m, s) for s in range(4)]
        src, lvS = island_resample(lv, UI, no_swap=True)
        assert np.allclose(lvS, np.log(V.mean()), rtol=0, atol=1e-12)
        counts += np.bincount(src, minlength=m)
    expect = m * V / V.sum()
    sd = np.sqrt(expect / reps)
    assert np.all(np.abs(counts / reps - expect) <= 5 * sd)


def test_no_swap_keeps_each_pairs_samples_and_weights():
    rng = np.random.Generator(np.random.PCG64(3))
    m = 64
    for trial in range(20):
        lv = rng.standard_normal(m) * 2
        for s in range(6):
            U = rng.random(m)
            p6, lv6, _ = island_stage(lv, U, s, no_swap=False)
            p7, lv7, _ = island_stage(lv, U, s, no_swap=True)
            assert np.array_equal(lv6, lv7)
            lo = np.nonzero((np.arange(m) >> s) & 1 == 0)[0]
            hi = lo + (1 << s)
            for a, b in zip(lo, hi):
                assert sorted((p6[a], p6[b])) == sorted((p7[a], p7[b]))
                assert {p7[a], p7[b]} <= {a, b}
                if (p6[a], p6[b]) == (b, a):
                    assert (p7[a], p7[b]) == (a, b)
                else:
                    assert (p7[a], p7[b]) == (p6[a], p6[b])


@pytest.mark.parametrize("M", [2, 16, 64])
def test_within_island_out_weight_and_locality(M):
    rng = np.random.Generator(np.random.PCG64(M))
    N = 256
    ell = rng.standard_normal(N) * 1.5
    U = rng.random(N)
    anc, lv, _ = group_resample(ell, U, M, 1, "multinomial")
    g = np.exp(ell)
    for k in range(N // M):
        isl = slice(k * M, (k + 1) * M)
        assert np.allclose(lv[isl], np.log(g[isl].mean()), rtol=0, atol=1e-13)
        assert np.all((anc[isl] >= k * M) & (anc[isl] < (k + 1) * M))


@pytest.mark.parametrize("resampler", ["multinomial", "systematic"])
def test_one_island_is_the_plain_bpf(resampler):
    model = W.random_stable_lg(2, 21)
    N, T = 512, 12
    _, ys = W.simulate(model, T, seed=8)
    orc = IslandOracle(model, N, N, resampler, seed=31, stream_id=2)
    st, recs = orc.run(ys, keep=True)
    xb, brecs = bpf.bpf_run(model, N, ys, seed=31, stream_id=2, resampler=resampler, keep=True)
    for a, b in zip(recs, brecs):
        assert np.array_equal(a["origin"], b["ancestors"])
        assert np.array_equal(a["mean"], b["mean"]) and np.array_equal(a["var"], b["var"])
        assert a["ess"] == b["ess"] and a["log_norm"] == b["log_norm"]
    assert np.array_equal(st.x, xb)


def test_step_structure():
    """One step: destination island k holds island src[k]'s within-island
    draws, in order; the output is unweighted; the record's stage count is
    log2 m."""
    model = W.ar1_model()
    N, M = 1024, 32
    orc = IslandOracle(model, N, M, seed=4)
    st = orc.init()
    st1, rec = orc.step(st, np.array([0.3]), keep=True)
    assert rec["stage"] == 5 and rec["radix"] == M
    src, within, origin = rec["src"], rec["within"], rec["origin"]
    for k in range(N // M):
        ks = src[k]
        assert np.array_equal(origin[k * M:(k + 1) * M], within[ks * M:(ks + 1) * M])
        assert np.all(origin[k * M:(k + 1) * M] // M == ks)
    assert np.all(st1.logw == 0.0) and st1.t == 1


def test_island_filter_against_kalman():
    """AR(1): N = 2^12 in 64 islands of 64; over 30 steps the filter means
    stay within a few posterior standard deviations / sqrt(ESS) of the Kalman
    means, and the log-likelihood is close."""
    model = W.ar1_model()
    T = 30
    _, ys = W.simulate(model, T, seed=12)
    kf = kalman.kalman_filter(model, ys)
    orc = IslandOracle(model, 1 << 12, 64, seed=17)
    st, recs = orc.run(ys)
    mu = np.array([r["mean"][0] for r in recs])
    sd = np.sqrt(kf["cov"][:, 0, 0])
    err = np.abs(mu - kf["mean"][:, 0]) / sd
    assert np.max(err) < 0.25, err
    assert abs(recs[-1]["log_norm"] - kf["loglik"]) < 1.0
