"""Pins of the within-group draw, the carried stage weight and full augmented
resampling: exact enumeration over the 24-bit uniform grid, Lemma 3 and
Proposition 1."""
import numpy as np
import pytest

from oracle import augmented, philox
from oracle import plan as P
from oracle.butterfly import MULTINOMIAL, SYSTEMATIC, group_resample

GRID = 1 << 24


def _weights(r, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    w = rng.gamma(0.7, size=r)
    return w


def _enumerate_multinomial(logw, chunk=1 << 20):
    """Ancestor of destination 0 for every uniform on the 24-bit grid, using
    the oracle's stage routine (one group per grid value)."""
    r = logw.shape[0]
    counts = np.zeros(r, dtype=np.int64)
    for g0 in range(0, GRID, chunk):
        u_grid = np.arange(g0, g0 + chunk, dtype=np.float64) / GRID
        ell = np.tile(logw, chunk)
        U = np.zeros(chunk * r)
        U[0::r] = u_grid
        anc, _, _ = group_resample(ell, U, r, 1, MULTINOMIAL)
        a0 = anc[0::r] - np.arange(chunk) * r
        counts += np.bincount(a0, minlength=r)
    return counts


@pytest.mark.parametrize("r,seed", [(2, 1), (4, 2), (8, 3)])
def test_multinomial_exact_enumeration(r, seed):
    """Over all 2^24 uniforms the draw picks member j with frequency p_j up to
    the grid resolution: E[O_j] = r p_j within r 2^-24."""
    w = _weights(r, seed)
    counts = _enumerate_multinomial(np.log(w))
    p = w / w.sum()
    assert counts.sum() == GRID
    assert np.all(np.abs(counts / GRID - p) <= 1.0 / GRID + 1e-15)
    assert np.all(np.abs(r * counts / GRID - r * p) <= r / GRID + 1e-12)


@pytest.mark.parametrize("r,seed", [(2, 4), (4, 5), (8, 6)])
def test_systematic_exact_enumeration(r, seed):
    """Systematic draw: over all 2^24 values of U_0, O_j is floor or ceil of
    r p_j and E[O_j] = r p_j within r 2^-24."""
    w = _weights(r, seed)
    p = w / w.sum()
    tot = np.zeros(r)
    chunk = 1 << 19
    for g0 in range(0, GRID, chunk):
        u0 = np.arange(g0, g0 + chunk, dtype=np.float64) / GRID
        ell = np.tile(np.log(w), chunk)
        U = np.repeat(u0, r)          # only member 0's uniform is used
        anc, _, _ = group_resample(ell, U, r, 1, SYSTEMATIC)
        j = (anc - np.repeat(np.arange(chunk) * r, r)).reshape(chunk, r)
        O = np.stack([np.sum(j == jj, axis=1) for jj in range(r)], axis=1)
        assert np.all(O.sum(1) == r)
        assert np.all((O == np.floor(r * p)) | (O == np.ceil(r * p)))
        tot += O.sum(0)
    assert np.all(np.abs(tot / GRID - r * p) <= r / GRID + 1e-12)


def test_weighted_unbiasedness_and_new_weight():
    """E[sum_{i in G} W'_i phi(xhat_i)] = sum_j w_j phi(x_j) with W' the
    carried group mean (eq. V_defn_proofs); checked exactly on the grid."""
    r = 4
    w = _weights(r, 9)
    phi = np.array([0.3, -1.2, 2.5, 0.7])
    counts = _enumerate_multinomial(np.log(w))
    _, new_lw, _ = group_resample(np.log(w), np.zeros(r), r, 1, MULTINOMIAL)
    assert np.allclose(np.exp(new_lw), w.mean(), rtol=1e-14)
    lhs = r * np.exp(new_lw[0]) * np.sum(counts / GRID * phi)
    assert abs(lhs - np.sum(w * phi)) <= r * np.max(np.abs(phi)) * w.sum() / GRID * 2


def test_zero_weight_never_chosen():
    r = 8
    ell = np.array([-1e4, 0.0, -1e4, -1e4, 1.0, -1e4, -1e4, -1e4])
    for res in (MULTINOMIAL, SYSTEMATIC):
        for u in (0.0, 0.25, 0.5, 1 - 2 ** -24):
            anc, _, _ = group_resample(ell, np.full(r, u), r, 1, res)
            assert set(anc.tolist()) <= {1, 4}


def test_ancestors_stay_in_group_and_margin():
    N, r = 256, 4
    pl = P.stage_plan(N, r)
    R = P.place_values(pl)
    rng = np.random.Generator(np.random.PCG64(3))
    ell = rng.normal(size=N)
    U = philox.resample_uniforms(1, 0, 1, N)
    for k in range(len(pl)):
        anc, lw, mg = group_resample(ell, U, pl[k], R[k], MULTINOMIAL)
        for g in P.groups(N, pl, k):
            assert set(anc[g].tolist()) <= set(g.tolist())
            assert np.allclose(lw[g], np.log(np.mean(np.exp(ell[g]))), rtol=1e-14)
        assert np.all(mg >= 0) and np.all(mg <= 1)


@pytest.mark.parametrize("N,r", [(8, 2), (16, 2), (64, 4), (64, 8), (32, 8), (1 << 12, 64)])
def test_lemma3_full_cycle_weights(N, r):
    """Lemma 3(c) / eq. V_k_unwind: carrying the group-mean weight through
    one full cycle of stages leaves every particle with the global mean."""
    pl = P.stage_plan(N, r)
    R = P.place_values(pl)
    rng = np.random.Generator(np.random.PCG64(N + r))
    ell0 = rng.normal(scale=2.0, size=N)
    lv = ell0
    for k in range(len(pl)):
        _, lv, _ = group_resample(lv, np.zeros(N), pl[k], R[k], MULTINOMIAL)
    assert np.allclose(lv, np.log(np.mean(np.exp(ell0))), rtol=0, atol=1e-12)
    if N <= 64:
        V = augmented.carried_weights(np.exp(ell0), pl)
        assert np.allclose(V[-1], np.mean(np.exp(ell0)), rtol=1e-12)


@pytest.mark.parametrize("N,r", [(4, 2), (8, 2), (8, 4), (16, 4)])
def test_prop1_unbiased_offspring_by_enumeration(N, r):
    """Proposition 1 (eq. aug_res_lack_of_bias): enumerating every ancestor
    path of full augmented resampling gives E[copies of j] = N g_j / sum g."""
    pl = P.stage_plan(N, r)
    g = _weights(N, 40 + N)
    E = augmented.expected_offspring_enumerated(g, pl)
    assert np.allclose(E, N * g / g.sum(), rtol=1e-12)


def test_augmented_sampler_matches_exact_law():
    """The oracle's Algorithm 3 sampler, run many times, reproduces the exact
    ancestor law within Monte Carlo error."""
    N, r = 8, 2
    pl = P.stage_plan(N, r)
    g = _weights(N, 77)
    Ts = augmented.transition_matrices(g, pl)
    law = np.eye(N)
    for T in Ts:
        law = T @ law          # law[i, j] = P(final i copies input j)
    reps = 1 << 14
    ell = np.tile(np.log(g), reps)
    NN = N * reps
    origin = np.arange(NN)
    lv = ell
    # reps independent copies laid out contiguously: add a high radix digit
    big = P.stage_plan(NN, r)
    Rb = P.place_values(big)
    for k in range(len(pl)):
        U = philox.resample_uniforms(5, 0, k + 1, NN)
        anc, lv, _ = group_resample(lv, U, big[k], Rb[k], MULTINOMIAL)
        origin = origin[anc]
    emp = np.zeros((N, N))
    src = origin.reshape(reps, N) % N
    for i in range(N):
        emp[i] = np.bincount(src[:, i], minlength=N) / reps
    assert np.max(np.abs(emp - law)) < 5 * np.sqrt(0.25 / reps)


def test_stage_uniforms_are_distinct_streams():
    """Stage 0 of a multi-stage step uses the step's ordinary uniforms; every
    later stage draws from its own block, on the same 24-bit grid."""
    u0 = philox.stage_uniforms(3, 1, 7, 64, 0)
    assert np.array_equal(u0, philox.resample_uniforms(3, 1, 7, 64))
    us = [philox.stage_uniforms(3, 1, 7, 64, s) for s in range(4)]
    for a in range(4):
        assert np.all((us[a] * 2 ** 24) == np.floor(us[a] * 2 ** 24))
        for b in range(a):
            assert not np.array_equal(us[a], us[b])


@pytest.mark.parametrize("N,r", [(8, 2), (16, 4), (64, 4), (1 << 10, 32)])
def test_full_cycle_step_leaves_equal_weights_and_unbiased_counts(N, r):
    """One full-cycle step of the filter oracle: after all S stages every
    log-weight is the log of the global mean (Lemma 3(c)); over many seeds
    the copies of each input particle average N g_j / sum g (Proposition 1)."""
    import workloads as W
    from oracle import ButterflyOracle, State
    model = W.ar1_model()
    rng = np.random.Generator(np.random.PCG64(N + r))
    x0 = rng.standard_normal((N, 1))
    lw0 = rng.standard_normal(N) * 0.3
    st = State(x=x0, logw=lw0 - lw0.max(), t=4, log_norm=0.0)
    y = np.array([0.4])
    orc = ButterflyOracle(model, N, r, seed=0, full_cycle=True)
    _, rec = orc.step(st, y, keep=True)
    ell = rec["ell"]
    reps = 400 if N <= 64 else 40
    counts = np.zeros(N)
    for sd in range(reps):
        o = ButterflyOracle(model, N, r, seed=sd, full_cycle=True)
        st1, rr = o.step(st, y, keep=True)
        assert np.max(np.abs(st1.logw)) < 1e-12       # all weights equal
        counts += np.bincount(rr["origin"], minlength=N)
    g = np.exp(ell - ell.max())
    expect = N * g / g.sum()
    sd_ = np.sqrt(np.maximum(expect, 1e-3) / reps)
    assert np.all(np.abs(counts / reps - expect) <= 6 * sd_ + 1e-9)
