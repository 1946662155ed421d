"""Pins of the oracle's effective sample size.

Section 1.2 defines the ESS of the bootstrap filter as the squared mean of
the weights over their mean square, and states its range: it lies in
[1/N, 1]. Both ends are attained: equal weights give 1 and a single
surviving particle gives 1/N. The checks below fix the value from facts that
do not restate the formula:

* the two ends of the range, exactly;
* k equal surviving weights among N give k/N;
* the identity ESS = 1 / (1 + CV^2), with CV^2 the population variance of
  the weights over their squared mean (computed by ``numpy.var``);
* invariance to a common factor on the weights (a shift of every
  log-weight);
* the range on random weights.

A dropped or doubled 1/N, a square on the wrong sum, or a missing
normalisation fails the first three. Each check runs on the two oracle
functions that report an ESS: ``weighted_estimate`` (the estimate record of
every filter) and ``adaptive.ess`` (the stage decisions of the ESS-gated
filter).
"""
import numpy as np
import pytest

from oracle.adaptive import ess as adaptive_ess
from oracle.butterfly import weighted_estimate


def _ess_estimate(ell):
    N = ell.shape[0]
    x = np.zeros((N, 1))
    return weighted_estimate(x, ell, np.zeros(N))["ess"]


ESS_FUNCS = [pytest.param(_ess_estimate, id="weighted_estimate"),
             pytest.param(adaptive_ess, id="adaptive.ess")]


@pytest.mark.parametrize("f", ESS_FUNCS)
@pytest.mark.parametrize("N", [1, 2, 7, 64, 4096])
def test_equal_weights_give_one(f, N):
    for level in (0.0, -3.5, 250.0):
        assert f(np.full(N, level)) == pytest.approx(1.0, rel=1e-14, abs=0)


@pytest.mark.parametrize("f", ESS_FUNCS)
@pytest.mark.parametrize("N", [2, 8, 1000, 4096])
def test_one_survivor_gives_one_over_n(f, N):
    # exp(-1e4) is exactly 0 in FP64: one particle carries all the weight
    ell = np.full(N, -1.0e4)
    ell[N // 3] = 1.25
    assert f(ell) == pytest.approx(1.0 / N, rel=1e-14, abs=0)


@pytest.mark.parametrize("f", ESS_FUNCS)
def test_k_survivors_give_k_over_n(f):
    rng = np.random.default_rng(4)
    for N in (16, 512, 4096):
        for k in (1, 2, 3, N // 4, N - 1, N):
            ell = np.full(N, -1.0e4)
            ell[rng.choice(N, size=k, replace=False)] = -0.75
            assert f(ell) == pytest.approx(k / N, rel=1e-13, abs=0), (N, k)


@pytest.mark.parametrize("f", ESS_FUNCS)
def test_coefficient_of_variation_identity(f):
    rng = np.random.default_rng(11)
    for N in (3, 100, 4096):
        for spread in (0.1, 1.0, 4.0):
            ell = rng.normal(0.0, spread, size=N)
            w = np.exp(ell)
            cv2 = np.var(w) / np.mean(w) ** 2
            assert f(ell) == pytest.approx(1.0 / (1.0 + cv2), rel=1e-12), (N, spread)


@pytest.mark.parametrize("f", ESS_FUNCS)
def test_scale_invariance_and_range(f):
    rng = np.random.default_rng(12)
    for N in (2, 33, 4096):
        ell = rng.normal(0.0, 3.0, size=N)
        e = f(ell)
        assert 1.0 / N - 1e-15 <= e <= 1.0 + 1e-15
        assert f(ell + 123.0) == pytest.approx(e, rel=1e-12)
        assert f(ell - 40.0) == pytest.approx(e, rel=1e-12)


def test_two_level_weights():
    """Weights a on k particles and b on the rest: with b = a / 2 and
    k = N / 2 the mean is 3a/4 and the mean square 5a^2/8, so ESS = 9/10."""
    N = 1024
    ell = np.zeros(N)
    ell[N // 2:] = np.log(0.5)
    assert _ess_estimate(ell) == pytest.approx(0.9, rel=1e-14)
    assert adaptive_ess(ell) == pytest.approx(0.9, rel=1e-14)
