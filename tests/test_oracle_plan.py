"""Pins of the stage plan and butterfly groups against the paper's printed
examples (Figures 1 and 2), Lemma 1, Lemma 2 and the Kronecker definition."""
import itertools

import numpy as np
import pytest

from oracle import plan as P
from tests.conftest import read_golden


def test_fig2_pairs_m8():
    """Figure 2: radix-2 stage groups of m = 8 equal the drawn PE pairs."""
    rows = read_golden("fig2_pairs_m8.txt")
    pl = P.stage_plan(8, 2)
    assert pl == [2, 2, 2]
    for row in rows:
        s = int(row[0])
        pairs = sorted(tuple(int(v) - 1 for v in p.split("-")) for p in row[1:])
        got = sorted(tuple(int(v) for v in g) for g in P.groups(8, pl, s - 1))
        assert got == pairs


def test_fig1_matrices_m4_M3():
    """Figure 1: printed A_1, A_2 for m = 4 PEs of M = 3 particles."""
    rows = read_golden("fig1_A_m4_M3.txt")
    M = 3
    for row in rows:
        s = int(row[0])
        pattern = np.array([[int(ch) for ch in blk] for blk in row[1:]], dtype=float)
        printed = 0.5 * np.kron(pattern, np.full((M, M), 1.0 / M))
        assert np.allclose(P.block_interaction_matrix(4, M, 2, s - 1), printed, atol=0)
        assert np.allclose(P.paper_A(s, 2, M), printed, atol=0)
        assert np.all(np.isin(printed, [0.0, 1.0 / (2 * M)]))


@pytest.mark.parametrize("S,M", [(1, 1), (2, 1), (3, 1), (3, 2), (4, 3)])
def test_radix2_matches_kronecker_definition(S, M):
    """eq. A matrices: the digit-formula groups reproduce the Kronecker A_s."""
    m = 2 ** S
    for s in range(1, S + 1):
        A = P.paper_A(s, S, M)
        if M == 1:
            B = P.interaction_matrix(m, P.stage_plan(m, 2), s - 1)
        else:
            B = P.block_interaction_matrix(m, M, 2, s - 1)
        assert np.array_equal(A, B)


@pytest.mark.parametrize("S", [1, 2, 3, 4, 5])
def test_lemma1_explicit_nonzeros(S):
    """Lemma 1, eq. explicit nonzero elements (1-based): the two nonzero
    columns of row i at stage s."""
    m = 2 ** S
    pl = P.stage_plan(m, 2)
    for s in range(1, S + 1):
        for i in range(1, m + 1):
            want = {((i - 1) % 2 ** (s - 1)) + (q - 1) * 2 ** (s - 1)
                    + 2 ** s * ((i - 1) // 2 ** s) + 1 for q in (1, 2)}
            got = {int(j) + 1 for j in P.group_members(i - 1, m, pl, s - 1)}
            assert got == want


PLANS = [(N, r) for N in (2, 4, 8, 16, 32, 64) for r in (2, 4, 8, 16, 32, 64)]


@pytest.mark.parametrize("N,r", PLANS)
def test_lemma1_properties_and_partition(N, r):
    """Lemma 1: every A_k is symmetric, idempotent, doubly stochastic with
    diagonal 1/r_k; each stage's groups partition {0..N-1} (incl. mixed radix)."""
    pl = P.stage_plan(N, r)
    assert int(np.prod(pl)) == N
    for k in range(len(pl)):
        A = P.interaction_matrix(N, pl, k)
        assert np.array_equal(A, A.T)
        assert np.allclose(A @ A, A, atol=1e-15)
        assert np.allclose(A.sum(0), 1) and np.allclose(A.sum(1), 1)
        assert np.allclose(np.diag(A), 1.0 / pl[k])
        g = P.groups(N, pl, k)
        assert g.shape == (N // pl[k], pl[k])
        assert np.array_equal(np.sort(g.ravel()), np.arange(N))
        assert np.all(np.diff(g, axis=1) == P.place_values(pl)[k])
        for i in range(N):
            assert sorted(P.group_members(i, N, pl, k)) == sorted(g[np.any(g == i, axis=1)][0])


@pytest.mark.parametrize("N,r", PLANS)
def test_lemma2_products(N, r):
    """Lemma 2 and its proof's partial products: prod_{j<=k} A_j is
    block-diagonal with blocks 1_{1/R_{k+1}}; the full cycle is 1_{1/N}."""
    pl = P.stage_plan(N, r)
    R = P.place_values(pl) + [N]
    prod = np.eye(N)
    for k in range(len(pl)):
        prod = P.interaction_matrix(N, pl, k) @ prod
        blk = R[k + 1]
        want = np.kron(np.eye(N // blk), np.full((blk, blk), 1.0 / blk))
        assert np.allclose(prod, want, atol=1e-14)
    assert np.allclose(prod, np.full((N, N), 1.0 / N), atol=1e-14)


def test_mixed_radix_plans():
    assert P.stage_plan(1 << 20, 64) == [64, 64, 64, 4]
    assert P.stage_plan(1 << 20, 32) == [32] * 4
    assert P.stage_plan(1 << 20, 4) == [4] * 10
    assert P.stage_plan(1 << 24, 32) == [32] * 4 + [16]
    assert P.stage_plan(1 << 24, 1024) == [1024, 1024, 16]
    assert P.stage_plan(1 << 24, 256) == [256, 256, 256]
    assert P.stage_plan(1024, 1024) == [1024]
    assert P.stage_plan(1024, 4096) == [1024]
    for bad in [(3, 2), (1, 2), (8, 3), (8, 1)]:
        with pytest.raises(ValueError):
            P.stage_plan(*bad)


def test_stage_rotation():
    pl = [64, 64, 64, 4]
    assert [P.stage_of_step(t, pl) for t in range(9)] == [0, 1, 2, 3, 0, 1, 2, 3, 0]
