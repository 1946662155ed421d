"""Butterfly stage plan and interaction groups.

TEST INFRASTRUCTURE ONLY: part of the FP64 oracle.

Section 1.2, eq. ``A matrices``: with ``N = mM`` and ``S = log2 m`` (Assumption
A1) the stage-s interaction matrix is ``I_{2^{S-s}} (x) 1_{1/2} (x) I_{2^{s-1}}
(x) 1_{1/M}``; Lemma 1 (eq. ``explicit nonzero elements``) lists the nonzero
columns of row ``i``: the two indices that agree with ``i`` in every binary
digit except digit ``s - 1``. Remark 1 allows any doubly stochastic family
whose product is ``1_{1/N}``; the radix-r family below replaces ``1_{1/2}``
by ``1_{1/r}``.

Reading used here (particle-level groups, block factor 1): write the particle
index in mixed radix with digits ``delta_k(i) = floor(i / R_k) mod r_k``,
place values ``R_0 = 1``, ``R_{k+1} = R_k r_k``. Stage ``k`` lets the ``r_k``
particles that differ only in digit ``k`` interact:
``G_k(i) = { i + (q - delta_k(i)) R_k : q = 0..r_k-1 }``.
For ``r = 2`` this is Lemma 1's formula with ``s = k + 1`` (0-based indices).

When ``log2 N`` is not a multiple of ``log2 r`` the most significant digit
gets the leftover radix (mixed radix); ``r >= N`` gives one stage with the
whole population as the group (the plain bootstrap filter).
"""
from __future__ import annotations

import numpy as np


def is_pow2(n: int) -> bool:
    return n >= 1 and (n & (n - 1)) == 0


def stage_plan(N: int, radix: int):
    """Radices ``(r_0, ..., r_{S-1})`` with product ``N``.

    ``N`` and ``radix`` must be powers of two, ``N >= 2``, ``radix >= 2``.
    ``radix >= N`` gives the single global stage ``[N]``.
    """
    if not (is_pow2(N) and N >= 2):
        raise ValueError(f"N must be a power of two >= 2, got {N}")
    if not (is_pow2(radix) and radix >= 2):
        raise ValueError(f"radix must be a power of two >= 2, got {radix}")
    if radix >= N:
        return [N]
    b = radix.bit_length() - 1
    n = N.bit_length() - 1
    S = -(-n // b)
    last = n - (S - 1) * b
    return [radix] * (S - 1) + [1 << last]


def place_values(plan):
    R = [1]
    for r in plan[:-1]:
        R.append(R[-1] * r)
    return R


def stage_of_step(t: int, plan) -> int:
    """Stage used at time step ``t``: the stages rotate, ``k = t mod S``."""
    return t % len(plan)


def groups(N: int, plan, k: int) -> np.ndarray:
    """Groups of stage ``k`` as an ``(N / r_k, r_k)`` index array; row ``g``
    lists its members in increasing order (member position ``q`` = digit k)."""
    r = plan[k]
    R = place_values(plan)[k]
    idx = np.arange(N, dtype=np.int64).reshape(N // (r * R), r, R)
    return idx.transpose(0, 2, 1).reshape(N // r, r)


def group_members(i: int, N: int, plan, k: int) -> np.ndarray:
    """``G_k(i)`` from the digit formula, for one index."""
    r = plan[k]
    R = place_values(plan)[k]
    dk = (i // R) % r
    return np.array([i + (q - dk) * R for q in range(r)], dtype=np.int64)


def interaction_matrix(N: int, plan, k: int) -> np.ndarray:
    """Dense ``A_k`` with ``A^{ij} = 1/r_k`` iff ``j`` is in ``G_k(i)``."""
    r = plan[k]
    A = np.zeros((N, N))
    for g in groups(N, plan, k):
        A[np.ix_(g, g)] = 1.0 / r
    return A


def paper_A(s: int, S: int, M: int) -> np.ndarray:
    """The paper's ``A_s`` built literally with Kronecker products
    (eq. ``A matrices``); ``1_{1/k}`` is the k x k matrix of ones over k."""
    ones = lambda k: np.full((k, k), 1.0 / k)
    return np.kron(np.kron(np.kron(np.eye(2 ** (S - s)), ones(2)),
                           np.eye(2 ** (s - 1))), ones(M))


def block_interaction_matrix(m: int, M: int, radix: int, k: int) -> np.ndarray:
    """Stage-k matrix when every processing element holds ``M`` particles
    (index ``i = pe * M + j``): particles interact iff their PE indices are in
    the same PE-level group of stage ``k``; every nonzero entry is
    ``1 / (r_k M)`` (the block reading of Lemma 1)."""
    plan = stage_plan(m, radix)
    r = plan[k]
    R = place_values(plan)[k]
    N = m * M
    A = np.zeros((N, N))
    for i in range(N):
        pe = i // M
        dk = (pe // R) % r
        for q in range(r):
            pe2 = pe + (q - dk) * R
            A[i, pe2 * M:(pe2 + 1) * M] = 1.0 / (r * M)
    return A
