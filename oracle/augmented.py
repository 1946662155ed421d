"""Full augmented resampling (Algorithm 3, all S stages in one call), FP64.

TEST INFRASTRUCTURE ONLY: part of the FP64 oracle.

Algorithm 3: ``V_0 = g``; for ``s = 1..S``: ``V_s = A_s V_{s-1}`` and
``xi_s^i`` is drawn from ``sum_j A_s^{ij} V_{s-1}^j delta_{xi_{s-1}^j} / V_s^i``.
Stage ``s`` of the paper is stage ``k = s - 1`` of the digit plan.

``transition_matrices`` gives the exact law of the ancestor chain: stage ``k``
moves particle ``i`` to ancestor ``j`` with probability
``A_k^{ij} V_{k}^j / V_{k+1}^i`` (eq. ``P_in_terms_of_V_proofs``; the weights
are deterministic given the input, Lemma 3(a)). Proposition 1
(eq. ``aug_res_lack_of_bias``) says the composed chain leaves every input
particle ``j`` with expected offspring ``N g_j / sum g``.
"""
from __future__ import annotations

import numpy as np

from .butterfly import group_resample
from .plan import interaction_matrix, place_values


def augmented_resample(log_g: np.ndarray, uniforms, plan, resampler="multinomial",
                       detail: bool = False):
    """Run all stages of ``plan`` on input log-weights ``log_g``.

    ``uniforms[k]`` holds the destination uniforms of stage ``k``. Returns
    ``(origin, log V_S)``: ``origin[i]`` is the input particle that final
    particle ``i`` copies. With ``detail`` a third item lists, per stage,
    ``(ancestors, margins)`` of that stage's draws (see ``group_resample``).
    """
    N = log_g.shape[0]
    R = place_values(plan)
    origin = np.arange(N)
    lv = np.asarray(log_g, dtype=np.float64)
    stages = []
    for k, r in enumerate(plan):
        anc, lv_new, margin = group_resample(lv, uniforms[k], r, R[k], resampler)
        origin = origin[anc]
        lv = lv_new
        stages.append((anc, margin))
    if detail:
        return origin, lv, stages
    return origin, lv


def carried_weights(g: np.ndarray, plan):
    """``V_0 .. V_S`` from eq. ``V_defn_proofs`` with dense ``A_s``."""
    N = g.shape[0]
    V = [np.asarray(g, dtype=np.float64)]
    for k in range(len(plan)):
        V.append(interaction_matrix(N, plan, k) @ V[-1])
    return V


def transition_matrices(g: np.ndarray, plan):
    """Exact per-stage ancestor laws ``T_k[i, j] = A_k^{ij} V_k^j / V_{k+1}^i``."""
    N = g.shape[0]
    V = carried_weights(g, plan)
    Ts = []
    for k in range(len(plan)):
        A = interaction_matrix(N, plan, k)
        Ts.append(A * V[k][None, :] / V[k + 1][:, None])
    return Ts


def expected_offspring_enumerated(g: np.ndarray, plan):
    """Expected number of final copies of each input particle, by brute-force
    enumeration of every ancestor path (all choices of all particles at all
    stages, weighted by their probabilities). Exponential: tiny ``N`` only."""
    N = g.shape[0]
    Ts = transition_matrices(g, plan)
    # paths as a product of independent per-particle choices per stage: the
    # expectation of counts is linear, so enumerate per final particle the
    # sequences (j_S, ..., j_1) explicitly.
    counts = np.zeros(N)
    S = len(plan)

    def walk(i, k, prob):
        if k < 0:
            counts[i] += prob
            return
        for j in np.nonzero(Ts[k][i])[0]:
            walk(j, k - 1, prob * Ts[k][i, j])

    for i in range(N):
        walk(i, S - 1, 1.0)
    return counts
