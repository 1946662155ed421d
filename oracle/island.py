"""Augmented island resampling particle filter (AIRPF), FP64.

TEST INFRASTRUCTURE ONLY: part of the FP64 oracle.

Section 4 of the paper, Algorithms 4-7. The N = m M particles form m islands
of M consecutive particles (island k holds particles kM .. kM + M - 1; m and
M powers of two). One time step t with observation y_t (Algorithm 4):

1. Weight. The cloud is unweighted at the start of a step (the previous
   step ended with a full island resampling), so l_i = log g(x_i, y_t). The
   estimate and the log-normaliser increment come from this weighted cloud
   before resampling, exactly as in the butterfly filter.
2. Within-island resampling (Algorithm 5, A = I_m (x) 1_{1/M}). Each island
   draws M particles from its own M with probabilities proportional to g,
   and every output particle of island k carries the island mean of g
   (eq. ``out weight``). This is one group stage of radix M and stride 1.
3. Augmented island resampling (Algorithm 6, A_s = I (x) 1_{1/2} (x) I).
   S_I = log2 m stages over islands. At stage s (0-based here; s + 1 in the
   paper) island i is paired with island i XOR 2^s. Both carry the mean of
   the pair's weights, and each draws the island sample it holds next (its
   own or its partner's) with probability proportional to the previous
   weights. Whole islands are copied; no particle inside an island is
   chosen. With the modification of Algorithm 7 (the default), a pair whose
   two draws would exchange their samples keeps both in place.
4. Mutation of every particle. After the last island stage every island
   carries the global mean weight, so the new cloud is unweighted again.

Random numbers (readings of the paper, which fixes no generator):
* within-island draws use each particle's ordinary resampling uniform of
  step t (``philox.resample_uniforms`` at tau = t + 1);
* island draws use ``island_uniforms``: island i at stage s takes word
  i mod 4 of the Philox block with counter (floor(i / 4), tau,
  ISLAND_BLOCK + s, stream id), as a 24-bit uniform;
* the propagation uses the step's normals (``philox.normals`` at tau).
"""
from __future__ import annotations

import numpy as np

from . import models, philox
from .butterfly import MULTINOMIAL, State, group_resample, weighted_estimate

ISLAND_BLOCK = 1 << 16   # counter word 2 of the island-stage uniforms (particle blocks are < 2^16)
LN2 = float(np.log(2.0))


def island_uniforms(seed: int, stream_id: int, tau: int, m: int, stage: int) -> np.ndarray:
    """Uniform of island ``i < m`` at island stage ``stage`` of the step with
    counter word ``tau``."""
    k0, k1 = philox.seed_key(seed)
    q = np.arange((m + 3) // 4, dtype=np.uint64)
    w = np.stack(philox.philox4x32_10(q, tau, ISLAND_BLOCK + stage, stream_id, k0, k1), axis=1)
    return philox.word_to_uniform(w.reshape(-1)[:m])


def island_stage(lv: np.ndarray, U: np.ndarray, s: int, no_swap: bool = True):
    """One stage of augmented island resampling (Algorithm 6, stage s + 1;
    with ``no_swap`` the rule of Algorithm 7).

    ``lv``: log island weights V_s (length m); ``U``: one uniform per island.
    Returns ``(pick, lv_new, margin)``: island i holds, after the stage, the
    sample island ``pick[i]`` held before it (i itself or its partner); every
    member of a pair carries log((V_lo + V_hi) / 2); ``margin`` is the
    distance of each draw's target from the pair's cut point, relative to
    the pair total.
    """
    m = lv.shape[0]
    # the pair draw is one butterfly group of radix 2 and stride 2^s
    pick, lv_new, margin = group_resample(lv, U, 2, 1 << s, MULTINOMIAL)
    if no_swap:
        lo = np.nonzero((np.arange(m) >> s) & 1 == 0)[0]
        hi = lo + (1 << s)
        swap = (pick[lo] == hi) & (pick[hi] == lo)
        pick = pick.copy()
        pick[lo[swap]] = lo[swap]
        pick[hi[swap]] = hi[swap]
    return pick, lv_new, margin


def island_resample(lvI: np.ndarray, uniforms, no_swap: bool = True, detail: bool = False):
    """All S_I = log2 m stages (Algorithm 6 or 7) on island log-weights.

    ``uniforms[s]`` holds the island uniforms of stage s. Returns
    ``(src, lv_S)``: destination island k holds the sample of input island
    ``src[k]``. With ``detail`` a third item lists ``(pick, margin)`` per
    stage.
    """
    m = lvI.shape[0]
    S_I = m.bit_length() - 1
    if 1 << S_I != m:
        raise ValueError("the island count must be a power of two")
    src = np.arange(m)
    lv = np.asarray(lvI, dtype=np.float64)
    stages = []
    for s in range(S_I):
        pick, lv, margin = island_stage(lv, uniforms[s], s, no_swap)
        src = src[pick]
        stages.append((pick, margin))
    if detail:
        return src, lv, stages
    return src, lv


def pair_outcome_law(p_lo: float, no_swap: bool = True):
    """Law of one pair stage by enumeration of the two independent draws:
    island lo keeps its sample with probability ``p_lo`` (else takes hi's),
    island hi takes lo's with probability ``p_lo`` (else keeps its own).
    Returns ``{(sample at lo, sample at hi): probability}`` with samples
    named "lo" and "hi"."""
    law = {}
    for a_lo, pa in (("lo", p_lo), ("hi", 1.0 - p_lo)):
        for a_hi, pb in (("lo", p_lo), ("hi", 1.0 - p_lo)):
            out = (a_lo, a_hi)
            if no_swap and out == ("hi", "lo"):
                out = ("lo", "hi")
            law[out] = law.get(out, 0.0) + pa * pb
    return law


def island_expected_counts(lvI: np.ndarray, no_swap: bool = True) -> np.ndarray:
    """Expected number of destination islands holding each input island's
    sample after all stages, by enumeration of every draw of every stage
    (the draws of stage s go through ``island_stage`` with uniforms 0 or
    1 - 2^-24, i.e. the lower or the upper member). Exponential in m log m:
    tiny m only."""
    m = lvI.shape[0]
    S_I = m.bit_length() - 1
    counts = np.zeros(m)
    u_lo, u_hi = 0.0, 1.0 - 2.0 ** -24

    def walk(s, src, lv, prob):
        if s == S_I:
            np.add.at(counts, src, prob)
            return
        mx = np.maximum(lv, lv[np.arange(m) ^ (1 << s)])
        p_self_lo = np.exp(lv - mx)  # unnormalised, per island
        for code in range(1 << m):
            U = np.array([u_hi if (code >> i) & 1 else u_lo for i in range(m)])
            pr = 1.0
            for i in range(m):
                lo = i & ~(1 << s)
                hi = lo | (1 << s)
                plo = p_self_lo[lo] / (p_self_lo[lo] + p_self_lo[hi])
                pr *= (1.0 - plo) if (code >> i) & 1 else plo
            if pr == 0.0:
                continue
            pick, lv_new, _ = island_stage(lv, U, s, no_swap)
            walk(s + 1, src[pick], lv_new, prob * pr)

    walk(0, np.arange(m), np.asarray(lvI, dtype=np.float64), 1.0)
    return counts


class IslandOracle:
    """Augmented island resampling particle filter (Algorithm 4), FP64."""

    def __init__(self, model, N: int, M: int, resampler: str = MULTINOMIAL,
                 seed: int = 0, stream_id: int = 0, no_swap: bool = True):
        """``M`` particles per island (power of two, 2 <= M <= N); ``no_swap``
        selects Algorithm 7 (else Algorithm 6) for the island stages."""
        self.model = model
        self.N = int(N)
        self.M = int(M)
        if self.N % self.M or self.M < 2 or self.M & (self.M - 1) or self.N & (self.N - 1):
            raise ValueError("N and M must be powers of two with 2 <= M <= N")
        self.m = self.N // self.M
        self.S_I = self.m.bit_length() - 1
        self.resampler = resampler
        self.seed = int(seed)
        self.stream_id = int(stream_id)
        self.no_swap = bool(no_swap)

    def init(self) -> State:
        """Algorithm 4, initialisation: x_0 ~ pi_0 from the tau = 0 normals."""
        z = philox.normals(self.seed, self.stream_id, 0, self.N, self.model.d)
        x = models.sample_prior(self.model, z)
        return State(x=x, logw=np.zeros(self.N), t=0, log_norm=0.0)

    def step(self, st: State, y, keep=True):
        """One AIRPF step with observation ``y``; returns ``(state, record)``.
        ``st.logw`` may be non-zero (a state set from outside): it enters the
        weights as in the butterfly filter; the output is unweighted."""
        t = st.t
        tau = t + 1
        ell = st.logw + models.log_g(self.model, st.x, y)
        est = weighted_estimate(st.x, ell, st.logw)
        U = philox.resample_uniforms(self.seed, self.stream_id, tau, self.N)
        # Algorithm 5: one group of M consecutive particles per island
        anc_w, lv_w, margin_w = group_resample(ell, U, self.M, 1, self.resampler)
        lvI = lv_w[::self.M]
        UI = [island_uniforms(self.seed, self.stream_id, tau, self.m, s) for s in range(self.S_I)]
        src, lvS, stages = island_resample(lvI, UI, self.no_swap, detail=True)
        # destination particle kM + j copies particle j of island src[k]
        # after its within-island draw
        k = np.arange(self.N) // self.M
        j = np.arange(self.N) % self.M
        origin = anc_w[src[k] * self.M + j]
        z = philox.normals(self.seed, self.stream_id, tau, self.N, self.model.d)
        x = models.propagate(self.model, st.x[origin], z)
        log_norm = st.log_norm + est["dlog"]
        rec = dict(t=t, stage=self.S_I, radix=self.M, mean=est["mean"], var=est["var"],
                   ess=est["ess"], log_norm=log_norm, max_ell=est["max_ell"])
        if keep:
            rec.update(origin=origin, within=anc_w, margin=margin_w, island_lv=lvI,
                       src=src, island_stages=stages, ell=ell)
        return State(x=x, logw=np.zeros(self.N), t=t + 1, log_norm=log_norm), rec

    def run(self, ys, keep=False, state: State | None = None):
        st = self.init() if state is None else state
        recs = []
        for y in ys:
            st, rec = self.step(st, y, keep=keep)
            recs.append(rec)
        return st, recs
