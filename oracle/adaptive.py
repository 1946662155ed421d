"""Butterfly filter with ESS-gated stages and a rotating start, FP64.

TEST INFRASTRUCTURE ONLY: part of the FP64 oracle.

Section 1.2 of the paper (the "fully adapted" scheme) evaluates the
effective sample size before resampling and after every stage of augmented
resampling, and goes on to the next stage only while it is below a
threshold theta in (1/N, 1]. Section 6.4 proposes starting each time step's
resampling at the stage after the last one executed, instead of always at
the first. One time step t with observation y_t:

1. l = logW + log g(x, y_t); the estimate and the log-normaliser increment
   of the weighted cloud, as in the butterfly filter;
2. E = ESS(l) = (sum w)^2 / (N sum w^2) with w = exp(l - max l);
3. while E < theta and fewer than S stages ran: run stage k (the group
   resampling of Algorithm 3 with the group means carried, eq.
   ``V_defn_proofs``), then k <- (k + 1) mod S and E <- ESS of the carried
   weights; the j-th stage run of the step draws the uniforms of
   ``philox.stage_uniforms`` (j = 0: the step's own);
4. the next step starts at the stage after the last one run (unchanged if
   none ran); gather, carry the weights, propagate with the step's normals.

After S stages every weight is the global mean (ESS = 1), so a step runs at
most S stages; theta = 1 runs all S every step (starting at 0 each time:
the rotation returns to its start), which is the full-cycle filter.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import models, philox
from .butterfly import MULTINOMIAL, State, group_resample, weighted_estimate
from .plan import place_values, stage_plan


@dataclass
class AdaptiveState(State):
    next_stage: int = 0     # the stage the next resampling starts at


def ess(lv: np.ndarray) -> float:
    """(sum w)^2 / (N sum w^2) of log-weights ``lv`` (Section 1.2)."""
    w = np.exp(lv - np.max(lv))
    return float(np.sum(w) ** 2 / (lv.shape[0] * np.sum(w * w)))


class AdaptiveOracle:
    """Butterfly filter whose stages are gated by the ESS (FP64)."""

    def __init__(self, model, N: int, radix: int, theta: float, resampler: str = MULTINOMIAL,
                 seed: int = 0, stream_id: int = 0):
        self.model = model
        self.N = int(N)
        self.radix = int(radix)
        self.theta = float(theta)
        self.plan = stage_plan(self.N, self.radix)
        self.R = place_values(self.plan)
        self.resampler = resampler
        self.seed = int(seed)
        self.stream_id = int(stream_id)

    @property
    def S(self) -> int:
        return len(self.plan)

    def init(self) -> AdaptiveState:
        z = philox.normals(self.seed, self.stream_id, 0, self.N, self.model.d)
        x = models.sample_prior(self.model, z)
        return AdaptiveState(x=x, logw=np.zeros(self.N), t=0, log_norm=0.0, next_stage=0)

    def step(self, st: AdaptiveState, y, keep=True):
        t = st.t
        tau = t + 1
        ell = st.logw + models.log_g(self.model, st.x, y)
        est = weighted_estimate(st.x, ell, st.logw)
        lv = ell
        origin = np.arange(self.N)
        k = st.next_stage
        e = ess(lv)
        essays = [e]
        run = []
        draws = []
        while e < self.theta and len(run) < self.S:
            U = philox.stage_uniforms(self.seed, self.stream_id, tau, self.N, len(run))
            anc, lv, margin = group_resample(lv, U, self.plan[k], self.R[k], self.resampler)
            origin = origin[anc]
            draws.append((anc, margin))
            run.append(k)
            k = (k + 1) % self.S
            e = ess(lv)
            essays.append(e)
        nxt = (run[-1] + 1) % self.S if run else st.next_stage
        xhat = st.x[origin]
        logw = lv - np.max(lv)
        z = philox.normals(self.seed, self.stream_id, tau, self.N, self.model.d)
        x = models.propagate(self.model, xhat, z)
        log_norm = st.log_norm + est["dlog"]
        rec = dict(t=t, stage=len(run), radix=self.radix, stages_run=run, ess_trace=essays,
                   mean=est["mean"], var=est["var"], ess=est["ess"], log_norm=log_norm,
                   max_ell=est["max_ell"])
        if keep:
            rec.update(origin=origin, stages=draws, ell=ell, logw_new=lv)
        return AdaptiveState(x=x, logw=logw, t=t + 1, log_norm=log_norm, next_stage=nxt), rec

    def run(self, ys, keep=False, state: AdaptiveState | None = None):
        st = self.init() if state is None else state
        recs = []
        for y in ys:
            st, rec = self.step(st, y, keep=keep)
            recs.append(rec)
        return st, recs
