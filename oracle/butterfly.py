"""FP64 oracle of the butterfly-interaction bootstrap particle filter.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import this module;
it exists so that tests, the smoke check and the CPU baseline have a slow,
plain reference to compare the device kernels against.

What one time step computes (the steps in the paper's order):

* Algorithm 1 (particle filter): initialise ``zeta_0^i ~ pi_0``; then per step
  resample with ``g_n`` and mutate ``zeta_{n+1}^i ~ f(zeta_hat_n^i, .)``.
* Algorithm 3 (augmented resampling) with one stage per time step: the stage
  weight is ``V_s = A_s V_{s-1}`` (eq. ``V_defn_proofs``: the group mean) and
  each particle draws its ancestor inside its group with probability
  proportional to the previous stage weights (eq. ``P_in_terms_of_V_proofs``).
  The stage rotates with the time step, ``k = t mod S`` (Section 1.2 allows
  stopping after any stage and moving to the next time step; Section 6.4
  proposes rotating the starting stage). The carried stage weight becomes the
  incoming log-weight of the next step.
* ``r >= N`` is one stage whose group is the whole population:
  Algorithm 2 (multinomial resampling) of the plain bootstrap filter.
* ``full_cycle``: every step runs all ``S`` stages of Algorithm 3 instead of
  one (``_step_full``).

Step ``t`` in detail (log domain, FP64):

1. ``l_i = logW_i + log g(x_i, y_t)``
2. estimate before resampling: ``M = max l``, ``w_i = exp(l_i - M)``,
   weighted mean and variance of ``x``, ``ESS = (sum w)^2 / (N sum w^2)``
   (the effective-sample-size form of Section 1.2 applied to ``w``),
   ``Lambda += (M + ln sum w) - ln sum exp(logW)``
3. per group of stage ``k`` (members in increasing index order):
   ``m_G = max l``; ``c_q = sum_{p<=q} exp(l_p - m_G)`` (sequential);
   new log-weight ``m_G + ln c_{r-1} - ln r`` for every member
4. ancestors: destination ``q`` with uniform ``U``; multinomial target
   ``U c_{r-1}``, systematic target ``(q + U_0) c_{r-1} / r`` with ``U_0``
   the uniform of the group's first member; the ancestor is the first ``p``
   with ``c_p > target`` (clamped to ``r - 1``)
5. gather ``xhat_i = x_{a(i)}``; subtract ``max`` of the new log-weights
6. propagate ``x_i = f(xhat_i, z_i)`` with the step's normals.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import models, philox
from .plan import place_values, stage_plan

MULTINOMIAL = "multinomial"
SYSTEMATIC = "systematic"


@dataclass
class State:
    x: np.ndarray          # (N, d) FP64
    logw: np.ndarray       # (N,)   FP64, max == 0
    t: int                 # number of completed steps
    log_norm: float        # running log-normaliser Lambda


def count_le(C: np.ndarray, tgt: np.ndarray) -> np.ndarray:
    """Row-wise ``#{p : C[g, p] <= tgt[g, q]}`` for non-decreasing rows of
    ``C`` (shape ``(G, r)``); ``tgt`` has shape ``(G, r')``."""
    G, r = C.shape
    out = np.empty(tgt.shape, dtype=np.int64)
    if r <= 64:
        step = max(1, (1 << 24) // (r * tgt.shape[1]))
        for g0 in range(0, G, step):
            c = C[g0:g0 + step]
            t = tgt[g0:g0 + step]
            out[g0:g0 + step] = np.sum(c[:, None, :] <= t[:, :, None], axis=2)
    else:
        for g in range(G):
            out[g] = np.searchsorted(C[g], tgt[g], side="right")
    return out


def group_resample(ell: np.ndarray, U: np.ndarray, r: int, R: int, resampler: str,
                   detail: bool = False):
    """One butterfly stage on log-weights ``ell`` (shape ``(N,)``).

    Groups are the ``r`` indices ``h r R + q R + lo`` (``q = 0..r-1``).
    Returns ``(ancestor index (N,), new log-weight (N,), margin (N,))``;
    ``margin`` is the distance from the draw's target to the nearest
    cumulative weight, relative to the group total. With ``detail`` a fourth
    item gives, per destination, the draw's target and the cumulative
    weights bounding every member's interval (``cdf[i, q]`` is
    ``c_q`` of destination i's group), all relative to the group total.
    """
    N = ell.shape[0]
    nh = N // (r * R)
    # (groups, members) view, members in increasing index order
    l2 = ell.reshape(nh, r, R).transpose(0, 2, 1).reshape(-1, r)
    u2 = U.reshape(nh, r, R).transpose(0, 2, 1).reshape(-1, r)
    m = np.max(l2, axis=1, keepdims=True)
    w = np.exp(l2 - m)
    C = np.cumsum(w, axis=1)
    total = C[:, -1:]
    new_lw = m + np.log(total) - np.log(r)
    if resampler == MULTINOMIAL:
        tgt = u2 * total
    elif resampler == SYSTEMATIC:
        q = np.arange(r, dtype=np.float64)[None, :]
        tgt = (q + u2[:, :1]) * total / r
    else:
        raise ValueError(resampler)
    qa = np.minimum(count_le(C, tgt), r - 1)
    lo_nb = np.take_along_axis(C, np.maximum(qa - 1, 0), axis=1)
    lo_nb = np.where(qa > 0, lo_nb, -np.inf)
    hi_nb = np.take_along_axis(C, qa, axis=1)
    margin = np.minimum(np.abs(tgt - lo_nb), np.abs(hi_nb - tgt)) / total
    qpos = np.arange(r)[None, :]
    # back to index order
    shape3 = (nh, R, r)
    anc_off = ((qa - qpos) * R).reshape(shape3).transpose(0, 2, 1).reshape(N)
    anc = np.arange(N, dtype=np.int64) + anc_off
    new_lw = np.broadcast_to(new_lw, (l2.shape[0], r)).reshape(shape3).transpose(0, 2, 1).reshape(N)
    margin = margin.reshape(shape3).transpose(0, 2, 1).reshape(N)
    if not detail:
        return anc, np.ascontiguousarray(new_lw), np.ascontiguousarray(margin)
    # per destination (index order): its group's row in (groups, members) form
    row = (np.arange(l2.shape[0]).reshape(nh, R)[:, None, :]
           * np.ones((1, r, 1), dtype=np.int64)).reshape(N)
    tgt_i = (tgt / total).reshape(shape3).transpose(0, 2, 1).reshape(N)
    info = dict(row=row, target=tgt_i, cdf=C / total)
    return anc, np.ascontiguousarray(new_lw), np.ascontiguousarray(margin), info


def weighted_estimate(x: np.ndarray, ell: np.ndarray, logw: np.ndarray):
    """Estimate from the weighted cloud before resampling (see module doc)."""
    N = ell.shape[0]
    M = np.max(ell)
    w = np.exp(ell - M)
    sw = np.sum(w)
    mean = (w @ x) / sw
    var = (w @ (x - mean) ** 2) / sw
    ess = sw * sw / (N * np.sum(w * w))
    dlog = (M + np.log(sw)) - np.log(np.sum(np.exp(logw)))
    return dict(mean=mean, var=var, ess=float(ess), dlog=float(dlog),
                max_ell=float(M), sum_w=float(sw))


class ButterflyOracle:
    """Butterfly particle filter, one rotating stage per step (FP64)."""

    def __init__(self, model, N: int, radix: int, resampler: str = MULTINOMIAL,
                 seed: int = 0, stream_id: int = 0, full_cycle: bool = False):
        """``full_cycle``: every time step runs all ``S`` stages (Algorithm 3
        in full) instead of the one rotating stage ``k = t mod S``."""
        self.full_cycle = bool(full_cycle)
        self.model = model
        self.N = int(N)
        self.radix = int(radix)
        self.plan = stage_plan(self.N, self.radix)
        self.R = place_values(self.plan)
        self.resampler = resampler
        self.seed = int(seed)
        self.stream_id = int(stream_id)

    @property
    def S(self) -> int:
        return len(self.plan)

    def init(self) -> State:
        """Algorithm 1, initialisation: ``x_0^i ~ pi_0`` with the ``tau = 0``
        normals; unit weights (``logW = 0``)."""
        z = philox.normals(self.seed, self.stream_id, 0, self.N, self.model.d)
        x = models.sample_prior(self.model, z)
        return State(x=x, logw=np.zeros(self.N), t=0, log_norm=0.0)

    def step(self, st: State, y, keep=True):
        """Advance one time step with observation ``y``; returns
        ``(new_state, record)``."""
        if self.full_cycle:
            return self._step_full(st, y, keep)
        t = st.t
        k = t % self.S
        r, R = self.plan[k], self.R[k]
        tau = t + 1
        ell = st.logw + models.log_g(self.model, st.x, y)
        est = weighted_estimate(st.x, ell, st.logw)
        U = philox.resample_uniforms(self.seed, self.stream_id, tau, self.N)
        if keep:
            anc, new_lw, margin, info = group_resample(ell, U, r, R, self.resampler, detail=True)
        else:
            anc, new_lw, margin = group_resample(ell, U, r, R, self.resampler)
        xhat = st.x[anc]
        c = np.max(new_lw)
        logw = new_lw - c
        z = philox.normals(self.seed, self.stream_id, tau, self.N, self.model.d)
        x = models.propagate(self.model, xhat, z)
        log_norm = st.log_norm + est["dlog"]
        rec = dict(t=t, stage=k, radix=r, stride=R, mean=est["mean"],
                   var=est["var"], ess=est["ess"], log_norm=log_norm,
                   max_ell=est["max_ell"], offset=float(c))
        if keep:
            rec.update(ancestors=anc, margin=margin, logw_new=new_lw, ell=ell, draw=info)
        return State(x=x, logw=logw, t=t + 1, log_norm=log_norm), rec

    def _step_full(self, st: State, y, keep):
        """One time step with all S stages (Algorithm 3): weight with
        ``y_t``, estimate, resample through stages 0..S-1 carrying the group
        means (after the last stage every weight is the global mean, Lemma
        3(c)), gather, propagate. Stage ``s`` draws the uniforms of
        ``philox.stage_uniforms``."""
        from .augmented import augmented_resample
        t = st.t
        tau = t + 1
        ell = st.logw + models.log_g(self.model, st.x, y)
        est = weighted_estimate(st.x, ell, st.logw)
        U = [philox.stage_uniforms(self.seed, self.stream_id, tau, self.N, k) for k in range(self.S)]
        origin, lv, stages = augmented_resample(ell, U, self.plan, self.resampler, detail=True)
        xhat = st.x[origin]
        c = np.max(lv)
        logw = lv - c
        z = philox.normals(self.seed, self.stream_id, tau, self.N, self.model.d)
        x = models.propagate(self.model, xhat, z)
        log_norm = st.log_norm + est["dlog"]
        rec = dict(t=t, stage=self.S, radix=self.radix, stride=1, mean=est["mean"],
                   var=est["var"], ess=est["ess"], log_norm=log_norm,
                   max_ell=est["max_ell"], offset=float(c))
        if keep:
            rec.update(origin=origin, stages=stages, ell=ell)
        return State(x=x, logw=logw, t=t + 1, log_norm=log_norm), rec

    def run(self, ys, keep=False, state: State | None = None):
        """Run ``len(ys)`` steps from ``state`` (default: a fresh init).
        Returns ``(final_state, records)``."""
        st = self.init() if state is None else state
        recs = []
        for y in ys:
            st, rec = self.step(st, y, keep=keep)
            recs.append(rec)
        return st, recs
