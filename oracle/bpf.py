"""Plain bootstrap particle filter (Algorithm 1 with Algorithm 2) in FP64.

TEST INFRASTRUCTURE ONLY: part of the FP64 oracle.

Written separately from the butterfly oracle. With one global group the
butterfly step must reproduce this routine exactly (same ancestors, states,
estimates and log-normaliser), because the stage weight of a single group is
the same for every particle and the renormalised log-weights are then zero.

Per step ``t`` (Algorithm 1, Algorithm 2, random numbers from the shared
Philox stream definition):
  weights ``g_t(x_i)``; estimate from ``w_i = exp(log g_i - max)``;
  ``Lambda += max + ln sum w - ln N`` (the usual ``(1/N) sum g`` estimator);
  multinomial draw: ancestor of ``i`` is the first ``j`` whose cumulative
  weight exceeds ``U_i`` times the total (systematic: ``(i + U_0) / N``);
  mutation ``x_i ~ f(x_{a(i)}, .)``.
"""
from __future__ import annotations

import numpy as np

from . import models, philox


def bpf_run(model, N: int, ys, seed: int, stream_id: int = 0,
            resampler: str = "multinomial", keep=False):
    z0 = philox.normals(seed, stream_id, 0, N, model.d)
    x = models.sample_prior(model, z0)
    log_norm = 0.0
    out = []
    for t, y in enumerate(ys):
        lg = models.log_g(model, x, y)
        top = np.max(lg)
        w = np.exp(lg - top)
        sw = np.sum(w)
        mean = (w @ x) / sw
        var = (w @ (x - mean) ** 2) / sw
        ess = sw * sw / (N * np.sum(w * w))
        log_norm = log_norm + ((top + np.log(sw)) - np.log(N))
        cdf = np.cumsum(w)
        total = cdf[-1]
        u = philox.resample_uniforms(seed, stream_id, t + 1, N)
        if resampler == "multinomial":
            target = u * total
        else:
            target = (np.arange(N, dtype=np.float64) + u[0]) * total / N
        a = np.minimum(np.searchsorted(cdf, target, side="right"), N - 1)
        z = philox.normals(seed, stream_id, t + 1, N, model.d)
        x = models.propagate(model, x[a], z)
        rec = dict(t=t, mean=mean, var=var, ess=float(ess), log_norm=float(log_norm))
        if keep:
            rec["ancestors"] = a
            rec["x_next"] = x
        out.append(rec)
    return x, out
