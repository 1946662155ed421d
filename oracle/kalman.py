"""Kalman filter in FP64 (closed form for linear-Gaussian models).

TEST INFRASTRUCTURE ONLY: part of the FP64 oracle.

Used as the exact target for the particle filters on LG models (the paper's
own experiments use a Kalman-tractable random walk for the same reason,
Section 6.1). Returns, per observation ``y_t`` (``t >= 0``), the filtering mean
and covariance of ``x_t`` given ``y_0..y_t``, the one-step predictive moments,
and the exact ``log p(y_0, ..., y_{T-1})``.
"""
from __future__ import annotations

import numpy as np


def kalman_filter(model, ys):
    A, H = model.A, model.H
    Q = model.Q_chol @ model.Q_chol.T
    R = model.R_chol @ model.R_chol.T
    m = model.m0.copy()
    P = model.P0_chol @ model.P0_chol.T
    d = model.d
    T = len(ys)
    means = np.empty((T, d))
    covs = np.empty((T, d, d))
    pred_means = np.empty((T, d))
    pred_covs = np.empty((T, d, d))
    loglik = 0.0
    for t, y in enumerate(ys):
        if t > 0:
            m = A @ m
            P = A @ P @ A.T + Q
        pred_means[t], pred_covs[t] = m, P
        S = H @ P @ H.T + R
        e = np.asarray(y, dtype=np.float64) - H @ m
        Sinv_e = np.linalg.solve(S, e)
        _, logdet = np.linalg.slogdet(S)
        loglik += -0.5 * (d * np.log(2 * np.pi) + logdet + e @ Sinv_e)
        K = np.linalg.solve(S, H @ P).T         # P H^T S^{-1}  (S symmetric)
        m = m + K @ e
        P = P - K @ S @ K.T
        P = 0.5 * (P + P.T)
        means[t], covs[t] = m, P
    return dict(mean=means, cov=covs, pred_mean=pred_means,
                pred_cov=pred_covs, loglik=float(loglik))


def steady_state_scalar(q: float, r: float):
    """Steady-state predictive variance ``p`` of the scalar random walk
    ``x_n = x_{n-1} + N(0, q)``, ``y_n = x_n + N(0, r)``: the positive root of
    ``p = p r / (p + r) + q``."""
    # p^2 - q p - q r = 0
    return 0.5 * (q + np.sqrt(q * q + 4.0 * q * r))
