"""Model functions of the hidden Markov model in FP64.

TEST INFRASTRUCTURE ONLY: part of the FP64 oracle.

Section 1.1, eq. ``HMM``: the filter needs a sampler of ``pi_0``, a sampler of
the Markov kernel ``f`` and the log-likelihood ``log g(x, y)`` (``g`` strictly
positive, Section 1.1 and Assumption A2). ``log g`` includes its normalising
constant so that the log-normaliser estimates ``log p(y_0, ..., y_{T-1})``.
"""
from __future__ import annotations

import numpy as np

LOG_2PI = float(np.log(2.0 * np.pi))


def log_g(model, x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """``log g(x_i, y)`` for every row ``x_i`` of ``x`` (shape ``(N, d)``)."""
    y = np.asarray(y, dtype=np.float64).reshape(model.d)
    if model.kind == "lg":
        # y - H x ~ N(0, R), R = L_R L_R^T:  -1/2 |L_R^{-1}(y - H x)|^2
        #   - sum log diag(L_R) - d/2 log(2 pi)
        e = y[None, :] - x @ model.H.T
        u = np.linalg.solve(model.R_chol, e.T).T
        return (-0.5 * np.sum(u * u, axis=1)
                - np.sum(np.log(np.diag(model.R_chol)))
                - 0.5 * model.d * LOG_2PI)
    # SV: y ~ N(0, beta^2 e^x)
    b2 = model.beta ** 2
    xx = x[:, 0]
    return (-0.5 * (LOG_2PI + np.log(b2)) - 0.5 * xx
            - (y[0] ** 2) * np.exp(-xx) / (2.0 * b2))


def sample_prior(model, z: np.ndarray) -> np.ndarray:
    """``x_0 = m0 + L_0 z`` (LG) or ``x_0 = sd_stat z`` (SV); ``z`` is ``(N, d)``."""
    if model.kind == "lg":
        return model.m0[None, :] + z @ model.P0_chol.T
    return model.sv_stationary_sd * z


def propagate(model, xhat: np.ndarray, z: np.ndarray) -> np.ndarray:
    """One draw from ``f(xhat, .)`` given standard normals ``z`` (``(N, d)``)."""
    if model.kind == "lg":
        return xhat @ model.A.T + z @ model.Q_chol.T
    return model.phi * xhat + model.sigma * z
