"""Point-mass (grid) filter for scalar AR(1)-state models, FP64.

TEST INFRASTRUCTURE ONLY: part of the FP64 oracle.

Brute-force quadrature of the filtering recursion for a scalar state with
transition ``x' = phi x + sigma z``: the density is carried on a uniform grid
spanning +-``width_sd`` stationary standard deviations; prediction applies the
Gaussian transition kernel sampled on the grid, the update multiplies
pointwise by ``g(x, y_t)``. Used as the reference filtering mean for the SV
model, where no closed form exists; on a linear-Gaussian observation it must
agree with the Kalman filter.
"""
from __future__ import annotations

import numpy as np


def grid_filter_1d(phi, sigma, x0_mean, x0_sd, log_lik, ys, n_nodes=4096,
                   width_sd=8.0):
    """``log_lik(xgrid, y)`` returns ``log g`` on the grid."""
    stat_sd = sigma / np.sqrt(1.0 - phi * phi) if abs(phi) < 1 else x0_sd
    half = width_sd * max(stat_sd, x0_sd)
    xg = np.linspace(x0_mean - half, x0_mean + half, n_nodes)
    dx = xg[1] - xg[0]
    diff = xg[None, :] - phi * xg[:, None]          # rows: from, cols: to
    K = np.exp(-0.5 * (diff / sigma) ** 2) / (sigma * np.sqrt(2 * np.pi))
    p = np.exp(-0.5 * ((xg - x0_mean) / x0_sd) ** 2) / (x0_sd * np.sqrt(2 * np.pi))
    means = np.empty(len(ys))
    varis = np.empty(len(ys))
    loglik = 0.0
    for t, y in enumerate(ys):
        if t > 0:
            p = (p @ K) * dx
        lg = log_lik(xg, float(np.asarray(y).reshape(-1)[0]))
        top = np.max(lg)
        post = p * np.exp(lg - top)
        z = np.sum(post) * dx
        loglik += np.log(z) + top
        p = post / z
        means[t] = np.sum(p * xg) * dx
        varis[t] = np.sum(p * (xg - means[t]) ** 2) * dx
    return dict(mean=means, var=varis, loglik=float(loglik))


def sv_grid_filter(model, ys, n_nodes=4096, width_sd=8.0):
    """Grid filter of the SV model ``y = beta exp(x/2) e``."""
    b2 = model.beta ** 2

    def ll(xg, y):
        return -0.5 * np.log(2 * np.pi * b2) - 0.5 * xg - y * y * np.exp(-xg) / (2 * b2)

    return grid_filter_1d(model.phi, model.sigma, 0.0, model.sv_stationary_sd, ll,
                          ys, n_nodes, width_sd)
