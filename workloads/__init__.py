"""Seeded synthetic inputs for the butterfly-interaction particle filter.

This module is shared by the FP64 oracle, the tests and the benchmark. It
holds model *parameters* and simulated *observations* only: no filtering
arithmetic (no weights, no resampling, no random numbers the filter draws).
The filter's own random numbers come from the counter-based Philox stream
that the oracle and the device code each implement separately.

Models follow the hidden Markov model of Section 1.1 (eq. ``HMM``):
``X_0 ~ pi_0``, ``X_n | X_{n-1} ~ f(X_{n-1}, .)``, ``Y_n | X_n ~ g(X_n, .)``.

* linear-Gaussian (LG): ``x_n = A x_{n-1} + L_Q z``, ``y_n = H x_n + L_R e``,
  ``x_0 = m0 + L_0 z``; the 1-D AR(1) model is LG with d = 1.
* stochastic volatility (SV): ``x_n = phi x_{n-1} + sigma z``,
  ``y_n = beta exp(x_n / 2) e``, ``x_0`` from the stationary law.
* the random walk of Section 6.1 (experimental setup): LG with ``A = I``,
  ``Q = I``, ``H = I``, ``R = I/4``, ``x_0 ~ N(0, I)``.

Observations are simulated in FP64 with ``numpy.random.Generator(PCG64(seed))``.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

__all__ = [
    "ModelSpec", "ar1_model", "lg_model", "lg8_model", "random_stable_lg",
    "dense_lg_model",
    "sv_model", "random_walk_model", "simulate", "CONFIGS", "config", "batched_workload",
    "haar_orthogonal",
]


@dataclass
class ModelSpec:
    """Parameters of one state-space model (host FP64 arrays).

    ``kind`` is ``"lg"`` or ``"sv"``. For LG every matrix is ``d x d``
    (row-major) and every vector has length ``d``; ``Q_chol``, ``R_chol`` and
    ``P0_chol`` are lower-triangular Cholesky factors. For SV only ``phi``,
    ``sigma`` and ``beta`` are used and ``d == 1``.
    """

    kind: str
    d: int
    A: Optional[np.ndarray] = None
    Q_chol: Optional[np.ndarray] = None
    H: Optional[np.ndarray] = None
    R_chol: Optional[np.ndarray] = None
    m0: Optional[np.ndarray] = None
    P0_chol: Optional[np.ndarray] = None
    phi: float = 0.0
    sigma: float = 0.0
    beta: float = 0.0
    name: str = ""
    meta: dict = field(default_factory=dict)

    def __post_init__(self):
        if self.kind not in ("lg", "sv"):
            raise ValueError(f"unknown model kind {self.kind!r}")
        if self.kind == "sv":
            if self.d != 1:
                raise ValueError("the SV model is one-dimensional")
            return
        d = self.d
        for nm in ("A", "Q_chol", "H", "R_chol", "P0_chol"):
            v = np.asarray(getattr(self, nm), dtype=np.float64)
            if v.shape != (d, d):
                raise ValueError(f"{nm} must be {d}x{d}, got {v.shape}")
            setattr(self, nm, np.ascontiguousarray(v))
        m0 = np.asarray(self.m0, dtype=np.float64).reshape(d)
        self.m0 = np.ascontiguousarray(m0)
        for nm in ("Q_chol", "R_chol", "P0_chol"):
            v = getattr(self, nm)
            if np.any(np.triu(v, 1) != 0.0):
                raise ValueError(f"{nm} must be lower-triangular")
            if np.any(np.diag(v) <= 0.0):
                raise ValueError(f"{nm} must have a positive diagonal")

    @property
    def sv_stationary_sd(self) -> float:
        return float(self.sigma / np.sqrt(1.0 - self.phi ** 2))


def lg_model(A, Q, H, R, m0, P0, name="lg") -> ModelSpec:
    """LG model from covariance matrices (Cholesky factors taken here)."""
    A = np.atleast_2d(np.asarray(A, dtype=np.float64))
    d = A.shape[0]
    return ModelSpec(
        kind="lg", d=d, A=A,
        Q_chol=np.linalg.cholesky(np.atleast_2d(np.asarray(Q, dtype=np.float64))),
        H=np.atleast_2d(np.asarray(H, dtype=np.float64)),
        R_chol=np.linalg.cholesky(np.atleast_2d(np.asarray(R, dtype=np.float64))),
        m0=np.asarray(m0, dtype=np.float64).reshape(d),
        P0_chol=np.linalg.cholesky(np.atleast_2d(np.asarray(P0, dtype=np.float64))),
        name=name)


def ar1_model(phi=0.9, q=1.0, r=1.0, p0=1.0) -> ModelSpec:
    """1-D AR(1): ``x_t = phi x_{t-1} + N(0, q)``, ``y_t = x_t + N(0, r)``."""
    return lg_model([[phi]], [[q]], [[1.0]], [[r]], [0.0], [[p0]], name="ar1")


def haar_orthogonal(d: int, seed: int) -> np.ndarray:
    """Haar-distributed orthogonal matrix from a seeded QR, sign-fixed so that
    ``diag(R) > 0`` (the standard Mezzadri construction)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    g = rng.standard_normal((d, d))
    q, r = np.linalg.qr(g)
    return q * np.sign(np.diag(r))[None, :]


def lg8_model(seed: int = 2, d: int = 8) -> ModelSpec:
    """8-D LG model: ``A = 0.9 I + 0.05 O`` (O Haar orthogonal), ``Q = I``,
    ``H = I``, ``R = 0.5 I``, ``x_0 ~ N(0, I)``."""
    O = haar_orthogonal(d, seed)
    A = 0.9 * np.eye(d) + 0.05 * O
    return lg_model(A, np.eye(d), np.eye(d), 0.5 * np.eye(d), np.zeros(d),
                    np.eye(d), name=f"lg{d}")


def random_stable_lg(d: int, seed: int, rho: float = 0.95) -> ModelSpec:
    """LG model with a seeded Gaussian ``B`` scaled to spectral radius ``rho``;
    ``Q = I``, ``H = I``, ``R = 0.5 I``, ``x_0 ~ N(0, I)``."""
    rng = np.random.Generator(np.random.PCG64(seed))
    B = rng.standard_normal((d, d))
    sr = float(np.max(np.abs(np.linalg.eigvals(B))))
    A = rho * B / sr
    return lg_model(A, np.eye(d), np.eye(d), 0.5 * np.eye(d), np.zeros(d),
                    np.eye(d), name=f"lg{d}_stable")


def dense_lg_model(d: int = 4, seed: int = 12) -> ModelSpec:
    """LG model with every matrix dense and non-symmetric where allowed: ``A``
    Gaussian scaled to spectral radius 0.8, ``Q = B B^T + 0.3 I``,
    ``H = I + 0.2 G``, ``R = C C^T + 2 I`` (moderately informative), ``P0 = I``.
    Exercises every term of the LG likelihood and transition."""
    rng = np.random.Generator(np.random.PCG64(seed))
    B = rng.standard_normal((d, d))
    A = 0.8 * B / float(np.max(np.abs(np.linalg.eigvals(B))))
    Qb = 0.2 * rng.standard_normal((d, d))
    H = np.eye(d) + 0.2 * rng.standard_normal((d, d))
    Rb = 0.5 * rng.standard_normal((d, d))
    m0 = np.linspace(0.5, -0.3, d)
    return lg_model(A, Qb @ Qb.T + 0.3 * np.eye(d), H, Rb @ Rb.T + 2.0 * np.eye(d),
                    m0, np.eye(d), name=f"lg{d}_dense")


def sv_model(phi=0.95, sigma=0.25, beta=0.6) -> ModelSpec:
    """Stochastic volatility: ``x_t = phi x_{t-1} + sigma z``,
    ``y_t = beta exp(x_t/2) e``; ``x_0`` from the stationary law."""
    return ModelSpec(kind="sv", d=1, phi=float(phi), sigma=float(sigma),
                     beta=float(beta), name="sv")


def random_walk_model(d: int = 7) -> ModelSpec:
    """Random-walk model of the paper's experiments (Section 6.1)."""
    return lg_model(np.eye(d), np.eye(d), np.eye(d), 0.25 * np.eye(d),
                    np.zeros(d), np.eye(d), name=f"rw{d}")


def simulate(model: ModelSpec, T: int, seed: int):
    """Simulate ``T`` steps of the HMM. Returns ``(x, y)`` of shape ``(T, d)``
    in FP64; ``y[t]`` is the observation of ``x[t]`` (observations start at
    ``n = 0``)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    d = model.d
    xs = np.empty((T, d))
    ys = np.empty((T, d))
    if model.kind == "lg":
        x = model.m0 + model.P0_chol @ rng.standard_normal(d)
        for t in range(T):
            if t > 0:
                x = model.A @ x + model.Q_chol @ rng.standard_normal(d)
            xs[t] = x
            ys[t] = model.H @ x + model.R_chol @ rng.standard_normal(d)
    else:
        x = model.sv_stationary_sd * rng.standard_normal()
        for t in range(T):
            if t > 0:
                x = model.phi * x + model.sigma * rng.standard_normal()
            xs[t, 0] = x
            ys[t, 0] = model.beta * np.exp(0.5 * x) * rng.standard_normal()
    return xs, ys


# ---------------------------------------------------------------------------
# The five workload configurations (synthetic stand-ins; the paper's own data
# set and seeds are not available).
# ---------------------------------------------------------------------------

def _c1():
    return dict(name="ar1_n1024", model=ar1_model(), N=1024, T=100,
                radices=[2, 1024], dtype="f64", seed_obs=1, seed_pf=101)


def _c2():
    return dict(name="lg8_n2p20", model=lg8_model(seed=2), N=1 << 20, T=500,
                radices=[2, 4, 32, 64, 1 << 20], dtype="f32", seed_obs=2,
                seed_pf=202)


def _c3():
    return dict(name="sv_n2p24", model=sv_model(), N=1 << 24, T=1000,
                radices=[32, 64, 256, 1024, 1 << 24], dtype="f32",
                seed_obs=3, seed_pf=303)


CONFIGS = {"c1": _c1, "c2": _c2, "c3": _c3}


def config(name: str) -> dict:
    """Return a fresh copy of a named workload configuration."""
    return CONFIGS[name]()


def batched_filters(n_filters: int = 4096, seed: int = 4):
    """Per-filter sizes of the batched workload: ``N_f = 2^u``,
    ``u ~ UniformInt{10..16}``, ``d_f`` uniform over ``{1, 4, 16}``; the model
    of filter ``f`` is ``random_stable_lg(d_f, 4000 + f)``."""
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.integers(10, 17, size=n_filters)
    dsel = rng.integers(0, 3, size=n_filters)
    ds = np.array([1, 4, 16])[dsel]
    return [dict(N=int(1 << int(uu)), d=int(dd), model_seed=4000 + f)
            for f, (uu, dd) in enumerate(zip(u, ds))]


def batched_workload(n_filters: int = 4096, T: int = 200, seed: int = 4):
    """The batched workload: per-filter models and sizes of
    ``batched_filters`` and their observations, simulated from each model
    (seed ``seed * 1_000_000 + f``) and packed per step in filter order.
    Returns ``(models, Ns, Y)`` with ``Y`` of shape ``(T, sum d_f)``."""
    spec = batched_filters(n_filters, seed)
    models = [random_stable_lg(s["d"], s["model_seed"]) for s in spec]
    Ns = [s["N"] for s in spec]
    cols = [simulate(m, T, seed=seed * 1_000_000 + f)[1].reshape(T, -1) for f, m in enumerate(models)]
    return models, Ns, np.concatenate(cols, axis=1)

