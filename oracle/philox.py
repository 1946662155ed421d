"""Philox4x32-10 counter-based generator and the filter's random-number stream.

TEST INFRASTRUCTURE ONLY: part of the FP64 oracle.

The paper does not specify a random-number generator. Both the oracle and the
device code implement Philox4x32-10 from its published definition (Salmon,
Moraes, Dror and Shaw, "Parallel Random Numbers: As Easy as 1, 2, 3", SC'11):
a 4 x 32-bit counter ``c`` and a 2 x 32-bit key ``k``; each of the 10 rounds
computes the two 32x32 -> 64-bit products ``M0 * c0`` and ``M1 * c2`` and
outputs ``(hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0))``;
the key is bumped by the Weyl constants between rounds.

Stream mapping (one call serves the particle pair ``(2p, 2p+1)``):

* key ``(k0, k1) = (seed mod 2^32, seed >> 32)``
* counter ``(p, tau, b, stream_id)``; ``tau = 0`` draws the prior,
  ``tau = t + 1`` draws the resampling uniforms and the propagation noise of
  time step ``t``; ``b`` is the block index.
* block 0: ``w0, w1`` are the resampling uniforms of ``2p`` and ``2p+1``,
  ``U = (w >> 8) 2^-24``; ``(w2, w3)`` feed one Box-Muller transform whose
  cosine branch is dimension 0 of particle ``2p`` and whose sine branch is
  dimension 0 of particle ``2p+1``.
* block ``b >= 1``: ``(w0, w1)`` give dimension ``2b - 1`` and ``(w2, w3)``
  give dimension ``2b`` with the same cosine/sine split.
* when one time step runs several resampling stages (all ``S`` stages of
  Algorithm 3), stage ``s >= 1`` takes its uniforms from words ``w0, w1`` of
  block 0 at counter word ``tau + s 2^24`` (``tau < 2^24``); stage 0 uses the
  step's own uniforms.
* Box-Muller (Box and Muller, 1958) on words ``(wa, wb)``:
  ``u1 = ((wa >> 8) + 1) 2^-24`` in ``(0, 1]``, ``u2 = (wb >> 8) 2^-24``,
  ``rho = sqrt(-2 ln u1)``, normals ``rho cos(2 pi u2)``, ``rho sin(2 pi u2)``.

Parity of this generator with the canonical Philox is pinned against
rocRAND's independent host-callable implementation in the tests.
"""
from __future__ import annotations

import numpy as np

M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK32 = 0xFFFFFFFF
TWO_M24 = 2.0 ** -24
STAGE_TAU = 1 << 24   # uniforms of stage s >= 1 of a multi-stage step: tau + s STAGE_TAU


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32-10. Inputs are arrays or scalars of unsigned
    32-bit values (any integer dtype); returns four ``uint32`` arrays."""
    c0 = np.asarray(c0, dtype=np.uint64) & MASK32
    c1 = np.asarray(c1, dtype=np.uint64) & MASK32
    c2 = np.asarray(c2, dtype=np.uint64) & MASK32
    c3 = np.asarray(c3, dtype=np.uint64) & MASK32
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    k0 = int(k0) & MASK32
    k1 = int(k1) & MASK32
    m0 = np.uint64(M0)
    m1 = np.uint64(M1)
    sh = np.uint64(32)
    mk = np.uint64(MASK32)
    for rnd in range(10):
        p0 = m0 * c0          # < 2^64, exact in uint64
        p1 = m1 * c2
        hi0, lo0 = p0 >> sh, p0 & mk
        hi1, lo1 = p1 >> sh, p1 & mk
        c0, c1, c2, c3 = (hi1 ^ c1 ^ np.uint64(k0), lo1,
                          hi0 ^ c3 ^ np.uint64(k1), lo0)
        if rnd < 9:
            k0 = (k0 + W0) & MASK32
            k1 = (k1 + W1) & MASK32
    return (c0.astype(np.uint32), c1.astype(np.uint32),
            c2.astype(np.uint32), c3.astype(np.uint32))


def seed_key(seed: int):
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return seed & MASK32, seed >> 32


def n_blocks(d: int) -> int:
    """Philox blocks per particle pair for state dimension ``d``."""
    return 1 + d // 2          # 1 + ceil((d - 1) / 2)


def _pair_words(seed, stream_id, tau, n_pairs, b):
    k0, k1 = seed_key(seed)
    p = np.arange(n_pairs, dtype=np.uint64)
    return philox4x32_10(p, tau, b, stream_id, k0, k1)


def word_to_uniform(w) -> np.ndarray:
    """24-bit uniform on ``[0, 1)``; exact in FP32 and FP64."""
    return (np.asarray(w, dtype=np.uint64) >> np.uint64(8)).astype(np.float64) * TWO_M24


def box_muller(wa, wb):
    """Two standard normals (cosine branch, sine branch) from two words."""
    u1 = ((np.asarray(wa, dtype=np.uint64) >> np.uint64(8)).astype(np.float64) + 1.0) * TWO_M24
    u2 = (np.asarray(wb, dtype=np.uint64) >> np.uint64(8)).astype(np.float64) * TWO_M24
    rho = np.sqrt(-2.0 * np.log(u1))
    ang = 2.0 * np.pi * u2
    return rho * np.cos(ang), rho * np.sin(ang)


def resample_uniforms(seed: int, stream_id: int, tau: int, n: int) -> np.ndarray:
    """Resampling uniform ``U_i`` of every destination ``i < n`` (n even)."""
    if n % 2:
        raise ValueError("the particle count must be even")
    w0, w1, _, _ = _pair_words(seed, stream_id, tau, n // 2, 0)
    u = np.empty(n)
    u[0::2] = word_to_uniform(w0)
    u[1::2] = word_to_uniform(w1)
    return u


def stage_uniforms(seed: int, stream_id: int, tau: int, n: int, stage: int) -> np.ndarray:
    """Destination uniforms of resampling stage ``stage`` of a multi-stage
    step (stage 0: the step's ordinary uniforms)."""
    if tau >= STAGE_TAU or not 0 <= stage < 256:
        raise ValueError("multi-stage steps need tau < 2^24 and fewer than 256 stages")
    return resample_uniforms(seed, stream_id, tau + stage * STAGE_TAU, n)


def normals(seed: int, stream_id: int, tau: int, n: int, d: int) -> np.ndarray:
    """Standard normals ``z[i, j]`` for particle ``i < n`` and dimension ``j < d``."""
    if n % 2:
        raise ValueError("the particle count must be even")
    npair = n // 2
    z = np.empty((n, d))
    _, _, w2, w3 = _pair_words(seed, stream_id, tau, npair, 0)
    zc, zs = box_muller(w2, w3)
    z[0::2, 0] = zc
    z[1::2, 0] = zs
    for b in range(1, n_blocks(d)):
        w0, w1, w2, w3 = _pair_words(seed, stream_id, tau, npair, b)
        for dim, (wa, wb) in ((2 * b - 1, (w0, w1)), (2 * b, (w2, w3))):
            if dim < d:
                zc, zs = box_muller(wa, wb)
                z[0::2, dim] = zc
                z[1::2, dim] = zs
    return z
