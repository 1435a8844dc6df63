"""Seeded N(0,1) start block drawn by the method itself (FP64 + 32-bit integer
arithmetic).

TEST INFRASTRUCTURE ONLY (see the package docstring).

When no initial guess is given, the eigensolver starts from a block of
standard normal deviates (the seeded random start of the one-element
workload), drawn from a counter-based generator so that any entry can be
produced independently:

* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
  easy as 1, 2, 3", SC 2011): a 128-bit counter (x0, x1, x2, x3) and a 64-bit
  key (k0, k1); each of ten rounds multiplies x0 and x2 by the constants
  0xD2511F53 and 0xCD9E8D57 into 64-bit products (hi, lo), sets
  (x0, x1, x2, x3) <- (hi(M1 x2) ^ x1 ^ k0, lo(M1 x2), hi(M0 x0) ^ x3 ^ k1,
  lo(M0 x0)), then bumps the key by (0x9E3779B9, 0xBB67AE85).
* For rows 2q and 2q + 1 of column j of batch element e the counter is
  (q, j, e, 0) and the key (seed mod 2^32, seed div 2^32).  The outputs
  (w0, w1, w2, w3) give two 53-bit uniforms u1 = (w0 2^21 + w1 div 2^11) / 2^53
  and u2 likewise from (w2, w3) (exact in FP64), and the Box-Muller transform
  (Box and Muller, 1958) gives
      x_{2q}     = sqrt(-2 ln(1 - u1)) cos(2 pi u2)
      x_{2q + 1} = sqrt(-2 ln(1 - u1)) sin(2 pi u2)
  (an odd N_g's last row takes x_{2q} only).
"""
from __future__ import annotations

import numpy as np

M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85
_MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr, key):
    """Philox4x32-10 on arrays: ctr (..., 4) and key (..., 2) of unsigned
    32-bit values (any integer dtype); returns (..., 4) uint64 holding 32-bit
    outputs."""
    x = [np.asarray(c, dtype=np.uint64) & _MASK for c in np.moveaxis(np.asarray(ctr), -1, 0)]
    k0, k1 = [np.asarray(c, dtype=np.uint64) & _MASK for c in np.moveaxis(np.asarray(key), -1, 0)]
    x0, x1, x2, x3 = np.broadcast_arrays(*x)
    for _ in range(10):
        p0 = np.uint64(M0) * x0
        p1 = np.uint64(M1) * x2
        x0, x1, x2, x3 = ((p1 >> np.uint64(32)) ^ x1 ^ k0, p1 & _MASK,
                          (p0 >> np.uint64(32)) ^ x3 ^ k1, p0 & _MASK)
        k0 = (k0 + np.uint64(W0)) & _MASK
        k1 = (k1 + np.uint64(W1)) & _MASK
    return np.stack([x0, x1, x2, x3], axis=-1)


def uniforms53(hi, lo):
    """(hi 2^21 + lo div 2^11) / 2^53 for 32-bit words hi, lo."""
    hi = np.asarray(hi, dtype=np.uint64)
    lo = np.asarray(lo, dtype=np.uint64)
    return ((hi << np.uint64(21)) | (lo >> np.uint64(11))).astype(np.float64) * 2.0 ** -53


def start_block(ng, n_states, elem, seed):
    """N_g x J start block (Fortran order) of batch element `elem`."""
    nq = (ng + 1) // 2
    q, j = np.meshgrid(np.arange(nq, dtype=np.uint64), np.arange(n_states, dtype=np.uint64),
                       indexing="ij")
    ctr = np.stack([q, j, np.full_like(q, elem), np.zeros_like(q)], axis=-1)
    key = np.array([seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF], dtype=np.uint64)
    w = philox4x32_10(ctr, key)
    u1 = uniforms53(w[..., 0], w[..., 1])
    u2 = uniforms53(w[..., 2], w[..., 3])
    r = np.sqrt(-2.0 * np.log1p(-u1))
    X = np.empty((2 * nq, n_states))
    X[0::2] = r * np.cos(2.0 * np.pi * u2)
    X[1::2] = r * np.sin(2.0 * np.pi * u2)
    return np.asfortranarray(X[:ng])
