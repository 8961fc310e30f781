"""Philox4x32-10 and the Box-Muller map of the thermostat noise (FP64 side).

TEST INFRASTRUCTURE ONLY.  Written from the published definition of the
Philox family (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
as 1, 2, 3", SC'11): a 4x32-bit counter and a 2x32-bit key; each of the 10
rounds multiplies counter words 0 and 2 by the constants 0xD2511F53 and
0xCD9E8D57, takes the 64-bit products apart into high and low halves, and
builds the new counter (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0); between
rounds the key is advanced by the Weyl constants (0x9E3779B9, 0xBB67AE85).

Stream layout used by the Langevin thermostat (same on both sides):
key = (seed mod 2^32, seed >> 32), counter = (tag, step mod 2^32, step >> 32, 0).
The four output words x0..x3 map to uniforms u = (x + 1/2) 2^-32 in (0, 1)
and to three normals by Box-Muller:
  z0 = sqrt(-2 ln u0) cos(2 pi u1), z1 = sqrt(-2 ln u0) sin(2 pi u1),
  z2 = sqrt(-2 ln u2) cos(2 pi u3).

Parity status: pinned by the published known-answer vectors of Philox4x32-10.
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint64(0x9E3779B9)
W1 = np.uint64(0xBB67AE85)
MASK = np.uint64(0xFFFFFFFF)
S32 = np.uint64(32)


def philox4x32_10(ctr, key):
    """Vectorized Philox4x32-10.

    ctr: uint array [..., 4]; key: uint array [..., 2] (broadcastable).
    Returns uint32 array [..., 4].
    """
    c = [np.asarray(ctr[..., q], dtype=np.uint64) & MASK for q in range(4)]
    k0 = np.asarray(key[..., 0], dtype=np.uint64) & MASK
    k1 = np.asarray(key[..., 1], dtype=np.uint64) & MASK
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
        p0 = M0 * c[0]
        p1 = M1 * c[2]
        hi0, lo0 = p0 >> S32, p0 & MASK
        hi1, lo1 = p1 >> S32, p1 & MASK
        c = [(hi1 ^ c[1] ^ k0) & MASK, lo1, (hi0 ^ c[3] ^ k1) & MASK, lo0]
    return np.stack([x.astype(np.uint32) for x in c], axis=-1)


def uniforms(words):
    """(x + 1/2) * 2^-32 in float64."""
    return (np.asarray(words, dtype=np.float64) + 0.5) * (2.0 ** -32)


def thermostat_normals(seed: int, tags, step: int):
    """Three standard normals per tag for Langevin step ``step``."""
    tags = np.asarray(tags, dtype=np.uint64)
    n = tags.shape[0]
    ctr = np.zeros((n, 4), dtype=np.uint64)
    ctr[:, 0] = tags
    ctr[:, 1] = np.uint64(step & 0xFFFFFFFF)
    ctr[:, 2] = np.uint64((step >> 32) & 0xFFFFFFFF)
    key = np.array([seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF], dtype=np.uint64)
    w = philox4x32_10(ctr, key[None, :])
    u = uniforms(w)
    r0 = np.sqrt(-2.0 * np.log(u[:, 0]))
    r1 = np.sqrt(-2.0 * np.log(u[:, 2]))
    z = np.stack([r0 * np.cos(2.0 * np.pi * u[:, 1]),
                  r0 * np.sin(2.0 * np.pi * u[:, 1]),
                  r1 * np.cos(2.0 * np.pi * u[:, 3])], axis=1)
    return z
