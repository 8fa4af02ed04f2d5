"""Counter-based Gaussian action noise (TEST INFRASTRUCTURE ONLY).

Philox4x64-10 as published by Salmon, Moraes, Dror and Shaw ("Parallel random
numbers: as easy as 1, 2, 3", SC'11): a 4-word counter and a 2-word key; each
of the 10 rounds multiplies words 0 and 2 by two fixed 64-bit constants,
forms the new words from the high/low halves of those products XORed with the
odd words and the round key, and the key is advanced by two Weyl constants
between rounds.

Noise for environment n, step t, stock d uses key (noise_key, 0) and counter
(n, t, d // 4, 0).  Each 64-bit output word w becomes a uniform
u = ((w >> 41) + 0.5) * 2^-23 in (0, 1) (exact in float32), and the pairs
(u0, u1), (u2, u3) become four standard normals by the Box-Muller transform;
stock d takes normal d % 4.  All arithmetic after the integer stage is float64.
"""
from __future__ import annotations

import numpy as np

U64 = np.uint64
_M32 = U64(0xFFFFFFFF)
PHILOX_M0 = U64(0xD2E7470EE14C6C93)
PHILOX_M1 = U64(0xCA5A826395121157)
PHILOX_W0 = U64(0x9E3779B97F4A7C15)   # golden ratio
PHILOX_W1 = U64(0xBB67AE8584CAA73B)   # sqrt(3) - 1
ROUNDS = 10


def _mulhilo(a, b):
    """(high, low) 64-bit halves of the 128-bit product a*b, elementwise on uint64 arrays."""
    a = np.asarray(a, dtype=U64)
    b = np.asarray(b, dtype=U64)
    a_lo, a_hi = a & _M32, a >> U64(32)
    b_lo, b_hi = b & _M32, b >> U64(32)
    ll = a_lo * b_lo
    hl = a_hi * b_lo
    lh = a_lo * b_hi
    hh = a_hi * b_hi
    mid = (ll >> U64(32)) + (hl & _M32) + (lh & _M32)
    lo = (ll & _M32) | ((mid & _M32) << U64(32))
    hi = hh + (hl >> U64(32)) + (lh >> U64(32)) + (mid >> U64(32))
    return hi, lo


def philox4x64_10(counter, key):
    """Philox4x64-10 block function.

    counter: uint64 array [..., 4]; key: uint64 array broadcastable to [..., 2].
    Returns uint64 [..., 4].
    """
    with np.errstate(over="ignore"):
        x = np.array(counter, dtype=U64, copy=True)
        k = np.broadcast_to(np.asarray(key, dtype=U64), x.shape[:-1] + (2,)).copy()
        x0, x1, x2, x3 = x[..., 0], x[..., 1], x[..., 2], x[..., 3]
        k0, k1 = k[..., 0], k[..., 1]
        for r in range(ROUNDS):
            if r > 0:
                k0 = k0 + PHILOX_W0
                k1 = k1 + PHILOX_W1
            hi0, lo0 = _mulhilo(PHILOX_M0, x0)
            hi1, lo1 = _mulhilo(PHILOX_M1, x2)
            x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
        return np.stack([x0, x1, x2, x3], axis=-1)


def uniforms_from_words(w):
    """u = ((w >> 41) + 0.5) * 2^-23: the top 23 bits, centred, in (0, 1); float64."""
    w = np.asarray(w, dtype=U64)
    return ((w >> U64(41)).astype(np.float64) + 0.5) * 2.0 ** -23


def box_muller(u_a, u_b):
    """Two independent standard normals from two uniforms in (0, 1) (float64)."""
    r = np.sqrt(-2.0 * np.log(u_a))
    ang = 2.0 * np.pi * u_b
    return r * np.cos(ang), r * np.sin(ang)


def normals_from_words(w):
    """Four normals from one Philox output block w [..., 4] -> float64 [..., 4]."""
    u = uniforms_from_words(w)
    z0, z1 = box_muller(u[..., 0], u[..., 1])
    z2, z3 = box_muller(u[..., 2], u[..., 3])
    return np.stack([z0, z1, z2, z3], axis=-1)


def noise_words(noise_key: int, env_ids, t: int, n_stocks: int):
    """Raw Philox blocks for envs env_ids at step t: uint64 [len(env_ids)][ceil(D/4)][4]."""
    env_ids = np.asarray(env_ids, dtype=U64)
    nblk = (n_stocks + 3) // 4
    ctr = np.zeros((env_ids.size, nblk, 4), dtype=U64)
    ctr[..., 0] = env_ids[:, None]
    ctr[..., 1] = U64(t)
    ctr[..., 2] = np.arange(nblk, dtype=U64)[None, :]
    key = np.array([noise_key, 0], dtype=U64)
    return philox4x64_10(ctr, key)


def noise(noise_key: int, env_ids, t: int, n_stocks: int) -> np.ndarray:
    """Standard normal eps[n][d] for step t (float64 [len(env_ids)][D])."""
    z = normals_from_words(noise_words(noise_key, env_ids, t, n_stocks))
    return z.reshape(z.shape[0], -1)[:, :n_stocks]
