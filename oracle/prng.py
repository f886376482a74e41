"""Counter-based randomness for the oracle (test infrastructure only).

The paper does not say how keys and noise are sampled (§3.2 only names
KeyGen and SymEnc).  The oracle and the library therefore each implement the
same *published* counter-based generator, Philox4x64-10 (Salmon, Moraes,
Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11), so that
both derive identical keys from a seed without sharing code.  This file is
the oracle's own implementation, written from that definition with numpy
uint64 arithmetic; it is pinned against ``numpy.random.Philox`` (which is
Philox4x64-10) in the tests.

Stream addressing (a reading made here; the paper is silent):
  key     = (seed, (party << 32) | obj)
  counter = (block, idx, 0, 0)
Block ``b`` of stream (seed, party, obj, idx) yields four u64 words; the
u32 draw number ``j`` is the low half (``j`` even) or high half (``j`` odd)
of u64 word ``j // 2`` of the concatenated blocks.

Discrete Gaussian-like noise with standard deviation 2^-s (torus units) is
the integer Irwin-Hall(12) sum: X = sum of 12 u32 draws - 6*2^32 has mean 0
and standard deviation 2^32, and e = floor((X + 2^(s-1)) / 2^s) mod 2^32.
Integer-only, so two independent implementations agree bit for bit.
"""
from __future__ import annotations

import numpy as np

M64 = np.uint64(0xFFFFFFFFFFFFFFFF)
_M32 = np.uint64(0xFFFFFFFF)
_PHILOX_M0 = np.uint64(0xD2E7470EE14C6C93)
_PHILOX_M1 = np.uint64(0xCA5A826395121157)
_PHILOX_W0 = np.uint64(0x9E3779B97F4A7C15)
_PHILOX_W1 = np.uint64(0xBB67AE8584CAA73B)

# Object identifiers of the stream addressing.
OBJ_CRS = 1
OBJ_SK_LWE = 2
OBJ_SK_RLWE = 3
OBJ_PK_E = 4
OBJ_BK_R = 5
OBJ_BK_E1 = 6
OBJ_BK_F1 = 7
OBJ_BK_E2 = 8
OBJ_KS_A = 9
OBJ_KS_E = 10
OBJ_ENC_A = 11
OBJ_ENC_E = 12
PUBLIC_PARTY = 0xFFFF


def _mulhilo(a, b):
    """Full 64x64 -> 128-bit product of uint64 arrays, as (hi, lo)."""
    a_lo, a_hi = a & _M32, a >> np.uint64(32)
    b_lo, b_hi = b & _M32, b >> np.uint64(32)
    ll = a_lo * b_lo
    hl = a_hi * b_lo
    lh = a_lo * b_hi
    hh = a_hi * b_hi
    cross = (ll >> np.uint64(32)) + (hl & _M32) + lh
    hi = hh + (hl >> np.uint64(32)) + (cross >> np.uint64(32))
    lo = a * b
    return hi, lo


def philox4x64_10(c0, c1, c2, c3, k0, k1):
    """Ten Philox rounds on uint64 arrays (broadcastable); returns 4 words."""
    with np.errstate(over="ignore"):
        x0, x1, x2, x3 = (np.asarray(v, dtype=np.uint64) for v in (c0, c1, c2, c3))
        k0 = np.asarray(k0, dtype=np.uint64)
        k1 = np.asarray(k1, dtype=np.uint64)
        for r in range(10):
            if r:
                k0 = k0 + _PHILOX_W0
                k1 = k1 + _PHILOX_W1
            hi0, lo0 = _mulhilo(_PHILOX_M0, x0)
            hi1, lo1 = _mulhilo(_PHILOX_M1, x2)
            x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
    return x0, x1, x2, x3


def draws_u32(seed: int, party: int, obj: int, idx, count: int):
    """u32 draws 0..count-1 of streams (seed, party, obj, i) for i in idx.

    Returns uint32[len(idx), count] (a 1-D array if ``idx`` is a scalar).
    """
    scalar = np.isscalar(idx)
    idx = np.atleast_1d(np.asarray(idx, dtype=np.uint64))
    nblk = (count + 7) // 8
    blk = np.arange(nblk, dtype=np.uint64)[None, :]
    k0 = np.uint64(seed & 0xFFFFFFFFFFFFFFFF)
    k1 = np.uint64(((party & 0xFFFFFFFF) << 32) | (obj & 0xFFFFFFFF))
    w = philox4x64_10(blk, idx[:, None], np.uint64(0), np.uint64(0), k0, k1)
    words = np.stack(w, axis=-1)                       # [len, nblk, 4] u64
    lo = (words & _M32).astype(np.uint32)
    hi = (words >> np.uint64(32)).astype(np.uint32)
    out = np.stack([lo, hi], axis=-1).reshape(len(idx), nblk * 8)[:, :count]
    return out[0] if scalar else out


def uniform_torus(seed, party, obj, idx, count):
    """Uniform Torus32 values: one u32 draw each."""
    return draws_u32(seed, party, obj, idx, count)


def binary(seed, party, obj, idx, count):
    """Uniform bits: bit 0 of one u32 draw each."""
    return (draws_u32(seed, party, obj, idx, count) & 1).astype(np.uint8)


def noise(seed, party, obj, idx, count, s):
    """Noise of standard deviation 2^-s: Irwin-Hall(12) from 12 draws each."""
    d = draws_u32(seed, party, obj, idx, 12 * count).astype(np.int64)
    d = d.reshape(d.shape[:-1] + (count, 12))
    x = d.sum(axis=-1) - 6 * (1 << 32)
    e = (x + (1 << (s - 1))) >> s                     # floor division by 2^s
    return (e & 0xFFFFFFFF).astype(np.uint32)
