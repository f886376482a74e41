"""Fixed-point gradient-descent linear regression (TEST INFRASTRUCTURE).

§3.4 Eqs. (4)-(5) give the gradient-descent iteration and §4.6 rescales it
to integers (Eqs. (12)-(14), printed garbled: the w update lacks x_i and
both updates use the same sum).  Reading used here, on Q8.8 int16 values
(8 fractional bits) with one model w of d features and no intercept:

    r_i  = sum_j mulq(x_ij, w_j) - y_i                  (mod 2^16)
    g_j  = sum_i mulq(x_ij, r_i)                        (mod 2^16)
    w_j <- w_j - (g_j >> 12)                            (arithmetic shift)

mulq(a, b) = floor(a*b / 2^8) mod 2^16 (bits 8..23 of the 32-bit product);
the shift by 12 applies the step 1/m * alpha = 2^-6 * 2^-6 for m = 64.

``replica_step`` is the plain integer definition; ``build_netlist`` is the
same step as a gate netlist over the oracle's operator builders.
"""
from __future__ import annotations

import numpy as np

from . import circuits as C

FRAC = 8
BITS = 16


def _wrap(v):
    v = np.asarray(v, dtype=np.int64) & 0xFFFF
    return np.where(v >= 0x8000, v - 0x10000, v)


def mulq(a, b):
    return _wrap((np.asarray(a, np.int64) * np.asarray(b, np.int64)) >> FRAC)


def replica_step(X, y, w, shift=12):
    """One iteration on plain integers (Q8.8 in int64 arrays)."""
    X, y, w = (np.asarray(v, np.int64) for v in (X, y, w))
    m, d = X.shape
    r = np.zeros(m, np.int64)
    for i in range(m):
        acc = 0
        for j in range(d):
            acc = _wrap(acc + mulq(X[i, j], w[j]))
        r[i] = _wrap(acc - y[i])
    g = np.zeros(d, np.int64)
    for j in range(d):
        acc = 0
        for i in range(m):
            acc = _wrap(acc + mulq(X[i, j], r[i]))
        g[j] = acc
    return _wrap(w - (g >> shift))


def build_netlist(m: int, d: int, shift: int = 12) -> C.Netlist:
    """Inputs (16 bits each, LSB first): X row-major, then y, then w.
    Outputs: the updated w (d x 16 bits)."""
    nl = C.Netlist(fold=True)
    X = [[[nl.input() for _ in range(BITS)] for _ in range(d)] for _ in range(m)]
    y = [[nl.input() for _ in range(BITS)] for _ in range(m)]
    w = [[nl.input() for _ in range(BITS)] for _ in range(d)]

    def mq(a, b):
        return C.multiply_into(nl, a, b)[FRAC:FRAC + BITS]

    def add(a, b):
        return nl.ripple_add(a, b, C.ZERO)

    def sub(a, b):
        return nl.ripple_add(a, [nl.gate(C.XOR, bi, C.ONE) for bi in b], C.ONE)

    r = []
    for i in range(m):
        acc = mq(X[i][0], w[0])
        for j in range(1, d):
            acc = add(acc, mq(X[i][j], w[j]))
        r.append(sub(acc, y[i]))
    out = []
    for j in range(d):
        acc = mq(X[0][j], r[0])
        for i in range(1, m):
            acc = add(acc, mq(X[i][j], r[i]))
        step = acc[shift:] + [acc[BITS - 1]] * shift      # arithmetic >> shift
        out.extend(sub(w[j], step))
    nl.outputs = out
    return nl


def input_bits(X, y, w):
    """u8[n_inputs, 1] in the input order of build_netlist."""
    from mk_inputs import to_bits
    vals = np.concatenate([np.asarray(X, np.int64).ravel(), np.asarray(y, np.int64),
                           np.asarray(w, np.int64)])
    return to_bits(vals, BITS).reshape(-1, 1)


def input_owner(m: int, d: int):
    """Party owning each input bit: party 0 holds features < d/2, y and w;
    party 1 holds the other features."""
    own = []
    for i in range(m):
        for j in range(d):
            own += [0 if j < (d + 1) // 2 else 1] * BITS
    own += [0] * (BITS * (m + d))
    return np.array(own, np.int64)
