"""Linear regression on encrypted integers (TEST INFRASTRUCTURE): the
gradient-descent method and the closed-form ("calculation formula") method.

Gradient descent.

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

Closed form (§3.4 Eqs. (2)-(3), Alg. 7).  One feature and m pairs.  The
paper computes x̄, then the slope ω, then the intercept b.  It states only
that the inputs are rounded to integers and that 8-bit operators are used.
The reading here takes 8-bit inputs, exact 8 x 8 -> 16-bit products, 16-bit
sums, 16-bit values for the slope and intercept with FRAC_F fractional
bits, and truncating signed division.  Every sum and difference wraps at its
stated width:

    S_x = sum x_i,  S_y = sum y_i                             (mod 2^16)
    x̄ = S_x / m,  ȳ = S_y / m       (16-bit dividers; low 8 bits kept)
    dx_i = x_i - x̄,  dy_i = y_i - ȳ                           (mod 2^8)
    num = sum dy_i dx_i,  den = sum dx_i dx_i                 (mod 2^16)
    ω = (num 2^F) / den             (32-bit dividend, 16-bit divisor)
    b = (S_y 2^F - ω S_x) / m       (32-bit dividend, 16-bit divisor)

In exact arithmetic Eq. (2)'s numerator sum y_i (x_i - x̄) equals
sum (y_i - ȳ)(x_i - x̄), and its denominator equals sum (x_i - x̄)^2.  With
x̄ and ȳ truncated to integers the centred forms are off by m e_x e_y and
m e_x^2 (e = the truncation errors, |e| < 1).  The printed forms would be off
by e_x S_y and e_x S_x, which are large when the data are not centred.  b is
Eq. (3) scaled by 2^F.  Division truncates toward zero and keeps the low 16
quotient bits.  The divider array returns exactly these bits, also when the
quotient does not fit.  ``formula_replica`` is this definition on plain
integers; ``build_formula_netlist`` is the same computation as gates.
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


# ------------------------------------------------- closed-form method ----

FX_IN, FX_W, FRAC_F = 8, 16, 8


def _wrap_to(v, bits):
    v = np.asarray(v, dtype=np.int64) & ((1 << bits) - 1)
    return np.where(v >= 1 << (bits - 1), v - (1 << bits), v)


def _tdiv(a, b):
    """Signed division truncating toward zero (Python ints)."""
    if b == 0:
        raise ZeroDivisionError("closed-form regression: zero divisor")
    q = abs(a) // abs(b)
    return q if (a < 0) == (b < 0) else -q


def formula_replica(x, y, frac=FRAC_F):
    """Slope and intercept, both Q(16-frac).frac int16, of one data set
    (x, y: m signed 8-bit integers), by the integer definition above."""
    x = [int(v) for v in x]
    y = [int(v) for v in y]
    m = len(x)
    w16 = lambda v: int(_wrap_to(v, FX_W))
    w32 = lambda v: int(_wrap_to(v, 2 * FX_W))
    sx = sy = 0
    for xi, yi in zip(x, y):
        sx, sy = w16(sx + xi), w16(sy + yi)
    xbar = int(_wrap_to(_tdiv(sx, m), FX_IN))
    ybar = int(_wrap_to(_tdiv(sy, m), FX_IN))
    dx = [int(_wrap_to(xi - xbar, FX_IN)) for xi in x]
    dy = [int(_wrap_to(yi - ybar, FX_IN)) for yi in y]
    num = den = 0
    for a, b in zip(dx, dy):
        num, den = w16(num + b * a), w16(den + a * a)
    omega = w16(_tdiv(num << frac, den))
    u = w32((sy << frac) - w32(omega * sx))
    return omega, w16(_tdiv(u, m))


def build_formula_netlist(m: int, frac: int = FRAC_F) -> C.Netlist:
    """Inputs (8 bits each, LSB first): x_0..x_{m-1}, then y_0..y_{m-1}.
    Outputs: the slope (16 bits), then the intercept (16 bits).  The
    constant m enters as constant wires."""
    nl = C.Netlist(fold=True)
    x = [[nl.input() for _ in range(FX_IN)] for _ in range(m)]
    y = [[nl.input() for _ in range(FX_IN)] for _ in range(m)]
    const_m = [C.ONE if (m >> t) & 1 else C.ZERO for t in range(FX_W)]

    def ext(v, bits):                       # sign extension (wiring only)
        return v + [v[-1]] * (bits - len(v))

    def shifted(v, bits):                   # v * 2^frac, sign-extended
        return ext([C.ZERO] * frac + v, bits)

    def add(a, b):
        return nl.ripple_add(a, b, C.ZERO)

    def sub(a, b):
        return nl.ripple_add(a, [nl.gate(C.XOR, bi, C.ONE) for bi in b], C.ONE)

    def total(terms):
        acc = terms[0]
        for t in terms[1:]:
            acc = add(acc, t)
        return acc

    sx = total([ext(v, FX_W) for v in x])
    sy = total([ext(v, FX_W) for v in y])
    xbar = C.divide_into(nl, sx, const_m)[0][:FX_IN]
    ybar = C.divide_into(nl, sy, const_m)[0][:FX_IN]
    dx = [sub(v, xbar) for v in x]
    dy = [sub(v, ybar) for v in y]
    num = total([C.multiply_into(nl, dy[i], dx[i]) for i in range(m)])
    den = total([C.multiply_into(nl, dx[i], dx[i]) for i in range(m)])
    omega = C.divide_into(nl, shifted(num, 2 * FX_W), den)[0]
    u = sub(shifted(sy, 2 * FX_W), C.multiply_into(nl, omega, sx))
    b = C.divide_into(nl, u, const_m)[0]
    nl.outputs = omega + b
    return nl


def formula_input_bits(x, y):
    """u8[n_inputs, sets] in the input order of build_formula_netlist
    (x, y: int64[sets, m])."""
    from mk_inputs import to_bits
    x, y = np.atleast_2d(x), np.atleast_2d(y)
    vals = np.concatenate([x, y], axis=1)               # [sets, 2m]
    return to_bits(vals.ravel(), FX_IN).reshape(vals.shape[0], -1).T.copy()


def formula_input_owner(m: int, k: int):
    """Party owning each input bit: every party encrypts its own pairs,
    pair i belonging to party i mod k."""
    own = [i % k for i in range(m)] * 2
    return np.repeat(np.array(own, np.int64), FX_IN)
