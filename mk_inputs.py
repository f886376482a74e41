"""Seeded synthetic workloads for multi-key gate bootstrapping.

This module is shared by the tests, the benchmark and the oracle.  It holds
no arithmetic of the encryption scheme: it only draws plaintext bits, gate
types, integer operands and fixed-point regression data from numpy's
PCG64 generator, so that every side of a comparison starts from the same
plaintexts.  Keys, encryption randomness and noise are NOT drawn here; each
implementation derives them from its own counter-based generator.

Workloads (sizes follow the paper's experiments, §5.1-§5.5, with the data
synthetic because the paper does not publish its data):

* ``gate_batch``      - independent two-input gates with uniform types and
                        uniform input bits (Table 2 style per-gate timing).
* ``truth_table``     - every gate type on every input combination.
* ``operand_pairs``   - k-bit two's-complement operand pairs (Tables 3-6).
* ``lr_data``         - fixed-point linear-regression data (§4.6, Table 8).
"""
from __future__ import annotations

import numpy as np

# Gate type codes shared by every side (plain enumeration, no arithmetic).
NAND, AND, OR, NOR, XOR, XNOR, NOT = 0, 1, 2, 3, 4, 5, 6
BOOTSTRAPPED_GATES = (NAND, AND, OR, NOR, XOR, XNOR)
GATE_NAMES = {NAND: "NAND", AND: "AND", OR: "OR", NOR: "NOR", XOR: "XOR",
              XNOR: "XNOR", NOT: "NOT"}


def plain_gate(t: int, m1: int, m2: int) -> int:
    """Boolean value of gate ``t`` on plaintext bits (for checking only)."""
    if t == NAND:
        return 1 - (m1 & m2)
    if t == AND:
        return m1 & m2
    if t == OR:
        return m1 | m2
    if t == NOR:
        return 1 - (m1 | m2)
    if t == XOR:
        return m1 ^ m2
    if t == XNOR:
        return 1 - (m1 ^ m2)
    if t == NOT:
        return 1 - m1
    raise ValueError(t)


def gate_batch(count: int, seed: int):
    """``count`` gates, types uniform over the six bootstrapped gates, input
    bits uniform.  Returns (types u8[count], m1 u8[count], m2 u8[count])."""
    rng = np.random.Generator(np.random.PCG64(seed))
    types = rng.integers(0, len(BOOTSTRAPPED_GATES), size=count).astype(np.uint8)
    m1 = rng.integers(0, 2, size=count).astype(np.uint8)
    m2 = rng.integers(0, 2, size=count).astype(np.uint8)
    return types, m1, m2


def truth_table(gates=(XOR, NAND)):
    """Every listed gate on all four input combinations, in a fixed order."""
    types, m1, m2 = [], [], []
    for t in gates:
        for a in (0, 1):
            for b in (0, 1):
                types.append(t)
                m1.append(a)
                m2.append(b)
    return (np.array(types, np.uint8), np.array(m1, np.uint8),
            np.array(m2, np.uint8))


def operand_pairs(count: int, bits: int, seed: int, nonzero_second=False):
    """``count`` pairs of ``bits``-bit two's-complement integers drawn
    uniformly from [-2^(bits-1), 2^(bits-1)).  With ``nonzero_second`` the
    second operand is redrawn until it is non-zero (divisors)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lo, hi = -(1 << (bits - 1)), 1 << (bits - 1)
    a = rng.integers(lo, hi, size=count, dtype=np.int64)
    b = rng.integers(lo, hi, size=count, dtype=np.int64)
    if nonzero_second:
        while np.any(b == 0):
            z = b == 0
            b[z] = rng.integers(lo, hi, size=int(z.sum()), dtype=np.int64)
    return a, b


def to_bits(values, bits: int):
    """Two's-complement bits, LSB first: u8[len(values), bits]."""
    v = np.asarray(values, dtype=np.int64) & ((1 << bits) - 1)
    return ((v[:, None] >> np.arange(bits)[None, :]) & 1).astype(np.uint8)


def from_bits(bitarr, signed=True):
    """Inverse of ``to_bits`` over the last axis."""
    b = np.asarray(bitarr, dtype=np.int64)
    bits = b.shape[-1]
    v = (b << np.arange(bits)).sum(axis=-1)
    if signed:
        v = np.where(v >= (1 << (bits - 1)), v - (1 << bits), v)
    return v


def lr_data(m: int, d: int, seed: int, frac_bits: int = 8, noise_std=0.1):
    """Synthetic linear data y = X w + noise, quantised to Q(16-f).f.

    X ~ N(0,1), w ~ U[-1,1], noise ~ N(0, noise_std^2).  Values are rounded
    to the nearest multiple of 2^-frac_bits and saturated to int16.
    Returns (Xq int64[m,d], yq int64[m], w_true float[d]).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    X = rng.standard_normal((m, d))
    w = rng.uniform(-1.0, 1.0, size=d)
    y = X @ w + rng.normal(0.0, noise_std, size=m)
    scale = float(1 << frac_bits)
    q = lambda v: np.clip(np.rint(v * scale), -32768, 32767).astype(np.int64)
    return q(X), q(y), w


def formula_lr_data(sets: int, m: int, seed: int, noise_std=2.0):
    """``sets`` independent one-feature data sets of ``m`` integer pairs for
    the closed-form regression: x uniform in [-16, 15], slope a ~ U[-3, 3],
    intercept c ~ U[-20, 20], y = round(a x + c + noise), noise ~
    N(0, noise_std^2), saturated to int8.  Returns (x int64[sets, m],
    y int64[sets, m], a float[sets], c float[sets])."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.integers(-16, 16, size=(sets, m), dtype=np.int64)
    a = rng.uniform(-3.0, 3.0, size=sets)
    c = rng.uniform(-20.0, 20.0, size=sets)
    y = a[:, None] * x + c[:, None] + rng.normal(0.0, noise_std, size=(sets, m))
    return x, np.clip(np.rint(y), -128, 127).astype(np.int64), a, c
