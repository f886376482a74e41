"""Gate netlists of the k-bit two's-complement operators (TEST INFRASTRUCTURE).

The oracle's own builders, written independently of the library's C++
builders; the tests check that both produce the same gate list and that every
netlist computes the right integer function.

Netlist conventions: wire 0 is the constant 0 and wire 1 the constant 1
(noiseless trivial ciphertexts); inputs follow; every gate appends one output
wire.  A gate is (type, in1, in2, out); NOT (type 6) is free (§4.1 Eq. (8)),
its in2 is 0.

Operators (§3.3 plain designs, §4.3-§4.5 homomorphic versions, Algs. 3-6):
* adder (k bits, Alg. 3): a ripple of k one-bit adders with carry-in the
  constant 0, each x = a XOR b, s = x XOR c, c' = (a AND b) OR (x AND c);
  5k gates as counted in §5.2 (the printed carrier uses 3 AND + 2 OR, which
  gives 7 gates per bit and contradicts the 5k count; this reading keeps 5k
  and the same function).  The final carry is computed and discarded.
* subtractor (Alg. 5): b is inverted by k bootstrapped XORs with the constant
  1, then added with carry-in 1: 6k gates as counted in §5.4.
* multiplier (signed k x k -> 2k bits): the figure of §3.3 is missing and
  Alg. 4's bounds are garbled, so this is a Baugh-Wooley carry-save array in
  the paper's style: AND partial products, NAND for the mixed-sign ones
  (negative weights folded into inversions), rows of full adders, a final
  ripple adder, and the constants 2^k (injected at weight k) and 2^(2k-1)
  (a free inversion of the top bit).
* divider (signed, truncating): operands are made non-negative by the
  compensation device of §3.3 (XOR with the sign, then add the sign), an
  array of CAS cells (§4.5: out = a XOR ((b XOR p) XOR c),
  c' = ((a OR c) AND (b XOR p)) OR (a AND c)) performs non-restoring
  division, the negative final remainder is corrected, and the quotient
  (sign sA XOR sB) and remainder (sign sA) are compensated back.  Results are
  mod 2^k.
Multiplier and divider fold gates with constant inputs (AND(x,0)=0, ...).
"""
from __future__ import annotations

import numpy as np

NAND, AND, OR, NOR, XOR, XNOR, NOT = 0, 1, 2, 3, 4, 5, 6
ZERO, ONE = 0, 1


class Netlist:
    def __init__(self, fold: bool):
        self.fold = fold
        self.n_wires = 2
        self.gates = []          # [type, in1, in2, out]
        self.inputs = []
        self.outputs = []
        self._not_of = {}        # wire -> the wire it is the NOT of

    def input(self):
        w = self.n_wires
        self.n_wires += 1
        self.inputs.append(w)
        return w

    def _new(self, t, a, b):
        w = self.n_wires
        self.n_wires += 1
        self.gates.append([t, a, b, w])
        return w

    def NOT(self, a):
        if self.fold:
            if a in (ZERO, ONE):
                return ONE - a
            if a in self._not_of:
                return self._not_of[a]
        w = self._new(NOT, a, 0)
        self._not_of[w] = a
        return w

    def gate(self, t, a, b):
        if self.fold:
            ca, cb = a in (ZERO, ONE), b in (ZERO, ONE)
            if ca and cb:
                return _plain(t, a, b)
            if ca:
                a, b = b, a
                cb = True
            if cb:                      # b is a constant, a a wire
                v = b
                if t == AND:
                    return a if v else ZERO
                if t == OR:
                    return ONE if v else a
                if t == XOR:
                    return self.NOT(a) if v else a
                if t == XNOR:
                    return a if v else self.NOT(a)
                if t == NAND:
                    return self.NOT(a) if v else ONE
                if t == NOR:
                    return ZERO if v else self.NOT(a)
        return self._new(t, a, b)

    # --- building blocks ---
    def full_add(self, a, b, c):
        """x = a^b, s = x^c, c' = (a&b) | (x&c): 5 gates."""
        x = self.gate(XOR, a, b)
        s = self.gate(XOR, x, c)
        t1 = self.gate(AND, a, b)
        t2 = self.gate(AND, x, c)
        return s, self.gate(OR, t1, t2)

    def half_add(self, a, b):
        return self.gate(XOR, a, b), self.gate(AND, a, b)

    def add_bits(self, bits, want_carry=True):
        """Sum of 1-3 bits of equal weight: (sum, carry or None)."""
        if len(bits) == 1:
            return bits[0], None
        if len(bits) == 2:
            if want_carry:
                return self.half_add(*bits)
            return self.gate(XOR, *bits), None
        if want_carry:
            return self.full_add(*bits)
        return self.gate(XOR, self.gate(XOR, bits[0], bits[1]), bits[2]), None

    def ripple_add(self, a, b, cin):
        """k-bit ripple-carry addition (mod 2^k) with full adders throughout."""
        out = []
        c = cin
        for ai, bi in zip(a, b):
            s, c = self.full_add(ai, bi, c)
            out.append(s)
        return out

    def compensate(self, x, s):
        """(x XOR s) + s: two's-complement absolute value / negation by a sign
        wire s (the compensation device of §3.3)."""
        y = [self.gate(XOR, xi, s) for xi in x]
        out = []
        c = s
        for i, yi in enumerate(y):
            out.append(self.gate(XOR, yi, c))
            if i + 1 < len(y):
                c = self.gate(AND, yi, c)
        return out


def _plain(t, a, b):
    if t == NAND:
        return 1 - (a & b)
    if t == AND:
        return a & b
    if t == OR:
        return a | b
    if t == NOR:
        return 1 - (a | b)
    if t == XOR:
        return a ^ b
    if t == XNOR:
        return 1 - (a ^ b)
    raise ValueError(t)


# ------------------------------------------------------------ operators ----

def adder(k: int) -> Netlist:
    """Alg. 3: k-bit two's-complement adder, 5k gates."""
    nl = Netlist(fold=False)
    a = [nl.input() for _ in range(k)]
    b = [nl.input() for _ in range(k)]
    nl.outputs = nl.ripple_add(a, b, ZERO)
    return nl


def subtractor(k: int) -> Netlist:
    """Alg. 5: a - b = a + NOT(b) + 1 with bootstrapped inversions, 6k gates."""
    nl = Netlist(fold=False)
    a = [nl.input() for _ in range(k)]
    b = [nl.input() for _ in range(k)]
    nb = [nl.gate(XOR, bi, ONE) for bi in b]
    nl.outputs = nl.ripple_add(a, nb, ONE)
    return nl


def multiply_into(nl: Netlist, a, b):
    """Signed k x k -> 2k product bits (LSB first) of wires a, b."""
    k = len(a)
    # partial products, mixed-sign ones inverted (NAND)
    q = [[nl.gate(NAND if (i == k - 1) != (j == k - 1) else AND, a[j], b[i])
          for j in range(k)] for i in range(k)]
    S = {w: q[0][w] for w in range(k)}      # sum bit per weight
    C = {}                                  # carry bit per weight
    out = [S.pop(0)]
    for i in range(1, k):
        S2, C2 = {}, {}
        for w in range(i, i + k):
            bits = [x for x in (S.get(w), C.get(w), q[i][w - i]) if x is not None]
            if i == 1 and w == k:
                bits.append(ONE)            # Baugh-Wooley constant 2^k
            s, c = nl.add_bits(bits)
            S2[w] = s
            if c is not None:
                C2[w + 1] = c
        S, C = S2, C2
        out.append(S.pop(i))
    c = None
    for w in range(k, 2 * k):
        bits = [x for x in (S.get(w), C.get(w), c) if x is not None]
        s, c = nl.add_bits(bits, want_carry=w < 2 * k - 1)
        out.append(s)
    out[2 * k - 1] = nl.NOT(out[2 * k - 1])   # Baugh-Wooley constant 2^(2k-1)
    return out


def multiplier(k: int) -> Netlist:
    nl = Netlist(fold=True)
    a = [nl.input() for _ in range(k)]
    b = [nl.input() for _ in range(k)]
    nl.outputs = multiply_into(nl, a, b)
    return nl


def cas(nl: Netlist, a, b, c, p):
    """Controlled add/subtract cell of §4.5 (7 gates before folding)."""
    t = nl.gate(XOR, b, p)
    u = nl.gate(XOR, t, c)
    out = nl.gate(XOR, a, u)
    cout = nl.gate(OR, nl.gate(AND, nl.gate(OR, a, c), t), nl.gate(AND, a, c))
    return out, cout


def divide_into(nl: Netlist, A, B):
    """Signed truncating division: (quotient, remainder) bits mod 2^k, with
    len(A) dividend bits (k or 2k) and k = len(B) divisor bits."""
    kA, k = len(A), len(B)
    sA, sB = A[kA - 1], B[k - 1]
    ua = nl.compensate(A, sA)                 # |A|, kA bits unsigned
    ub = nl.compensate(B, sB)                 # |B|, k bits unsigned
    D = ub + [ZERO]                           # k+1 bits
    R = [ZERO] * (k + 1)                      # partial remainder, k+1 bits
    q = []
    p = ONE                                   # first step subtracts
    for i in range(kA - 1, -1, -1):
        Rs = [ua[i]] + R[:k]                  # 2R + A_i (mod 2^(k+1))
        c = p
        newR = []
        for t in range(k + 1):
            o, c = cas(nl, Rs[t], D[t], c, p)
            newR.append(o)
        R = newR
        qi = nl.NOT(R[k])                     # 1 iff the remainder is >= 0
        q.append(qi)
        p = qi
    q = q[::-1]                               # LSB first
    # remainder correction: R < 0 -> R + D
    corr = [nl.gate(AND, D[t], R[k]) for t in range(k)]
    rem = nl.ripple_add(R[:k], corr, ZERO)
    sQ = nl.gate(XOR, sA, sB)
    quot = nl.compensate(q[:k], sQ)
    rem = nl.compensate(rem, sA)
    return quot, rem


def divider(k: int, dividend_bits: int | None = None) -> Netlist:
    nl = Netlist(fold=True)
    kA = dividend_bits or k
    A = [nl.input() for _ in range(kA)]
    B = [nl.input() for _ in range(k)]
    quot, rem = divide_into(nl, A, B)
    nl.outputs = quot + rem
    return nl


# ----------------------------------------------------------- evaluation ----

def naive_gate(t: int) -> Netlist:
    """The comparison design of Table 2 (left column): every gate built from
    bootstrapped NAND gates only, NOT included (NOT a = NAND(a, a)).  Inputs
    a, b (b unused by NOT); one output.  Depths: NAND and NOT 1, AND and OR
    2, NOR and XOR 3, XNOR 4."""
    nl = Netlist(fold=False)
    a, b = nl.input(), nl.input()

    def nand(x, y):
        return nl._new(NAND, x, y)

    def naive_or(x, y):
        return nand(nand(x, x), nand(y, y))

    def naive_xor(x, y):
        n = nand(x, y)
        return nand(nand(x, n), nand(y, n))

    if t == NAND:
        out = nand(a, b)
    elif t == AND:
        n = nand(a, b)
        out = nand(n, n)
    elif t == OR:
        out = naive_or(a, b)
    elif t == NOR:
        o = naive_or(a, b)
        out = nand(o, o)
    elif t == XOR:
        out = naive_xor(a, b)
    elif t == XNOR:
        x = naive_xor(a, b)
        out = nand(x, x)
    elif t == NOT:
        out = nand(a, a)
    else:
        raise ValueError("gate type")
    nl.outputs = [out]
    return nl


def eval_plain(nl: Netlist, in_bits) -> np.ndarray:
    """Evaluate on plaintext bits, vectorised over instances.
    in_bits: u8[n_inputs, B]; returns u8[n_outputs, B]."""
    in_bits = np.asarray(in_bits, np.uint8)
    Bn = in_bits.shape[1]
    val = np.zeros((nl.n_wires, Bn), np.uint8)
    val[ONE] = 1
    for w, row in zip(nl.inputs, in_bits):
        val[w] = row
    for t, a, b, o in nl.gates:
        x, y = val[a], val[b]
        if t == NOT:
            val[o] = 1 - x
        elif t == AND:
            val[o] = x & y
        elif t == OR:
            val[o] = x | y
        elif t == XOR:
            val[o] = x ^ y
        elif t == NAND:
            val[o] = 1 - (x & y)
        elif t == NOR:
            val[o] = 1 - (x | y)
        elif t == XNOR:
            val[o] = 1 - (x ^ y)
    return val[nl.outputs]


def eval_encrypted(nl: Netlist, keys, in_ct):
    """Evaluate gate by gate with the oracle's bootstrapped gates.
    in_ct: u32[n_inputs, B, kn+1]; returns u32[n_outputs, B, kn+1]."""
    from . import tfhe
    P = keys.params
    in_ct = np.asarray(in_ct, np.uint32)
    Bn = in_ct.shape[1]
    evk = keys.evaluation_key()
    val = {ZERO: np.repeat(tfhe.trivial(P, [0]), Bn, axis=0),
           ONE: np.repeat(tfhe.trivial(P, [1]), Bn, axis=0)}
    for w, ct in zip(nl.inputs, in_ct):
        val[w] = ct
    for t, a, b, o in nl.gates:
        if t == NOT:
            val[o] = tfhe.lwe_not(val[a])
        else:
            val[o] = np.stack([tfhe.bootstrapped_gate(keys, t, val[a][i], val[b][i], evk)
                               for i in range(Bn)])
    return np.stack([val[w] for w in nl.outputs])


def gate_count(nl: Netlist) -> int:
    """Bootstrapped gates (NOT is free)."""
    return sum(1 for g in nl.gates if g[0] != NOT)
