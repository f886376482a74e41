"""Pins of the oracle's operator netlists: exhaustive plaintext simulation
against integer arithmetic, gate counts against the paper, the LR netlist
against its plain-integer definition, and encrypted evaluation at toy shapes
(CPU only)."""
import os

import numpy as np
import pytest

import mk_inputs as mi
from oracle import circuits as C
from oracle import lr
from oracle import params as OP
from oracle import tfhe

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _all_pairs(k):
    v = np.arange(-(1 << (k - 1)), 1 << (k - 1))
    a, b = np.meshgrid(v, v, indexing="ij")
    return a.ravel(), b.ravel()


def _run(nl, k_in, a, b, kb=None):
    kb = kb or k_in
    bits = np.concatenate([mi.to_bits(a, k_in).T, mi.to_bits(b, kb).T])
    return C.eval_plain(nl, bits)


def _wrap(v, k):
    v = np.asarray(v, np.int64) & ((1 << k) - 1)
    return np.where(v >= 1 << (k - 1), v - (1 << k), v)


def _trunc_div(a, b):
    q = np.abs(a) // np.abs(b) * np.sign(a) * np.sign(b)
    return q, a - q * b


@pytest.mark.parametrize("k", range(1, 9))
def test_adder_subtractor_exhaustive(k):
    a, b = _all_pairs(k)
    add = mi.from_bits(_run(C.adder(k), k, a, b).T)
    sub = mi.from_bits(_run(C.subtractor(k), k, a, b).T)
    assert np.array_equal(add, _wrap(a + b, k))
    assert np.array_equal(sub, _wrap(a - b, k))


@pytest.mark.parametrize("k", range(2, 9))
def test_multiplier_exhaustive(k):
    a, b = _all_pairs(k)
    got = mi.from_bits(_run(C.multiplier(k), k, a, b).T)
    assert np.array_equal(got, a * b)       # 2k-bit product is exact


@pytest.mark.parametrize("k", range(2, 9))
def test_divider_exhaustive(k):
    a, b = _all_pairs(k)
    keep = b != 0
    a, b = a[keep], b[keep]
    out = _run(C.divider(k), k, a, b)
    q, r = mi.from_bits(out[:k].T), mi.from_bits(out[k:].T)
    qe, re = _trunc_div(a, b)
    assert np.array_equal(q, _wrap(qe, k))   # -2^(k-1) / -1 wraps
    assert np.array_equal(r, _wrap(re, k))


@pytest.mark.parametrize("k", [3, 5])
def test_divider_double_width_dividend(k):
    """Paper form (§3.3): 2k-bit dividend, k-bit divisor, small quotients."""
    rng = np.random.default_rng(k)
    b = rng.integers(-(1 << (k - 1)), 1 << (k - 1), 3000)
    b[b == 0] = 1
    q0 = rng.integers(-(1 << (k - 2)), 1 << (k - 2), 3000)
    r0 = rng.integers(0, np.abs(b))
    a = q0 * b + np.where(q0 * b < 0, -r0, r0)
    out = _run(C.divider(k, 2 * k), 2 * k, a, b, kb=k)
    q, r = mi.from_bits(out[:k].T), mi.from_bits(out[k:].T)
    qe, re = _trunc_div(a, b)
    assert np.array_equal(q, _wrap(qe, k)) and np.array_equal(r, _wrap(re, k))


def test_sixteen_bit_operators_random():
    a, b = mi.operand_pairs(3000, 16, seed=4, nonzero_second=True)
    assert np.array_equal(mi.from_bits(_run(C.adder(16), 16, a, b).T), _wrap(a + b, 16))
    assert np.array_equal(mi.from_bits(_run(C.subtractor(16), 16, a, b).T), _wrap(a - b, 16))
    assert np.array_equal(mi.from_bits(_run(C.multiplier(16), 16, a, b).T), a * b)
    out = _run(C.divider(16), 16, a, b)
    qe, re = _trunc_div(a, b)
    assert np.array_equal(mi.from_bits(out[:16].T), _wrap(qe, 16))
    assert np.array_equal(mi.from_bits(out[16:].T), _wrap(re, 16))


def test_gate_counts_against_paper():
    """Adder 5k and subtractor 6k as printed (Tables 3 and 5); the multiplier
    and divider are this design's arrays, reported beside 7k(k-1) and
    7k^2+2k+1."""
    rows = {}
    for line in open(os.path.join(GOLD, "paper_gate_counts.txt")):
        if line.startswith("#") or ":" not in line:
            continue
        name, *pairs = line.split()
        rows[name] = {int(p.split(":")[0]): int(p.split(":")[1]) for p in pairs}
    for k, n in rows["adder"].items():
        assert C.gate_count(C.adder(k)) == n == 5 * k
    for k, n in rows["subtractor"].items():
        assert C.gate_count(C.subtractor(k)) == n == 6 * k
    for k, n in rows["multiplier"].items():
        assert n == 7 * k * (k - 1)
        assert C.gate_count(C.multiplier(k)) <= n + 2 * k
    assert C.gate_count(C.multiplier(8)) == 333


def test_lr_netlist_matches_integer_replica():
    X, y, _ = mi.lr_data(6, 3, seed=5)
    w = np.array([100, -50, 7])
    nl = lr.build_netlist(6, 3)
    out = C.eval_plain(nl, lr.input_bits(X, y, w))
    got = mi.from_bits(out.reshape(3, 16))
    assert np.array_equal(got, lr.replica_step(X, y, w))


def test_lr_replica_tracks_float_gradient_descent():
    """The integer step is the float GD step of §3.4 up to fixed-point
    rounding: compare w after a few iterations from w = 0."""
    X, y, wt = mi.lr_data(64, 4, seed=5)
    w = np.zeros(4, np.int64)
    wf = np.zeros(4)
    Xf, yf = X / 256.0, y / 256.0
    for _ in range(3):
        w = lr.replica_step(X, y, w)
        wf = wf - (1 / 64) * (1 / 64) * (Xf.T @ (Xf @ wf - yf))
    assert np.abs(w / 256.0 - wf).max() < 0.02


@pytest.mark.slow
def test_lr_netlist_config5_size():
    X, y, _ = mi.lr_data(64, 4, seed=5)
    w = np.zeros(4, np.int64)
    nl = lr.build_netlist(64, 4)
    out = C.eval_plain(nl, lr.input_bits(X, y, w))
    assert np.array_equal(mi.from_bits(out.reshape(4, 16)), lr.replica_step(X, y, w))


def test_divider_quotient_bits_beyond_its_range():
    """The closed-form regression relies on the divider returning the low k
    bits of the truncated quotient for every dividend: 2k-bit dividends and
    k-bit divisors, exhaustively at k = 4, including quotients that overflow
    k bits."""
    k = 4
    a = np.arange(-(1 << (2 * k - 1)), 1 << (2 * k - 1))
    b = np.arange(-(1 << (k - 1)), 1 << (k - 1))
    a, b = (v.ravel() for v in np.meshgrid(a, b[b != 0], indexing="ij"))
    out = _run(C.divider(k, 2 * k), 2 * k, a, b, kb=k)
    qe, _ = _trunc_div(a, b)
    assert np.array_equal(mi.from_bits(out[:k].T), _wrap(qe, k))


def _least_squares(x, y):
    A = np.vstack([np.asarray(x, float), np.ones(len(x))]).T
    return np.linalg.lstsq(A, np.asarray(y, float), rcond=None)[0]


@pytest.mark.parametrize("m,sets", [(64, 150), (16, 100)])
def test_lr_formula_replica_tracks_least_squares(m, sets):
    """§3.4 Eqs. (2)-(3): the integer closed form against float least
    squares.  With x̄, ȳ truncated (errors below 1), the centred sums are off
    by less than m each, so the slope is off by at most
    m (1 + |ω|) / sum (x - x̄)^2 + 2^-F, and the intercept by that times |x̄|
    plus 2^-F."""
    x, y, _, _ = mi.formula_lr_data(sets, m, seed=m)
    f = 2.0 ** -lr.FRAC_F
    for xs, ys in zip(x, y):
        om, b = lr.formula_replica(xs, ys)
        w, c = _least_squares(xs, ys)
        sxx = ((xs - xs.mean()) ** 2).sum()
        slope_tol = m * (1 + abs(w)) / sxx + f
        assert abs(om * f - w) <= slope_tol
        assert abs(b * f - c) <= slope_tol * abs(xs.mean()) + f


def test_lr_formula_exact_on_a_centred_line():
    """With integer means the centred sums are exact: y = 2x + 3 over
    x = -3..3 (twice) gives slope 2 and intercept 3 exactly (Q8.8)."""
    x = np.tile(np.arange(-3, 4), 2)
    om, b = lr.formula_replica(x, 2 * x + 3)
    assert (om, b) == (512, 768)
    # constant y: slope 0, intercept y
    assert lr.formula_replica(x, np.full(14, -5)) == (0, -5 * 256)


def test_lr_formula_netlist_matches_replica():
    """The netlist equals the integer definition, including full-range int8
    data where every sum wraps, and on the regression workload."""
    rng = np.random.default_rng(12)
    x = rng.integers(-128, 128, size=(40, 5))
    y = rng.integers(-128, 128, size=(40, 5))
    xw, yw, _, _ = mi.formula_lr_data(4, 5, seed=3)
    x, y = np.concatenate([x, xw]), np.concatenate([y, yw])
    keep = []
    for i in range(len(x)):
        try:
            keep.append((i, lr.formula_replica(x[i], y[i])))
        except ZeroDivisionError:
            pass
    idx = [i for i, _ in keep]
    assert len(idx) > 30
    out = C.eval_plain(lr.build_formula_netlist(5), lr.formula_input_bits(x[idx], y[idx]))
    got = list(zip(mi.from_bits(out[:16].T).tolist(), mi.from_bits(out[16:].T).tolist()))
    assert got == [v for _, v in keep]


def test_lr_formula_netlist_workload_size():
    x, y, _, _ = mi.formula_lr_data(3, 64, seed=5)
    nl = lr.build_formula_netlist(64)
    out = C.eval_plain(nl, lr.formula_input_bits(x, y))
    got = list(zip(mi.from_bits(out[:16].T).tolist(), mi.from_bits(out[16:].T).tolist()))
    assert got == [lr.formula_replica(a, b) for a, b in zip(x, y)]


@pytest.mark.parametrize("op,k", [("add", 3), ("sub", 2), ("mul", 2), ("div", 2)])
def test_encrypted_operators_exhaustive_toy(op, k):
    """Encrypted evaluation of every operand pair at the toy shape: operand a
    encrypted by party 0, b by party 1; outputs decrypt to the integer result."""
    K = tfhe.generate(OP.TOY, 31)
    nl = {"add": C.adder, "sub": C.subtractor, "mul": C.multiplier, "div": C.divider}[op](k)
    a, b = _all_pairs(k)
    if op == "div":
        keep = b != 0
        a, b = a[keep], b[keep]
    ca = np.stack([tfhe.encrypt(K, 0, col, seed=100 + i)
                   for i, col in enumerate(mi.to_bits(a, k).T)])
    cb = np.stack([tfhe.encrypt(K, 1, col, seed=200 + i)
                   for i, col in enumerate(mi.to_bits(b, k).T)])
    outs = C.eval_encrypted(nl, K, np.concatenate([ca, cb]))
    dec = np.stack([tfhe.decrypt(K, o) for o in outs])
    assert np.array_equal(dec, _run(nl, k, a, b))


@pytest.mark.parametrize("t", [C.NAND, C.AND, C.OR, C.NOR, C.XOR, C.XNOR, C.NOT])
def test_naive_nand_gates(t):
    """Table 2's comparison design: every gate from bootstrapped NANDs only.
    Truth tables on all inputs (plain and encrypted at the toy shape); only
    NAND gates; the depths 1/2/2/3/3/4/1 that make its times multiples of one
    bootstrap."""
    nl = C.naive_gate(t)
    assert all(g[0] == C.NAND for g in nl.gates)
    a = np.array([0, 0, 1, 1], np.uint8)
    b = np.array([0, 1, 0, 1], np.uint8)
    want = [1 - x for x in a] if t == C.NOT else [mi.plain_gate(t, int(x), int(y)) for x, y in zip(a, b)]
    assert C.eval_plain(nl, np.stack([a, b]))[0].tolist() == want
    depth = {}
    for typ, x, y, o in nl.gates:
        depth[o] = 1 + max(depth.get(x, 0), depth.get(y, 0))
    assert depth[nl.outputs[0]] == {C.NAND: 1, C.AND: 2, C.OR: 2, C.NOR: 3, C.XOR: 3, C.XNOR: 4, C.NOT: 1}[t]
    K = tfhe.generate(OP.TOY, 32)
    ct = np.stack([tfhe.encrypt(K, 0, a, seed=40), tfhe.encrypt(K, 1, b, seed=41)])
    outs = C.eval_encrypted(nl, K, ct)
    assert tfhe.decrypt(K, outs[0]).tolist() == want
