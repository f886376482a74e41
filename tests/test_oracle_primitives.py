"""Pins of the oracle's primitives against definitions, textbook routines and
library routines (CPU only)."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import prng, tfhe
from oracle._native import negacyclic_mac

M32 = (1 << 32) - 1


# ----------------------------------------------------------- generator ----

@pytest.mark.parametrize("seed,party,obj,idx", [(0, 0, 1, 0), (123, 1, 9, 77),
                                                (2**63 + 5, 0xFFFF, 12, 2**40)])
def test_philox_matches_numpy(seed, party, obj, idx):
    """Philox4x64-10 (SC'11 definition) equals numpy.random.Philox.

    numpy increments its counter before each block, so numpy counter c-1
    produces our block c."""
    ours = prng.philox4x64_10(np.arange(1, 4, dtype=np.uint64), np.uint64(idx),
                              np.uint64(0), np.uint64(0), np.uint64(seed),
                              np.uint64((party << 32) | obj))
    bg = np.random.Philox(key=np.array([seed, (party << 32) | obj], np.uint64),
                          counter=np.array([0, idx, 0, 0], np.uint64))
    ref = bg.random_raw(12).reshape(3, 4)
    assert np.array_equal(np.stack(ours, axis=-1), ref)


def test_draw_order_and_determinism():
    d = prng.draws_u32(7, 1, 3, [5, 6], 20)
    w = prng.philox4x64_10(np.arange(3, dtype=np.uint64), np.uint64(5), 0, 0,
                           np.uint64(7), np.uint64((1 << 32) | 3))
    words = np.stack(w, axis=-1).reshape(-1)
    halves = np.stack([words & M32, words >> 32], axis=-1).reshape(-1)
    assert np.array_equal(d[0], halves[:20].astype(np.uint32))
    assert np.array_equal(d, prng.draws_u32(7, 1, 3, [5, 6], 20))
    assert not np.array_equal(d[0], d[1])


@pytest.mark.parametrize("s", [12, 15, 20, 30])
def test_noise_moments(s):
    e = prng.noise(11, 0, prng.OBJ_PK_E, np.arange(50), 4000, s).astype(np.int64)
    e = np.where(e >= 1 << 31, e - (1 << 32), e).astype(np.float64)
    sigma = 2.0 ** (32 - s)
    assert abs(e.mean()) < 0.02 * sigma + 1
    assert 0.97 < e.std() / sigma < 1.03 or (s == 30 and abs(e.std() - sigma) < 0.2)
    # Irwin-Hall(12) is bounded by 6 standard deviations
    assert np.abs(e).max() <= 6 * sigma + 1


def test_binary_and_uniform_balance():
    b = prng.binary(3, 0, prng.OBJ_SK_RLWE, 0, 100000)
    assert set(np.unique(b)) == {0, 1} and abs(b.mean() - 0.5) < 0.01
    u = prng.uniform_torus(3, 0, prng.OBJ_CRS, 0, 100000).astype(np.float64)
    assert abs(u.mean() / 2**32 - 0.5) < 0.01


# ---------------------------------------------------- negacyclic product ----

def _textbook(u, K):
    """Full integer product with numpy.convolve, then fold X^N = -1."""
    N = len(K)
    full = np.convolve(np.asarray(u, dtype=object), np.asarray(K, dtype=object))
    full = np.concatenate([full, np.zeros(2 * N - len(full), dtype=object)])
    return np.array([(full[m] - full[m + N]) % (1 << 32) for m in range(N)],
                    dtype=np.uint64)


def _brute(u, K):
    """Monomial-by-monomial product with explicit reduction of exponents."""
    N = len(K)
    out = [0] * N
    for p, up in enumerate(u):
        for q, kq in enumerate(K):
            e, sgn = p + q, 1
            while e >= N:
                e, sgn = e - N, -sgn
            out[e] += sgn * int(up) * int(kq)
    return [v % (1 << 32) for v in out]


@pytest.mark.parametrize("N", [1, 2, 4, 8])
def test_negacyclic_bruteforce_small(N):
    rng = np.random.default_rng(N)
    for _ in range(20):
        u = rng.integers(-128, 128, N)
        K = rng.integers(0, 1 << 32, N, dtype=np.uint64).astype(np.uint32)
        acc = np.zeros(N, np.uint32)
        negacyclic_mac(acc, u, K)
        assert acc.tolist() == _brute(u, K)


@pytest.mark.parametrize("N", [64, 256, 1024])
def test_negacyclic_matches_textbook(N):
    rng = np.random.default_rng(N + 1)
    u = rng.integers(-128, 128, N)
    u[:3] = [-128, 127, 0]
    K = rng.integers(0, 1 << 32, N, dtype=np.uint64).astype(np.uint32)
    K[:2] = [M32, 1 << 31]
    acc = rng.integers(0, 1 << 32, N, dtype=np.uint64).astype(np.uint32)
    start = acc.astype(np.uint64)
    negacyclic_mac(acc, u, K)
    ref = (_textbook(u, K) + start) & M32
    assert np.array_equal(acc.astype(np.uint64), ref)


def test_negacyclic_commutes_for_integer_polys():
    rng = np.random.default_rng(5)
    N = 128
    a = rng.integers(-100, 100, N)
    b = rng.integers(-100, 100, N)
    x = np.zeros(N, np.uint32)
    y = np.zeros(N, np.uint32)
    negacyclic_mac(x, a, tfhe.u32(b))
    negacyclic_mac(y, b, tfhe.u32(a))
    assert np.array_equal(x, y)


# ------------------------------------------------- rotation / mod switch ----

def _monomial_neg(a, N):
    """X^(-a) as an integer polynomial mod X^N + 1."""
    e = (2 * N - a) % (2 * N)
    u = np.zeros(N, np.int64)
    if e < N:
        u[e] = 1
    else:
        u[e - N] = -1
    return u


@pytest.mark.parametrize("a", [0, 1, 5, 63, 64, 65, 100, 127])
def test_rotate_is_monomial_product(a):
    N = 64
    rng = np.random.default_rng(a)
    P = rng.integers(0, 1 << 32, N, dtype=np.uint64).astype(np.uint32)
    ref = np.zeros(N, np.uint32)
    negacyclic_mac(ref, _monomial_neg(a, N), P)
    assert np.array_equal(tfhe.rotate(P, a), ref)


def test_rotate_group_laws():
    N = 32
    P = np.arange(1, N + 1, dtype=np.uint32) * 7919
    assert np.array_equal(tfhe.rotate(P, 2 * N), P)                       # X^2N = 1
    assert np.array_equal(tfhe.rotate(P, N), tfhe.u32(-P.astype(np.int64)))  # X^N = -1
    assert np.array_equal(tfhe.rotate(tfhe.rotate(P, 7), 9), tfhe.rotate(P, 16))


def test_modulus_switch_is_rounding():
    N = 1024
    xs = [0, 1, (1 << 20) - 1, 1 << 20, (1 << 21) - 1, 1 << 31, M32, M32 - (1 << 20),
          M32 - (1 << 20) + 1, 123456789]
    rng = np.random.default_rng(0)
    xs += rng.integers(0, 1 << 32, 200, dtype=np.uint64).tolist()
    got = tfhe.modulus_switch(np.array(xs, dtype=np.uint64).astype(np.uint32), N)
    for x, g in zip(xs, got):
        f = Fraction(int(x) * 2 * N, 1 << 32)
        ref = int(f + Fraction(1, 2)) % (2 * N)      # round half up, mod 2N
        assert g == ref, (x, g, ref)


# ------------------------------------------------------- decomposition ----

def _balanced_digits(R, beta, ell):
    """Digits of R (mod 2^(beta*ell)) in balanced base 2^beta, MSB first,
    by repeated division with remainders in [-2^(beta-1), 2^(beta-1))."""
    B = 1 << beta
    out = []
    R %= 1 << (beta * ell)
    for _ in range(ell):
        r = R % B
        if r >= B // 2:
            r -= B
        out.append(r)
        R = (R - r) // B
    return out[::-1]


@pytest.mark.parametrize("beta,ell", [(8, 2), (8, 3), (7, 3), (10, 2)])
def test_decompose_matches_balanced_base(beta, ell):
    rng = np.random.default_rng(beta * 10 + ell)
    step = 1 << (32 - beta * ell)
    xs = [0, 1, M32, 1 << 31, step // 2, step // 2 - 1, step - 1, (1 << 31) - step // 2]
    xs += rng.integers(0, 1 << 32, 500, dtype=np.uint64).tolist()
    x = np.array(xs, dtype=np.uint64).astype(np.uint32)
    d = tfhe.decompose(x, beta, ell)
    half = 1 << (beta - 1)
    assert d.min() >= -half and d.max() < half
    for i, xv in enumerate(xs):
        R = (int(xv) + step // 2) // step          # round half up to the grid
        assert d[:, i].tolist() == _balanced_digits(R, beta, ell)
        rec = sum(int(d[p, i]) << (32 - beta * (p + 1)) for p in range(ell))
        diff = (rec - int(xv)) % (1 << 32)
        diff = diff - (1 << 32) if diff >= 1 << 31 else diff
        assert -step // 2 < diff <= step // 2
    assert not tfhe.decompose(np.zeros(4, np.uint32), beta, ell).any()
