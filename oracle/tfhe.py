"""Plain CPU oracle of multi-key TFHE gate bootstrapping (TEST INFRASTRUCTURE).

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this module.  The product library never calls it.

What is computed, and where it comes from
-----------------------------------------
Torus elements (§3.1) are Torus32 words: x in [0,1) is held as round(x*2^32)
mod 2^32, and every sum below wraps mod 2^32.

* §3.2 MKTFHE.Setup/KeyGen: a common reference string (CRS) a in T_N[X]^ell,
  and for each party i a binary LWE key s_i (dim n), a binary ring key z_i
  (dim N), a public key b_i = -z_i*a + e, a bootstrapping key of n
  uni-encryptions of the bits of s_i under z_i, and a key-switching key from
  z_i to s_i.  The paper names these objects but prints none of their
  construction; it follows the MKTFHE scheme the paper builds on (Chen,
  Chillotti, Song 2019).  Reading used here:
      uni-encryption of mu under z with fresh binary r:
          d_l  = r*a_l + mu*g_l + e1_l
          f1_l = uniform
          f0_l = -z*f1_l + e2_l + r*g_l          (gadget g_l = 2^(32-beta*l))
      KS_i[q][p][v] = LWE_{s_i}(v * z_{i,q} * 2^(32-log2(B')*(p+1))),  v=1..B'-1
* §3.2 SymEnc: b + <a, s> ~ mu/4, i.e. b = mu*2^30 - <a,s> + e; the
  ciphertext of party i is extended to k slots by zero-padding (§4.1).
* §3.2 SymDec: the mu in {0,1} nearest to the phase b + sum_i <a_i, s_i>,
  i.e. 1 iff the phase lies in [1/8, 5/8).
* §4.1 Eqs. (6)-(11) and Table 1: a gate is a linear combination
  (0, const) + s1*c1 + s2*c2 (LweAdd/LweSub/LweMul, Algs. 1-2) followed by
  one bootstrapping and the multi-key key switch.  Constants (readings in
  CAPITALS differ from the printed equations, which fail the truth table):
      NAND 5/8, -1, -1   AND -1/8, +1, +1   OR 1/8, +1, +1
      NOR  3/8 (PRINTED 1/8 GIVES AND), -1, -1
      XOR  0, +2, -2     XNOR 1/2 (PRINTED 1/4 HAS ZERO MARGIN), -2, +2
      NOT  1/4 - c, no bootstrapping (Eq. (8)).
* §3.2 MKTFHE.NAND "evaluates the decryption circuit": the bootstrapping
  maps a phase in [1/4, 3/4) to 1/4 and any other phase to 0.  Steps:
  modulus switch to Z_2N, blind rotation by k*n hybrid-product CMux steps
  (party-major, bits ascending), sample extraction plus 1/8, key switching.

Every step is written in the paper's (or the cited scheme's) order with no
blocking or fusion; products of polynomials call the schoolbook routine in
``negacyclic.c``.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import prng
from ._native import negacyclic_mac
from .params import Params

M32 = 0xFFFFFFFF

# Gate codes (same enumeration as the shared input generators).
NAND, AND, OR, NOR, XOR, XNOR, NOT = 0, 1, 2, 3, 4, 5, 6

#: gate -> (constant added to b, scale of c1, scale of c2); §4.1, Table 1.
GATE_TABLE = {
    NAND: (0xA0000000, -1, -1),   # 5/8 - c1 - c2
    AND:  (0xE0000000, +1, +1),   # -1/8 + c1 + c2          Eq. (6)
    OR:   (0x20000000, +1, +1),   # 1/8 + c1 + c2           Eq. (7)
    NOR:  (0x60000000, -1, -1),   # 3/8 - c1 - c2           Eq. (9), reading
    XOR:  (0x00000000, +2, -2),   # 2 (c1 - c2)             Eq. (10)
    XNOR: (0x80000000, -2, +2),   # 1/2 - 2 (c1 - c2)       Eq. (11), reading
}
QUARTER = 0x40000000   # 1/4, the encoding scale of SymEnc (§3.2)
EIGHTH = 0x20000000    # 1/8


def u32(x):
    return (np.asarray(x, dtype=np.int64) & M32).astype(np.uint32)


# ---------------------------------------------------------------- keys ----

@dataclass
class PartyKeys:
    s: np.ndarray      # u8[n]          LWE secret
    z: np.ndarray      # u8[N]          ring secret
    pk: np.ndarray     # u32[ell, N]    public key b_i
    bk: np.ndarray     # u32[n, 3, ell, N]   (d, f0, f1) per bit of s_i
    ks: np.ndarray     # u32[N, t, B'-1, n+1] rows (b, a) per (q, p, v)


@dataclass
class Keys:
    params: Params
    crs: np.ndarray                      # u32[ell, N]
    parties: list = field(default_factory=list)

    def evaluation_key(self) -> np.ndarray:
        """(b_0 := -a, b_1..b_k) as u32[k+1, ell, N]: the server-side
        "reconstruction" of the parties' public keys (Alg. 7/8 step 1)."""
        rows = [u32(-self.crs.astype(np.int64))]
        rows += [p.pk for p in self.parties]
        return np.stack(rows)


def gadget(params: Params) -> np.ndarray:
    """g_l = 2^(32 - beta*l) for l = 1..ell, as Python ints."""
    return [1 << (32 - params.bk_log_base * l) for l in range(1, params.bk_ell + 1)]


def setup(params: Params, seed: int) -> Keys:
    """§3.2 Setup: sample the CRS a in T_N[X]^ell."""
    crs = prng.uniform_torus(seed, prng.PUBLIC_PARTY, prng.OBJ_CRS,
                             np.arange(params.bk_ell), params.N)
    return Keys(params=params, crs=crs)


def poly_mul(u, K) -> np.ndarray:
    """u * K in T_N[X] (u integer, K torus)."""
    acc = np.zeros(K.shape[-1], np.uint32)
    negacyclic_mac(acc, u, K)
    return acc


def keygen(keys: Keys, party: int, seed: int) -> PartyKeys:
    """§3.2 KeyGen for one party; appends and returns its keys."""
    P = keys.params
    n, N, ell, t = P.n, P.N, P.bk_ell, P.ks_t
    g = gadget(P)
    s = prng.binary(seed, party, prng.OBJ_SK_LWE, 0, n)
    z = prng.binary(seed, party, prng.OBJ_SK_RLWE, 0, N)
    # public key b_l = -z*a_l + e_l
    e = prng.noise(seed, party, prng.OBJ_PK_E, np.arange(ell), N, P.bk_noise_log2)
    pk = np.zeros((ell, N), np.uint32)
    for l in range(ell):
        pk[l] = u32(-poly_mul(z, keys.crs[l]).astype(np.int64) + e[l])
    # bootstrapping key: uni-encryption of each bit of s under z
    r_all = prng.binary(seed, party, prng.OBJ_BK_R, np.arange(n), N)
    idx = np.arange(n * ell)
    e1 = prng.noise(seed, party, prng.OBJ_BK_E1, idx, N, P.bk_noise_log2).reshape(n, ell, N)
    f1 = prng.uniform_torus(seed, party, prng.OBJ_BK_F1, idx, N).reshape(n, ell, N)
    e2 = prng.noise(seed, party, prng.OBJ_BK_E2, idx, N, P.bk_noise_log2).reshape(n, ell, N)
    bk = np.zeros((n, 3, ell, N), np.uint32)
    for j in range(n):
        r = r_all[j].astype(np.int64)
        mu = int(s[j])
        for l in range(ell):
            d = poly_mul(r, keys.crs[l]).astype(np.int64) + e1[j, l]
            d[0] += mu * g[l]
            f0 = -poly_mul(z, f1[j, l]).astype(np.int64) + e2[j, l] + r * g[l]
            bk[j, 0, l] = u32(d)
            bk[j, 1, l] = u32(f0)
            bk[j, 2, l] = f1[j, l]
    # key-switching key from z (dim N) to s (dim n)
    Bp = 1 << P.ks_log_base
    nrow = N * t * (Bp - 1)
    ridx = np.arange(nrow)
    a = prng.uniform_torus(seed, party, prng.OBJ_KS_A, ridx, n)
    ek = prng.noise(seed, party, prng.OBJ_KS_E, ridx, 1, P.ks_noise_log2)[:, 0]
    q = ridx // (t * (Bp - 1))
    p = (ridx // (Bp - 1)) % t
    v = ridx % (Bp - 1) + 1
    msg = v * z[q].astype(np.int64) * (1 << 32 >> (P.ks_log_base * (p + 1)))
    b = msg - (a.astype(np.int64) @ s.astype(np.int64)) + ek
    ks = np.concatenate([u32(b)[:, None], a], axis=1).reshape(N, t, Bp - 1, n + 1)
    pkeys = PartyKeys(s=s, z=z, pk=pk, bk=bk, ks=ks)
    keys.parties.append(pkeys)
    return pkeys


def generate(params: Params, seed: int) -> Keys:
    """Setup plus KeyGen of all k parties; party i uses seed + 1 + i."""
    keys = setup(params, seed)
    for i in range(params.k):
        keygen(keys, i, party_seed(seed, i))
    return keys


def party_seed(seed: int, party: int) -> int:
    return (seed + 1 + party) & 0xFFFFFFFFFFFFFFFF


# ----------------------------------------------------- encrypt/decrypt ----

def encrypt(keys: Keys, party: int, bits, seed: int) -> np.ndarray:
    """§3.2 SymEnc by ``party`` plus extension to k slots: u32[count, kn+1]."""
    P = keys.params
    bits = np.asarray(bits, dtype=np.int64)
    cnt = bits.shape[0]
    s = keys.parties[party].s.astype(np.int64)
    a = prng.uniform_torus(seed, party, prng.OBJ_ENC_A, np.arange(cnt), P.n)
    e = prng.noise(seed, party, prng.OBJ_ENC_E, np.arange(cnt), 1, P.lwe_noise_log2)[:, 0]
    b = bits * QUARTER - a.astype(np.int64) @ s + e
    out = np.zeros((cnt, P.lwe_words), np.uint32)
    out[:, 0] = u32(b)
    out[:, 1 + party * P.n: 1 + (party + 1) * P.n] = a
    return out


def trivial(params: Params, bits) -> np.ndarray:
    """Noiseless ciphertexts (b = mu/4, a = 0) for constants and carries."""
    bits = np.atleast_1d(np.asarray(bits, dtype=np.int64))
    out = np.zeros((bits.shape[0], params.lwe_words), np.uint32)
    out[:, 0] = u32(bits * QUARTER)
    return out


def phase(keys: Keys, c) -> np.ndarray:
    """b + sum_i <a_i, s_i> mod 2^32 for ciphertexts u32[..., kn+1]."""
    P = keys.params
    c = np.atleast_2d(c).astype(np.int64)
    ph = c[:, 0].copy()
    for i, pk in enumerate(keys.parties):
        ph += c[:, 1 + i * P.n: 1 + (i + 1) * P.n] @ pk.s.astype(np.int64)
    return u32(ph)


def decrypt(keys: Keys, c) -> np.ndarray:
    """§3.2 SymDec: nearest of {0, 1/4}; 1 iff the phase is in [1/8, 5/8)."""
    ph = phase(keys, c).astype(np.int64)
    return ((ph >= EIGHTH) & (ph < 5 * EIGHTH)).astype(np.uint8)


# --------------------------------------------------------------- gates ----

def gate_combine(gate: int, c1, c2) -> np.ndarray:
    """(0, const) + s1*c1 + s2*c2 (ModToT, LweAdd/LweSub/LweMul; §4.1-4.2)."""
    const, s1, s2 = GATE_TABLE[gate]
    out = s1 * np.asarray(c1, np.int64) + s2 * np.asarray(c2, np.int64)
    out[..., 0] += const
    return u32(out)


def lwe_not(c) -> np.ndarray:
    """MKNOT, Eq. (8): (0, 1/4) - c, no bootstrapping."""
    out = -np.asarray(c, np.int64)
    out[..., 0] += QUARTER
    return u32(out)


def modulus_switch(x, N: int) -> np.ndarray:
    """Round Torus32 words to Z_2N: floor((x + 2^(31-log2 2N)) / 2^(32-log2 2N))."""
    L = (2 * N).bit_length() - 1
    y = (np.asarray(x, np.int64) + (1 << (31 - L))) & M32
    return (y >> (32 - L)).astype(np.int64)


def rotate(P, a: int) -> np.ndarray:
    """X^(-a) * P in T_N[X] for a in Z_2N."""
    N = P.shape[-1]
    idx = np.arange(N) + (int(a) % (2 * N))
    src = np.asarray(P, np.int64)[..., idx % N]
    sign = np.where((idx // N) % 2 == 0, 1, -1)
    return u32(src * sign)


def decompose(x, beta: int, ell: int) -> np.ndarray:
    """Signed gadget decomposition, most significant digit first.

    Returns int64[ell, ...] with digits in [-2^(beta-1), 2^(beta-1)) such that
    sum_p digit_p * 2^(32-beta*p) equals x rounded to a multiple of
    2^(32-beta*ell) (ties up), mod 2^32.
    """
    half = 1 << (beta - 1)
    offset = 1 << (31 - beta * ell)
    for p in range(1, ell + 1):
        offset += half << (32 - beta * p)
    y = (np.asarray(x, np.int64) + offset) & M32
    return np.stack([((y >> (32 - beta * p)) & ((1 << beta) - 1)) - half
                     for p in range(1, ell + 1)])


def test_vector(N: int) -> np.ndarray:
    """v with v_j = -1/8 for j < N/2 and +1/8 for j >= N/2, so that the
    constant coefficient of X^(-phi) v is +1/8 iff phi in [N/2, 3N/2)."""
    v = np.full(N, EIGHTH, np.uint32)
    v[: N // 2] = (1 << 32) - EIGHTH
    return v


def hybrid_product(params: Params, c, bk_bit, evk, party: int) -> np.ndarray:
    """Hybrid product of a k-party RLWE ciphertext c = (c_0..c_k) with the
    uni-encryption (d, f0, f1) of a bit mu of party ``party``; the result's
    phase is mu * phase(c) plus noise.

      u_j  = g^-1(c_j)                         j = 0..k
      c'_j = sum_l u_{j,l} * d_l
      w    = sum_j sum_l u_{j,l} * b_{j,l}      (b_0 = -a, b_j = pk_j)
      v    = g^-1(w)
      c'_0 += sum_l v_l * f0_l ;  c'_party += sum_l v_l * f1_l
    """
    k, ell, beta = params.k, params.bk_ell, params.bk_log_base
    N = params.N
    u = [decompose(c[j], beta, ell) for j in range(k + 1)]
    out = np.zeros((k + 1, N), np.uint32)
    w = np.zeros(N, np.uint32)
    for j in range(k + 1):
        for l in range(ell):
            negacyclic_mac(out[j], u[j][l], bk_bit[0, l])
            negacyclic_mac(w, u[j][l], evk[j, l])
    v = decompose(w, beta, ell)
    for l in range(ell):
        negacyclic_mac(out[0], v[l], bk_bit[1, l])
        negacyclic_mac(out[1 + party], v[l], bk_bit[2, l])
    return out


def blind_rotate(keys: Keys, abar, evk=None, max_steps=None) -> np.ndarray:
    """ACC = (X^-b v, 0..0), then for parties i and bits l in order:
    ACC += HbProd(X^-a_{i,l} ACC - ACC, BK_{i,l}).  Returns u32[k+1, N].

    ``max_steps`` stops after that many CMux steps (for partial checks).
    """
    P = keys.params
    k, n, N = P.k, P.n, P.N
    if evk is None:
        evk = keys.evaluation_key()
    acc = np.zeros((k + 1, N), np.uint32)
    acc[0] = rotate(test_vector(N), int(abar[0]))
    step = 0
    for i in range(k):
        for l in range(n):
            if max_steps is not None and step >= max_steps:
                return acc
            step += 1
            a = int(abar[1 + i * n + l])
            diff = u32(rotate(acc, a).astype(np.int64) - acc)
            acc = u32(acc.astype(np.int64)
                      + hybrid_product(P, diff, keys.parties[i].bk[l], evk, i))
    return acc


def sample_extract(acc) -> np.ndarray:
    """Constant coefficient of the RLWE phase as an LWE sample under the
    concatenated ring keys: b = c_0[0], a_j[0] = c_j[0], a_j[q] = -c_j[N-q]."""
    k1, N = acc.shape
    out = np.zeros(1 + (k1 - 1) * N, np.int64)
    out[0] = acc[0, 0]
    for j in range(1, k1):
        a = np.empty(N, np.int64)
        a[0] = acc[j, 0]
        a[1:] = -acc[j, N - 1:0:-1].astype(np.int64)
        out[1 + (j - 1) * N: 1 + j * N] = a
    return u32(out)


def key_switch(keys: Keys, big) -> np.ndarray:
    """§3.2 MKKeySwitch: per party, switch a_i (under z_i, dim N) to s_i.

    Each a_{i,q} is rounded to t base-B' digits (most significant first) and
    row KS_i[q][p][v] is added for every non-zero digit v.
    """
    P = keys.params
    k, n, N, t, lb = P.k, P.n, P.N, P.ks_t, P.ks_log_base
    out = np.zeros(P.lwe_words, np.int64)
    out[0] = int(big[0])
    prec = lb * t
    for i in range(k):
        a = big[1 + i * N: 1 + (i + 1) * N].astype(np.int64)
        abar = ((a + (1 << (31 - prec))) & M32) >> (32 - prec)
        ks = keys.parties[i].ks
        for p in range(t):
            v = (abar >> (lb * (t - 1 - p))) & ((1 << lb) - 1)
            q = np.nonzero(v)[0]
            rows = ks[q, p, v[q] - 1].astype(np.int64)      # [len(q), n+1]
            out[0] += rows[:, 0].sum()
            out[1 + i * n: 1 + (i + 1) * n] += rows[:, 1:].sum(axis=0)
    return u32(out)


def bootstrap(keys: Keys, c, evk=None) -> np.ndarray:
    """Gate bootstrapping of a combined ciphertext: output encrypts 1/4 iff
    its phase is in [1/4, 3/4), else 0 (then key-switched to the s_i)."""
    P = keys.params
    abar = modulus_switch(c, P.N)
    acc = blind_rotate(keys, abar, evk)
    big = sample_extract(acc)
    big[0] = np.uint32((int(big[0]) + EIGHTH) & M32)
    return key_switch(keys, big)


def bootstrapped_gate(keys: Keys, gate: int, c1, c2, evk=None) -> np.ndarray:
    """MKBoots{NAND,AND,OR,NOR,XOR,XNOR} of §4.1 on one pair of ciphertexts."""
    return bootstrap(keys, gate_combine(gate, c1, c2), evk)
