"""Shared test helpers: parameter conversion and cached key worlds.

A "world" holds one parameter set with keys generated twice, independently:
by the oracle (CPU reference) and by the library (mk_setup/mk_keygen).  The
tests check that both key sets are byte-identical before comparing anything
computed from them.
"""
from __future__ import annotations

import functools

import numpy as np

from oracle import params as OP
from oracle import tfhe

FIELDS = ("k", "n", "N", "bk_ell", "ks_t", "bk_noise_log2", "ks_noise_log2",
          "lwe_noise_log2", "bk_log_base", "ks_log_base")
SEEDS = {"C1": 0, "C1B": 5, "C1B4": 6, "C1S": 7, "C2": 2, "C3": 3, "C8": 11, "TOY": 9, "TOYB3": 10}
HEADER_BYTES = 4 + 4 + 40 + 4


def lib_params(P):
    import paper_2205_05825_amd as mk
    return mk.Params(**{f: getattr(P, f) for f in FIELDS})


def split_export(P, blob):
    """Parse a library key export of a party into named numpy arrays."""
    o = HEADER_BYTES
    out = {}
    Bm1 = (1 << P.ks_log_base) - 1
    for name, cnt, dt, shape in (
            ("s", P.n, np.uint8, (P.n,)), ("z", P.N, np.uint8, (P.N,)),
            ("pk", P.bk_ell * P.N, np.uint32, (P.bk_ell, P.N)),
            ("bk", P.n * 3 * P.bk_ell * P.N, np.uint32, (P.n, 3, P.bk_ell, P.N)),
            ("ks", P.N * P.ks_t * Bm1 * (P.n + 1), np.uint32, (P.N, P.ks_t, Bm1, P.n + 1))):
        nb = cnt * np.dtype(dt).itemsize
        out[name] = np.frombuffer(blob[o:o + nb], dt).reshape(shape)
        o += nb
    assert o == len(blob)
    return out


@functools.lru_cache(maxsize=None)
def oracle_keys(name):
    P = getattr(OP, name)
    return tfhe.generate(P, SEEDS[name])


@functools.lru_cache(maxsize=None)
def lib_context(name):
    import paper_2205_05825_amd as mk
    P = getattr(OP, name)
    seed = SEEDS[name]
    ctx = mk.Context(lib_params(P), seed)
    for i in range(P.k):
        ctx.keygen(i, tfhe.party_seed(seed, i))
    return ctx


def assert_same_keys(name):
    P = getattr(OP, name)
    K = oracle_keys(name)
    ctx = lib_context(name)
    crs = np.frombuffer(ctx.export_keys(-1)[HEADER_BYTES:], np.uint32).reshape(P.bk_ell, P.N)
    assert np.array_equal(crs, K.crs)
    for i in range(P.k):
        got = split_export(P, ctx.export_keys(i))
        ref = K.parties[i]
        for f in ("s", "z", "pk", "bk", "ks"):
            assert np.array_equal(got[f], getattr(ref, f)), (name, i, f)


def oracle_gates(name, types, c1, c2, idx=None, workers=8):
    """Oracle outputs of bootstrapped gates ``idx`` (threads: the oracle's C
    product releases the GIL)."""
    from concurrent.futures import ThreadPoolExecutor
    K = oracle_keys(name)
    evk = K.evaluation_key()
    idx = range(len(types)) if idx is None else idx
    W = K.params.lwe_words

    def one(g):
        return tfhe.bootstrapped_gate(K, int(types[g]), c1[g, :W], c2[g, :W], evk)

    with ThreadPoolExecutor(max_workers=workers) as ex:
        return np.stack(list(ex.map(one, idx)))


def gpu_world(name):
    """Library context for `name` with keys checked against the oracle and
    the evaluation key uploaded to the current GPU."""
    assert_same_keys(name)
    ctx = lib_context(name)
    if not getattr(ctx, "_uploaded", False):
        ctx.upload()
        ctx._uploaded = True
    return oracle_keys(name), ctx


def oracle_circuit(name, nl, in_ct, workers=8):
    """Oracle gate-by-gate evaluation of netlist nl on in_ct[n_in, B, words],
    one instance per thread."""
    from concurrent.futures import ThreadPoolExecutor
    from oracle import circuits as C
    K = oracle_keys(name)
    W = K.params.lwe_words
    Bn = in_ct.shape[1]
    with ThreadPoolExecutor(max_workers=workers) as ex:
        outs = list(ex.map(lambda b: C.eval_encrypted(nl, K, in_ct[:, b:b + 1, :W]), range(Bn)))
    return np.concatenate(outs, axis=1)


def encrypt_operands(K, values, bits, party, seed):
    """u32[bits, B, words]: bit i of every value, encrypted by `party`."""
    import mk_inputs as mi
    cols = mi.to_bits(values, bits).T
    return np.stack([tfhe.encrypt(K, party, col, seed=seed + 1000 * i) for i, col in enumerate(cols)])


def sampled_level_parity(name, circ, in_ct, evaluate, samples, seed, workers=8):
    """Per-gate parity inside a full-size circuit run.

    `samples` (gate, instance) items are drawn (seeded) from the bootstrapped
    gates; the circuit is evaluated on the GPU with those gates' input and
    output wires appended to its outputs (evaluate(circuit) -> u32[n_out, B,
    words]); then the oracle recomputes each sampled gate from the GPU's own
    input ciphertexts (constants as trivial ciphertexts, inputs as given) and
    the result must equal the GPU's output word for word.  By induction over
    the levels this checks every level at these shapes.  Returns the GPU
    outputs of the original circuit's outputs."""
    from concurrent.futures import ThreadPoolExecutor
    import paper_2205_05825_amd as mk
    K = oracle_keys(name)
    P = K.params
    W = P.lwe_words
    rng = np.random.default_rng(seed)
    boot = [i for i, g in enumerate(circ.gates) if g[0] != mk.NOT]
    picks = [(int(rng.choice(boot)), int(rng.integers(0, in_ct.shape[1]))) for _ in range(samples)]
    extra = []
    for gi, _ in picks:
        _, a, b, o = (int(x) for x in circ.gates[gi])
        extra += [a, b, o]
    n0 = len(circ.outputs)
    ext = mk.Circuit(circ.n_wires, circ.inputs, np.concatenate([circ.outputs, np.array(extra, np.int32)]),
                     circ.gates)
    got = evaluate(ext)
    input_pos = {int(w): i for i, w in enumerate(circ.inputs)}
    evk = K.evaluation_key()

    def wire_ct(w, row, inst):
        if w in (0, 1):
            return tfhe.trivial(P, [w])[0]
        if w in input_pos:
            return np.asarray(in_ct[input_pos[w], inst, :W], np.uint32)
        return got[row, inst, :W]

    def check(k):
        gi, inst = picks[k]
        t, a, b, _ = (int(x) for x in circ.gates[gi])
        base = n0 + 3 * k
        c1, c2 = wire_ct(a, base, inst), wire_ct(b, base + 1, inst)
        return np.array_equal(tfhe.bootstrapped_gate(K, t, c1, c2, evk), got[base + 2, inst, :W])

    with ThreadPoolExecutor(max_workers=workers) as ex:
        ok = list(ex.map(check, range(len(picks))))
    assert all(ok), [p for p, f in zip(picks, ok) if not f]
    return got[:n0]
