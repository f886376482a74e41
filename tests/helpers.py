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
SEEDS = {"C1": 0, "C1B": 5, "C1B4": 6, "C1S": 7, "C2": 2, "C3": 3, "C8": 11, "TOY": 9, "TOYB3": 10, "C1SB3": 12}
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


_POOL = None


def oracle_pool():
    """Process pool for oracle work (the oracle's numpy steps hold the GIL,
    so threads do not run gates in parallel).  The forkserver start method
    gives workers that never inherited this process's GPU state; each worker
    regenerates a parameter set's keys from its seed on first use."""
    global _POOL
    if _POOL is None:
        import multiprocessing as mp
        import os
        from concurrent.futures import ProcessPoolExecutor
        _POOL = ProcessPoolExecutor(max_workers=max(1, min(16, os.cpu_count() or 1)),
                                    mp_context=mp.get_context("forkserver"))
    return _POOL


@functools.lru_cache(maxsize=None)
def _evk(name):
    return oracle_keys(name).evaluation_key()


def _oracle_gate_job(name, t, c1, c2):
    return tfhe.bootstrapped_gate(oracle_keys(name), int(t), c1, c2, _evk(name))


def _oracle_rotation_job(name, abar, steps):
    return tfhe.blind_rotate(oracle_keys(name), np.asarray(abar, np.int64), _evk(name),
                             max_steps=None if steps < 0 else steps)


def oracle_gates(name, types, c1, c2, idx=None):
    """Oracle outputs of bootstrapped gates ``idx`` (all by default),
    computed in the oracle process pool."""
    W = getattr(OP, name).lwe_words
    idx = list(range(len(types))) if idx is None else list(idx)
    jobs = [oracle_pool().submit(_oracle_gate_job, name, int(types[g]), np.ascontiguousarray(c1[g, :W]),
                                 np.ascontiguousarray(c2[g, :W])) for g in idx]
    return np.stack([j.result() for j in jobs])


def oracle_rotations(name, abar, steps=-1):
    """Oracle blind rotations of the rows of abar (first `steps` CMux steps,
    all if negative), in the oracle process pool."""
    jobs = [oracle_pool().submit(_oracle_rotation_job, name, np.ascontiguousarray(row), steps) for row in abar]
    return np.stack([np.asarray(j.result()) for j in jobs])


def gpu_world(name):
    """Library context for `name` with keys checked against the oracle and
    the evaluation key uploaded to the current GPU."""
    assert_same_keys(name)
    ctx = lib_context(name)
    if not getattr(ctx, "_uploaded", False):
        ctx.upload()
        ctx._uploaded = True
    return oracle_keys(name), ctx


def oracle_circuit(name, nl, in_ct):
    """Oracle gate-by-gate evaluation of netlist nl on in_ct[n_in, B, words],
    one instance per pool worker."""
    W = getattr(OP, name).lwe_words
    Bn = in_ct.shape[1]
    jobs = [oracle_pool().submit(_oracle_circuit_job, name, nl, np.ascontiguousarray(in_ct[:, b:b + 1, :W]))
            for b in range(Bn)]
    return np.concatenate([j.result() for j in jobs], axis=1)


def _oracle_circuit_job(name, nl, in_ct):
    from oracle import circuits as C
    return C.eval_encrypted(nl, oracle_keys(name), in_ct)


def encrypt_operands(K, values, bits, party, seed):
    """u32[bits, B, words]: bit i of every value, encrypted by `party`."""
    import mk_inputs as mi
    cols = mi.to_bits(values, bits).T
    return np.stack([tfhe.encrypt(K, party, col, seed=seed + 1000 * i) for i, col in enumerate(cols)])


def live_levels(circ):
    """Bootstrapping level of every live bootstrapped gate of a netlist, as
    the engine levels it: NOT gates are free (a NOT's output has its
    input's level), inputs and constants are level 0, a bootstrapped gate is
    one above its deepest input; gates no output depends on are dropped.
    Returns {gate index: level}."""
    NOT = 6
    gates = [tuple(int(x) for x in g) for g in circ.gates]
    base = {}       # wire -> producing bootstrapped gate's output wire (or None)
    level = {}
    for w in list(circ.inputs) + [0, 1]:
        base[int(w)] = None
        level[int(w)] = 0
    for t, a, b, o in gates:
        if t == NOT:
            base[o] = base[a]
            level[o] = level[a]
        else:
            base[o] = o
            level[o] = 1 + max(level[a], level[b])
    needed = set()
    for w in circ.outputs:
        if base[int(w)] is not None:
            needed.add(base[int(w)])
    for t, a, b, o in reversed(gates):
        if t == NOT or o not in needed:
            continue
        for w in (a, b):
            if base[w] is not None:
                needed.add(base[w])
    return {gi: level[g[3]] for gi, g in enumerate(gates) if g[0] != NOT and g[3] in needed}


def sampled_level_parity(name, circ, in_ct, evaluate, seed, max_levels=64, check_unmodified=True):
    """Per-gate oracle parity inside a full-size circuit run, at every level.

    One (gate, instance) item is drawn (seeded) from the live bootstrapped
    gates of every bootstrapping level; circuits deeper than max_levels get
    every s-th level from a seeded offset (s = ceil(levels / max_levels)),
    plus the first and the last.  The circuit is evaluated twice on the GPU
    (evaluate(circuit) -> u32[n_out, B, words]): as given, and with the
    sampled gates' input and output wires appended to its outputs.  The
    sampled gates are live already, so both runs evaluate the same gates in
    the same levels and only the wire slots differ: the original outputs
    must equal the first outputs of the extended run word for word.  Then
    the oracle recomputes each sampled gate from the GPU's own input
    ciphertexts (constants as trivial ciphertexts, inputs as given) and the
    result must equal the GPU's output word for word; with a sample at every
    level this checks each level given the one before.  Returns the
    original run's outputs and the list of (gate, instance) items.  With
    check_unmodified=False only the extended circuit runs (for sub-circuits
    that are not a user's circuit) and its first outputs are returned."""
    import paper_2205_05825_amd as mk
    K = oracle_keys(name)
    P = K.params
    W = P.lwe_words
    rng = np.random.default_rng(seed)
    lv = live_levels(circ)
    by_level = {}
    for gi, l in lv.items():
        by_level.setdefault(l, []).append(gi)
    levels = sorted(by_level)
    if len(levels) > max_levels:
        step = -(-len(levels) // max_levels)
        off = int(rng.integers(0, step))
        keep = set(levels[off::step]) | {levels[0], levels[-1]}
        levels = [l for l in levels if l in keep]
    picks = [(int(rng.choice(by_level[l])), int(rng.integers(0, in_ct.shape[1]))) for l in levels]
    extra = []
    for gi, _ in picks:
        _, a, b, o = (int(x) for x in circ.gates[gi])
        extra += [a, b, o]
    n0 = len(circ.outputs)
    ext = mk.Circuit(circ.n_wires, circ.inputs, np.concatenate([circ.outputs, np.array(extra, np.int32)]),
                     circ.gates)
    got = evaluate(ext)
    if check_unmodified:
        plain = evaluate(circ)
        assert np.array_equal(plain, got[:n0]), "exposing internal wires changed the outputs"
    else:
        plain = got[:n0]
    input_pos = {int(w): i for i, w in enumerate(circ.inputs)}

    def wire_ct(w, row, inst):
        if w in (0, 1):
            return tfhe.trivial(P, [w])[0]
        if w in input_pos:
            return np.asarray(in_ct[input_pos[w], inst, :W], np.uint32)
        return got[row, inst, :W]

    jobs = []
    for k, (gi, inst) in enumerate(picks):
        t, a, b, _ = (int(x) for x in circ.gates[gi])
        base = n0 + 3 * k
        jobs.append(oracle_pool().submit(_oracle_gate_job, name, t, np.ascontiguousarray(wire_ct(a, base, inst)),
                                         np.ascontiguousarray(wire_ct(b, base + 1, inst))))
    bad = [p for k, (p, j) in enumerate(zip(picks, jobs))
           if not np.array_equal(j.result(), got[n0 + 3 * k + 2, p[1], :W])]
    assert not bad, bad
    return plain, picks


def split_by_levels(circ, parts):
    """Cuts a netlist into `parts` consecutive sub-netlists by bootstrapping
    level (as the engine levels it), keeping the wire numbering.  Part k
    holds the live bootstrapped gates of its level range and the NOT gates
    at those levels; its inputs are the wires it reads that earlier parts
    (or the circuit's inputs) define, its outputs the wires it defines that
    later parts read or the circuit outputs.  Evaluating the parts in order
    computes exactly the gates of the whole circuit.  Returns a list of
    paper_2205_05825_amd.Circuit."""
    import paper_2205_05825_amd as mk
    NOT = 6
    gates = [tuple(int(x) for x in g) for g in circ.gates]
    level = {int(w): 0 for w in list(circ.inputs) + [0, 1]}
    for t, a, b, o in gates:
        level[o] = level[a] if t == NOT else 1 + max(level[a], level[b])
    needed = set(int(w) for w in circ.outputs)
    for t, a, b, o in reversed(gates):
        if o in needed:
            needed.update([a] if t == NOT else [a, b])
    L = max([level[o] for t, a, b, o in gates if o in needed] + [1])
    part_of = lambda lv: 0 if lv <= 0 else min(parts - 1, (lv - 1) * parts // L)
    owner = {}
    members = [[] for _ in range(parts)]
    for t, a, b, o in gates:
        if o not in needed:
            continue
        k = part_of(level[o])
        owner[o] = k
        members[k].append((t, a, b, o))
    later_reads = [set() for _ in range(parts)]
    for k in range(parts):
        for t, a, b, o in members[k]:
            for w in ([a] if t == NOT else [a, b]):
                if w in owner and owner[w] < k:
                    later_reads[owner[w]].add(w)
    out = []
    for k in range(parts):
        defined = {o for _, _, _, o in members[k]}
        ins = []
        for t, a, b, o in members[k]:
            for w in ([a] if t == NOT else [a, b]):
                if w not in defined and w not in (0, 1) and w not in ins:
                    ins.append(w)
        outs = sorted(w for w in defined if w in later_reads[k] or w in set(int(x) for x in circ.outputs))
        g = np.array([list(x) for x in members[k]], np.int32).reshape(-1, 4)
        out.append(mk.Circuit(circ.n_wires, np.array(ins, np.int32), np.array(outs, np.int32), g))
    return out
