"""Benchmark: bootstrapped multi-key gates per second on one MI355X.

Headline workload: a batch of 1024 independent bootstrapped gates, types
uniform over AND/OR/NOR/XOR/XNOR/NAND, uniform input bits, 2 parties (input 1
encrypted by party 0, input 2 by party 1), n=560, N=1024, gadget base 2^8 with
ell=3, key-switching base 2^2 with t=8 (Table 7 shape with B = 2^8).  One
"step" is the whole gate pipeline on the batch: pre-combination and modulus
switch, blind rotation (k*n = 1120 hybrid-product CMux steps), sample
extraction and multi-key key switching.  Ciphertexts and keys are resident in
HBM before timing starts; key generation and upload are excluded.

The default run also times, with every output decrypted and checked: the
plain 32-bit integer path on the same batch (outputs bit-identical to the
MFMA path), the 4-party 8-bit multiplier on 256 pairs, the 16-bit adder,
subtractor (4096 pairs each), multiplier and divider (256 pairs each),
one encrypted gradient-descent step of linear regression (m=64, d=4), larger
batches, 4 and 8 parties, the scheme's gates against NAND-composed ones, and
the CPU oracle on bounded samples (C2 and the 8-gate C1 workload, one core
and all cores).  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import mk_inputs as mi  # noqa: E402

C2 = dict(k=2, n=560, N=1024, bk_ell=3, ks_t=8, bk_noise_log2=30, ks_noise_log2=15,
          lwe_noise_log2=15)
SEED = 2
BATCH = 1024
PEAK_INT8_OPS = 5.0e15          # MI355X dense int8 MFMA
# An exact Torus32 multiply-add on the vector ALU takes at least two full-rate
# 24-bit multiply-adds (one per half of the key word): 256 CUs x 64 lanes x
# 2.4 GHz / 2.
PEAK_VALU_TORUS_MACS = 256 * 64 * 2.4e9 / 2


CSRC = os.path.join(ROOT, "paper_2205_05825_amd", "csrc")
# HBM traffic summaries (rocprofv3 FETCH_SIZE/WRITE_SIZE, copy-calibrated)
# and the sources each kernel is built from: a summary counts only while the
# sha256 of those sources matches the one it records.
TRAFFIC = {
    "gemm1": (os.path.join(ROOT, "profiles", "mfma_gemm1_c2_1024gates_hbm_traffic.md"),
              [os.path.join(CSRC, "mk_mfma.hip"), os.path.join(CSRC, "mk_mfma_core.h")]),
    "persist": (os.path.join(ROOT, "profiles", "persist_rotation_c2_1024gates_hbm_traffic.md"),
                [os.path.join(CSRC, "mk_persist.hip"), os.path.join(CSRC, "mk_mfma_core.h"),
                 os.path.join(CSRC, "mk_ks_core.h")]),
}
PERSIST_KERNEL = "persist_rotation_kernel<32, 8>"


# Stage-1 GEMM instantiation run for each tile shape (the shape table of
# mk_mfma.hip), as rocprofv3 names the kernel.
GEMM1_KERNEL = {0: "mfma_gemm1_limb_kernel<8, 1, 2>", 1: "mfma_gemm1_limb_kernel<4, 2, 2>",
                2: "mfma_gemm1_limb_kernel<4, 1, 3>", 3: "mfma_gemm1_kernel<2, 1, 2>",
                4: "mfma_gemm1_limb_kernel<8, 2, 1>", 5: "mfma_gemm1_split_kernel<2, 1>",
                6: "mfma_gemm1_split_kernel<1, 1>", 7: "mfma_gemm1_split_kernel<1, 2>"}


def sources_sha(paths):
    import hashlib
    h = hashlib.sha256()
    for p in paths:
        h.update(open(p, "rb").read())
    return h.hexdigest()


def measured_traffic(which, kernel):
    """HBM bytes per launch of `kernel` from its committed traffic summary,
    or None when that kernel was not measured or its sources changed since
    the counters were taken."""
    import re
    path, srcs = TRAFFIC[which]
    try:
        text = open(path).read()
        src = sources_sha(srcs)
    except OSError:
        return None
    m = re.search(r"HBM bytes per launch \[%s\]: (\d+)" % re.escape(kernel), text)
    h = re.search(r"sha256 ([0-9a-f]{64})", text)
    if not m or not h or h.group(1) != src:
        return None
    return int(m.group(1))


def macs_per_gate(p):
    """Exact Torus32 multiply-adds of one blind rotation: k*n CMux steps, each
    (2k+4)*ell negacyclic products of N^2 multiply-adds."""
    return p["k"] * p["n"] * (2 * p["k"] + 4) * p["bk_ell"] * p["N"] ** 2


def executed_int8_ops_per_gate(p):
    """Int8 operations the MFMA rotation executes per gate: in party i's
    steps only the accumulator slots j < L = min(k+1, i+2) can be non-zero,
    so a step runs 2 L ell products in stage 1 (c'_j and the w sum) and
    2 ell in stage 2, each N^2 Torus32 multiply-adds of 4 int8 limb
    products, 2 operations per multiply-add."""
    k, n, ell, N = p["k"], p["n"], p["bk_ell"], p["N"]
    return sum(n * (2 * min(k + 1, i + 2) * ell + 2 * ell) for i in range(k)) * 8 * N * N


# ------------------------------------------------------- CPU baseline ----
_CPU = {}


def _cpu_gate(g):
    from oracle import tfhe
    K, evk, types, c1, c2 = _CPU["state"]
    return tfhe.bootstrapped_gate(K, int(types[g]), c1[g], c2[g], evk)


def _cpu_rate(ctx, K, types, m1, m2, c1, c2, sample, cores):
    """Gates/s of the oracle over `sample` on `cores` processes (1 = in this
    process), with every output decrypted against its truth table."""
    from oracle import tfhe
    _CPU["state"] = (K, K.evaluation_key(), types, c1, c2)
    t0 = time.perf_counter()
    if cores == 1:
        outs = [_cpu_gate(g) for g in sample]
    else:
        with ctx.Pool(cores) as pool:
            outs = pool.map(_cpu_gate, sample, chunksize=1)
    dt = time.perf_counter() - t0
    want = [mi.plain_gate(int(types[g]), int(m1[g]), int(m2[g])) for g in sample]
    ok = tfhe.decrypt(K, np.stack(outs)).tolist() == want
    return len(sample) / dt, dt, ok


def cpu_baseline(gates_per_core: int):
    """The oracle, as it stands, on bounded samples of the workloads, one
    process per host core for the all-core rates (fork before any GPU use):
    the C2 gate mix (the headline workload: gates_per_core gates per core
    on all cores, and four gates on one core), the 8-gate C1 truth-table
    workload (all 8 gates on one core and on all cores), and one 4-party
    gate per core at the C3 shape (the basis of the config 3
    extrapolation)."""
    import multiprocessing as mp

    from oracle import params as OP
    from oracle import tfhe
    cores = min(os.cpu_count() or 1, 16)
    ctx = mp.get_context("fork")
    K = tfhe.generate(OP.C2, SEED)
    types, m1, m2 = mi.gate_batch(BATCH, seed=SEED)
    c1 = tfhe.encrypt(K, 0, m1, seed=200)
    c2 = tfhe.encrypt(K, 1, m2, seed=201)
    all_rate, all_dt, all_ok = _cpu_rate(ctx, K, types, m1, m2, c1, c2, list(range(cores * gates_per_core)), cores)
    one_rate, one_dt, one_ok = _cpu_rate(ctx, K, types, m1, m2, c1, c2, list(range(4)), 1)
    K1 = tfhe.generate(OP.C1, 0)
    t1, a1, b1 = mi.truth_table(gates=(mi.XOR, mi.NAND))
    e1, e2 = tfhe.encrypt(K1, 0, a1, seed=0), tfhe.encrypt(K1, 1, b1, seed=1)
    c1_one = _cpu_rate(ctx, K1, t1, a1, b1, e1, e2, list(range(len(t1))), 1)
    c1_all = _cpu_rate(ctx, K1, t1, a1, b1, e1, e2, list(range(len(t1))), min(cores, len(t1)))
    # one 4-party gate per core (the C3 shape), for the C3 extrapolation
    K3 = tfhe.generate(OP.C3, 3)
    t3, p3, q3 = mi.gate_batch(cores, seed=3)
    d1, d2 = tfhe.encrypt(K3, 0, p3, seed=300), tfhe.encrypt(K3, OP.C3.k - 1, q3, seed=301)
    c3_all = _cpu_rate(ctx, K3, t3, p3, q3, d1, d2, list(range(cores)), cores)
    return {"value": all_rate, "unit": "gates/s", "cores": cores, "kind": "oracle",
            "sample": "%d of the %d workload gates (%d per core) on %d cores, %.1f s wall, decrypt %s"
                      % (cores * gates_per_core, BATCH, gates_per_core, cores, all_dt, "ok" if all_ok else "FAILED"),
            "one_core": {"value": one_rate, "unit": "gates/s", "cores": 1,
                         "sample": "gates 0..3 of the workload, %.1f s, decrypt %s" % (one_dt, "ok" if one_ok else "FAILED")},
            "c1_truth_table": {"gates": len(t1), "one_core_gates_per_s": c1_one[0],
                               "all_core_gates_per_s": c1_all[0], "all_core_processes": min(cores, len(t1)),
                               "decrypts_to_truth_table": bool(c1_one[2] and c1_all[2]),
                               "note": "C1 (k=2, n=64, N=256, ell=2, toy noise): 4 XOR + 4 NAND on every "
                                       "input pair"},
            "c3_four_party": {"value": c3_all[0], "unit": "gates/s", "cores": cores,
                              "sample": "%d mixed gates at k=4 (one per core), %.1f s wall, decrypt %s"
                                        % (cores, c3_all[1], "ok" if c3_all[2] else "FAILED")}}


# ---------------------------------------------------------------- GPU ----
OPERATORS = {"add": "OP_ADD", "sub": "OP_SUB", "mul": "OP_MUL", "div": "OP_DIV"}


def _operator_want(op, a, b, bits=16):
    """Expected integer outputs (LSB-first bit rows are compared after
    decoding): sum, difference (mod 2^bits), exact product, or truncated
    quotient and remainder."""
    wrap = lambda v: ((v + (1 << (bits - 1))) & ((1 << bits) - 1)) - (1 << (bits - 1))
    if op == "add":
        return [wrap(a + b)]
    if op == "sub":
        return [wrap(a - b)]
    if op == "mul":
        return [a * b]
    q = np.abs(a) // np.abs(b) * np.sign(a) * np.sign(b)
    return [wrap(q), wrap(a - q * b)]


def operator_rate(torch, mk, ctx, pairs, op="add", bits=16, graph=True, sub=0, parties=(0, 1), seed=4):
    """`bits`-bit two's-complement operator (adder 5k gates, Alg. 3;
    subtractor 6k, Alg. 5; array multiplier; divider) on `pairs` operand
    pairs drawn uniformly (divisors non-zero), a encrypted by parties[0] and
    b by parties[1].  With `graph` the whole evaluation is captured as HIP
    graph pieces and the timed launch follows one warm-up launch; otherwise
    one eager call is timed; with `sub` (< pairs) the pairs run eagerly in
    sub-batches of that size, one progress line each.  Every output is
    decrypted and checked against plain integer arithmetic."""
    circ = mk.build_operator(getattr(mk, OPERATORS[op]), bits)
    levels, live, width, _ = mk.circuit_stats(circ)
    a, b = mi.operand_pairs(pairs, bits, seed=seed, nonzero_second=op == "div")
    words = ctx.params.lwe_words
    cols = np.concatenate([mi.to_bits(a, bits).T, mi.to_bits(b, bits).T])
    in_ct = np.stack([ctx.encrypt(parties[0] if i < bits else parties[1], col, seed=400 + i)
                      for i, col in enumerate(cols)])
    dev = torch.device("cuda:0")
    sub = sub if 0 < sub < pairs else pairs
    graph = graph and sub == pairs
    w = 1
    while w <= width:            # level batch sizes the autotuner sees first
        ctx.autotune(w * sub)
        w *= 2
    name = "%s%d" % (op, bits)
    print("bench: %s autotuned; %s" % (name, "capturing the graph" if graph else "running"),
          file=sys.stderr, flush=True)
    pieces = 0
    host_out = []
    if graph:
        inp = torch.from_numpy(np.ascontiguousarray(in_ct).view(np.int32)).to(dev)
        out = torch.zeros((len(circ.outputs), pairs, words), dtype=torch.int32, device=dev)
        g = ctx.circuit_graph(circ, inp, out)
        try:
            pieces = g.info()[2]
            print("bench: graph of %d pieces captured; launching" % pieces, file=sys.stderr, flush=True)
            g.launch()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            g.launch()
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
        finally:
            g.close()
        host_out.append(out.cpu().numpy().view(np.uint32))
    else:
        dt = 0.0
        for s0 in range(0, pairs, sub):
            inp = torch.from_numpy(np.ascontiguousarray(in_ct[:, s0:s0 + sub]).view(np.int32)).to(dev)
            out = torch.zeros((len(circ.outputs), inp.shape[1], words), dtype=torch.int32, device=dev)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.eval_circuit(circ, inp, out)
            torch.cuda.synchronize()
            dt += time.perf_counter() - t0
            host_out.append(out.cpu().numpy().view(np.uint32))
            if sub < pairs:
                print("bench: %s pairs %d..%d done" % (name, s0, s0 + inp.shape[1]), file=sys.stderr, flush=True)
    ctx.device_status()
    dec = np.stack([ctx.decrypt(x) for x in np.concatenate(host_out, axis=1)])
    want = _operator_want(op, a, b, bits)
    per = len(circ.outputs) // len(want)
    for k, wv in enumerate(want):
        assert np.array_equal(mi.from_bits(dec[k * per:(k + 1) * per].T), wv), "%s outputs" % name
    print("bench: %s on %d pairs: %.1f s, every output correct" % (name, pairs, dt), file=sys.stderr, flush=True)
    return {"operator": name, "pairs": pairs, "levels": levels, "gates_per_pair": live,
            "seconds": dt, "operators_per_s": pairs / dt, "gates_per_s": pairs * live / dt,
            "graph": graph, "graph_pieces": pieces, "sub_batch": sub, "outputs_checked": "all"}


def _party_context(mk, k):
    P = mk.Params(**PARTY_SETS[k])
    ctx = mk.Context(P, SEED + k)
    for i in range(k):
        ctx.keygen(i, (SEED + 100 * k + i) & 0xFFFFFFFFFFFFFFFF)
    ctx.upload()
    return ctx


def c3_multiplier(torch, mk, pairs):
    """Config 3: the 8-bit array multiplier on `pairs` pairs from [-128, 127]
    with 4 parties (a from party 0, b from party 3), one eager evaluation
    level by level; every product decrypted."""
    ctx = _party_context(mk, 4)
    try:
        r = operator_rate(torch, mk, ctx, pairs, "mul", bits=8, graph=False, parties=(0, 3), seed=3)
    finally:
        ctx.close()
        torch.cuda.empty_cache()
    r["parties"] = 4
    return r


def _wrap16(v):
    v = np.asarray(v, np.int64) & 0xFFFF
    return np.where(v >= 0x8000, v - 0x10000, v)


def _gd_step_plain(X, y, w, shift=12):
    """One gradient-descent step on Q8.8 integers as the netlist computes it:
    r_i = sum_j X_ij w_j - y_i and g_j = sum_i X_ij r_i with every product
    (a b) >> 8 and every sum wrapped to 16 bits, then w_j - (g_j >> shift)
    (learning rate 2^-6 times 1/m = 2^-6 as one arithmetic shift)."""
    mul = lambda a, b: _wrap16((np.int64(a) * np.int64(b)) >> 8)
    m, d = X.shape
    r = []
    for i in range(m):
        acc = mul(X[i, 0], w[0])
        for j in range(1, d):
            acc = _wrap16(acc + mul(X[i, j], w[j]))
        r.append(_wrap16(acc - y[i]))
    out = []
    for j in range(d):
        acc = mul(X[0, j], r[0])
        for i in range(1, m):
            acc = _wrap16(acc + mul(X[i, j], r[i]))
        out.append(_wrap16(w[j] - (int(acc) >> shift)))
    return np.array(out, np.int64)


def c5_lr_step(torch, mk, ctx, m=64, d=4):
    """Config 5: one encrypted gradient-descent iteration of linear
    regression on m samples and d features (Q8.8, 16-bit), features split
    between the two parties (features < d/2, y and w from party 0, the rest
    from party 1), one eager evaluation level by level; the new weights are
    decrypted and checked against the plain integer step."""
    circ = mk.build_lr_step(m, d)
    levels, live, width, _ = mk.circuit_stats(circ)
    X, y, w_true = mi.lr_data(m, d, seed=5)
    w = np.clip(np.rint(w_true * 256 * 0.5), -32768, 32767).astype(np.int64)
    bits = mi.to_bits(np.concatenate([X.ravel(), y, w]), 16).reshape(-1)
    owner = np.concatenate([np.repeat([0 if j < (d + 1) // 2 else 1 for j in range(d)] * m, 16),
                            np.zeros(16 * (m + d), np.int64)])
    words = ctx.params.lwe_words
    in_ct = np.zeros((len(bits), 1, words), np.uint32)
    for p in (0, 1):
        sel = np.nonzero(owner == p)[0]
        in_ct[sel, 0] = ctx.encrypt(p, bits[sel], seed=900 + p)
    dev = torch.device("cuda:0")
    inp = torch.from_numpy(in_ct.view(np.int32)).to(dev)
    out = torch.zeros((len(circ.outputs), 1, words), dtype=torch.int32, device=dev)
    print("bench: LR step (%d levels, %d gates) running" % (levels, live), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.eval_circuit(circ, inp, out)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.device_status()
    dec = np.stack([ctx.decrypt(o) for o in out.cpu().numpy().view(np.uint32)])[:, 0]
    got = mi.from_bits(dec.reshape(d, 16))
    assert np.array_equal(got, _gd_step_plain(X, y, w)), "LR step weights"
    print("bench: LR step %.1f s, weights correct" % dt, file=sys.stderr, flush=True)
    return {"m": m, "d": d, "levels": levels, "gates": live, "widest_level": width, "seconds": dt,
            "gates_per_s": live / dt, "steps_per_s": 1.0 / dt, "outputs_checked": "all"}


def formula_lr(torch, mk, ctx, sets, m=64, frac=8):
    """Closed-form one-feature regression (§3.4 Eqs. (2)-(3), Alg. 7) on
    `sets` data sets of m pairs of 8-bit integers, pair i encrypted by party
    i mod 2, evaluated level by level in one eager call.  Every slope and
    intercept is decrypted and checked against float least squares within
    the rounding bound of the integer formula: m (1 + |w|) / sum (x - x̄)^2
    + 2^-frac for the slope, that times |x̄| plus 2^-frac for the intercept."""
    circ = mk.build_lr_formula(m, frac)
    levels, live, width, _ = mk.circuit_stats(circ)
    x, y, _, _ = mi.formula_lr_data(sets, m, seed=5)
    vals = np.concatenate([x, y], axis=1)                         # [sets, 2m]
    bits = mi.to_bits(vals.ravel(), 8).reshape(sets, -1).T       # [16m, sets]
    owner = np.repeat(np.array([i % 2 for i in range(m)] * 2), 8)
    in_ct = np.stack([ctx.encrypt(int(owner[i]), bits[i], seed=800 + i) for i in range(len(bits))])
    dev = torch.device("cuda:0")
    inp = torch.from_numpy(np.ascontiguousarray(in_ct).view(np.int32)).to(dev)
    out = torch.zeros((32, sets, in_ct.shape[2]), dtype=torch.int32, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.eval_circuit(circ, inp, out)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    dec = np.stack([ctx.decrypt(o) for o in out.cpu().numpy().view(np.uint32)])
    slope, icpt = mi.from_bits(dec[:16].T) / 2.0 ** frac, mi.from_bits(dec[16:].T) / 2.0 ** frac
    f = 2.0 ** -frac
    for s in range(sets):
        A = np.vstack([x[s].astype(float), np.ones(m)]).T
        w, c = np.linalg.lstsq(A, y[s].astype(float), rcond=None)[0]
        tol = m * (1 + abs(w)) / ((x[s] - x[s].mean()) ** 2).sum() + f
        assert abs(slope[s] - w) <= tol and abs(icpt[s] - c) <= tol * abs(x[s].mean()) + f, \
            "closed-form regression output %d off the least-squares fit" % s
    return {"sets": sets, "m": m, "levels": levels, "gates_per_set": live, "widest_level": width,
            "seconds": dt, "gates_per_s": sets * live / dt, "ms_per_level": dt * 1e3 / levels}


PARTY_SETS = {4: dict(C2, k=4), 8: dict(C2, k=8, bk_noise_log2=31, ks_noise_log2=16)}


def party_scaling(torch, mk, batch, ks):
    """Table 8's party counts on the bootstrapped gate: `batch` mixed gates at
    the Table 7 shape with k parties (k = 8 with the retuned key noise), in1
    from party 0 and in2 from party k-1, tile shapes autotuned; the second
    of two runs is timed and every output is decrypted."""
    dev = torch.device("cuda:0")
    res = {}
    for k in ks:
        P = mk.Params(**PARTY_SETS[k])
        ctx = mk.Context(P, SEED + k)
        for i in range(k):
            ctx.keygen(i, (SEED + 100 * k + i) & 0xFFFFFFFFFFFFFFFF)
        ctx.upload()
        types, m1, m2 = mi.gate_batch(batch, seed=SEED)
        c1, c2 = ctx.encrypt(0, m1, seed=200), ctx.encrypt(k - 1, m2, seed=201)
        t = torch.from_numpy(types).to(dev)
        a = torch.from_numpy(c1.view(np.int32)).to(dev)
        b = torch.from_numpy(c2.view(np.int32)).to(dev)
        out = torch.zeros_like(a)
        tiles = ctx.autotune(batch)
        for _ in range(2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.bootstrap_gate(t, a, b, out)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
        want = np.array([mi.plain_gate(int(x), int(y), int(z)) for x, y, z in zip(types, m1, m2)])
        assert np.array_equal(ctx.decrypt(out.cpu().numpy().view(np.uint32)), want), "k=%d" % k
        res[str(k)] = {"gates_per_s": batch / dt, "ms_per_batch": dt * 1e3, "tiles": list(tiles[:2]),
                       "cmux_steps": k * P.n}
        ctx.close()
        del a, b, out
        torch.cuda.empty_cache()
        print("bench: %d parties measured" % k, file=sys.stderr, flush=True)
    return res


def batch_scaling(torch, mk, ctx, sizes):
    """The headline gate mix at larger batches (wide circuit levels run at
    these sizes): tile shapes autotuned per size, the second of two runs
    timed, every output decrypted."""
    dev = torch.device("cuda:0")
    res = {}
    for n in sizes:
        types, m1, m2 = mi.gate_batch(n, seed=SEED)
        c1, c2 = ctx.encrypt(0, m1, seed=200), ctx.encrypt(1, m2, seed=201)
        t = torch.from_numpy(types).to(dev)
        a = torch.from_numpy(c1.view(np.int32)).to(dev)
        b = torch.from_numpy(c2.view(np.int32)).to(dev)
        out = torch.zeros_like(a)
        tiles = ctx.autotune(n)
        for _ in range(2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.bootstrap_gate(t, a, b, out)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
        want = np.array([mi.plain_gate(int(x), int(y), int(z)) for x, y, z in zip(types, m1, m2)])
        assert np.array_equal(ctx.decrypt(out.cpu().numpy().view(np.uint32)), want), "batch %d" % n
        res[str(n)] = {"gates_per_s": n / dt, "ms_per_batch": dt * 1e3, "tiles": list(tiles[:2]),
                       "persistent_team_rows": ctx.get_team_rows(n),
                       "whole_gate_int8_tops": 8 * macs_per_gate(C2) * n / dt / 1e12}
    print("bench: batch sizes measured", file=sys.stderr, flush=True)
    return res


def naive_comparison(torch, mk, ctx, batch):
    """Table 2 on one MI355X: every gate type run as the scheme's single
    bootstrapped gate (NOT: the free linear NOT) and as its NAND-only
    composition, on the same `batch` input pairs; the second of two runs is
    timed, and every output is decrypted against the truth table."""
    dev = torch.device("cuda:0")
    _, m1, m2 = mi.gate_batch(batch, seed=6)
    c1, c2 = ctx.encrypt(0, m1, seed=600), ctx.encrypt(1, m2, seed=601)
    ta = torch.from_numpy(c1.view(np.int32)).to(dev)
    tb = torch.from_numpy(c2.view(np.int32)).to(dev)
    inp = torch.stack([ta, tb])
    res = {}
    names = {mk.NAND: "NAND", mk.AND: "AND", mk.OR: "OR", mk.NOR: "NOR", mk.XOR: "XOR", mk.XNOR: "XNOR",
             mk.NOT: "NOT"}
    for t, name in names.items():
        want = 1 - m1 if t == mk.NOT else np.array([mi.plain_gate(t, int(x), int(y)) for x, y in zip(m1, m2)])
        out = torch.zeros_like(ta)
        types = torch.full((batch,), t, dtype=torch.uint8, device=dev)

        def scheme():
            if t == mk.NOT:
                ctx.lwe_not(ta, out)
            else:
                ctx.bootstrap_gate(types, ta, tb, out)

        circ = mk.build_naive_gate(t)
        nout = torch.zeros((1, batch, ta.shape[1]), dtype=torch.int32, device=dev)

        def naive():
            ctx.eval_circuit(circ, inp, nout)

        times = []
        for fn, o in ((scheme, out), (naive, nout[0])):
            for rep in range(2):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                fn()
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
            assert np.array_equal(ctx.decrypt(o.cpu().numpy().view(np.uint32)), want), name
            times.append(dt)
        levels, gates, _, _ = mk.circuit_stats(circ)
        res[name] = {"scheme_ms": times[0] * 1e3, "nand_composed_ms": times[1] * 1e3,
                     "nand_gates": gates, "nand_depth": levels, "speedup": times[1] / times[0]}
    return {"pairs": batch, "gates": res}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--plain-steps", type=int, default=1)
    ap.add_argument("--path", choices=["mfma", "i32"], default="mfma")
    ap.add_argument("--cpu-gates-per-core", type=int, default=8)
    ap.add_argument("--c3-pairs", type=int, default=256,
                    help="operand pairs of the 4-party 8-bit multiplier (config 3; 0: skip)")
    ap.add_argument("--c4", default="add=4096,sub=4096,mul=256,div=256",
                    help="16-bit operators and their operand pairs (config 4; empty: skip); the adder, "
                         "subtractor and multiplier run through HIP graphs, the divider eagerly")
    ap.add_argument("--c5", type=int, default=1, help="run the LR gradient-descent step (config 5; 0: skip)")
    ap.add_argument("--batch-sizes", default="256,512,2048,4096",
                    help="other batch sizes of the same gate mix to time (comma list; 0 or empty: skip)")
    ap.add_argument("--operator-subbatch", type=int, default=0,
                    help="run the 16-bit multiplier and divider eagerly in sub-batches of this many pairs "
                         "(0: one batch)")
    ap.add_argument("--party-gates", type=int, default=1024,
                    help="gates per batch of the 4- and 8-party runs (0: skip)")
    ap.add_argument("--formula-sets", type=int, default=0,
                    help="data sets of the closed-form regression run (m = 64 pairs each; 0: skip)")
    ap.add_argument("--naive-pairs", type=int, default=1024,
                    help="input pairs of the scheme-vs-NAND-composed gate comparison (0: skip)")
    ap.add_argument("--tiles", default="", metavar="G1,G2",
                    help="force the two GEMM tile shapes instead of autotuning")
    ap.add_argument("--rotation", choices=["auto", "stream", "persistent"], default="auto",
                    help="schedule of the MFMA rotation for every run of this process (mk_set_rotation)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run one device-to-device copy of MIB MiB (reference "
                         "kernel for scaling HBM byte counters) and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.int32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4}))
        return
    if args.gpus != 1:
        print("bench.py: the path runs on exactly one GPU (its work is per GPU; "
              "--gpus %d is not supported)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    cpu = None if args.no_cpu_baseline else cpu_baseline(args.cpu_gates_per_core)

    import torch

    import paper_2205_05825_amd as mk
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    P = mk.Params(**C2)
    ctx = mk.Context(P, SEED)
    for i in range(P.k):
        ctx.keygen(i, (SEED + 1 + i) & 0xFFFFFFFFFFFFFFFF)
    ctx.upload()
    ctx.set_rotation({"auto": mk.ROT_AUTO, "stream": mk.ROT_STREAM, "persistent": mk.ROT_PERSISTENT}[args.rotation])
    types, m1, m2 = mi.gate_batch(BATCH, seed=SEED)
    c1 = ctx.encrypt(0, m1, seed=200)
    c2 = ctx.encrypt(1, m2, seed=201)
    t = torch.from_numpy(types).to(dev)
    a = torch.from_numpy(c1.view(np.int32)).to(dev)
    b = torch.from_numpy(c2.view(np.int32)).to(dev)
    want = np.array([mi.plain_gate(int(x), int(y), int(z)) for x, y, z in zip(types, m1, m2)])

    def run(path, out):
        ctx.bootstrap_gate(t, a, b, out, path=path)

    paths = {"mfma": mk.PATH_MFMA_I8, "i32": mk.PATH_I32}
    head = paths[args.path]
    # the autotuner times every GEMM tile shape for this batch size
    tiles = ctx.autotune(BATCH)
    if args.tiles:
        v1, v2 = (int(x) for x in args.tiles.split(","))
        ctx.set_tiles(v1, v2)
        tiles = (v1, v2, tiles[2])
    # correctness gate before timing: outputs decrypt and both paths agree
    outs = {}
    for name, path in paths.items():
        o = torch.zeros_like(a)
        try:
            run(path, o)
        except mk.MkError as e:
            if path == mk.PATH_MFMA_I8 and head != path:
                continue
            raise
        torch.cuda.synchronize()
        outs[name] = o.cpu().numpy().view(np.uint32)
        assert np.array_equal(ctx.decrypt(outs[name]), want), name
    if len(outs) == 2:
        assert np.array_equal(outs["mfma"], outs["i32"]), "paths differ"

    def timed(path, steps, warmup, level=2):
        out = torch.zeros_like(a)
        for _ in range(warmup):
            run(path, out)
        torch.cuda.synchronize()
        ctx.get_profile(reset=True)
        ctx.set_profiling(level)
        t0 = time.perf_counter()
        for _ in range(steps):
            run(path, out)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ctx.set_profiling(0)
        ms, launches = ctx.get_profile(reset=True)
        return dt / steps, ms, launches

    sec, hms, hln = timed(head, args.steps, args.warmup, level=1)
    value = BATCH / sec
    # one more step with events around every rotation kernel: per-kernel times
    _, ms, ln = timed(head, 1, 0, level=2)
    br_ms = ms[1] / max(ln[1], 1)
    macs = macs_per_gate(C2) * BATCH
    persistent = head == mk.PATH_MFMA_I8 and ln[4] > 0 and ln[5] == 0
    # extraction and key switching inside the persistent launch: no
    # separate key-switching stage was timed
    ks_fused = persistent and ln[2] == 0
    if persistent:
        # dominant kernel: the persistent rotation (all 1120 CMux steps of
        # the batch in one launch); executed int8 ops with live-slot
        # skipping.  With key switching fused the launch also switches the
        # batch (0.3-0.4% of its time); those ops are not counted, so the
        # achieved rate is slightly conservative.
        ops = executed_int8_ops_per_gate(C2) * BATCH
        kms = ms[4] / ln[4]
        achieved = ops / (kms * 1e-3)
        traffic = measured_traffic("persist", PERSIST_KERNEL)
        roof = {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK_INT8_OPS / 1e12,
                "unit": "TOP/s", "frac": achieved / PEAK_INT8_OPS, "traffic": traffic,
                "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                "kernel": PERSIST_KERNEL, "avg_launch_ms": kms, "launches": ln[4],
                "int8_ops_per_launch": ops,
                "launch_includes": ("rotation, extraction and key switching (ops: rotation only)"
                                    if ks_fused else "rotation"),
                "hbm_GBs": traffic / (kms * 1e-3) / 1e9 if traffic else None,
                "full_hybrid_product_tops": 8 * macs / (kms * 1e-3) / 1e12}
    elif head == mk.PATH_MFMA_I8:
        # dominant kernel: the stage-1 GEMM.  During party i's steps only the
        # live accumulator slots j <= i+1 are non-zero, so a launch computes
        # 2*live*ell of the products (c'_j and w_j for live j); int8 ops =
        # 2 (multiply + add) * 4 limbs * Torus32 MACs.
        k, ell, N = C2["k"], C2["bk_ell"], C2["N"]
        live = [min(k + 1, i + 2) for i in range(k)]
        g1_ops = 8 * (sum(2 * lv * ell for lv in live) / k) * N * N * BATCH
        g1_ms = ms[4] / max(ln[4], 1)
        achieved = g1_ops / (g1_ms * 1e-3)
        kname = GEMM1_KERNEL[tiles[0]]
        traffic = measured_traffic("gemm1", kname)
        roof = {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK_INT8_OPS / 1e12,
                "unit": "TOP/s", "frac": achieved / PEAK_INT8_OPS, "traffic": traffic,
                "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                "kernel": kname, "avg_launch_ms": g1_ms, "launches": ln[4],
                "hbm_GBs": traffic / (g1_ms * 1e-3) / 1e9 if traffic else None,
                "whole_rotation_tops": 8 * macs / (br_ms * 1e-3) / 1e12}
    else:
        achieved = macs / (br_ms * 1e-3)
        roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_VALU_TORUS_MACS / 1e12,
                "unit": "T Torus32-MAC/s", "frac": achieved / PEAK_VALU_TORUS_MACS, "traffic": None,
                "kernel": "br_plain_kernel", "avg_launch_ms": br_ms}
    ctx.device_status()
    print("bench: headline measured", file=sys.stderr, flush=True)
    res = {
        "metric": "bootstrapped MK gates/sec on 1 MI355X (int8-MFMA batched vs int32 plain), bit-exact",
        "value": value, "unit": "gates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": sec * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "int8" if head == mk.PATH_MFMA_I8 else "int32", "data": "synthetic",
        "config": {"workload": "1024 mixed bootstrapped MK gates (AND/OR/NOR/XOR/XNOR/NAND), "
                               "k=2 n=560 N=1024 B=2^8 ell=3 B'=2^2 t=8",
                   "global_batch": BATCH, "path": args.path, "parallelism": "single GPU"},
        "tiles": {"gemm1_shape": tiles[0], "gemm2_shape": tiles[1], "candidate_ms": tiles[2],
                  "sub_batches": ctx.get_split(BATCH)},
        # stage times of the timed steps (HIP events around each stage, per
        # step); kernel times from one extra step with events around every
        # rotation kernel as well
        "stage_ms_per_step": {"precombine": hms[0] / args.steps, "blind_rotate": hms[1] / args.steps,
                              "extract_keyswitch": hms[2] / args.steps},
        "kernel_ms_instrumented_step": ({"persistent_rotation": ms[4], "blind_rotate_stage": ms[1]}
                                        if persistent else
                                        {"mfma_gemm1": ms[4], "mfma_gemm2": ms[5], "rotdec": ms[6],
                                         "wdec": ms[7], "blind_rotate_stage": ms[1]}),
        "rotation_schedule": "persistent" if persistent else "stream-ordered",
        "key_switch_fused": ks_fused,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    if head == mk.PATH_MFMA_I8 and args.c3_pairs > 0:
        res["c3_multiplier8_4party"] = c3_multiplier(torch, mk, args.c3_pairs)
    c4 = dict((kv.split("=")[0], int(kv.split("=")[1])) for kv in args.c4.split(",") if "=" in kv)
    if head == mk.PATH_MFMA_I8 and c4:
        res["c4_operators_16bit"] = {
            op: operator_rate(torch, mk, ctx, pairs, op, graph=op != "div",
                              sub=args.operator_subbatch if op in ("mul", "div") else 0)
            for op, pairs in c4.items() if pairs > 0}
    if head == mk.PATH_MFMA_I8 and args.c5:
        res["c5_lr_step"] = c5_lr_step(torch, mk, ctx)
    sizes = [int(x) for x in args.batch_sizes.split(",") if x.strip() and int(x) > 0]
    if head == mk.PATH_MFMA_I8 and sizes:
        res["batch_scaling"] = batch_scaling(torch, mk, ctx, sizes)
    if head == mk.PATH_MFMA_I8 and args.party_gates > 0:
        res["party_scaling"] = party_scaling(torch, mk, args.party_gates, (4, 8))
        res["party_scaling"]["2"] = {"gates_per_s": value, "ms_per_batch": sec * 1e3,
                                     "tiles": list(tiles[:2]), "cmux_steps": C2["k"] * C2["n"]}
    if head == mk.PATH_MFMA_I8 and args.formula_sets > 0:
        res["lr_formula"] = formula_lr(torch, mk, ctx, args.formula_sets)
        print("bench: closed-form regression measured", file=sys.stderr, flush=True)
    if head == mk.PATH_MFMA_I8 and args.naive_pairs > 0:
        res["naive_nand_gates"] = naive_comparison(torch, mk, ctx, args.naive_pairs)
        print("bench: NAND-composed gates measured", file=sys.stderr, flush=True)
    if head == mk.PATH_MFMA_I8 and "i32" in outs and args.plain_steps > 0:
        psec, pms, pln = timed(mk.PATH_I32, args.plain_steps, 0, level=1)
        res["plain_i32"] = {"value": BATCH / psec, "ms_per_step": psec * 1e3,
                            "blind_rotate_ms": pms[1] / max(pln[1], 1)}
        res["mfma_vs_plain"] = value / (BATCH / psec)
    if cpu:
        res["cpu_baseline"]["extrapolated"] = oracle_extrapolation(cpu, res)
    print(json.dumps(res))


def oracle_extrapolation(cpu, res):
    """Seconds the oracle would take on the host cores for the configs 3-5
    workloads just run on the GPU: their bootstrapped-gate counts over the
    oracle's measured all-core rate (the 4-party sample for config 3, the
    2-party C2 sample otherwise).  An extrapolation, not a measurement."""
    out = {"basis": "gate count / measured all-core oracle rate on %d cores; not run" % cpu["cores"]}
    rate2, rate4 = cpu["value"], cpu["c3_four_party"]["value"]
    jobs = []
    c3 = res.get("c3_multiplier8_4party")
    if c3:
        jobs.append(("c3_mul8", c3["gates_per_pair"] * c3["pairs"], rate4, c3["seconds"]))
    for op, r in res.get("c4_operators_16bit", {}).items():
        jobs.append(("c4_%s16" % op, r["gates_per_pair"] * r["pairs"], rate2, r["seconds"]))
    c5 = res.get("c5_lr_step")
    if c5:
        jobs.append(("c5_lr_step", c5["gates"], rate2, c5["seconds"]))
    for name, gates, rate, gpu_s in jobs:
        out[name] = {"gates": gates, "oracle_s": gates / rate, "gpu_s": gpu_s,
                     "gpu_speedup": gates / rate / gpu_s}
    return out


if __name__ == "__main__":
    main()
