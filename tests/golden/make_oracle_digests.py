"""Writes oracle_c2_digests.txt: SHA-256 digests of oracle outputs at the
Table 7 shape (parameter set C2: k=2, n=560, N=1024, ell=3, t=8), for GPU
parity tests that compare every output word without running the oracle on
the GPU machine for minutes (it takes about 4 s per gate on one core).

Calls only oracle/ and the plaintext workload generator mk_inputs.  Two
records, each one digest per row over the row's uint32 words (little endian):

  gate <g> <hex>   the 1024-gate mixed workload: types and bits from
                   mk_inputs.gate_batch(1024, seed=2), in1 encrypted by party 0
                   with seed 200, in2 by party 1 with seed 201; the digest
                   covers the kn+1 output words of the bootstrapped gate g.
  rot <g> <hex>    full blind rotations (all k n = 1120 CMux steps, both
                   parties) of 8 modulus-switched inputs drawn uniformly from
                   [0, 2N) by numpy.random.default_rng(4); the digest covers
                   the (k+1) N accumulator words.

Usage: python tests/golden/make_oracle_digests.py [workers]
"""
from __future__ import annotations

import hashlib
import os
import sys
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import mk_inputs as mi  # noqa: E402
from oracle import params as OP  # noqa: E402
from oracle import tfhe  # noqa: E402

SEED = 2          # key seed of C2 in the tests
GATES = 1024
ROT_GATES = 8
OUT = os.path.join(HERE, "oracle_c2_digests.txt")

_K = None


def _keys():
    global _K
    if _K is None:
        _K = tfhe.generate(OP.C2, SEED)
    return _K


def digest(words) -> str:
    return hashlib.sha256(np.ascontiguousarray(words, dtype="<u4").tobytes()).hexdigest()


_W = None


def workload():
    global _W
    if _W is not None:
        return _W
    K = _keys()
    types, m1, m2 = mi.gate_batch(GATES, seed=2)
    c1 = tfhe.encrypt(K, 0, m1, seed=200)
    c2 = tfhe.encrypt(K, K.params.k - 1, m2, seed=201)
    _W = (types, c1, c2)
    return _W


def rotation_inputs():
    P = OP.C2
    return np.random.default_rng(4).integers(0, 2 * P.N, (ROT_GATES, P.lwe_words)).astype(np.uint32)


def _gate(g):
    K = _keys()
    types, c1, c2 = workload()
    out = tfhe.bootstrapped_gate(K, int(types[g]), c1[g], c2[g], K.evaluation_key())
    return "gate", g, digest(out)


def _rot(g):
    K = _keys()
    acc = tfhe.blind_rotate(K, rotation_inputs()[g].astype(np.int64))
    return "rot", g, digest(np.asarray(acc).reshape(-1))


def main(workers: int):
    jobs = [(_rot, g) for g in range(ROT_GATES)] + [(_gate, g) for g in range(GATES)]
    with ProcessPoolExecutor(max_workers=workers, initializer=_keys) as ex:
        futs = [ex.submit(f, g) for f, g in jobs]
        rows = [f.result() for f in futs]
    with open(OUT, "w") as fh:
        fh.write("# SHA-256 of oracle outputs at the Table 7 shape (C2); written by\n")
        fh.write("# make_oracle_digests.py, which calls only oracle/ and mk_inputs.\n")
        for kind, g, h in rows:
            fh.write("%s %d %s\n" % (kind, g, h))
    print("wrote", OUT, len(rows), "digests")


def load(path=OUT):
    """{('gate'|'rot', index): hex digest}"""
    out = {}
    with open(path) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            kind, g, h = line.split()
            out[(kind, int(g))] = h
    return out


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else os.cpu_count() or 1)
