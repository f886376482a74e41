"""Full-size workloads on the GPU (needs an MI355X).  Ciphertexts come from
the library's own encryption; every output is decrypted and compared with
integer arithmetic.  Bit parity with the oracle at these shapes is covered
per gate (the oracle is too slow for whole circuits here); whole-circuit
parity runs at small shapes in test_gpu_circuits.py."""
import time

import numpy as np
import pytest

import mk_inputs as mi
from oracle import params as OP
from oracle import tfhe
from tests import helpers

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def _enc_operand(ctx, values, bits, party, seed):
    cols = mi.to_bits(values, bits).T
    return np.stack([ctx.encrypt(party, col, seed=seed + 1000 * i) for i, col in enumerate(cols)])


def _words(torch, ctx, circ, in_ct, path=1):
    d = torch.device("cuda:0")
    inp = torch.from_numpy(np.ascontiguousarray(in_ct).view(np.int32)).to(d)
    out = torch.zeros((len(circ.outputs), in_ct.shape[1], in_ct.shape[2]), dtype=torch.int32, device=d)
    t0 = time.perf_counter()
    ctx.eval_circuit(circ, inp, out, path=path)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return out.cpu().numpy().view(np.uint32), dt


def _run(torch, ctx, circ, in_ct, path=1):
    o, dt = _words(torch, ctx, circ, in_ct, path)
    return np.stack([ctx.decrypt(x) for x in o]), dt


def _wrap(v, k):
    v = np.asarray(v, np.int64) & ((1 << k) - 1)
    return np.where(v >= 1 << (k - 1), v - (1 << k), v)


def test_c3_gate_parity_four_parties(torch_cuda):
    """Single gates at the 4-party Table 7 shape, word for word."""
    K, ctx = helpers.gpu_world("C3")
    types, m1, m2 = mi.gate_batch(40, seed=33)
    c1 = tfhe.encrypt(K, 0, m1, seed=300)
    c2 = tfhe.encrypt(K, 3, m2, seed=301)
    d = torch_cuda.device("cuda:0")
    t = torch_cuda.from_numpy(types).to(d)
    a = torch_cuda.from_numpy(c1.view(np.int32)).to(d)
    b = torch_cuda.from_numpy(c2.view(np.int32)).to(d)
    out = torch_cuda.zeros_like(a)
    ctx.bootstrap_gate(t, a, b, out, path=1)
    torch_cuda.cuda.synchronize()
    got = out.cpu().numpy().view(np.uint32)
    want = [mi.plain_gate(int(x), int(y), int(z)) for x, y, z in zip(types, m1, m2)]
    assert tfhe.decrypt(K, got).tolist() == want
    idx = [0, 17, 39]
    assert np.array_equal(got[idx], helpers.oracle_gates("C3", types, c1, c2, idx))


def test_c8_gate_parity_eight_parties(torch_cuda):
    """Single gates with 8 parties (Table 8's largest party count) at the
    Table 7 shape with the retuned key noise: in1 from party 0, in2 from
    party 7; every output decrypted, three word for word against the
    oracle."""
    K, ctx = helpers.gpu_world("C8")
    types, m1, m2 = mi.gate_batch(48, seed=38)
    c1 = tfhe.encrypt(K, 0, m1, seed=380)
    c2 = tfhe.encrypt(K, 7, m2, seed=381)
    d = torch_cuda.device("cuda:0")
    t = torch_cuda.from_numpy(types).to(d)
    a = torch_cuda.from_numpy(c1.view(np.int32)).to(d)
    b = torch_cuda.from_numpy(c2.view(np.int32)).to(d)
    out = torch_cuda.zeros_like(a)
    ctx.bootstrap_gate(t, a, b, out, path=1)
    torch_cuda.cuda.synchronize()
    got = out.cpu().numpy().view(np.uint32)
    want = [mi.plain_gate(int(x), int(y), int(z)) for x, y, z in zip(types, m1, m2)]
    assert tfhe.decrypt(K, got).tolist() == want
    idx = [0, 23, 47]
    assert np.array_equal(got[idx], helpers.oracle_gates("C8", types, c1, c2, idx))


def test_c8_adder_circuit(torch_cuda):
    """A 4-bit adder through the circuit engine with 8 parties: operand a
    from party 0, b from party 7, 16 pairs covering the range; every sum
    decrypts to a + b (mod 16) and two sampled gates match the oracle."""
    import paper_2205_05825_amd as mk
    K, ctx = helpers.gpu_world("C8")
    circ = mk.build_operator(mk.OP_ADD, 4)
    a = np.arange(-8, 8)
    b = np.roll(np.arange(-8, 8), 5)
    in_ct = np.concatenate([_enc_operand(ctx, a, 4, 0, 31), _enc_operand(ctx, b, 4, 7, 32)])
    outs, _ = helpers.sampled_level_parity("C8", circ, in_ct, lambda c: _words(torch_cuda, ctx, c, in_ct)[0], seed=88)
    dec = np.stack([ctx.decrypt(x) for x in outs])
    assert np.array_equal(mi.from_bits(dec.T), _wrap(a + b, 4))


def test_c3_multiplier_256_pairs(torch_cuda):
    """8-bit signed multiplier, 256 pairs in [-128, 127], 4 parties; a from
    party 0, b from party 1; one batch per bootstrapping level.  Six sampled
    (gate, pair) items match the oracle word for word, recomputed from the
    GPU's own inputs; every product decrypts to a * b."""
    import paper_2205_05825_amd as mk
    K, ctx = helpers.gpu_world("C3")
    circ = mk.build_operator(mk.OP_MUL, 8)
    a, b = mi.operand_pairs(256, 8, seed=3)
    in_ct = np.concatenate([_enc_operand(ctx, a, 8, 0, 1), _enc_operand(ctx, b, 8, 1, 2)])
    timing = {}

    def evaluate(c):
        words, timing["dt"] = _words(torch_cuda, ctx, c, in_ct)
        return words

    outs, _ = helpers.sampled_level_parity("C3", circ, in_ct, evaluate, seed=33)
    dec, dt = np.stack([ctx.decrypt(x) for x in outs]), timing["dt"]
    levels, live, width, _ = mk.circuit_stats(circ)
    print("C3 8-bit multiplier: %d pairs, %d levels, %d gates/pair, %.2f s, %.0f gates/s"
          % (256, levels, live, dt, live * 256 / dt))
    assert np.array_equal(mi.from_bits(dec.T), a * b)


@pytest.mark.parametrize("op", ["add", "sub", "mul", "div"])
def test_c4_operators_subset(torch_cuda, op):
    """16-bit operators at the 2-party shape on 32 pairs each (a sample of
    the 4096-pair workload), divisors non-zero."""
    import paper_2205_05825_amd as mk
    K, ctx = helpers.gpu_world("C2")
    code = {"add": mk.OP_ADD, "sub": mk.OP_SUB, "mul": mk.OP_MUL, "div": mk.OP_DIV}[op]
    circ = mk.build_operator(code, 16)
    a, b = mi.operand_pairs(32, 16, seed=4, nonzero_second=True)
    in_ct = np.concatenate([_enc_operand(ctx, a, 16, 0, 5), _enc_operand(ctx, b, 16, 1, 6)])
    timing = {}

    def evaluate(c):
        words, timing["dt"] = _words(torch_cuda, ctx, c, in_ct)
        return words

    # six sampled (gate, pair) items recomputed by the oracle from the GPU's inputs
    outs, _ = helpers.sampled_level_parity("C2", circ, in_ct, evaluate, seed=40 + code)
    dec = np.stack([ctx.decrypt(x) for x in outs])
    _, live, _, _ = mk.circuit_stats(circ)
    print("C4 16-bit %s: 32 pairs, %d gates/pair, %.2f s" % (op, live, timing["dt"]))
    v = mi.from_bits(dec.T)
    if op == "add":
        assert np.array_equal(v, _wrap(a + b, 16))
    elif op == "sub":
        assert np.array_equal(v, _wrap(a - b, 16))
    elif op == "mul":
        assert np.array_equal(v, a * b)
    else:
        q = np.abs(a) // np.abs(b) * np.sign(a) * np.sign(b)
        assert np.array_equal(mi.from_bits(dec[:16].T), _wrap(q, 16))
        assert np.array_equal(mi.from_bits(dec[16:].T), _wrap(a - q * b, 16))


@pytest.mark.timeout(600)
def test_c5_lr_step_full(torch_cuda):
    """Config 5: one encrypted gradient-descent step on m=64 samples, d=4
    features split between the two parties, 16-bit Q8.8 values, learning rate
    2^-6 as an arithmetic shift; the new weights decrypt to the integer
    replica's, and sampled gates match the oracle word for word."""
    import paper_2205_05825_amd as mk
    from oracle import lr
    K, ctx = helpers.gpu_world("C2")
    m, d = 64, 4
    X, y, w_true = mi.lr_data(m, d, seed=5)
    w = np.clip(np.rint(w_true * 256 * 0.5), -32768, 32767).astype(np.int64)   # a starting point
    circ = mk.build_lr_step(m, d)
    bits = lr.input_bits(X, y, w)[:, 0]
    owner = lr.input_owner(m, d)
    in_ct = np.zeros((len(bits), 1, K.params.lwe_words), np.uint32)
    for p in (0, 1):
        sel = np.nonzero(owner == p)[0]
        in_ct[sel, 0] = ctx.encrypt(p, bits[sel], seed=900 + p)
    timing = {}

    def evaluate(c):
        words, timing["dt"] = _words(torch_cuda, ctx, c, in_ct)
        return words

    outs, _ = helpers.sampled_level_parity("C2", circ, in_ct, evaluate, seed=55)
    dec = np.stack([ctx.decrypt(x) for x in outs])[:, 0]
    levels, live, width, _ = mk.circuit_stats(circ)
    print("C5 LR step: %d levels, %d gates, widest level %d, %.1f s, %.0f gates/s"
          % (levels, live, width, timing["dt"], live / timing["dt"]))
    assert np.array_equal(mi.from_bits(dec.reshape(d, 16)), lr.replica_step(X, y, w))



def test_add16_2200_pairs_chunked_levels(torch_cuda):
    """The 16-bit adder on 2200 pairs at the Table 7 shape: its widest level
    (31 gates x 2200 pairs = 68 200 gates) is more than one rotation launch
    takes (65 536), so it runs in two chunks that read and write the wire
    buffer while the level is in flight (the case a slot-reuse bug once
    broke).  Every sum decrypts to a + b, the unmodified circuit's outputs
    equal the extended run's, and one gate per level matches the oracle."""
    import paper_2205_05825_amd as mk
    K, ctx = helpers.gpu_world("C2")
    circ = mk.build_operator(mk.OP_ADD, 16)
    assert mk.circuit_stats(circ)[2] * 2200 > 65536
    a, b = mi.operand_pairs(2200, 16, seed=22)
    in_ct = np.concatenate([_enc_operand(ctx, a, 16, 0, 2201), _enc_operand(ctx, b, 16, 1, 2202)])
    outs, picks = helpers.sampled_level_parity("C2", circ, in_ct, lambda c: _words(torch_cuda, ctx, c, in_ct)[0],
                                               seed=2203)
    assert len(picks) == mk.circuit_stats(circ)[0]
    dec = np.stack([ctx.decrypt(x) for x in outs])
    assert np.array_equal(mi.from_bits(dec.T), _wrap(a + b, 16))


@pytest.mark.parametrize("op", ["add"])
def test_full_circuit_oracle_pairs_table7(torch_cuda, op):
    """4-bit adder on 256 pairs at the Table 7 shape (levels of 256 gates
    and more: the persistent rotation with key switching fused, teams sized
    to each level); three seeded pairs run through the whole circuit in the
    oracle (about a minute on the host's cores), from the same input
    ciphertexts, and every output word of those pairs equals the GPU's.  All
    256 sums decrypt."""
    import paper_2205_05825_amd as mk
    from oracle import circuits as C
    K, ctx = helpers.gpu_world("C2")
    k, pairs = 4, 256
    code, build = {"add": (mk.OP_ADD, C.adder), "sub": (mk.OP_SUB, C.subtractor)}[op]
    circ = mk.build_operator(code, k)
    a, b = mi.operand_pairs(pairs, k, seed=70 + code)
    in_ct = np.concatenate([helpers.encrypt_operands(K, a, k, 0, 7000 + code),
                            helpers.encrypt_operands(K, b, k, 1, 7100 + code)])
    words, _ = _words(torch_cuda, ctx, circ, in_ct)
    pick = [0] + sorted(np.random.default_rng(code).choice(np.arange(1, pairs - 1), 1, replace=False).tolist()) + [pairs - 1]
    ref = helpers.oracle_circuit("C2", build(k), np.ascontiguousarray(in_ct[:, pick]))
    assert np.array_equal(words[:, pick, :K.params.lwe_words], ref)
    dec = np.stack([tfhe.decrypt(K, o) for o in words])
    want = _wrap(a + b, k) if op == "add" else _wrap(a - b, k)
    assert np.array_equal(mi.from_bits(dec.T), want)
