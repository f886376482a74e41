"""GPU evaluation of the operator netlists through mk_eval_circuit: parity
with the oracle's gate-by-gate evaluation, and full-size workloads checked by
decryption against integer arithmetic (needs an MI355X)."""
import numpy as np
import pytest

import mk_inputs as mi
from oracle import circuits as C
from oracle import lr
from oracle import tfhe
from tests import helpers

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def _eval(torch, ctx, circ, in_ct, path):
    d = torch.device("cuda:0")
    inp = torch.from_numpy(np.ascontiguousarray(in_ct).view(np.int32)).to(d)
    out = torch.full((len(circ.outputs), in_ct.shape[1], in_ct.shape[2]), -1,
                     dtype=torch.int32, device=d)
    ctx.eval_circuit(circ, inp, out, path=path)
    torch.cuda.synchronize()
    return out.cpu().numpy().view(np.uint32)


def _trunc_div(a, b):
    q = np.abs(a) // np.abs(b) * np.sign(a) * np.sign(b)
    return q, a - q * b


def _wrap(v, k):
    v = np.asarray(v, np.int64) & ((1 << k) - 1)
    return np.where(v >= 1 << (k - 1), v - (1 << k), v)


OPS = {"add": (0, C.adder), "sub": (1, C.subtractor), "mul": (2, C.multiplier),
       "div": (3, C.divider)}


@pytest.mark.parametrize("path", [0, 1])
@pytest.mark.parametrize("op", ["add", "sub", "mul", "div"])
def test_operator_parity_c1b(torch_cuda, op, path):
    """4-bit operators on 3 operand pairs (a from party 0, b from party 1):
    every output word equals the oracle's, outputs decrypt correctly."""
    import paper_2205_05825_amd as mk
    K, ctx = helpers.gpu_world("C1B")
    code, build = OPS[op]
    k = 4
    circ = mk.build_operator(code, k)
    a, b = np.array([5, -8, 7]), np.array([-3, 3, -1])
    in_ct = np.concatenate([helpers.encrypt_operands(K, a, k, 0, 11),
                            helpers.encrypt_operands(K, b, k, 1, 12)])
    got = _eval(torch_cuda, ctx, circ, in_ct, path)
    ref = helpers.oracle_circuit("C1B", build(k), in_ct)
    assert np.array_equal(got, ref)
    dec = np.stack([tfhe.decrypt(K, o) for o in got])
    want = C.eval_plain(build(k), np.concatenate([mi.to_bits(a, k).T, mi.to_bits(b, k).T]))
    assert np.array_equal(dec, want)


def test_paths_agree_on_a_circuit(torch_cuda):
    import paper_2205_05825_amd as mk
    K, ctx = helpers.gpu_world("C1B")
    circ = mk.build_operator(mk.OP_MUL, 6)
    a, b = mi.operand_pairs(40, 6, seed=3)
    in_ct = np.concatenate([helpers.encrypt_operands(K, a, 6, 0, 21),
                            helpers.encrypt_operands(K, b, 6, 1, 22)])
    x = _eval(torch_cuda, ctx, circ, in_ct, 0)
    y = _eval(torch_cuda, ctx, circ, in_ct, 1)
    assert np.array_equal(x, y)
    dec = mi.from_bits(np.stack([tfhe.decrypt(K, o) for o in y]).T)
    assert np.array_equal(dec, a * b)


def test_four_party_circuit_parity(torch_cuda):
    """k = 4 parties at a small shape: operand bits spread over all parties."""
    import paper_2205_05825_amd as mk
    K, ctx = helpers.gpu_world("C1B4")
    circ = mk.build_operator(mk.OP_ADD, 3)
    a, b = np.array([3, -4]), np.array([-2, 1])
    in_ct = np.concatenate([helpers.encrypt_operands(K, a, 3, 0, 31),
                            helpers.encrypt_operands(K, b, 3, 3, 32)])
    got = _eval(torch_cuda, ctx, circ, in_ct, 1)
    ref = helpers.oracle_circuit("C1B4", C.adder(3), in_ct)
    assert np.array_equal(got, ref)
    dec = mi.from_bits(np.stack([tfhe.decrypt(K, o) for o in got]).T)
    assert np.array_equal(dec, _wrap(a + b, 3))


def test_lr_step_small(torch_cuda):
    """One encrypted gradient-descent step (m=2, d=2) against the replica."""
    import paper_2205_05825_amd as mk
    K, ctx = helpers.gpu_world("C1B")
    X, y, _ = mi.lr_data(2, 2, seed=7)
    w = np.array([40, -25])
    circ = mk.build_lr_step(2, 2)
    bits = lr.input_bits(X, y, w)[:, 0]
    owner = lr.input_owner(2, 2)
    in_ct = np.stack([tfhe.encrypt(K, int(owner[i]), [bits[i]], seed=500 + i)
                      for i in range(len(bits))])
    got = _eval(torch_cuda, ctx, circ, in_ct, 1)
    dec = np.stack([tfhe.decrypt(K, o) for o in got])[:, 0]
    assert np.array_equal(mi.from_bits(dec.reshape(2, 16)), lr.replica_step(X, y, w))


def test_wide_level_runs_in_chunks(torch_cuda):
    """An 8-bit multiplier on 1100 operand pairs: its partial-product level
    has 64 x 1100 = 70 400 gates, more than one rotation launch takes
    (65 536), so the engine runs it in two chunks.  Sampled gates match the
    oracle word for word; every product decrypts to a * b."""
    import paper_2205_05825_amd as mk
    K, ctx = helpers.gpu_world("C1B")
    circ = mk.build_operator(mk.OP_MUL, 8)
    _, _, width, _ = mk.circuit_stats(circ)
    pairs = 1100
    assert width * pairs > 65536
    a, b = mi.operand_pairs(pairs, 8, seed=21)
    in_ct = np.concatenate([helpers.encrypt_operands(K, a, 8, 0, 2100),
                            helpers.encrypt_operands(K, b, 8, 1, 2200)])
    outs, _ = helpers.sampled_level_parity("C1B", circ, in_ct, lambda c: _eval(torch_cuda, ctx, c, in_ct, 1), seed=23)
    dec = np.stack([tfhe.decrypt(K, o) for o in outs])
    assert np.array_equal(mi.from_bits(dec.T), a * b)


def test_chunked_level_reading_reused_slots(torch_cuda):
    """A 16-bit adder on 2200 operand pairs: its widest level (31 x 2200 =
    68 200 gates) runs in two chunks.  The first chunk's outputs must not
    land in wire slots that the second chunk still reads, so a level's
    output range never reuses slots its own gates read.  Every sum decrypts
    to a + b (mod 2^16) and sampled gates match the oracle."""
    import paper_2205_05825_amd as mk
    K, ctx = helpers.gpu_world("C1B")
    circ = mk.build_operator(mk.OP_ADD, 16)
    _, _, width, _ = mk.circuit_stats(circ)
    pairs = 2200
    assert width * pairs > 65536
    a, b = mi.operand_pairs(pairs, 16, seed=22)
    in_ct = np.concatenate([helpers.encrypt_operands(K, a, 16, 0, 2300),
                            helpers.encrypt_operands(K, b, 16, 1, 2400)])
    outs, _ = helpers.sampled_level_parity("C1B", circ, in_ct, lambda c: _eval(torch_cuda, ctx, c, in_ct, 1), seed=24)
    dec = np.stack([tfhe.decrypt(K, o) for o in outs])
    assert np.array_equal(mi.from_bits(dec.T), _wrap(a + b, 16))


def test_lr_formula_small(torch_cuda):
    """Closed-form regression (Alg. 7) on 4 data sets of m = 8 pairs, pair i
    encrypted by party i mod 2: sampled gates word for word against the
    oracle, slopes and intercepts decrypted against the integer replica."""
    import paper_2205_05825_amd as mk
    K, ctx = helpers.gpu_world("C1B")
    m, sets = 8, 4
    x, y, _, _ = mi.formula_lr_data(sets, m, seed=17)
    circ = mk.build_lr_formula(m)
    bits = lr.formula_input_bits(x, y)
    owner = lr.formula_input_owner(m, 2)
    in_ct = np.stack([tfhe.encrypt(K, int(owner[i]), bits[i], seed=700 + i) for i in range(len(bits))])
    outs, _ = helpers.sampled_level_parity("C1B", circ, in_ct, lambda c: _eval(torch_cuda, ctx, c, in_ct, 1), seed=71)
    dec = np.stack([tfhe.decrypt(K, o) for o in outs])
    got = list(zip(mi.from_bits(dec[:16].T).tolist(), mi.from_bits(dec[16:].T).tolist()))
    assert got == [lr.formula_replica(a, b) for a, b in zip(x, y)]


@pytest.mark.parametrize("path", [0, 1])
def test_graph_replays_match_eager(torch_cuda, path):
    """An operator captured as a HIP graph: three replays on new inputs, with
    eager evaluations on the same stream in between; every replay equals the
    eager result word for word and decrypts to the integer results."""
    import paper_2205_05825_amd as mk
    K, ctx = helpers.gpu_world("C1B")
    k = 4
    circ = mk.build_operator(0, k)                      # 4-bit adder
    d = torch_cuda.device("cuda:0")
    W = K.params.lwe_words + 2                          # padded rows
    batch = 5
    inp = torch_cuda.zeros((2 * k, batch, W), dtype=torch_cuda.int32, device=d)
    out = torch_cuda.full((len(circ.outputs), batch, W), -1, dtype=torch_cuda.int32, device=d)
    g = ctx.circuit_graph(circ, inp, out, path=path)
    try:
        levels, gates, pieces = g.info()
        assert levels >= 1 and gates == batch * mk.circuit_stats(circ)[1]
        if path == 1:   # 4 kernels per CMux step, k*n = 128 steps per level
            assert pieces >= levels * 4 * 128 // 1024
        rng = np.random.default_rng(70 + path)
        for rep in range(3):
            a = rng.integers(-8, 8, batch)
            b = rng.integers(-8, 8, batch)
            in_ct = np.concatenate([helpers.encrypt_operands(K, a, k, 0, 700 + rep),
                                    helpers.encrypt_operands(K, b, k, 1, 710 + rep)])
            padded = np.zeros((2 * k, batch, W), np.uint32)
            padded[:, :, :in_ct.shape[2]] = in_ct
            inp.copy_(torch_cuda.from_numpy(padded.view(np.int32)).to(d))
            g.launch()
            torch_cuda.cuda.synchronize()
            got = out.cpu().numpy().view(np.uint32).copy()
            eager = _eval(torch_cuda, ctx, circ, padded, path)     # eager work in between
            assert np.array_equal(got[:, :, :K.params.lwe_words], eager[:, :, :K.params.lwe_words]), rep
            dec = np.stack([tfhe.decrypt(K, o[:, :K.params.lwe_words]) for o in got])
            assert np.array_equal(mi.from_bits(dec.T), _wrap(a + b, k)), rep
    finally:
        g.close()


def test_graph_of_a_table7_operator(torch_cuda):
    """A 16-bit adder at the 2-party Table 7 shape captured as a graph (about
    4500 kernels per level, cut into bounded pieces): two launches equal the
    eager evaluation word for word and decrypt to the sums."""
    import paper_2205_05825_amd as mk
    K, ctx = helpers.gpu_world("C2")
    k, batch = 16, 6
    circ = mk.build_operator(mk.OP_ADD, k)
    a, b = mi.operand_pairs(batch, k, seed=8)
    in_ct = np.concatenate([helpers.encrypt_operands(K, a, k, 0, 800),
                            helpers.encrypt_operands(K, b, k, 1, 810)])
    d = torch_cuda.device("cuda:0")
    inp = torch_cuda.from_numpy(np.ascontiguousarray(in_ct).view(np.int32)).to(d)
    out = torch_cuda.zeros((k, batch, in_ct.shape[2]), dtype=torch_cuda.int32, device=d)
    g = ctx.circuit_graph(circ, inp, out, path=1)
    try:
        levels, _, pieces = g.info()
        assert pieces >= levels * 4 * K.params.k * K.params.n // 1024
        eager = _eval(torch_cuda, ctx, circ, in_ct, 1)
        for _ in range(2):
            out.fill_(0)
            g.launch()
            torch_cuda.cuda.synchronize()
            assert np.array_equal(out.cpu().numpy().view(np.uint32), eager)
    finally:
        g.close()
    dec = np.stack([tfhe.decrypt(K, o) for o in eager])
    assert np.array_equal(mi.from_bits(dec.T), _wrap(a + b, k))


def test_graph_of_persistent_levels_table7(torch_cuda):
    """A 4-bit adder on 256 pairs at the Table 7 shape captured as a graph:
    its levels of 256 gates and more run the persistent rotation (teams of
    32, 16 or 8 by width) with key switching inside the launch.  Three
    launches, with an eager evaluation between them, equal the eager words,
    and the sums decrypt."""
    import paper_2205_05825_amd as mk
    K, ctx = helpers.gpu_world("C2")
    k, batch = 4, 256
    circ = mk.build_operator(mk.OP_ADD, k)
    a, b = mi.operand_pairs(batch, k, seed=9)
    in_ct = np.concatenate([helpers.encrypt_operands(K, a, k, 0, 900),
                            helpers.encrypt_operands(K, b, k, 1, 910)])
    d = torch_cuda.device("cuda:0")
    inp = torch_cuda.from_numpy(np.ascontiguousarray(in_ct).view(np.int32)).to(d)
    out = torch_cuda.zeros((k, batch, in_ct.shape[2]), dtype=torch_cuda.int32, device=d)
    g = ctx.circuit_graph(circ, inp, out, path=1)
    try:
        eager = _eval(torch_cuda, ctx, circ, in_ct, 1)
        for _ in range(3):
            out.fill_(0)
            g.launch()
            torch_cuda.cuda.synchronize()
            ctx.device_status()
            assert np.array_equal(out.cpu().numpy().view(np.uint32), eager)
            _eval(torch_cuda, ctx, circ, in_ct, 1)
    finally:
        g.close()
    dec = np.stack([tfhe.decrypt(K, o) for o in eager])
    assert np.array_equal(mi.from_bits(dec.T), _wrap(a + b, k))


@pytest.mark.parametrize("t", range(7))
def test_naive_gates_parity(torch_cuda, t):
    """NAND-composed gates (Table 2's comparison design) through the engine:
    every output word equals the oracle's gate-by-gate evaluation, and the
    outputs decrypt to the truth table."""
    import paper_2205_05825_amd as mk
    K, ctx = helpers.gpu_world("C1B")
    circ = mk.build_naive_gate(t)
    a = np.array([0, 0, 1, 1, 1, 0], np.uint8)
    b = np.array([0, 1, 0, 1, 1, 1], np.uint8)
    in_ct = np.stack([tfhe.encrypt(K, 0, a, seed=60 + t), tfhe.encrypt(K, 1, b, seed=70 + t)])
    got = _eval(torch_cuda, ctx, circ, in_ct, 1)
    assert np.array_equal(got, helpers.oracle_circuit("C1B", C.naive_gate(t), in_ct))
    want = [1 - x for x in a] if t == mk.NOT else [mi.plain_gate(t, int(x), int(y)) for x, y in zip(a, b)]
    assert tfhe.decrypt(K, got[0]).tolist() == want


@pytest.mark.parametrize("piece", [64, 4096])
def test_graph_piece_sizes(torch_cuda, piece):
    """Graphs cut into pieces of 64 and of 4096 kernels (the bounds
    mk_set_graph_piece accepts): two replays equal the eager evaluation word
    for word, and the piece count follows the size."""
    import paper_2205_05825_amd as mk
    K, ctx = helpers.gpu_world("C1B")
    k, batch = 4, 7
    circ = mk.build_operator(0, k)
    W = K.params.lwe_words
    d = torch_cuda.device("cuda:0")
    a = np.arange(batch) - 3
    b = 5 - 2 * np.arange(batch)
    in_ct = np.concatenate([helpers.encrypt_operands(K, a, k, 0, 7200 + piece),
                            helpers.encrypt_operands(K, b, k, 1, 7300 + piece)])
    inp = torch_cuda.from_numpy(np.ascontiguousarray(in_ct).view(np.int32)).to(d)
    out = torch_cuda.full((len(circ.outputs), batch, W), -1, dtype=torch_cuda.int32, device=d)
    eager = _eval(torch_cuda, ctx, circ, in_ct, 1)
    ctx.set_graph_piece(piece)
    try:
        g = ctx.circuit_graph(circ, inp, out, path=1)
    finally:
        ctx.set_graph_piece(1024)
    try:
        pieces = g.info()[2]
        levels = mk.circuit_stats(circ)[0]
        # 4 kernels per stream-ordered CMux step (k n = 128 steps per level)
        assert pieces >= levels * 4 * 128 // piece
        for _ in range(2):
            g.launch()
            torch_cuda.cuda.synchronize()
            assert np.array_equal(out.cpu().numpy().view(np.uint32), eager)
    finally:
        g.close()
    dec = np.stack([tfhe.decrypt(K, o) for o in eager])
    assert np.array_equal(mi.from_bits(dec.T), _wrap(a + b, k))
