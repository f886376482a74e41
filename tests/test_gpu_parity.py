"""GPU parity of the bootstrapping pipeline against the oracle, bit for bit,
through the C ABI (needs an MI355X)."""
import numpy as np
import pytest

import mk_inputs as mi
from oracle import params as OP
from oracle import tfhe
from tests import helpers
from tests.golden.make_oracle_digests import digest, load as golden_digests, rotation_inputs

pytestmark = pytest.mark.gpu

PATHS = [0, 1]   # MK_PATH_I32, MK_PATH_MFMA_I8


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def _gates_on_gpu(torch, ctx, types, c1, c2, path):
    d = torch.device("cuda:0")
    t = torch.from_numpy(np.ascontiguousarray(types, np.uint8)).to(d)
    a = torch.from_numpy(np.ascontiguousarray(c1).view(np.int32)).to(d)
    b = torch.from_numpy(np.ascontiguousarray(c2).view(np.int32)).to(d)
    out = torch.full_like(a, -1)
    ctx.bootstrap_gate(t, a, b, out, path=path)
    torch.cuda.synchronize()
    return out.cpu().numpy().view(np.uint32)


def _workload(K, types, m1, m2, seed, stride=None):
    P = K.params
    c1 = tfhe.encrypt(K, 0, m1, seed=seed)
    c2 = tfhe.encrypt(K, P.k - 1 if P.k > 1 else 0, m2, seed=seed + 1)
    if stride:
        pad = np.zeros((len(types), stride - P.lwe_words), np.uint32)
        c1, c2 = np.hstack([c1, pad]), np.hstack([c2, pad])
    return c1, c2


@pytest.mark.parametrize("path", PATHS)
def test_c1_truth_table_workload(torch_cuda, path):
    """4 XOR + 4 NAND on every input pair, seed 0: every output word."""
    K, ctx = helpers.gpu_world("C1")
    types, m1, m2 = mi.truth_table(gates=(mi.XOR, mi.NAND))
    c1, c2 = _workload(K, types, m1, m2, seed=0)
    got = _gates_on_gpu(torch_cuda, ctx, types, c1, c2, path)
    ref = helpers.oracle_gates("C1", types, c1, c2)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("path", PATHS)
def test_c1b_random_batch_decrypts_and_matches(torch_cuda, path):
    K, ctx = helpers.gpu_world("C1B")
    types, m1, m2 = mi.gate_batch(77, seed=31)
    c1, c2 = _workload(K, types, m1, m2, seed=40)
    got = _gates_on_gpu(torch_cuda, ctx, types, c1, c2, path)
    ref = helpers.oracle_gates("C1B", types, c1, c2)
    assert np.array_equal(got, ref)
    want = [mi.plain_gate(int(t), int(a), int(b)) for t, a, b in zip(types, m1, m2)]
    assert tfhe.decrypt(K, got).tolist() == want


@pytest.mark.parametrize("path", PATHS)
def test_blind_rotate_stage_c1(torch_cuda, path):
    """Arbitrary modulus-switched inputs, including zero shifts."""
    K, ctx = helpers.gpu_world("C1")
    P = K.params
    rng = np.random.default_rng(3)
    abar = rng.integers(0, 2 * P.N, (5, P.lwe_words)).astype(np.uint32)
    abar[1, 1::2] = 0                    # skipped steps
    abar[2, :] = 0
    abar[3, :] = 2 * P.N - 1
    d = torch_cuda.device("cuda:0")
    ta = torch_cuda.from_numpy(abar.view(np.int32)).to(d)
    acc = torch_cuda.zeros((5, (P.k + 1) * P.N), dtype=torch_cuda.int32, device=d)
    ctx.blind_rotate(ta, acc, path=path)
    torch_cuda.cuda.synchronize()
    got = acc.cpu().numpy().view(np.uint32).reshape(5, P.k + 1, P.N)
    for g in range(5):
        assert np.array_equal(got[g], tfhe.blind_rotate(K, abar[g].astype(np.int64))), g


@pytest.mark.parametrize("path", PATHS)
def test_blind_rotate_partial_c2(torch_cuda, path):
    """First 12 CMux steps of 96 C2 gates (several workgroups, ragged)."""
    K, ctx = helpers.gpu_world("C2")
    P = K.params
    rng = np.random.default_rng(4)
    cnt = 96
    abar = rng.integers(0, 2 * P.N, (cnt, P.lwe_words)).astype(np.uint32)
    d = torch_cuda.device("cuda:0")
    ta = torch_cuda.from_numpy(abar.view(np.int32)).to(d)
    acc = torch_cuda.zeros((cnt, (P.k + 1) * P.N), dtype=torch_cuda.int32, device=d)
    ctx.blind_rotate(ta, acc, max_steps=12, path=path)
    torch_cuda.cuda.synchronize()
    got = acc.cpu().numpy().view(np.uint32).reshape(cnt, P.k + 1, P.N)
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(8) as ex:
        refs = list(ex.map(lambda g: tfhe.blind_rotate(K, abar[g].astype(np.int64), max_steps=12),
                           range(cnt)))
    for g in range(cnt):
        assert np.array_equal(got[g], refs[g]), g


def _keyswitch_case(torch_cuda, name, cnt, path, seed):
    K, ctx = helpers.gpu_world(name)
    P = K.params
    rng = np.random.default_rng(seed)
    acc = rng.integers(0, 1 << 32, (cnt, (P.k + 1) * P.N), dtype=np.uint64).astype(np.uint32)
    acc[1] = 0
    acc[2, :] = 0xFFFFFFFF       # every digit at its maximum after rounding
    d = torch_cuda.device("cuda:0")
    tacc = torch_cuda.from_numpy(acc.view(np.int32)).to(d)
    stride = P.lwe_words + 3
    out = torch_cuda.full((cnt, stride), 7, dtype=torch_cuda.int32, device=d)
    ctx.extract_keyswitch(tacc, out, path=path)
    torch_cuda.cuda.synchronize()
    got = out.cpu().numpy().view(np.uint32)
    for g in range(cnt):
        big = tfhe.sample_extract(acc[g].reshape(P.k + 1, P.N))
        big[0] = np.uint32((int(big[0]) + tfhe.EIGHTH) & 0xFFFFFFFF)
        assert np.array_equal(got[g, :P.lwe_words], tfhe.key_switch(K, big)), (name, g)
        assert (got[g, P.lwe_words:] == 7).all()      # padding untouched


@pytest.mark.parametrize("path", PATHS)
def test_extract_keyswitch_stage_c2(torch_cuda, path):
    _keyswitch_case(torch_cuda, "C2", 6, path, 5)


@pytest.mark.parametrize("name,cnt", [("C1", 70), ("C1B4", 33), ("TOYB3", 41)])
def test_extract_keyswitch_shapes(torch_cuda, name, cnt):
    """Key switching on both paths: t = 6 digits (padded one-hot blocks),
    k = 4 parties (column 0 summed over parties), base-8 digits (generic
    one-hot, two K-blocks per coefficient), ragged gate tiles."""
    for path in PATHS:
        _keyswitch_case(torch_cuda, name, cnt, path, 50 + cnt)


# (path, rotation schedule) pairs: the i32 path, and the MFMA path with the
# stream-ordered and the persistent blind rotation
SCHEDULES = [(0, -1), (1, 0), (1, 1)]


def _with_rotation(ctx, kind, fn):
    ctx.set_rotation(kind)
    try:
        return fn()
    finally:
        ctx.set_rotation(-1)


@pytest.mark.parametrize("path,rot", SCHEDULES)
def test_c2_batch_1024(torch_cuda, path, rot):
    """The 1024-gate mixed workload at the Table 7 shape: every output word
    of every gate equals the oracle's (SHA-256 digests of the oracle's rows
    written by tests/golden/make_oracle_digests.py), every output decrypts
    to the plaintext gate, and two gates are recomputed by the oracle live."""
    K, ctx = helpers.gpu_world("C2")
    types, m1, m2 = mi.gate_batch(1024, seed=2)
    c1, c2 = _workload(K, types, m1, m2, seed=200)
    got = _with_rotation(ctx, rot, lambda: _gates_on_gpu(torch_cuda, ctx, types, c1, c2, path))
    ctx.device_status()
    want = [mi.plain_gate(int(t), int(a), int(b)) for t, a, b in zip(types, m1, m2)]
    assert tfhe.decrypt(K, got).tolist() == want
    dig = golden_digests()
    bad = [g for g in range(1024) if digest(got[g]) != dig[("gate", g)]]
    assert not bad, bad[:20]
    idx = [int(i) for i in np.random.default_rng(6 + path + rot).choice(1024, 2, replace=False)]
    assert np.array_equal(got[idx], helpers.oracle_gates("C2", types, c1, c2, idx))


@pytest.mark.parametrize("path,rot", SCHEDULES)
def test_c2_full_rotation(torch_cuda, path, rot):
    """All k n = 1120 CMux steps of 8 gates at the Table 7 shape, every
    accumulator word against the oracle's digests."""
    K, ctx = helpers.gpu_world("C2")
    P = K.params
    abar = rotation_inputs()
    d = torch_cuda.device("cuda:0")
    ta = torch_cuda.from_numpy(abar.view(np.int32)).to(d)
    acc = torch_cuda.zeros((len(abar), (P.k + 1) * P.N), dtype=torch_cuda.int32, device=d)
    _with_rotation(ctx, rot, lambda: ctx.blind_rotate(ta, acc, path=path))
    torch_cuda.cuda.synchronize()
    ctx.device_status()
    got = acc.cpu().numpy().view(np.uint32)
    dig = golden_digests()
    bad = [g for g in range(len(abar)) if digest(got[g]) != dig[("rot", g)]]
    assert not bad, bad


@pytest.mark.parametrize("path", PATHS)
def test_edge_cases(torch_cuda, path):
    K, ctx = helpers.gpu_world("C1")
    P = K.params
    d = torch_cuda.device("cuda:0")
    # empty batch is a no-op
    e = torch_cuda.zeros((0, P.lwe_words), dtype=torch_cuda.int32, device=d)
    ctx.bootstrap_gate(torch_cuda.zeros(0, dtype=torch_cuda.uint8, device=d), e, e, e, path=path)
    # padded stride, single gate, trivial (noiseless) inputs: all mask shifts 0
    stride = P.lwe_words + 5
    for types, c1, c2 in [
        (np.array([mi.AND], np.uint8), *_workload(K, [mi.AND], [1], [1], 9, stride)),
        (np.array([mi.XOR, mi.NOR], np.uint8),
         np.hstack([tfhe.trivial(P, [1, 0]), np.zeros((2, 5), np.uint32)]),
         np.hstack([tfhe.trivial(P, [0, 0]), np.zeros((2, 5), np.uint32)])),
    ]:
        got = _gates_on_gpu(torch_cuda, ctx, types, c1, c2, path)
        ref = helpers.oracle_gates("C1", types, c1, c2)
        assert np.array_equal(got[:, :P.lwe_words], ref)
        assert (got[:, P.lwe_words:] == 0xFFFFFFFF).all()


@pytest.mark.parametrize("path", PATHS)
def test_repeat_is_deterministic(torch_cuda, path):
    K, ctx = helpers.gpu_world("C1")
    types, m1, m2 = mi.gate_batch(300, seed=8)
    c1, c2 = _workload(K, types, m1, m2, seed=80)
    a = _gates_on_gpu(torch_cuda, ctx, types, c1, c2, path)
    b = _gates_on_gpu(torch_cuda, ctx, types, c1, c2, path)
    assert np.array_equal(a, b)


def test_not_gate(torch_cuda):
    K, ctx = helpers.gpu_world("C1")
    c = tfhe.encrypt(K, 0, [0, 1, 1], seed=5)
    d = torch_cuda.device("cuda:0")
    t = torch_cuda.from_numpy(c.view(np.int32)).to(d)
    out = torch_cuda.empty_like(t)
    ctx.lwe_not(t, out)
    torch_cuda.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy().view(np.uint32), tfhe.lwe_not(c))


@pytest.mark.parametrize("shape", [0, 1, 2, 3, 4, 5, 6, 7])
def test_every_tile_shape_is_bit_identical(torch_cuda, shape):
    """The GEMM tile shapes only change speed: outputs of every shape equal
    the oracle's (C1 gates) and each other's (C2 partial rotation)."""
    K, ctx = helpers.gpu_world("C1")
    types, m1, m2 = mi.gate_batch(70, seed=12)
    c1, c2 = _workload(K, types, m1, m2, seed=120)
    ctx.set_tiles(shape, shape)
    try:
        got = _gates_on_gpu(torch_cuda, ctx, types, c1, c2, 1)
    finally:
        ctx.set_tiles(-1, -1)
    assert np.array_equal(got, helpers.oracle_gates("C1", types, c1, c2))
    K2, ctx2 = helpers.gpu_world("C2")
    P = K2.params
    abar = np.random.default_rng(9).integers(0, 2 * P.N, (200, P.lwe_words)).astype(np.uint32)
    d = torch_cuda.device("cuda:0")
    ta = torch_cuda.from_numpy(abar.view(np.int32)).to(d)
    outs = []
    for sh in (0, shape):
        acc = torch_cuda.zeros((200, (P.k + 1) * P.N), dtype=torch_cuda.int32, device=d)
        ctx2.set_tiles(sh, sh)
        try:
            ctx2.blind_rotate(ta, acc, max_steps=600, path=1)   # crosses into party 1
        finally:
            ctx2.set_tiles(-1, -1)
        torch_cuda.cuda.synchronize()
        outs.append(acc.cpu().numpy())
    assert np.array_equal(outs[0], outs[1])


def test_large_batch_runs_in_chunks(torch_cuda):
    """70 000 gates in one call, more than one rotation launch takes (65 536):
    the call runs two chunks.  Gates on both sides of the chunk boundary
    match the oracle word for word, and every output decrypts to its truth
    table value."""
    K, ctx = helpers.gpu_world("C1B")
    types, m1, m2 = mi.gate_batch(70000, seed=31)
    c1, c2 = _workload(K, types, m1, m2, seed=310)
    got = _gates_on_gpu(torch_cuda, ctx, types, c1, c2, 1)
    want = [mi.plain_gate(int(x), int(y), int(z)) for x, y, z in zip(types, m1, m2)]
    assert tfhe.decrypt(K, got).tolist() == want
    idx = [0, 65535, 65536, 69999]
    assert np.array_equal(got[idx], helpers.oracle_gates("C1B", types, c1, c2, idx))


def test_split_batches_are_bit_identical(torch_cuda):
    """A batch run as two sub-batches on two streams gives the same words as
    the whole batch and as the oracle (ragged halves: 70 gates -> 64 + 6)."""
    K, ctx = helpers.gpu_world("C1")
    types, m1, m2 = mi.gate_batch(70, seed=15)
    c1, c2 = _workload(K, types, m1, m2, seed=150)
    ref = helpers.oracle_gates("C1", types, c1, c2)
    outs = []
    for parts in (2, 1):
        ctx.set_split(70, parts)
        assert ctx.get_split(70) == parts
        try:
            outs.append(_gates_on_gpu(torch_cuda, ctx, types, c1, c2, 1))
        finally:
            ctx.set_split(70, 0)
    assert np.array_equal(outs[0], ref) and np.array_equal(outs[1], ref)
    K2, ctx2 = helpers.gpu_world("C2")
    P = K2.params
    abar = np.random.default_rng(19).integers(0, 2 * P.N, (300, P.lwe_words)).astype(np.uint32)
    d = torch_cuda.device("cuda:0")
    ta = torch_cuda.from_numpy(abar.view(np.int32)).to(d)
    accs = []
    for parts in (1, 2):
        acc = torch_cuda.zeros((300, (P.k + 1) * P.N), dtype=torch_cuda.int32, device=d)
        ctx2.set_split(300, parts)
        try:
            ctx2.blind_rotate(ta, acc, max_steps=600, path=1)
        finally:
            ctx2.set_split(300, 0)
        torch_cuda.cuda.synchronize()
        accs.append(acc.cpu().numpy())
    assert np.array_equal(accs[0], accs[1])


def test_smallest_ring_shapes(torch_cuda):
    """N = 128 (4 K-blocks): the 256-row shapes are refused, the default for
    large batches is the first shape that fits, and every admissible shape
    matches the oracle, ragged gate tiles included."""
    K, ctx = helpers.gpu_world("C1S")
    assert ctx.get_tiles(100) == (5, 6) and ctx.get_tiles(1000) == (1, 3)
    for bad in (0, 4):
        with pytest.raises(Exception):
            ctx.set_tiles(bad, bad)
    types, m1, m2 = mi.gate_batch(45, seed=14)
    c1, c2 = _workload(K, types, m1, m2, seed=140)
    ref = helpers.oracle_gates("C1S", types, c1, c2)
    for shape in (1, 2, 3, 5, 6, 7):
        ctx.set_tiles(shape, shape)
        try:
            got = _gates_on_gpu(torch_cuda, ctx, types, c1, c2, 1)
        finally:
            ctx.set_tiles(-1, -1)
        assert np.array_equal(got, ref), shape
    v1, v2, ms = ctx.autotune(45)
    assert v1 in (1, 2, 3, 5, 6, 7) and v2 in (1, 2, 3, 5, 6, 7)
    assert ms[0] == 0 and ms[4] == 0 and ms[8] == 0 and ms[12] == 0


def test_autotune_picks_valid_shapes(torch_cuda):
    K, ctx = helpers.gpu_world("C1")
    v1, v2, ms = ctx.autotune(300)
    assert v1 in range(8) and v2 in range(8)
    assert ctx.get_tiles(300) == (v1, v2)
    assert all(m > 0 for m in ms)     # N/32 = 8 admits every shape
    types, m1, m2 = mi.gate_batch(300, seed=13)
    c1, c2 = _workload(K, types, m1, m2, seed=130)
    got = _gates_on_gpu(torch_cuda, ctx, types, c1, c2, 1)
    ref = helpers.oracle_gates("C1", types, c1, c2, idx=[0, 150, 299])
    assert np.array_equal(got[[0, 150, 299]], ref)
