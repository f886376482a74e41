"""The persistent blind rotation (one launch for all CMux steps, XCD-local
teams of workgroups) against the oracle and against the stream-ordered
schedule, word for word, through the C ABI (needs an MI355X)."""
import numpy as np
import pytest

import mk_inputs as mi
from oracle import tfhe
from paper_2205_05825_amd import MkError
from tests import helpers

pytestmark = pytest.mark.gpu

STREAM, PERSISTENT = 0, 1


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def _gates(torch, ctx, types, c1, c2, rot, fuse=True, rows=0):
    d = torch.device("cuda:0")
    t = torch.from_numpy(np.ascontiguousarray(types, np.uint8)).to(d)
    a = torch.from_numpy(np.ascontiguousarray(c1).view(np.int32)).to(d)
    b = torch.from_numpy(np.ascontiguousarray(c2).view(np.int32)).to(d)
    out = torch.full_like(a, -1)
    ctx.set_rotation(rot)
    ctx.set_ks_fusion(fuse)
    if rows:
        ctx.set_team_rows(rows)
    try:
        ctx.bootstrap_gate(t, a, b, out, path=1)
    finally:
        ctx.set_rotation(-1)
        ctx.set_ks_fusion(True)
        ctx.set_team_rows(0)
    torch.cuda.synchronize()
    ctx.device_status()
    return out.cpu().numpy().view(np.uint32)


def _rotate(torch, ctx, abar, steps, rot, rows=0):
    P = ctx.params
    d = torch.device("cuda:0")
    ta = torch.from_numpy(np.ascontiguousarray(abar).view(np.int32)).to(d)
    acc = torch.zeros((len(abar), (P.k + 1) * P.N), dtype=torch.int32, device=d)
    ctx.set_rotation(rot)
    ctx.set_team_rows(rows)
    try:
        ctx.blind_rotate(ta, acc, max_steps=steps, path=1)
    finally:
        ctx.set_rotation(-1)
        ctx.set_team_rows(0)
    torch.cuda.synchronize()
    ctx.device_status()
    return acc.cpu().numpy().view(np.uint32)


def _workload(K, cnt, seed):
    types, m1, m2 = mi.gate_batch(cnt, seed=seed)
    c1 = tfhe.encrypt(K, 0, m1, seed=seed + 1)
    c2 = tfhe.encrypt(K, K.params.k - 1, m2, seed=seed + 2)
    return types, m1, m2, c1, c2


@pytest.mark.parametrize("name,cnt", [("C1B", 70), ("C1S", 45), ("C1B4", 97), ("C1SB3", 75), ("C1B", 1)])
def test_gates_every_word(torch_cuda, name, cnt):
    """Whole gates with the persistent rotation forced (extraction and key
    switching inside its launch): every output word equals the oracle's
    (N = 256 and N = 128 rings, k = 2, 3 and 4 parties, base-4 and base-8
    key switching, ragged gate tiles, a single gate) and decrypts to the
    plaintext gate (the C1B noise levels make every gate decrypt; C1's do
    not)."""
    K, ctx = helpers.gpu_world(name)
    types, m1, m2, c1, c2 = _workload(K, cnt, 60 + cnt)
    got = _gates(torch_cuda, ctx, types, c1, c2, PERSISTENT)
    assert np.array_equal(got, helpers.oracle_gates(name, types, c1, c2))
    want = [mi.plain_gate(int(t), int(a), int(b)) for t, a, b in zip(types, m1, m2)]
    assert tfhe.decrypt(K, got).tolist() == want


@pytest.mark.parametrize("name,cnt", [("C1SB3", 300), ("C1B", 1100), ("C2", 1100)])
def test_fused_key_switch(torch_cuda, name, cnt):
    """Extraction and key switching inside the persistent launch give the
    same words as the separate kernels after it and as the stream-ordered
    schedule; three gates equal the oracle's and every gate decrypts.  At
    the Table 7 shape 1100 gates are 35 tiles, more than the 4 teams an XCD
    holds at once, so teams switch two tiles each."""
    K, ctx = helpers.gpu_world(name)
    types, m1, m2, c1, c2 = _workload(K, cnt, 80 + cnt)
    fused = _gates(torch_cuda, ctx, types, c1, c2, PERSISTENT)
    apart = _gates(torch_cuda, ctx, types, c1, c2, PERSISTENT, fuse=False)
    strm = _gates(torch_cuda, ctx, types, c1, c2, STREAM)
    assert np.array_equal(fused, apart)
    assert np.array_equal(fused, strm)
    idx = [0, cnt // 2, cnt - 1]
    assert np.array_equal(fused[idx], helpers.oracle_gates(name, types, c1, c2, idx))
    want = [mi.plain_gate(int(t), int(a), int(b)) for t, a, b in zip(types, m1, m2)]
    assert tfhe.decrypt(K, fused).tolist() == want


@pytest.mark.parametrize("rows", [2, 4, 8])
def test_team_sizes_match_stream(torch_cuda, rows):
    """Every team size of the persistent rotation at the Table 7 shape (32,
    16 and 8 workgroups per tile) gives the stream-ordered schedule's words
    on 300 gates (10 tiles, a ragged last one: one or two per XCD, so with
    teams of 32 one team runs two tiles), with key switching fused; sampled
    gates equal the oracle's and every gate decrypts."""
    K, ctx = helpers.gpu_world("C2")
    types, m1, m2, c1, c2 = _workload(K, 300, 77)
    per = _gates(torch_cuda, ctx, types, c1, c2, PERSISTENT, rows=rows)
    strm = _gates(torch_cuda, ctx, types, c1, c2, STREAM)
    assert np.array_equal(per, strm)
    idx = [0, 299]
    assert np.array_equal(per[idx], helpers.oracle_gates("C2", types, c1, c2, idx))
    want = [mi.plain_gate(int(t), int(a), int(b)) for t, a, b in zip(types, m1, m2)]
    assert tfhe.decrypt(K, per).tolist() == want


@pytest.mark.parametrize("cnt", [1100, 1280, 1344])
def test_ragged_wide_batch_split(torch_cuda, cnt):
    """The automatic schedule on batches just over one full round of teams
    (32 tiles at the Table 7 shape): 1100 and 1280 gates run 1024 gates on
    teams of 8, then the remainder as a second launch (76 gates on the
    stream-ordered kernels, 256 gates on teams of 32); 1344 gates (10 tiles
    over) stay in one launch.  Every word equals the stream-ordered
    schedule's for the whole batch, and every gate decrypts."""
    K, ctx = helpers.gpu_world("C2")
    types, m1, m2, c1, c2 = _workload(K, cnt, 91)
    auto = _gates(torch_cuda, ctx, types, c1, c2, -1)
    strm = _gates(torch_cuda, ctx, types, c1, c2, STREAM)
    assert np.array_equal(auto, strm)
    want = [mi.plain_gate(int(t), int(a), int(b)) for t, a, b in zip(types, m1, m2)]
    assert tfhe.decrypt(K, auto).tolist() == want


@pytest.mark.parametrize("rows", [2, 4])
def test_narrow_teams_partial_rotation(torch_cuda, rows):
    """Teams of 32 and 16 workgroups over 1061 gates (34 tiles: a team runs
    up to five tiles phase by phase) for 600 CMux steps, across the party
    boundary: the same words as the stream-ordered schedule."""
    K, ctx = helpers.gpu_world("C2")
    P = K.params
    abar = np.random.default_rng(rows).integers(0, 2 * P.N, (1061, P.lwe_words)).astype(np.uint32)
    per = _rotate(torch_cuda, ctx, abar, 600, PERSISTENT, rows=rows)
    strm = _rotate(torch_cuda, ctx, abar, 600, STREAM)
    assert np.array_equal(per, strm)


@pytest.mark.parametrize("name,cnt,steps", [("C2", 200, 600), ("C2", 1061, 40), ("C3", 97, 600),
                                            ("C8", 40, 1200)])
def test_partial_rotation_matches_stream(torch_cuda, name, cnt, steps):
    """Partial blind rotations that cross party boundaries (live slots grow
    from 2 to k + 1): the persistent and the stream-ordered schedules give
    the same words, and sampled gates equal the oracle's.  1061 gates leave
    a ragged last tile and more tiles than the XCDs divide evenly."""
    K, ctx = helpers.gpu_world(name)
    P = K.params
    abar = np.random.default_rng(cnt + steps).integers(0, 2 * P.N, (cnt, P.lwe_words)).astype(np.uint32)
    abar[0, :] = 0                      # every step skipped
    abar[1, ::3] = 0
    per = _rotate(torch_cuda, ctx, abar, steps, PERSISTENT)
    strm = _rotate(torch_cuda, ctx, abar, steps, STREAM)
    assert np.array_equal(per, strm)
    idx = [0, 1, cnt - 1]
    ref = helpers.oracle_rotations(name, abar[idx], steps)
    assert np.array_equal(per[idx], ref.reshape(len(idx), -1))


def test_batch_sizes_around_the_team_grid(torch_cuda):
    """Gate counts around multiples of the tile (32 gates) and of the XCD
    count: persistent and stream-ordered outputs are identical and decrypt."""
    K, ctx = helpers.gpu_world("C1B")
    types, m1, m2, c1, c2 = _workload(K, 1100, 90)
    want = np.array([mi.plain_gate(int(t), int(a), int(b)) for t, a, b in zip(types, m1, m2)])
    for cnt in (31, 33, 255, 257, 1100):
        a = _gates(torch_cuda, ctx, types[:cnt], c1[:cnt], c2[:cnt], PERSISTENT)
        b = _gates(torch_cuda, ctx, types[:cnt], c1[:cnt], c2[:cnt], STREAM)
        assert np.array_equal(a, b), cnt
        assert np.array_equal(tfhe.decrypt(K, a), want[:cnt]), cnt


def test_status_reports_bad_gate_types(torch_cuda):
    """A gate type outside NAND..XNOR is evaluated as NAND and flagged in the
    device status word; reading the status clears it."""
    K, ctx = helpers.gpu_world("C1")
    types, m1, m2, c1, c2 = _workload(K, 4, 70)
    types = np.array([mi.NAND, 9, mi.AND, mi.XOR], np.uint8)
    d = torch_cuda.device("cuda:0")
    out = torch_cuda.full((4, c1.shape[1]), -1, dtype=torch_cuda.int32, device=d)
    ctx.bootstrap_gate(torch_cuda.from_numpy(types).to(d), torch_cuda.from_numpy(c1.view(np.int32)).to(d),
                       torch_cuda.from_numpy(c2.view(np.int32)).to(d), out, path=1)
    with pytest.raises(MkError):
        ctx.device_status()
    ctx.device_status()                 # cleared by the read
    got = out.cpu().numpy().view(np.uint32)
    as_nand = types.copy()
    as_nand[1] = mi.NAND
    assert np.array_equal(got, helpers.oracle_gates("C1", as_nand, c1, c2))
