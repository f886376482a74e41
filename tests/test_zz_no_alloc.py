"""mk_bootstrap_gate_noalloc (every scratch buffer in the library's fixed
per-GPU block) against mk_bootstrap_gate, word for word, through the C ABI:
two calls in a row on each path, the second smaller, and a batch beyond the
block refused before any work (needs an MI355X)."""
import numpy as np
import pytest

import mk_inputs as mi
from oracle import tfhe
from paper_2205_05825_amd import MkError
from tests import helpers
from tests.golden.make_oracle_digests import digest, load as golden_digests

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def _run(torch, ctx, types, c1, c2, path, noalloc):
    d = torch.device("cuda:0")
    t = torch.from_numpy(np.ascontiguousarray(types, np.uint8)).to(d)
    a = torch.from_numpy(np.ascontiguousarray(c1).view(np.int32)).to(d)
    b = torch.from_numpy(np.ascontiguousarray(c2).view(np.int32)).to(d)
    out = torch.full_like(a, -1)
    ctx.bootstrap_gate(t, a, b, out, path=path, noalloc=noalloc)
    torch.cuda.synchronize()
    ctx.device_status()
    return out.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("path", [1, 0])
def test_noalloc_matches_bootstrap_gate_c2(torch_cuda, path):
    """1024 gates (the whole Table 7 workload: every word also against the
    oracle's digests), then 100 gates: both equal mk_bootstrap_gate."""
    K, ctx = helpers.gpu_world("C2")
    P = K.params
    types, m1, m2 = mi.gate_batch(1024, seed=2)
    c1 = tfhe.encrypt(K, 0, m1, seed=200)
    c2 = tfhe.encrypt(K, P.k - 1, m2, seed=201)
    got = _run(torch_cuda, ctx, types, c1, c2, path, True)
    dig = golden_digests()
    assert [g for g in range(1024) if digest(got[g]) != dig[("gate", g)]] == []
    assert np.array_equal(got, _run(torch_cuda, ctx, types, c1, c2, path, False))
    sl = slice(300, 400)
    small = _run(torch_cuda, ctx, types[sl], c1[sl], c2[sl], path, True)
    assert np.array_equal(small, _run(torch_cuda, ctx, types[sl], c1[sl], c2[sl], path, False))
    assert np.array_equal(small, got[sl])


def test_noalloc_small_ring_and_refusal(torch_cuda):
    """C1B: 257 gates then 33 gates on the MFMA path equal the allocating
    entry point's; at C2 a batch of 1100 gates needs more than the 64 MiB
    block and is refused with MK_EINVAL, leaving the output untouched."""
    K, ctx = helpers.gpu_world("C1B")
    types, m1, m2 = mi.gate_batch(257, seed=21)
    c1 = tfhe.encrypt(K, 0, m1, seed=210)
    c2 = tfhe.encrypt(K, 1, m2, seed=211)
    for cnt in (257, 33):
        a = _run(torch_cuda, ctx, types[:cnt], c1[:cnt], c2[:cnt], 1, True)
        assert np.array_equal(a, _run(torch_cuda, ctx, types[:cnt], c1[:cnt], c2[:cnt], 1, False)), cnt
    K2, ctx2 = helpers.gpu_world("C2")
    d = torch_cuda.device("cuda:0")
    n = 1100
    t = torch_cuda.zeros(n, dtype=torch_cuda.uint8, device=d)
    x = torch_cuda.zeros((n, K2.params.lwe_words), dtype=torch_cuda.int32, device=d)
    out = torch_cuda.full_like(x, 7)
    with pytest.raises(MkError) as e:
        ctx2.bootstrap_gate(t, x, x, out, path=1, noalloc=True)
    assert e.value.code == -1
    torch_cuda.cuda.synchronize()
    assert bool((out == 7).all())
