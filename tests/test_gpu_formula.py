"""Closed-form regression (§3.4 Eqs. (2)-(3), Alg. 7) at the Table 7 shape:
one data set of m = 2 pairs (x, y 8-bit, pair i encrypted by party i) and
its 4 093-level netlist, run as four consecutive level ranges, one test item
each, so that each item ends well inside a minute (the whole netlist is
about 150 s of narrow levels).  In every range one (gate, instance) item per
level (ranges deeper than 64 levels: a seeded stride) is recomputed by the
oracle from the GPU's own inputs; the last item decrypts the slope and the
intercept against the integer definition (needs an MI355X)."""
import numpy as np
import pytest

import mk_inputs as mi
from oracle import lr
from oracle import tfhe
from tests import helpers

pytestmark = pytest.mark.gpu

PARTS = 4
M, SETS = 2, 2
_STATE = {}


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def _setup():
    if "parts" in _STATE:
        return
    import paper_2205_05825_amd as mk
    K, ctx = helpers.gpu_world("C2")
    x, y, _, _ = mi.formula_lr_data(SETS, M, seed=23)
    circ = mk.build_lr_formula(M)
    bits = lr.formula_input_bits(x, y)
    owner = lr.formula_input_owner(M, 2)
    in_ct = np.stack([tfhe.encrypt(K, int(owner[i]), bits[i], seed=1700 + i) for i in range(len(bits))])
    _STATE.update(K=K, ctx=ctx, x=x, y=y, circ=circ, parts=helpers.split_by_levels(circ, PARTS),
                  wires={int(w): in_ct[i] for i, w in enumerate(circ.inputs)}, done=-1)


def _run_part(torch, k):
    _setup()
    while _STATE["done"] < k - 1:            # a part run on its own first runs the earlier ones
        _run_part(torch, _STATE["done"] + 1)
    if _STATE["done"] >= k:
        return
    ctx, part, wires = _STATE["ctx"], _STATE["parts"][k], _STATE["wires"]
    in_ct = np.stack([wires[int(w)] for w in part.inputs])
    d = torch.device("cuda:0")

    def evaluate(c):
        inp = torch.from_numpy(np.ascontiguousarray(in_ct).view(np.int32)).to(d)
        out = torch.zeros((len(c.outputs), SETS, in_ct.shape[2]), dtype=torch.int32, device=d)
        ctx.eval_circuit(c, inp, out)
        torch.cuda.synchronize()
        return out.cpu().numpy().view(np.uint32)

    outs, picks = helpers.sampled_level_parity("C2", part, in_ct, evaluate, seed=90 + k, check_unmodified=False)
    for i, w in enumerate(part.outputs):
        wires[int(w)] = outs[i]
    _STATE["done"] = k
    return picks


@pytest.mark.parametrize("k", range(PARTS))
def test_formula_part(torch_cuda, k):
    _run_part(torch_cuda, k)
    if k == PARTS - 1:
        K, circ, wires = _STATE["K"], _STATE["circ"], _STATE["wires"]
        P = K.params

        def ct(w):
            w = int(w)
            return wires[w] if w > 1 else np.stack([tfhe.trivial(P, [w])[0]] * SETS)

        dec = np.stack([tfhe.decrypt(K, ct(w)) for w in circ.outputs])
        got = list(zip(mi.from_bits(dec[:16].T).tolist(), mi.from_bits(dec[16:].T).tolist()))
        assert got == [lr.formula_replica(a, b) for a, b in zip(_STATE["x"], _STATE["y"])]
