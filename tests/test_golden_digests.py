"""The stored oracle digests at the Table 7 shape (tests/golden/
oracle_c2_digests.txt) are the oracle's: a few rows are recomputed here and
must hash to the stored values (CPU only)."""
import numpy as np

from tests import helpers
from tests.golden import make_oracle_digests as G


def test_digest_file_is_complete():
    d = G.load()
    assert sorted(k for k in d if k[0] == "gate") == [("gate", g) for g in range(G.GATES)]
    assert sorted(k for k in d if k[0] == "rot") == [("rot", g) for g in range(G.ROT_GATES)]
    assert all(len(h) == 64 for h in d.values())


def test_digests_match_a_recomputation():
    d = G.load()
    types, c1, c2 = G.workload()
    idx = [0, 517, G.GATES - 1]
    got = helpers.oracle_gates("C2", types, c1, c2, idx)
    for g, row in zip(idx, got):
        assert G.digest(row) == d[("gate", g)], g
    rot = helpers.oracle_rotations("C2", G.rotation_inputs()[[3]])
    assert G.digest(np.asarray(rot[0]).reshape(-1)) == d[("rot", 3)]
