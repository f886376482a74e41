"""Host-side checks of the C-ABI library (CPU only, no GPU calls):
exported symbols, keygen/encryption parity with the oracle, serialisation
and error codes."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import params as OP
from oracle import tfhe
from tests import helpers

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "mk_tfhe.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mk_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    import paper_2205_05825_amd as mk
    lib = ctypes.CDLL(mk.LIB_PATH)
    declared = _declared_symbols()
    assert len(declared) >= 16
    for name in declared:
        assert hasattr(lib, name), name
    assert set(declared) == set(mk.EXPORTED)


@pytest.mark.parametrize("name", ["C1", "TOY"])
def test_keygen_bytes_match_oracle(name):
    helpers.assert_same_keys(name)


@pytest.mark.slow
def test_keygen_bytes_match_oracle_c2():
    helpers.assert_same_keys("C2")


def test_encrypt_matches_oracle_and_decrypts():
    K = helpers.oracle_keys("C1")
    ctx = helpers.lib_context("C1")
    rng = np.random.default_rng(0)
    bits = rng.integers(0, 2, 100).astype(np.uint8)
    for party in range(OP.C1.k):
        got = ctx.encrypt(party, bits, seed=1000 + party)
        ref = tfhe.encrypt(K, party, bits, seed=1000 + party)
        assert np.array_equal(got, ref)
        assert np.array_equal(ctx.decrypt(got), bits)
        assert np.array_equal(tfhe.decrypt(K, got), bits)
    # padded stride: extra words are zero, the rest identical
    got = ctx.encrypt(1, bits[:5], seed=3, stride=OP.C1.lwe_words + 7)
    ref = tfhe.encrypt(K, 1, bits[:5], seed=3)
    assert np.array_equal(got[:, :OP.C1.lwe_words], ref) and not got[:, OP.C1.lwe_words:].any()
    assert np.array_equal(ctx.decrypt(got), bits[:5])


def test_trivial_matches_oracle():
    ctx = helpers.lib_context("C1")
    bits = np.array([0, 1, 1], np.uint8)
    assert np.array_equal(ctx.trivial(bits), tfhe.trivial(OP.C1, bits))


def test_export_import_roundtrip():
    import paper_2205_05825_amd as mk
    src = helpers.lib_context("TOY")
    dst = mk.Context(helpers.lib_params(OP.TOY), 12345)
    for p in range(-1, OP.TOY.k):
        dst.import_keys(p, src.export_keys(p))
        assert dst.export_keys(p) == src.export_keys(p)
    c = src.encrypt(0, [1, 0, 1], seed=4)
    assert dst.decrypt(c).tolist() == [1, 0, 1]


def test_error_codes():
    import paper_2205_05825_amd as mk
    bad = mk.Params(k=2, n=64, N=100, bk_ell=2, ks_t=6, bk_noise_log2=20,
                    ks_noise_log2=20, lwe_noise_log2=12)
    with pytest.raises(mk.MkError) as e:
        mk.Context(bad, 0)
    assert e.value.code == -5
    b9 = mk.Params(k=2, n=560, N=1024, bk_ell=3, ks_t=8, bk_noise_log2=30,
                   ks_noise_log2=15, lwe_noise_log2=15, bk_log_base=9)
    with pytest.raises(mk.MkError) as e:        # Table 7's B = 2^9: digits not int8
        mk.Context(b9, 0)
    assert e.value.code == -5
    ctx = mk.Context(helpers.lib_params(OP.TOY), 1)
    with pytest.raises(mk.MkError) as e:
        ctx.keygen(5, 0)
    assert e.value.code == -1
    with pytest.raises(mk.MkError) as e:
        ctx.encrypt(0, [1], seed=0)
    assert e.value.code == -4
    with pytest.raises(mk.MkError) as e:
        ctx.import_keys(0, b"\0" * 10)
    assert e.value.code == -1
    with pytest.raises(mk.MkError) as e:        # no keys: upload refused on the host
        ctx.upload(stream=0)
    assert e.value.code == -4


def test_tile_shape_arguments():
    import paper_2205_05825_amd as mk
    ctx = mk.Context(helpers.lib_params(OP.C1), 3)
    assert ctx.get_tiles(1000) == (0, 3)
    # untuned small batches take the K-split and skewed shapes
    assert ctx.get_tiles(20) == (6, 6) and ctx.get_tiles(100) == (5, 6) and ctx.get_tiles(300) == (3, 5)
    ctx.set_tiles(2, 1)
    assert ctx.get_tiles(1000) == (2, 1)
    ctx.set_tiles(-1, -1)
    assert ctx.get_tiles(1000) == (0, 3)
    with pytest.raises(mk.MkError):
        ctx.set_tiles(8, 0)
    assert ctx.get_split(1000) == 1
    ctx.set_split(1000, 2)
    assert ctx.get_split(1000) == 2 and ctx.get_split(1024) == 2 and ctx.get_split(900) == 1
    ctx.set_split(1000, 0)
    assert ctx.get_split(1000) == 1
    assert ctx.get_split(20) == 1
    for bad in (-1, 3):
        with pytest.raises(mk.MkError):
            ctx.set_split(1000, bad)
    small = mk.Context(helpers.lib_params(OP.C1S), 3)   # N/32 = 4: 256-row shapes refused
    assert small.get_tiles(1000) == (1, 3)
    with pytest.raises(mk.MkError):
        small.set_tiles(0, 1)
    with pytest.raises(mk.MkError):
        small.set_tiles(1, 4)
    with pytest.raises(mk.MkError) as e:      # needs the uploaded key
        ctx.autotune(64, stream=0)
    assert e.value.code == -4


def test_schedule_switch_arguments():
    """Rotation schedule and key-switch fusion setters take their documented
    values only (host checks, no device work)."""
    import paper_2205_05825_amd as mk
    ctx = mk.Context(helpers.lib_params(OP.C1), 3)
    for kind in (mk.ROT_AUTO, mk.ROT_STREAM, mk.ROT_PERSISTENT):
        ctx.set_rotation(kind)
    for on in (False, True):
        ctx.set_ks_fusion(on)
    for bad in (-2, 2):
        with pytest.raises(mk.MkError) as e:
            ctx.set_rotation(bad)
        assert e.value.code == -1
    from paper_2205_05825_amd import _lib
    assert _lib._L.mk_set_ks_fusion(ctx._h, 2) == -1
    assert _lib._L.mk_set_ks_fusion(None, 1) == -1
    big = mk.Context(helpers.lib_params(OP.C2), 3)          # N = 1024: three team sizes
    for rows in (2, 4, 8, 0):
        big.set_team_rows(rows)
        assert big.get_team_rows(4096) == 0                 # no XCDs probed: stream-ordered
    for bad in (1, 3, 16, -1):
        with pytest.raises(mk.MkError):
            big.set_team_rows(bad)
    with pytest.raises(mk.MkError):                         # fixed size at N = 256
        ctx.set_team_rows(4)
    ctx.set_team_rows(0)
    assert ctx.get_team_rows(1000) == 0


def test_builder_and_parameter_limits():
    """Argument checks on the host: netlist builder ranges, the party limit,
    and the int8 exactness bound (k+1)*ell*N*2^14 < 2^31, which the
    eight-party set meets and a doubled ring at eight parties does not."""
    import paper_2205_05825_amd as mk
    from paper_2205_05825_amd import _lib
    n_g, n_w = ctypes.c_int32(), ctypes.c_int32()
    for m, frac in ((0, 8), (4097, 8), (4, -1), (4, 16)):
        assert _lib._L.mk_build_lr_formula(m, frac, None, ctypes.byref(n_g), ctypes.byref(n_w), None, None) == -1
    for t in (-1, 7):
        assert _lib._L.mk_build_naive_gate(t, None, ctypes.byref(n_g), ctypes.byref(n_w), None, None) == -1
    assert _lib._L.mk_build_lr_formula(4, 8, None, None, None, None, None) == -1
    mk.Context(helpers.lib_params(OP.C8), 1).close()
    fields = {f: getattr(OP.C8, f) for f in helpers.FIELDS}
    for change in ({"k": 9}, {"N": 8192}):
        with pytest.raises(mk.MkError) as e:
            mk.Context(mk.Params(**{**fields, **change}), 1)
        assert e.value.code == -5, change


def test_import_fails_loudly_without_the_library(tmp_path):
    """A copy of the package without libmktfhe.so refuses to import (there is
    no fallback implementation to run instead)."""
    import shutil
    import subprocess
    import sys
    src = os.path.join(ROOT, "paper_2205_05825_amd")
    dst = tmp_path / "paper_2205_05825_amd"
    dst.mkdir()
    for f in os.listdir(src):
        if f.endswith(".py"):
            shutil.copy(os.path.join(src, f), dst / f)
    r = subprocess.run([sys.executable, "-c", "import paper_2205_05825_amd"], cwd=tmp_path,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "ImportError" in r.stderr and "libmktfhe.so is not built" in r.stderr


def test_bench_refuses_more_than_one_gpu():
    """The path is per GPU: bench.py --gpus 2 exits with status 2 and says so."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2 and "one GPU" in r.stderr and not r.stdout
