"""ctypes binding of libmktfhe.so (the C ABI declared in include/mk_tfhe.h).

Argument marshalling only: every step of the bootstrapping runs inside the
library's HIP kernels.  Device buffers are torch tensors on the current
HIP device (``tensor.data_ptr()``); host buffers are numpy arrays.  If the
library has not been built, importing this module raises ImportError: there
is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmktfhe.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        "libmktfhe.so is not built; run `python -m paper_2205_05825_amd.build` "
        "(hipcc, gfx950) first")

# torch first: its streams and device pointers are handed to the library,
# so both must run on one HIP runtime.  torch loads its own copy of the
# runtime library, which then also satisfies this library's dependency (same
# soname); loading this library first would bind a second runtime.
import torch  # noqa: E402,F401

_L = ctypes.CDLL(LIB_PATH)

MK_OK, MK_EINVAL, MK_ENOMEM, MK_EDEVICE, MK_ESTATE, MK_EPARAM = 0, -1, -2, -3, -4, -5
PATH_I32, PATH_MFMA_I8 = 0, 1
ROT_AUTO, ROT_STREAM, ROT_PERSISTENT = -1, 0, 1
TILE_SHAPES = 8
NAND, AND, OR, NOR, XOR, XNOR, NOT = 0, 1, 2, 3, 4, 5, 6


class MkParams(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int32) for name in (
        "k", "n", "N", "bk_log_base", "bk_ell", "ks_log_base", "ks_t",
        "bk_noise_log2", "ks_noise_log2", "lwe_noise_log2")]


class MkGate(ctypes.Structure):
    _fields_ = [("type", ctypes.c_int32), ("in1", ctypes.c_int32),
                ("in2", ctypes.c_int32), ("out", ctypes.c_int32)]


class MkCircuit(ctypes.Structure):
    _fields_ = [("n_wires", ctypes.c_int32),
                ("n_inputs", ctypes.c_int32), ("inputs", ctypes.POINTER(ctypes.c_int32)),
                ("n_outputs", ctypes.c_int32), ("outputs", ctypes.POINTER(ctypes.c_int32)),
                ("n_gates", ctypes.c_int32), ("gates", ctypes.POINTER(MkGate))]


_vp, _sz, _i, _u64 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_uint64
_SIGS = {
    "mk_setup": ([ctypes.POINTER(MkParams), _u64, ctypes.POINTER(_vp)], _i),
    "mk_keygen": ([_vp, _i, _u64], _i),
    "mk_export_keys": ([_vp, _i, _vp, ctypes.POINTER(_sz)], _i),
    "mk_import_keys": ([_vp, _i, _vp, _sz], _i),
    "mk_upload_eval_key": ([_vp, _vp], _i),
    "mk_encrypt": ([_vp, _i, _vp, _sz, _u64, _vp, _sz], _i),
    "mk_decrypt": ([_vp, _vp, _sz, _sz, _vp], _i),
    "mk_trivial": ([_vp, _vp, _sz, _vp, _sz], _i),
    "mk_not": ([_vp, _vp, _vp, _sz, _sz, _vp], _i),
    "mk_bootstrap_gate": ([_vp, _vp, _vp, _vp, _vp, _sz, _sz, _i, _vp], _i),
    "mk_bootstrap_gate_noalloc": ([_vp, _vp, _vp, _vp, _vp, _sz, _sz, _i, _vp], _i),
    "mk_eval_circuit": ([_vp, ctypes.POINTER(MkCircuit), _vp, _vp, _sz, _sz, _i, _vp], _i),
    "mk_circuit_graph_create": ([_vp, ctypes.POINTER(MkCircuit), _vp, _vp, _sz, _sz, _i,
                                 ctypes.POINTER(_vp)], _i),
    "mk_graph_launch": ([_vp, _vp], _i),
    "mk_graph_info": ([_vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64),
                       ctypes.POINTER(ctypes.c_int32)], _i),
    "mk_graph_destroy": ([_vp], _i),
    "mk_blind_rotate": ([_vp, _vp, _vp, _sz, _i, _i, _vp], _i),
    "mk_extract_keyswitch": ([_vp, _vp, _vp, _sz, _sz, _i, _vp], _i),
    "mk_build_operator": ([_i, _i, ctypes.POINTER(MkGate), ctypes.POINTER(ctypes.c_int32),
                           ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                           ctypes.POINTER(ctypes.c_int32)], _i),
    "mk_build_naive_gate": ([_i, ctypes.POINTER(MkGate), ctypes.POINTER(ctypes.c_int32),
                             ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                             ctypes.POINTER(ctypes.c_int32)], _i),
    "mk_build_lr_step": ([_i, _i, _i, ctypes.POINTER(MkGate), ctypes.POINTER(ctypes.c_int32),
                          ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                          ctypes.POINTER(ctypes.c_int32)], _i),
    "mk_build_lr_formula": ([_i, _i, ctypes.POINTER(MkGate), ctypes.POINTER(ctypes.c_int32),
                             ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                             ctypes.POINTER(ctypes.c_int32)], _i),
    "mk_circuit_stats": ([ctypes.POINTER(MkCircuit), ctypes.POINTER(ctypes.c_int32),
                          ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32),
                          ctypes.POINTER(ctypes.c_int32)], _i),
    "mk_circuit_slots": ([ctypes.POINTER(MkCircuit), ctypes.POINTER(ctypes.c_int32),
                          ctypes.POINTER(ctypes.c_int32)], _i),
    "mk_set_graph_piece": ([_vp, _i], _i),
    "mk_set_split": ([_vp, _sz, _i], _i),
    "mk_get_split": ([_vp, _sz, ctypes.POINTER(ctypes.c_int32)], _i),
    "mk_autotune": ([_vp, _sz, _vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                     ctypes.POINTER(ctypes.c_float)], _i),
    "mk_set_tiles": ([_vp, _i, _i], _i),
    "mk_get_tiles": ([_vp, _sz, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)], _i),
    "mk_set_rotation": ([_vp, _i], _i),
    "mk_set_ks_fusion": ([_vp, _i], _i),
    "mk_set_team_rows": ([_vp, _i], _i),
    "mk_get_team_rows": ([_vp, _sz, ctypes.POINTER(ctypes.c_int32)], _i),
    "mk_device_status": ([_vp, _vp], _i),
    "mk_set_profiling": ([_vp, _i], _i),
    "mk_get_profile": ([_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64), _i], _i),
    "mk_last_error": ([], ctypes.c_char_p),
    "mk_free": ([_vp], None),
}
for _name, (_args, _res) in _SIGS.items():
    _f = getattr(_L, _name)
    _f.argtypes = _args
    _f.restype = _res

EXPORTED = tuple(_SIGS)


class MkError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (code %d)" % (msg, code))
        self.code = code


def _check(rc):
    if rc != MK_OK:
        raise MkError(rc, _L.mk_last_error().decode())


def _stream(stream):
    """hipStream_t handle of a torch stream (current stream if None)."""
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


_WORD_DTYPES = None


def _dev(t, name, ndim, dtypes=None):
    """Checks that `t` is a contiguous tensor of rank `ndim` with 32-bit
    words (or one of `dtypes`); where it lives is checked by _on_device once
    all shapes are known.  A wrong element size, rank or a non-contiguous
    view would make the kernels read or write out of bounds."""
    global _WORD_DTYPES
    if _WORD_DTYPES is None:
        _WORD_DTYPES = tuple(d for d in (torch.int32, getattr(torch, "uint32", None)) if d is not None)
    if not isinstance(t, torch.Tensor):
        raise ValueError("%s: expected a torch tensor, got %s" % (name, type(t).__name__))
    if t.dtype not in (dtypes or _WORD_DTYPES):
        raise ValueError("%s: dtype %s not accepted" % (name, t.dtype))
    if t.dim() != ndim:
        raise ValueError("%s: expected %d dimensions, got shape %s" % (name, ndim, tuple(t.shape)))
    if not t.is_contiguous():
        raise ValueError("%s: tensor must be contiguous" % name)
    return t


def _on_device(**tensors):
    """Every tensor is on the current HIP device (the library's device)."""
    for name, t in tensors.items():
        if not t.is_cuda:
            raise ValueError("%s: expected a device tensor, got one on %s" % (name, t.device))
        if t.device.index != torch.cuda.current_device():
            raise ValueError("%s: tensor is on %s, the current device is cuda:%d"
                             % (name, t.device, torch.cuda.current_device()))


def _same(name, got, want):
    if tuple(got) != tuple(want):
        raise ValueError("%s: expected shape %s, got %s" % (name, tuple(want), tuple(got)))


def _host(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data_as(ctypes.c_void_p)


@dataclass(frozen=True)
class Params:
    k: int
    n: int
    N: int
    bk_ell: int
    ks_t: int
    bk_noise_log2: int
    ks_noise_log2: int
    lwe_noise_log2: int
    bk_log_base: int = 8
    ks_log_base: int = 2

    def c(self) -> MkParams:
        return MkParams(self.k, self.n, self.N, self.bk_log_base, self.bk_ell,
                        self.ks_log_base, self.ks_t, self.bk_noise_log2,
                        self.ks_noise_log2, self.lwe_noise_log2)

    @property
    def lwe_words(self):
        return self.k * self.n + 1


class Context:
    """Owns an mk_ctx: keys on the host and the evaluation key on the GPU."""

    def __init__(self, params: Params, crs_seed: int):
        self.params = params
        h = ctypes.c_void_p()
        _check(_L.mk_setup(ctypes.byref(params.c()), crs_seed, ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            _L.mk_free(self._h)
            self._h = None

    def __del__(self):
        self.close()

    # ---- host ----
    def keygen(self, party: int, seed: int):
        _check(_L.mk_keygen(self._h, party, seed))

    def export_keys(self, party: int) -> bytes:
        n = ctypes.c_size_t(0)
        _check(_L.mk_export_keys(self._h, party, None, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        _check(_L.mk_export_keys(self._h, party, buf, ctypes.byref(n)))
        return buf.raw

    def import_keys(self, party: int, data: bytes):
        buf = ctypes.create_string_buffer(bytes(data), len(data))
        _check(_L.mk_import_keys(self._h, party, buf, len(data)))

    def upload(self, stream=None):
        _check(_L.mk_upload_eval_key(self._h, _stream(stream)))

    def encrypt(self, party: int, bits, seed: int, stride: int | None = None) -> np.ndarray:
        b, bp = _host(bits, np.uint8)
        stride = stride or self.params.lwe_words
        out = np.zeros((b.shape[0], stride), np.uint32)
        _check(_L.mk_encrypt(self._h, party, bp, b.shape[0], seed,
                             out.ctypes.data_as(ctypes.c_void_p), stride))
        return out

    def decrypt(self, ct) -> np.ndarray:
        c, cp = _host(ct, np.uint32)
        c = c.reshape(-1, c.shape[-1])
        out = np.zeros(c.shape[0], np.uint8)
        _check(_L.mk_decrypt(self._h, c.ctypes.data_as(ctypes.c_void_p), c.shape[0],
                             c.shape[1], out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def trivial(self, bits, stride: int | None = None) -> np.ndarray:
        b, bp = _host(bits, np.uint8)
        stride = stride or self.params.lwe_words
        out = np.zeros((b.shape[0], stride), np.uint32)
        _check(_L.mk_trivial(self._h, bp, b.shape[0], out.ctypes.data_as(ctypes.c_void_p), stride))
        return out

    # ---- tile shapes of the MFMA rotation ----
    def autotune(self, count: int, stream=None):
        """Times every GEMM tile shape for batches of `count` gates, keeps the
        fastest; returns (gemm1 shape, gemm2 shape, ms[2 * TILE_SHAPES])."""
        v1, v2 = ctypes.c_int32(), ctypes.c_int32()
        ms = (ctypes.c_float * (2 * TILE_SHAPES))()
        _check(_L.mk_autotune(self._h, count, _stream(stream), ctypes.byref(v1), ctypes.byref(v2), ms))
        return v1.value, v2.value, list(ms)

    def set_tiles(self, gemm1_shape: int = -1, gemm2_shape: int = -1):
        _check(_L.mk_set_tiles(self._h, gemm1_shape, gemm2_shape))

    def set_split(self, count: int, parts: int):
        _check(_L.mk_set_split(self._h, count, parts))

    def get_split(self, count: int) -> int:
        p = ctypes.c_int32()
        _check(_L.mk_get_split(self._h, count, ctypes.byref(p)))
        return p.value

    def get_tiles(self, count: int):
        v1, v2 = ctypes.c_int32(), ctypes.c_int32()
        _check(_L.mk_get_tiles(self._h, count, ctypes.byref(v1), ctypes.byref(v2)))
        return v1.value, v2.value

    def set_graph_piece(self, kernels: int = 1024):
        _check(_L.mk_set_graph_piece(self._h, int(kernels)))

    def set_rotation(self, kind: int = ROT_AUTO):
        """Schedule of the MFMA rotation: ROT_STREAM (four kernels per CMux
        step), ROT_PERSISTENT (one launch per rotation) or ROT_AUTO."""
        _check(_L.mk_set_rotation(self._h, int(kind)))

    def set_ks_fusion(self, on: bool = True):
        """Extraction and key switching inside the persistent rotation's
        launch (True, default) or as separate kernels after it (False)."""
        _check(_L.mk_set_ks_fusion(self._h, int(bool(on))))

    def set_team_rows(self, rows: int = 0):
        """Row tiles per task of the persistent rotation at N = 1024 (2, 4 or
        8; 0 = chosen by batch width)."""
        _check(_L.mk_set_team_rows(self._h, int(rows)))

    def get_team_rows(self, count: int) -> int:
        r = ctypes.c_int32()
        _check(_L.mk_get_team_rows(self._h, int(count), ctypes.byref(r)))
        return r.value

    def device_status(self, stream=None):
        """Waits for the stream; raises MkError if a persistent rotation gave
        up waiting (its outputs are then invalid)."""
        _check(_L.mk_device_status(self._h, _stream(stream)))

    # ---- profiling ----
    def set_profiling(self, level: int):
        """0 off, 1 pipeline stages, 2 stages and each MFMA-rotation kernel."""
        _check(_L.mk_set_profiling(self._h, int(level)))

    def get_profile(self, reset: bool = False):
        """(ms[8], launches[8]): precombine, rotation, keyswitch, circuit,
        MFMA gemm1, MFMA gemm2, rotate+decompose, w decompose."""
        ms = (ctypes.c_double * 8)()
        ln = (ctypes.c_int64 * 8)()
        _check(_L.mk_get_profile(self._h, ms, ln, int(bool(reset))))
        return list(ms), list(ln)

    # ---- device (torch tensors; shapes checked before any call) ----
    def _rows(self, t, name):
        """[count, stride] ciphertext rows, stride >= kn+1."""
        _dev(t, name, 2)
        if t.shape[1] < self.params.lwe_words:
            raise ValueError("%s: row stride %d < kn+1 = %d" % (name, t.shape[1], self.params.lwe_words))
        return t

    def lwe_not(self, inp, out, stream=None):
        self._rows(inp, "inp")
        _same("out", self._rows(out, "out").shape, inp.shape)
        _on_device(inp=inp, out=out)
        _check(_L.mk_not(self._h, _ptr(inp), _ptr(out), inp.shape[0], inp.shape[1],
                         _stream(stream)))

    def bootstrap_gate(self, types, in1, in2, out, path=PATH_MFMA_I8, stream=None, noalloc=False):
        """Bootstrapped gates out[g] = types[g](in1[g], in2[g]); with
        `noalloc` through mk_bootstrap_gate_noalloc (fixed scratch block)."""
        self._rows(in1, "in1")
        _same("in2", self._rows(in2, "in2").shape, in1.shape)
        _same("out", self._rows(out, "out").shape, in1.shape)
        _same("types", _dev(types, "types", 1, (torch.uint8,)).shape, (in1.shape[0],))
        _on_device(types=types, in1=in1, in2=in2, out=out)
        fn = _L.mk_bootstrap_gate_noalloc if noalloc else _L.mk_bootstrap_gate
        _check(fn(self._h, _ptr(types), _ptr(in1), _ptr(in2), _ptr(out), in1.shape[0], in1.shape[1], path,
                  _stream(stream)))

    def blind_rotate(self, abar, acc, max_steps=-1, path=PATH_MFMA_I8, stream=None):
        P = self.params
        _dev(abar, "abar", 2)
        _same("abar", abar.shape, (abar.shape[0], P.lwe_words))
        _same("acc", _dev(acc, "acc", 2).shape, (abar.shape[0], (P.k + 1) * P.N))
        _on_device(abar=abar, acc=acc)
        _check(_L.mk_blind_rotate(self._h, _ptr(abar), _ptr(acc), abar.shape[0], max_steps,
                                  path, _stream(stream)))

    def extract_keyswitch(self, acc, out, path=PATH_MFMA_I8, stream=None):
        P = self.params
        _dev(acc, "acc", 2)
        _same("acc", acc.shape, (acc.shape[0], (P.k + 1) * P.N))
        _same("out rows", self._rows(out, "out").shape[:1], acc.shape[:1])
        _on_device(acc=acc, out=out)
        _check(_L.mk_extract_keyswitch(self._h, _ptr(acc), _ptr(out), acc.shape[0],
                                       out.shape[1], path, _stream(stream)))

    def _circuit_io(self, circuit, inp, out):
        _dev(inp, "inp", 3)
        _dev(out, "out", 3)
        if inp.shape[2] < self.params.lwe_words:
            raise ValueError("inp: row stride %d < kn+1 = %d" % (inp.shape[2], self.params.lwe_words))
        _same("inp", inp.shape, (len(circuit.inputs), inp.shape[1], inp.shape[2]))
        _same("out", out.shape, (len(circuit.outputs), inp.shape[1], inp.shape[2]))
        _on_device(inp=inp, out=out)

    def circuit_graph(self, circuit: "Circuit", inp, out, path=PATH_MFMA_I8) -> "Graph":
        return Graph(self, circuit, inp, out, path)

    def eval_circuit(self, circuit: "Circuit", inp, out, path=PATH_MFMA_I8, stream=None):
        self._circuit_io(circuit, inp, out)
        batch = inp.shape[1]
        _check(_L.mk_eval_circuit(self._h, ctypes.byref(circuit.c()), _ptr(inp), _ptr(out),
                                  batch, inp.shape[2], path, _stream(stream)))


class Graph:
    """A circuit evaluation captured as a HIP graph on fixed buffers (see
    mk_circuit_graph_create); launch() replays it on the current inputs."""

    def __init__(self, ctx: "Context", circuit: "Circuit", inp, out, path=PATH_MFMA_I8):
        ctx._circuit_io(circuit, inp, out)
        self._ctx = ctx                      # keeps the context alive
        self._bufs = (inp, out)              # the graph reads/writes these
        self._c = circuit.c()
        h = ctypes.c_void_p()
        _check(_L.mk_circuit_graph_create(ctx._h, ctypes.byref(self._c), _ptr(inp), _ptr(out),
                                          inp.shape[1], inp.shape[2], path, ctypes.byref(h)))
        self._h = h

    def launch(self, stream=None):
        _check(_L.mk_graph_launch(self._h, _stream(stream)))

    def info(self):
        """(levels, bootstrapped gates per launch, graph pieces)."""
        lv, g, pc = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int32()
        _check(_L.mk_graph_info(self._h, ctypes.byref(lv), ctypes.byref(g), ctypes.byref(pc)))
        return lv.value, g.value, pc.value

    def close(self):
        if getattr(self, "_h", None):
            _L.mk_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()


@dataclass
class Circuit:
    """A netlist in the layout of mk_circuit (arrays of int32)."""
    n_wires: int
    inputs: np.ndarray
    outputs: np.ndarray
    gates: np.ndarray        # int32[n_gates, 4]: type, in1, in2, out

    def c(self) -> MkCircuit:
        self._keep = (np.ascontiguousarray(self.inputs, np.int32),
                      np.ascontiguousarray(self.outputs, np.int32),
                      np.ascontiguousarray(self.gates, np.int32))
        i, o, g = self._keep
        return MkCircuit(self.n_wires,
                         len(i), i.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                         len(o), o.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                         len(g), g.ctypes.data_as(ctypes.POINTER(MkGate)))


OP_ADD, OP_SUB, OP_MUL, OP_DIV, OP_DIV2 = 0, 1, 2, 3, 4


def _netlist(call, n_in, n_out) -> "Circuit":
    ng, nw = ctypes.c_int32(0), ctypes.c_int32(0)
    P32 = ctypes.POINTER(ctypes.c_int32)
    _check(call(None, ctypes.byref(ng), ctypes.byref(nw), None, None))
    gates = np.zeros((ng.value, 4), np.int32)
    inputs = np.zeros(n_in, np.int32)
    outputs = np.zeros(n_out, np.int32)
    _check(call(gates.ctypes.data_as(ctypes.POINTER(MkGate)), ctypes.byref(ng), ctypes.byref(nw),
                inputs.ctypes.data_as(P32), outputs.ctypes.data_as(P32)))
    return Circuit(nw.value, inputs, outputs, gates)


def build_operator(op: int, kbits: int) -> "Circuit":
    """Netlist of a k-bit operator from the library's builders."""
    n_in = {OP_DIV2: 3 * kbits}.get(op, 2 * kbits)
    n_out = {OP_ADD: kbits, OP_SUB: kbits}.get(op, 2 * kbits)
    return _netlist(lambda *a: _L.mk_build_operator(op, kbits, *a), n_in, n_out)


def build_naive_gate(gate_type: int) -> "Circuit":
    """Gate `gate_type` made of bootstrapped NAND gates only (Table 2's
    comparison design)."""
    return _netlist(lambda *a: _L.mk_build_naive_gate(gate_type, *a), 2, 1)


def build_lr_step(m: int, d: int, shift: int = 12) -> "Circuit":
    """Netlist of one fixed-point gradient-descent step (16-bit values)."""
    return _netlist(lambda *a: _L.mk_build_lr_step(m, d, shift, *a), 16 * (m * d + m + d), 16 * d)


def build_lr_formula(m: int, frac: int = 8) -> "Circuit":
    """Netlist of the closed-form one-feature regression on m pairs of 8-bit
    integers: outputs the slope and the intercept, 16 bits each with `frac`
    fractional bits."""
    return _netlist(lambda *a: _L.mk_build_lr_formula(m, frac, *a), 16 * m, 32)


def circuit_stats(c: "Circuit"):
    """(levels, bootstrapped gates evaluated, widest level, slots per instance)."""
    nl, ng, mw, sl = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
    _check(_L.mk_circuit_stats(ctypes.byref(c.c()), ctypes.byref(nl), ctypes.byref(ng),
                               ctypes.byref(mw), ctypes.byref(sl)))
    return nl.value, ng.value, mw.value, sl.value


def circuit_slots(c: "Circuit"):
    """(slot, level) per wire as int32 arrays: the wire slot that holds each
    ciphertext and its bootstrapping level (-1 for wires with no slot)."""
    slot = np.empty(c.n_wires, np.int32)
    level = np.empty(c.n_wires, np.int32)
    _check(_L.mk_circuit_slots(ctypes.byref(c.c()), slot.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                               level.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
    return slot, level
