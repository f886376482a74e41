"""MI355X-native multi-key TFHE gate bootstrapping (binding of libmktfhe.so).

The library behind this package implements the bootstrapped gates of §4.1 and
the k-bit operators of §4.3-§4.5 of Jiang et al., "Privacy-Preserving
Distributed Machine Learning Made Faster", as hand-written HIP kernels for
gfx950.  Import fails if the HIP library has not been built (no fallback).
"""
from ._lib import (AND, NAND, NOR, NOT, OR, PATH_I32, PATH_MFMA_I8, XNOR, XOR,  # noqa: F401
                   Circuit, Context, Graph, MkError, Params, build_operator, build_lr_step,
                   build_lr_formula, build_naive_gate, circuit_stats, circuit_slots, EXPORTED, LIB_PATH, OP_ADD, OP_SUB, OP_MUL, OP_DIV, OP_DIV2,
                   ROT_AUTO, ROT_STREAM, ROT_PERSISTENT)
