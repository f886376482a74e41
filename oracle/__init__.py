"""CPU oracle for multi-key TFHE gate bootstrapping — TEST INFRASTRUCTURE.

This package is the plain, slow, independent reference that the HIP library
is checked against, bit for bit.  It shares no code with the library
(``paper_2205_05825_amd``) and never imports it.  Only ``tests/``,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may
import, call or link anything under ``oracle/``; the product path must not.

Modules
  prng      Philox4x64-10 streams and the integer noise sampler
  params    parameter sets
  tfhe      keys, encryption, gates, bootstrapping (blind rotation, sample
            extraction, key switching)
  circuits  k-bit two's-complement adder/subtractor/multiplier/divider
            netlists, plaintext and encrypted evaluation
  lr        fixed-point gradient-descent linear regression replica
  _native   gcc build of negacyclic.c (the schoolbook polynomial product)
"""
from . import params, prng  # noqa: F401
