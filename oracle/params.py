"""Parameter sets of the multi-key TFHE oracle (test infrastructure only).

Symbols follow the paper's Table 7 (LWE n, alpha, B', d'; RLWE N, beta, B, d)
with the party count k of §3.1.  The gadget base is B = 2^bk_log_base with
bk_ell digits; the key-switching base is B' = 2^ks_log_base with ks_t digits.
Noise levels are given as s with standard deviation 2^-s in torus units.

Readings (the paper prints one parameter set, Table 7, with B = 2^9 and
beta = 3.72e-9): the evaluated sets use B = 2^8 so that gadget digits are
exactly int8, and RLWE key noise 2^-30; LWE noise 2^-15 matches Table 7's
alpha = 3.05e-5.
"""
from __future__ import annotations

from dataclasses import dataclass


@dataclass(frozen=True)
class Params:
    k: int                 # parties
    n: int                 # LWE dimension
    N: int                 # ring dimension (power of two)
    bk_ell: int            # gadget length
    ks_t: int              # key-switching digits
    bk_noise_log2: int     # public key / uni-encryption noise 2^-s
    ks_noise_log2: int     # key-switching key noise 2^-s
    lwe_noise_log2: int    # fresh encryption noise 2^-s
    bk_log_base: int = 8   # log2 B
    ks_log_base: int = 2   # log2 B'

    @property
    def lwe_words(self) -> int:
        """Words of a k-party LWE ciphertext (b, a_1..a_k)."""
        return self.k * self.n + 1

    @property
    def log2_2N(self) -> int:
        return (2 * self.N).bit_length() - 1


# Toy shape, keys with noise 2^-20 and encryptions 2^-12 (parity only: the
# blind-rotation noise at this shape exceeds the decryption margin).
C1 = Params(k=2, n=64, N=256, bk_ell=2, ks_t=6,
            bk_noise_log2=20, ks_noise_log2=20, lwe_noise_log2=12)
# Same shape with key noise 2^-26, where gates decrypt correctly.
C1B = Params(k=2, n=64, N=256, bk_ell=2, ks_t=6,
             bk_noise_log2=26, ks_noise_log2=20, lwe_noise_log2=12)
# C1B shape with 4 parties.
C1B4 = Params(k=4, n=64, N=256, bk_ell=2, ks_t=6,
              bk_noise_log2=26, ks_noise_log2=20, lwe_noise_log2=12)
# Smallest ring the int8-MFMA path takes (N/32 = 4 K-blocks), parity only.
C1S = Params(k=2, n=32, N=128, bk_ell=2, ks_t=6,
             bk_noise_log2=26, ks_noise_log2=20, lwe_noise_log2=12)
# Table 7 shape with 2 parties.
C2 = Params(k=2, n=560, N=1024, bk_ell=3, ks_t=8,
            bk_noise_log2=30, ks_noise_log2=15, lwe_noise_log2=15)
# Table 7 shape with 4 parties.
C3 = Params(k=4, n=560, N=1024, bk_ell=3, ks_t=8,
            bk_noise_log2=30, ks_noise_log2=15, lwe_noise_log2=15)
# Table 7 shape with 8 parties, retuned.  With the Table 7 noise the
# rotation's phase error grows with k n N (k N + 2) to about 2^-5.4 at k = 8,
# which leaves the gate windows a margin of only 3.6 standard deviations
# (a failure rate near 4e-4 per gate).  Key noise 2^-31 on the bootstrapping
# key and 2^-16 on the key-switching key restore about 6.8 deviations, the
# margin of the 4-party set.
C8 = Params(k=8, n=560, N=1024, bk_ell=3, ks_t=8,
            bk_noise_log2=31, ks_noise_log2=16, lwe_noise_log2=15)
# Small shapes for fast encrypted tests (decryptable).
TOY = Params(k=2, n=16, N=64, bk_ell=3, ks_t=8,
             bk_noise_log2=30, ks_noise_log2=24, lwe_noise_log2=20)


# Toy shape with base-8 key switching (3-bit digits), 3 parties.
TOYB3 = Params(k=3, n=16, N=64, bk_ell=3, ks_t=5,
               bk_noise_log2=30, ks_noise_log2=24, lwe_noise_log2=20, ks_log_base=3)


# Smallest MFMA ring with 3 parties and base-8 key switching (3-bit
# digits): the general one-hot code of the int8-MFMA key switch.
C1SB3 = Params(k=3, n=32, N=128, bk_ell=2, ks_t=5,
               bk_noise_log2=26, ks_noise_log2=20, lwe_noise_log2=12, ks_log_base=3)


def toy(k: int) -> Params:
    return Params(k=k, n=16, N=64, bk_ell=3, ks_t=8,
                  bk_noise_log2=30, ks_noise_log2=24, lwe_noise_log2=20)
