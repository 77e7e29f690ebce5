"""Parameter conditions stated by the paper.

* Theorem 1 (Sec. 3.1): LWE compression decrypts correctly when the additive plaintext
  modulus exceeds q + n q^2 (uniform secret: the largest plaintext sum is below it).
* ZipPIR correctness condition (Sec. 4.2): q/p > 2 p sigma sqrt(2 d0 ln(2/delta)), with d0
  the number of entries a query covers (here the number of database columns).
"""
from __future__ import annotations

import math


def compression_bound(n: int, q: int = 1 << 32) -> int:
    """q + n q^2: the plaintext modulus must be strictly larger (Theorem 1)."""
    return q + n * q * q


def compression_ok(N: int, n: int, q: int = 1 << 32) -> bool:
    return N > compression_bound(n, q)


def zippir_noise_ok(cols: int, p: int = 256, q: int = 1 << 32, sigma: float = 6.4,
                    fail_prob: float = 2.0 ** -40) -> bool:
    """q/p > 2 p sigma sqrt(2 d0 ln(2/delta))."""
    return q / p > 2 * p * sigma * math.sqrt(2 * cols * math.log(2 / fail_prob))
