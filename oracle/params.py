"""Parameter conditions stated by the paper.

* Theorem 1 (Sec. 3.1): LWE compression decrypts correctly when the additive plaintext
  modulus exceeds q + n q^2 (uniform secret: the largest plaintext sum is below it).
* ZipPIR correctness condition (Sec. 4.2): q/p > 2 p sigma sqrt(2 d0 ln(2/delta)), with d0
  the number of entries a query covers (here the number of database columns).
* Sizes (Sec. 5.1): an LWE ciphertext (a, b) in Z_q^n x Z_q against one additive (Paillier)
  ciphertext modulo N^2; the number of values packed into one additive plaintext,
  floor(log2 m / log2 delta) (Sec. 3.2, Sec. 3.3).
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


def lwe_ciphertext_bits(n: int, log_q: int) -> int:
    """(n + 1) log2 q: the vector a in Z_q^n and the scalar b."""
    return (n + 1) * log_q


def additive_ciphertext_bits(N_bits: int) -> int:
    """A Paillier ciphertext lives modulo N^2."""
    return 2 * N_bits


def size_reduction(n: int, log_q: int, N_bits: int) -> float:
    """1 - |compressed| / |uncompressed| for one LWE ciphertext."""
    return 1.0 - additive_ciphertext_bits(N_bits) / lwe_ciphertext_bits(n, log_q)


def pack_count(m_bits: int, delta: int) -> int:
    """Values of size below delta that fit one plaintext of an m_bits-bit modulus:
    floor(log2 m / log2 delta), with log2 m taken as m_bits."""
    return int(m_bits // math.log2(delta))


def packed_key_ciphertexts(n: int, q: int, N_bits: int, binary: bool) -> int:
    """ceil(n / digits per ciphertext) with the smallest admissible delta (Sec. 3.2):
    delta > q + n q^2, or delta > q + n q for a binary key."""
    delta = (q + n * q) if binary else compression_bound(n, q)
    per = pack_count(N_bits, delta + 1)
    return -(-n // per)
