"""LWE encryption (Alg. 1, Sec. 2.1) and the SimplePIR-style query/extract of ZipPIR (Alg. 5).

Orientation: the database is a ``rows x cols`` matrix D; the client retrieves column
``col``.  The paper writes the same protocol with D transposed (it retrieves a row of
D^T); the two are identical up to that transpose.

All values live in Z_q with q = 2^32 unless a different ``q`` is passed.
"""
from __future__ import annotations

import numpy as np

MASK32 = 0xFFFFFFFF


def delta(q: int, p: int) -> int:
    """Delta = round(q/p) (Sec. 2.1); exact integer rounding, ties upward."""
    return (2 * q + p) // (2 * p)


def round_div(x: int, y: int) -> int:
    """round(x/y) for non-negative integers, ties upward."""
    return (2 * x + y) // (2 * y)


# ----------------------------------------------------------------------------- Alg. 1

def lwe_encrypt(sk, a, mu: int, e: int, q: int, p: int) -> int:
    """b = <a, sk> + Delta*mu + e mod q (Alg. 1, LWEEncrypt; ``a`` supplied by the caller)."""
    acc = 0
    for ai, si in zip(a, sk):
        acc += int(ai) * int(si)
    return (acc + delta(q, p) * mu + e) % q


def lwe_phase(sk, a, b: int, q: int) -> int:
    """mu* = b - <a, sk> mod q (Alg. 1, LWEDecrypt, first step)."""
    acc = 0
    for ai, si in zip(a, sk):
        acc += int(ai) * int(si)
    return (int(b) - acc) % q


def lwe_decrypt(sk, a, b: int, q: int, p: int) -> int:
    """mu' = round(mu*/Delta) (Alg. 1), reduced into Z_p."""
    return round_div(lwe_phase(sk, a, b, q), delta(q, p)) % p


# ----------------------------------------------------------------------------- Alg. 5

def matvec_mod32(M: np.ndarray, v: np.ndarray) -> np.ndarray:
    """M.v mod 2^32 for a uint32-valued matrix ``M`` and vector ``v`` (exact)."""
    prod = M.astype(np.uint64) @ v.astype(np.uint64)   # wraps modulo 2^64
    return (prod & np.uint64(MASK32)).astype(np.uint32)


def pir_query(A: np.ndarray, s: np.ndarray, e: np.ndarray, col: int, p: int = 256) -> np.ndarray:
    """qu = A.s + e + Delta*u_col mod 2^32 (Alg. 5, Query), one entry per database column.

    ``A`` is ``cols x n`` uint32, ``s`` the n-entry secret, ``e`` the cols-entry signed
    error, ``u_col`` the selection vector of column ``col``.
    """
    q = 1 << 32
    As = matvec_mod32(A, s).astype(np.int64)
    u = np.zeros(A.shape[0], dtype=np.int64)
    u[col] = 1
    return ((As + e.astype(np.int64) + delta(q, p) * u) % q).astype(np.uint32)


def pir_extract_value(mu: int, p: int = 256, q: int = 1 << 32) -> int:
    """f = round((mu mod q) * p / q) mod p (Alg. 5, Extract; ties upward)."""
    return round_div((mu % q) * p, q) % p
