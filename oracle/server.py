"""Server-side quantities of ZipPIR, written as their plain definitions.

Orientation: D is ``rows x cols`` uint8 (p = 256), A is ``cols x n`` uint32, a query is a
``cols``-entry uint32 vector and an answer a ``rows``-entry uint32 vector.

* Global hint (Alg. 5 preamble; reused by all clients, Sec. 4.3):   H = D.A mod 2^32
* Exponents (Alg. 2 multiplies ck[i] by (q - a[i]); Alg. 4 takes it mod q):
                                                                     E = (-H) mod 2^32
* Client hint (Alg. 5, Hint = PaillierMatMul(H, ck)):                K_j = prod_k ck_k^{E_jk} mod N^2
* Online answer (Alg. 5, Response, first line):                     b = D.qu mod 2^32
* Combined response (Sec. 4.3, "Smaller responses w/ Paillier addition"):
                                                                     c_j = K_j (+) Enc(b_j; 1)
                                                                         = K_j * (N+1)^{b_j} mod N^2

Matrix products use numpy uint64 arithmetic, which wraps modulo 2^64 and is therefore
exact modulo 2^32 after masking.  Paillier quantities use Python integers and ``pow``.
"""
from __future__ import annotations

import numpy as np

MASK32 = np.uint64(0xFFFFFFFF)


def answer(D: np.ndarray, qu: np.ndarray, chunk_rows: int = 1024) -> np.ndarray:
    """b[j] = sum_i D[j,i] * qu[i] mod 2^32."""
    rows, cols = D.shape
    assert qu.shape == (cols,)
    q64 = qu.astype(np.uint64)
    out = np.empty(rows, dtype=np.uint32)
    for r0 in range(0, rows, chunk_rows):
        r1 = min(rows, r0 + chunk_rows)
        out[r0:r1] = ((D[r0:r1].astype(np.uint64) @ q64) & MASK32).astype(np.uint32)
    return out


def answer_rows(D: np.ndarray, qu: np.ndarray, rows) -> np.ndarray:
    """b restricted to the listed rows."""
    rows = np.asarray(rows, dtype=np.int64)
    return ((D[rows].astype(np.uint64) @ qu.astype(np.uint64)) & MASK32).astype(np.uint32)


def answer_batch(D: np.ndarray, Q: np.ndarray) -> np.ndarray:
    """B[c] = D.Q[c] mod 2^32 for each query c -- one independent answer per query."""
    return np.stack([answer(D, Q[c]) for c in range(Q.shape[0])])


def global_hint(D: np.ndarray, A: np.ndarray, rows=None, chunk_rows: int = 64) -> np.ndarray:
    """H[j,k] = sum_i D[j,i] * A[i,k] mod 2^32 (all rows, or the listed rows in order)."""
    sel = np.arange(D.shape[0]) if rows is None else np.asarray(rows, dtype=np.int64)
    A64 = A.astype(np.uint64)
    out = np.empty((len(sel), A.shape[1]), dtype=np.uint32)
    for r0 in range(0, len(sel), chunk_rows):
        r1 = min(len(sel), r0 + chunk_rows)
        out[r0:r1] = ((D[sel[r0:r1]].astype(np.uint64) @ A64) & MASK32).astype(np.uint32)
    return out


def exponents(H: np.ndarray) -> np.ndarray:
    """E = (q - H) mod q with q = 2^32: the non-negative representative of -H."""
    return ((np.uint64(1 << 32) - H.astype(np.uint64)) & MASK32).astype(np.uint32)


def client_hint_row(ck, e_row, N: int) -> int:
    """K_j = prod_k ck_k^{E_jk} mod N^2: the k-sum of E_jk (x) ck_k under (+)."""
    N2 = N * N
    acc = 1
    for c, e in zip(ck, e_row):
        acc = acc * pow(int(c), int(e), N2) % N2
    return acc


def client_hint(ck, E: np.ndarray, N: int) -> list[int]:
    return [client_hint_row(ck, E[j], N) for j in range(E.shape[0])]


def compress_row(K_j: int, b_j: int, N: int) -> int:
    """c_j = K_j (+) Enc(b_j; 1) = K_j * (N+1)^{b_j} mod N^2."""
    N2 = N * N
    return int(K_j) * pow(N + 1, int(b_j), N2) % N2


def compress(K, b, N: int) -> list[int]:
    return [compress_row(k, int(x), N) for k, x in zip(K, b)]


def hint_plaintext_row(e_row, s) -> int:
    """The integer sum_k E_jk * s_k that Dec(K_j) must equal when it stays below N."""
    return sum(int(e) * int(x) for e, x in zip(e_row, s))


# ----------------------------------------------------------------------------- batched compression
# Alg. 3 (BatchedLWECompress, Sec. 3.3) in the combined form of ZipPIR (Sec. 4.3, "Batched
# compression for smaller responses"): the compressed rows x_j of a group of ell rows are
# folded into one ciphertext x = (+)_j gamma^j (x) x_j.  Correct when N > gamma^ell and
# gamma >= q + n q^2 (Theorem 2, Sec. 3.3).

def packing_scale_min(n: int, q: int = 1 << 32) -> int:
    """q + n q^2, the smallest admissible gamma (Theorem 2)."""
    return q + n * q * q


def compress_packed(K, b, N: int, ell: int, gamma: int) -> list[int]:
    """c_g = prod_{j<ell} c_{g ell + j}^{gamma^j} mod N^2, c_r the combined row r (last group may be short)."""
    N2 = N * N
    rows = len(K)
    out = []
    for g0 in range(0, rows, ell):
        acc = 1
        for j in range(min(ell, rows - g0)):
            acc = acc * pow(compress_row(K[g0 + j], int(b[g0 + j]), N), gamma ** j, N2) % N2
        out.append(acc)
    return out


def packed_digits(mu: int, ell: int, gamma: int) -> list[int]:
    """mu_j = floor(mu / gamma^j) mod gamma for j < ell (ModifiedBatchedLWEDecrypt, Alg. 3)."""
    return [(mu // gamma ** j) % gamma for j in range(ell)]
