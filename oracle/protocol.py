"""The paper's full ZipPIR protocol (Alg. 5 with the Sec. 4.3 optimizations), written as plain
definitions.  Test infrastructure only: nothing on the product path imports this package.

In the full protocol the per-query hint is built from random ciphertexts instead of an
encryption of the LWE secret, and the secret enters online through an offset vector:

* Setup (Alg. 5):      ck_r uniform ciphertexts, pt_r = Dec(ck_r) (client side)
* Hint (Alg. 5):       k_j = prod_k ck_r,k^{E_jk} mod N^2, E = (-H) mod q    (same map as K)
* Query (Alg. 5):      ck_o = (s - pt_r) mod N, one entry per LWE coordinate
* Response (Alg. 5):   b = D.qu mod q, then t_j = (b_j + sum_k E_jk ck_o,k) mod N
* Extract (Alg. 5):    mu = (t_j + Dec(k_j)) mod N,  f = round((mu mod q) p / q) mod p
* Sec. 4.3, "Smaller responses w/ Paillier addition": the server may send
                       c_j = k_j (+) Enc(t_j; 1) = k_j (1 + t_j N) mod N^2
  instead of (k_j, t_j); then mu = Dec(c_j).

* Sec. 4.3, "Batched compression for smaller responses", applied to this protocol: the rows
  of a group of ell share one key k_g = prod_j k_{g ell + j}^{gamma^j} and one offset answer
  t_g = sum_j gamma^j t_{g ell + j} mod N (scaling is linear, so it splits into the offline
  key and the online answer); the client splits (t_g + Dec(k_g)) mod N into base-gamma digits.

Correctness (appendix proof of the ZipPIR correctness theorem): t_j + Dec(k_j) equals
b_j + sum_k E_jk s_k mod N, which is the integer itself while it stays below N; packed, the
digits are these integers when gamma exceeds each of them and gamma^ell < N (Theorem 2).
Orientation as in ``oracle.server``: rows of D, H, E, k and t are database rows.
"""
from __future__ import annotations

import numpy as np

from oracle import lwe, paillier


def random_key_plaintexts(sk: paillier.SecretKey, ck_r) -> list[int]:
    """pt_r = Dec(ck_r), entry by entry (Alg. 5, Setup)."""
    return [paillier.decrypt(sk, int(c)) for c in ck_r]


def query_offset(s, pt_r, N: int) -> list[int]:
    """ck_o = (s - pt_r) mod N (Alg. 5, Query)."""
    return [(int(x) - int(p)) % N for x, p in zip(s, pt_r)]


def offset_answer_row(b_j: int, e_row, cko, N: int) -> int:
    """t_j = (b_j + sum_k E_jk ck_o,k) mod N (Alg. 5, Response, second line)."""
    acc = int(b_j)
    for e, c in zip(e_row, cko):
        acc += int(e) * int(c)
    return acc % N


def offset_answer(b: np.ndarray, E: np.ndarray, cko, N: int, rows=None) -> list[int]:
    """t for every row (or the listed rows, in order); ``E`` holds all rows."""
    sel = range(E.shape[0]) if rows is None else [int(r) for r in rows]
    return [offset_answer_row(int(b[j]), E[j], cko, N) for j in sel]


def combine_offset(k_j: int, t_j: int, N: int) -> int:
    """c_j = k_j (+) Enc(t_j; 1) = k_j (N+1)^{t_j} = k_j (1 + t_j N) mod N^2 (Sec. 4.3)."""
    N2 = N * N
    return int(k_j) * pow(N + 1, int(t_j), N2) % N2


def extract(sk: paillier.SecretKey, k_j: int, t_j: int, p: int = 256, q: int = 1 << 32) -> int:
    """f from the pair (k_j, t_j) (Alg. 5, Extract)."""
    mu = (int(t_j) + paillier.decrypt(sk, int(k_j))) % sk.pk.N
    return lwe.pir_extract_value(mu, p, q)


def extract_combined(sk: paillier.SecretKey, c_j: int, p: int = 256, q: int = 1 << 32) -> int:
    """f from one combined ciphertext c_j (Sec. 4.3)."""
    return lwe.pir_extract_value(paillier.decrypt(sk, int(c_j)), p, q)


def offset_answer_packed(t, ell: int, gamma: int, N: int) -> list[int]:
    """t_g = sum_{j<ell} gamma^j t_{g ell + j} mod N (the last group may be short)."""
    return [sum(gamma ** j * int(t[g0 + j]) for j in range(min(ell, len(t) - g0))) % N
            for g0 in range(0, len(t), ell)]


def packed_keys(k, ell: int, gamma: int, N: int) -> list[int]:
    """k_g = prod_{j<ell} k_{g ell + j}^(gamma^j) mod N^2."""
    N2 = N * N
    out = []
    for g0 in range(0, len(k), ell):
        acc = 1
        for j in range(min(ell, len(k) - g0)):
            acc = acc * pow(int(k[g0 + j]), gamma ** j, N2) % N2
        out.append(acc)
    return out


def extract_packed(sk: paillier.SecretKey, k_g: int, t_g: int, rows: int, gamma: int,
                   p: int = 256, q: int = 1 << 32) -> list[int]:
    """The `rows` values of one group: base-gamma digits of (t_g + Dec(k_g)) mod N."""
    mu = (int(t_g) + paillier.decrypt(sk, int(k_g))) % sk.pk.N
    return [lwe.pir_extract_value((mu // gamma ** j) % gamma, p, q) for j in range(rows)]
