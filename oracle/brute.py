"""Pure-Python recomputation of the server quantities for tiny inputs.

No numpy and no built-in ``pow``: the modular exponentiation is a hand-written
right-to-left square-and-multiply, and every sum is an explicit loop over Python
integers reduced once at the end.  Used to cross-check ``oracle.server`` on tiny sizes.
"""
from __future__ import annotations


def modexp(base: int, exp: int, mod: int) -> int:
    """base^exp mod mod by square-and-multiply (exp >= 0)."""
    result = 1 % mod
    b = base % mod
    e = exp
    while e > 0:
        if e & 1:
            result = result * b % mod
        b = b * b % mod
        e >>= 1
    return result


def matvec(D, v, modulus: int = 1 << 32):
    """[sum_i D[j][i] v[i] mod modulus for j] with lists of ints."""
    return [sum(int(D[j][i]) * int(v[i]) for i in range(len(v))) % modulus for j in range(len(D))]


def matmul(D, A, modulus: int = 1 << 32):
    rows, inner, cols = len(D), len(A), len(A[0])
    return [[sum(int(D[j][i]) * int(A[i][k]) for i in range(inner)) % modulus for k in range(cols)]
            for j in range(rows)]


def negate(x: int, modulus: int = 1 << 32) -> int:
    return (modulus - x) % modulus


def hint_row(ck, e_row, N: int) -> int:
    N2 = N * N
    acc = 1
    for c, e in zip(ck, e_row):
        acc = acc * modexp(int(c), int(e), N2) % N2
    return acc


def combine(K_j: int, b_j: int, N: int) -> int:
    """K_j times the unit-randomness encryption of b_j, i.e. (N+1)^{b_j}."""
    N2 = N * N
    return int(K_j) * modexp(N + 1, int(b_j), N2) % N2


def offset_row(b_j: int, e_row, cko, N: int) -> int:
    """b_j + sum_k E_jk ck_o,k reduced mod N once, by an explicit loop."""
    acc = int(b_j)
    for k in range(len(e_row)):
        acc = acc + int(e_row[k]) * int(cko[k])
    return acc - (acc // N) * N
