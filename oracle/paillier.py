"""The Paillier cryptosystem (Sec. 2.1; Paillier 1999), textbook form with generator g = N+1.

The paper fixes only the interface: plaintexts in Z_N, ciphertexts in Z_{N^2}, addition
(+) and plaintext multiplication (x).  This oracle uses the standard instantiation:

    Enc(m; r) = g^m * r^N mod N^2,            g = N + 1, r in Z*_N
    Dec(c)    = L(c^lambda mod N^2) * mu mod N,  L(x) = (x - 1) / N,
                lambda = lcm(P-1, Q-1),  mu = L(g^lambda mod N^2)^{-1} mod N
    c1 (+) c2 = c1 * c2 mod N^2                (adds plaintexts)
    k  (x) c  = c^k mod N^2                    (multiplies the plaintext by k)

Decryption is written out directly, without the CRT shortcut, so it can be checked by eye.
"""
from __future__ import annotations

import math
from dataclasses import dataclass


@dataclass(frozen=True)
class PublicKey:
    N: int

    @property
    def N2(self) -> int:
        return self.N * self.N

    @property
    def g(self) -> int:
        return self.N + 1


@dataclass(frozen=True)
class SecretKey:
    pk: PublicKey
    lam: int
    mu: int


def _L(x: int, N: int) -> int:
    assert (x - 1) % N == 0, "L() applied to a value not congruent to 1 mod N"
    return (x - 1) // N


def keygen(P: int, Q: int) -> SecretKey:
    """Key pair from two distinct primes P, Q (the caller supplies them)."""
    if P == Q:
        raise ValueError("Paillier primes must differ")
    N = P * Q
    pk = PublicKey(N)
    lam = (P - 1) * (Q - 1) // math.gcd(P - 1, Q - 1)
    mu = pow(_L(pow(pk.g, lam, pk.N2), N), -1, N)
    return SecretKey(pk, lam, mu)


def encrypt(pk: PublicKey, m: int, r: int) -> int:
    """Enc(m; r) = g^m r^N mod N^2 with g = N+1; ``m`` is reduced into Z_N."""
    if math.gcd(r, pk.N) != 1 or not (0 < r < pk.N):
        raise ValueError("randomness must lie in Z*_N")
    return pow(pk.g, m % pk.N, pk.N2) * pow(r, pk.N, pk.N2) % pk.N2


def decrypt(sk: SecretKey, c: int) -> int:
    """Dec(c) = L(c^lambda mod N^2) * mu mod N."""
    N, N2 = sk.pk.N, sk.pk.N2
    if not (0 <= c < N2) or math.gcd(c, N) != 1:
        raise ValueError("not a ciphertext")
    return _L(pow(c, sk.lam, N2), N) * sk.mu % N


def add(pk: PublicKey, c1: int, c2: int) -> int:
    """c1 (+) c2: the ciphertext of the sum of the plaintexts."""
    return c1 * c2 % pk.N2


def scalar_mul(pk: PublicKey, k: int, c: int) -> int:
    """k (x) c: the ciphertext of k times the plaintext (k a non-negative integer)."""
    return pow(c, k, pk.N2)


def add_plain(pk: PublicKey, c: int, m: int) -> int:
    """c (+) Enc(m; 1): adds a known plaintext with unit randomness (deterministic)."""
    return c * pow(pk.g, m % pk.N, pk.N2) % pk.N2
