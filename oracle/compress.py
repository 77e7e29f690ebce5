"""Standalone compression of LWE and RLWE ciphertexts into Paillier ciphertexts (Sec. 3 and
the appendix), written as plain definitions.  Test infrastructure only.

* Alg. 2, LWECompress_q(ck, (a, b)): x = b (+) sum_i (q - a_i) (x) ck_i, where (+) is the
  Paillier product and k (x) c = c^k; b enters as Enc(b; 1) = (N+1)^b.  With reading
  (q - a_i) mod q every exponent lies in [0, q).
* Alg. 2, ModifiedLWEDecrypt: mu** = Dec(x) mod q, mu'' = round(mu** / Delta) mod p.
* Alg. 6 (appendix A, Sec. 3.2): packed compression keys.  t = floor(0.5 log2 m / log2 delta)
  secret digits share one ciphertext pck_i = Enc(delta^-(t-1) sum_j s[it+j] delta^j mod m);
  the server unpacks ck[it+j] = delta^(t-1-j) (x) pck_i, and the client decrypts with
  y = delta^(t-1) Dec(x) mod m, mu** = floor(y / delta^(t-1)) mod q.  delta must exceed the
  largest digit (q + n q^2, or q + n q for a binary key) and be a multiple of q, so that the
  digits above delta^(t-1) vanish modulo q; the oracle takes delta as an argument.
* Alg. 8 (appendix B): RLWECompressCoefficient(ck, (A, B), k) for R_q = Z_q[X]/(X^Nr + 1):
  x = B[k] (+) sum_{i<=k} (q - A[k-i]) (x) ck_i (+) sum_{i>k} A[Nr+k-i] (x) ck_i.

Paillier arithmetic uses Python integers and ``pow``; polynomial products are schoolbook.
"""
from __future__ import annotations

import math

from oracle import lwe, paillier


# ----------------------------------------------------------------------------- Alg. 2

def lwe_compress(ck, a, b: int, q: int, N: int) -> int:
    """x = (N+1)^b prod_i ck_i^((q - a_i) mod q) mod N^2."""
    N2 = N * N
    x = pow(N + 1, int(b) % q, N2)
    for c, ai in zip(ck, a):
        x = x * pow(int(c), (q - int(ai)) % q, N2) % N2
    return x


def modified_lwe_decrypt(sk: paillier.SecretKey, x: int, q: int, p: int) -> int:
    """mu'' = round((Dec(x) mod q) / Delta) mod p."""
    mu = paillier.decrypt(sk, int(x)) % q
    return lwe.round_div(mu, lwe.delta(q, p)) % p


def lwe_phase_plaintext(a, b: int, s, q: int) -> int:
    """The integer b + sum_i ((q - a_i) mod q) s_i that Dec(x) equals below the modulus."""
    return int(b) + sum(((q - int(ai)) % q) * int(si) for ai, si in zip(a, s))


# ----------------------------------------------------------------------------- Alg. 6 (packed keys)

def packed_digits_per_key(m_bits: int, delta: int) -> int:
    """t = floor(0.5 log2 m / log2 delta), log2 m taken as m_bits."""
    return int((0.5 * m_bits) // math.log2(delta))


def generate_packed_key(pk: paillier.PublicKey, s, delta: int, t: int, rands) -> list[int]:
    """pck_i = Enc(delta^-(t-1) sum_{j<t} s[it+j] delta^j mod N; rands[i]); missing digits are 0."""
    N = pk.N
    inv = pow(delta, -(t - 1), N)
    out = []
    for i in range(-(-len(s) // t)):
        acc = 0
        for j in range(t):
            if i * t + j < len(s):
                acc += int(s[i * t + j]) * delta ** j
        out.append(paillier.encrypt(pk, inv * acc % N, int(rands[i])))
    return out


def unpack_compression_key(pck, delta: int, t: int, n: int, N: int) -> list[int]:
    """ck[it+j] = pck_i^(delta^(t-1-j)) mod N^2 for it + j < n."""
    N2 = N * N
    return [pow(int(pck[k // t]), delta ** (t - 1 - k % t), N2) for k in range(n)]


def modified_decrypt_packed_key(sk: paillier.SecretKey, x: int, delta: int, t: int, q: int,
                                p: int) -> int:
    """y = delta^(t-1) Dec(x) mod N, mu** = floor(y / delta^(t-1)) mod q, mu'' = round(mu**/Delta)."""
    N = sk.pk.N
    y = delta ** (t - 1) * paillier.decrypt(sk, int(x)) % N
    mu = (y // delta ** (t - 1)) % q
    return lwe.round_div(mu, lwe.delta(q, p)) % p


# ----------------------------------------------------------------------------- RLWE (Alg. 7, Alg. 8)

def negacyclic_mul(A, S, q: int) -> list[int]:
    """A(X) S(X) mod (X^Nr + 1, q), schoolbook."""
    Nr = len(A)
    out = [0] * Nr
    for i in range(Nr):
        for j in range(Nr):
            k = i + j
            if k < Nr:
                out[k] += int(A[i]) * int(S[j])
            else:
                out[k - Nr] -= int(A[i]) * int(S[j])
    return [v % q for v in out]


def rlwe_encrypt(S, mu, A, E, q: int, p: int) -> list[int]:
    """B = A S + Delta mu + E in R_q (Alg. 7); A and E supplied by the caller."""
    AS = negacyclic_mul(A, S, q)
    d = lwe.delta(q, p)
    return [(AS[k] + d * int(mu[k]) + int(E[k])) % q for k in range(len(A))]


def rlwe_decrypt_coefficient(S, A, B, k: int, q: int, p: int) -> int:
    """Coefficient k of round((B - A S) / Delta) (Alg. 7)."""
    phase = (int(B[k]) - negacyclic_mul(A, S, q)[k]) % q
    return lwe.round_div(phase, lwe.delta(q, p)) % p


def rlwe_compress_coefficient(ck, A, B, k: int, q: int, N: int) -> int:
    """Alg. 8: x = Enc(B[k]; 1) times ck_i^(q - A[k-i]) for i <= k and ck_i^(A[Nr+k-i]) for i > k."""
    N2 = N * N
    Nr = len(A)
    x = pow(N + 1, int(B[k]) % q, N2)
    for i in range(Nr):
        e = (q - int(A[k - i])) % q if i <= k else int(A[Nr + k - i]) % q
        x = x * pow(int(ck[i]), e, N2) % N2
    return x


def rlwe_extract_lwe(A, B, k: int, q: int):
    """The LWE ciphertext (a, b) of coefficient k: b - <a, S> equals coefficient k of B - A S,
    a_i = A[k-i] for i <= k and -A[Nr+k-i] mod q for i > k (eq. of appendix B)."""
    Nr = len(A)
    a = [int(A[k - i]) % q if i <= k else (q - int(A[Nr + k - i])) % q for i in range(Nr)]
    return a, int(B[k]) % q
