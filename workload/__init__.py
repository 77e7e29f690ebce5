"""Seeded synthetic inputs for the ZipPIR server path.

This module only draws random material: database bytes, the public LWE matrix, LWE
secrets and errors, the selected column, Paillier prime factors and randomness, uniform
residues, request arrival times and database updates.  It performs none of the
protocol's arithmetic (no LWE encryption, no Paillier operation, no matrix product), so
the CPU oracle and the GPU path can both be fed from it without sharing any of the
method's computation.

Every stream is a numpy PCG64 generator keyed by ``SeedSequence([cfg, role, client])``.
Large integers (Paillier primes, residues) are assembled from 32-bit words drawn from
such a stream, so they are reproducible across machines.

The shapes and distributions follow the paper's PIR setting (Alg. 5 and Sec. 6.2):
``D`` uniform over Z_p with p = 256, ``A`` uniform over Z_q with q = 2^32, the secret
uniform over Z_q (the uniform-secret reading of the compression theorem), and the error a
rounded Gaussian of standard deviation 6.4.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

ROLE = {
    "db": 0,
    "lwe_a": 1,
    "secret": 2,
    "error": 3,
    "column": 4,
    "primes": 5,
    "paillier_r": 6,
    "arrivals": 7,
    "update": 8,
    "cipher": 9,
    "query": 10,
}

Q_BITS = 32
P_PLAIN = 256
SIGMA = 6.4


def rng(cfg: int, role: str, client: int = 0) -> np.random.Generator:
    """A reproducible generator for one (config, role, client) stream."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(cfg), ROLE[role], int(client)])))


# ----------------------------------------------------------------------------- matrices

DB_CHUNK_ROWS = 256


def _db_chunk(cfg: int, chunk: int, nrows: int, cols: int) -> np.ndarray:
    # every block of DB_CHUNK_ROWS rows has its own stream, so any rows can be regenerated alone
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(cfg), ROLE["db"], 1 << 20, chunk])))
    return g.integers(0, 256, size=(nrows, cols), dtype=np.uint8)


def database(cfg: int, rows: int, cols: int, threads: int = 8) -> np.ndarray:
    """Uniform uint8 database of ``rows x cols`` (row-major)."""
    from concurrent.futures import ThreadPoolExecutor
    out = np.empty((rows, cols), dtype=np.uint8)

    def fill(c):
        r0 = c * DB_CHUNK_ROWS
        r1 = min(rows, r0 + DB_CHUNK_ROWS)
        out[r0:r1] = _db_chunk(cfg, c, r1 - r0, cols)

    nchunks = (rows + DB_CHUNK_ROWS - 1) // DB_CHUNK_ROWS
    with ThreadPoolExecutor(max_workers=max(1, threads)) as ex:
        list(ex.map(fill, range(nchunks)))
    return out


def database_rows(cfg: int, rows: int, cols: int, idx) -> np.ndarray:
    """The listed rows of ``database(cfg, rows, cols)`` without generating the rest."""
    idx = np.asarray(idx, dtype=np.int64)
    out = np.empty((len(idx), cols), dtype=np.uint8)
    cache = {}
    for k, r in enumerate(idx):
        c = int(r) // DB_CHUNK_ROWS
        if c not in cache:
            r0 = c * DB_CHUNK_ROWS
            cache[c] = _db_chunk(cfg, c, min(rows, r0 + DB_CHUNK_ROWS) - r0, cols)
        out[k] = cache[c][int(r) - c * DB_CHUNK_ROWS]
    return out


def lwe_matrix(cfg: int, cols: int, n: int) -> np.ndarray:
    """Public LWE matrix A, uniform over Z_{2^32}, ``cols x n`` row-major (one row per DB column)."""
    return rng(cfg, "lwe_a").integers(0, 1 << 32, size=(cols, n), dtype=np.uint32)


def secret(cfg: int, client: int, n: int) -> np.ndarray:
    """LWE secret, uniform over Z_{2^32}."""
    return rng(cfg, "secret", client).integers(0, 1 << 32, size=n, dtype=np.uint32)


def error(cfg: int, client: int, length: int, sigma: float = SIGMA) -> np.ndarray:
    """Rounded Gaussian LWE error (no tail cut), as signed int64."""
    z = rng(cfg, "error", client).standard_normal(length)
    return np.rint(sigma * z).astype(np.int64)


def column(cfg: int, client: int, cols: int) -> int:
    """The database column a client retrieves."""
    return int(rng(cfg, "column", client).integers(0, cols))


def uniform_queries(cfg: int, batch: int, cols: int) -> np.ndarray:
    """``batch`` uniform uint32 vectors of length ``cols`` (timing-only query stand-ins)."""
    return rng(cfg, "query").integers(0, 1 << 32, size=(batch, cols), dtype=np.uint32)


# ----------------------------------------------------------------------------- big integers

def _words_to_int(words: np.ndarray) -> int:
    return int.from_bytes(np.asarray(words, dtype="<u4").tobytes(), "little")


def random_bits(g: np.random.Generator, bits: int) -> int:
    """A uniform integer in [0, 2^bits) from 32-bit words."""
    nwords = (bits + 31) // 32
    x = _words_to_int(g.integers(0, 1 << 32, size=nwords, dtype=np.uint32))
    return x & ((1 << bits) - 1)


def uniform_below(g: np.random.Generator, bound: int) -> int:
    """A uniform integer in [0, bound) by rejection sampling."""
    bits = bound.bit_length()
    while True:
        x = random_bits(g, bits)
        if x < bound:
            return x


def uniform_unit(g: np.random.Generator, modulus: int) -> int:
    """A uniform element of the unit group Z*_modulus, by rejection."""
    while True:
        x = uniform_below(g, modulus)
        if x > 0 and math.gcd(x, modulus) == 1:
            return x


_SMALL_PRIMES = [p for p in range(3, 2000) if all(p % d for d in range(2, int(p ** 0.5) + 1))]


def _probable_prime(x: int, g: np.random.Generator, rounds: int = 40) -> bool:
    """Miller-Rabin with seeded random bases."""
    if x < 2:
        return False
    for p in _SMALL_PRIMES:
        if x % p == 0:
            return x == p
    d, s = x - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for _ in range(rounds):
        a = 2 + uniform_below(g, x - 3)
        y = pow(a, d, x)
        if y in (1, x - 1):
            continue
        for _ in range(s - 1):
            y = y * y % x
            if y == x - 1:
                break
        else:
            return False
    return True


def seeded_prime(g: np.random.Generator, bits: int) -> int:
    """Next probable prime at or above a random odd integer with its top two bits set."""
    x = random_bits(g, bits) | (3 << (bits - 2)) | 1
    while not _probable_prime(x, g):
        x += 2
    return x


@dataclass(frozen=True)
class PaillierPrimes:
    P: int
    Q: int


def paillier_primes(cfg: int, client: int, n_bits: int) -> PaillierPrimes:
    """Two distinct primes of ``n_bits/2`` bits each whose product has exactly ``n_bits`` bits."""
    g = rng(cfg, "primes", client)
    half = n_bits // 2
    while True:
        P = seeded_prime(g, half)
        Q = seeded_prime(g, n_bits - half)
        if P != Q and (P * Q).bit_length() == n_bits:
            return PaillierPrimes(P, Q)


def paillier_randomness(cfg: int, client: int, count: int, N: int) -> list[int]:
    """``count`` uniform elements of Z*_N (the Paillier encryption randomness)."""
    g = rng(cfg, "paillier_r", client)
    return [uniform_unit(g, N) for _ in range(count)]


def uniform_ciphertexts(cfg: int, client: int, count: int, N: int) -> list[int]:
    """``count`` uniform elements of Z*_{N^2}.

    Every such element is a valid Paillier ciphertext (encryption is a bijection from
    Z_N x Z*_N onto Z*_{N^2}); the paper's setup samples its random compression-key
    component the same way, directly from the ciphertext space (Sec. 4.1, Alg. 5).
    """
    g = rng(cfg, "cipher", client)
    N2 = N * N
    return [uniform_unit(g, N2) for _ in range(count)]


# ----------------------------------------------------------------------------- serving / updates

def arrivals(cfg: int, rate_qps: float, duration_s: float) -> np.ndarray:
    """Poisson arrival times (seconds) at ``rate_qps`` over ``duration_s``."""
    g = rng(cfg, "arrivals")
    n_est = int(rate_qps * duration_s * 1.5) + 64
    t = np.cumsum(g.exponential(1.0 / rate_qps, size=n_est))
    while t[-1] < duration_s:
        more = t[-1] + np.cumsum(g.exponential(1.0 / rate_qps, size=n_est))
        t = np.concatenate([t, more])
    return t[t < duration_s]


def db_choices(cfg: int, count: int, weights) -> np.ndarray:
    """Which database each arriving request targets, by the given mix weights."""
    w = np.asarray(weights, dtype=np.float64)
    return rng(cfg, "arrivals", 1).choice(len(w), size=count, p=w / w.sum())


def update_rows(cfg: int, rows: int, cols: int, fraction: float = 0.01):
    """``ceil(fraction*rows)`` distinct rows (sorted) and fresh uniform bytes for them."""
    g = rng(cfg, "update")
    k = math.ceil(fraction * rows)
    idx = np.sort(g.permutation(rows)[:k]).astype(np.uint32)
    new = g.integers(0, 256, size=(k, cols), dtype=np.uint8)
    return idx, new


# ----------------------------------------------------------------------------- limb packing

def int_to_limbs(x: int, nlimbs: int) -> np.ndarray:
    """Little-endian uint32 limbs of a non-negative integer (raises if it does not fit)."""
    if x < 0 or x.bit_length() > 32 * nlimbs:
        raise ValueError("integer does not fit in the limb count")
    return np.frombuffer(x.to_bytes(4 * nlimbs, "little"), dtype="<u4").astype(np.uint32)


def limbs_to_int(limbs) -> int:
    return int.from_bytes(np.ascontiguousarray(limbs, dtype="<u4").tobytes(), "little")


def ints_to_limbs(xs, nlimbs: int) -> np.ndarray:
    out = np.empty((len(xs), nlimbs), dtype=np.uint32)
    for i, x in enumerate(xs):
        out[i] = int_to_limbs(x, nlimbs)
    return out
