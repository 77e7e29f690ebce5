"""Seeded PIR instances built from ``workload`` draws and the oracle's client-side math.

Tests use these to feed the same inputs to the oracle and to the GPU library.  The
client side (Paillier key generation and encryption of the LWE secret, the LWE query)
is computed by the oracle; the server-side expected values are computed by the oracle
from the same inputs.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from multiprocessing import Pool

import numpy as np

import workload as wl
from oracle import lwe, paillier, server


@dataclass
class Client:
    cid: int
    sk: paillier.SecretKey
    s: np.ndarray            # LWE secret (uint32)
    ck: list                 # Paillier ciphertexts, one per LWE coordinate
    col: int = 0
    e: np.ndarray = None
    qu: np.ndarray = None    # LWE query vector (uint32, one entry per DB column)

    @property
    def N(self) -> int:
        return self.sk.pk.N


@dataclass
class Instance:
    cfg: int
    rows: int
    cols: int
    n: int
    n_bits: int
    D: np.ndarray
    A: np.ndarray
    clients: list = field(default_factory=list)


def _enc_one(args):
    N, m, r = args
    return paillier.encrypt(paillier.PublicKey(N), m, r)


def make_client(cfg: int, cid: int, A: np.ndarray, n_bits: int, encrypt_secret: bool = True,
                pool: Pool | None = None) -> Client:
    cols, n = A.shape
    pr = wl.paillier_primes(cfg, cid, n_bits)
    sk = paillier.keygen(pr.P, pr.Q)
    N = sk.pk.N
    s = wl.secret(cfg, cid, n)
    if encrypt_secret:
        rs = wl.paillier_randomness(cfg, cid, n, N)
        jobs = [(N, int(s[k]), rs[k]) for k in range(n)]
        ck = pool.map(_enc_one, jobs) if pool is not None else [_enc_one(j) for j in jobs]
    else:
        # uniform elements of Z*_{N^2}: valid ciphertexts of unknown plaintexts
        ck = wl.uniform_ciphertexts(cfg, cid, n, N)
    col = wl.column(cfg, cid, cols)
    e = wl.error(cfg, cid, cols)
    qu = lwe.pir_query(A, s, e, col)
    return Client(cid, sk, s, ck, col, e, qu)


def make_instance(cfg: int, rows: int, cols: int, n: int, n_bits: int, nclients: int = 1,
                  encrypt_secret: bool = True, zero_row: int | None = None, pool=None) -> Instance:
    D = wl.database(cfg, rows, cols)
    if zero_row is not None:
        D[zero_row] = 0
    A = wl.lwe_matrix(cfg, cols, n)
    inst = Instance(cfg, rows, cols, n, n_bits, D, A)
    for c in range(nclients):
        inst.clients.append(make_client(cfg, c, A, n_bits, encrypt_secret, pool))
    return inst


def _hint_row_job(args):
    ck, e_row, N = args
    return server.client_hint_row(ck, e_row, N)


def oracle_client_hint(ck, E: np.ndarray, N: int, rows=None, pool=None) -> dict:
    """{row: K_row} for the listed rows (all rows by default), optionally in a pool."""
    sel = list(range(E.shape[0])) if rows is None else [int(r) for r in rows]
    jobs = [(ck, E[j], N) for j in sel]
    vals = pool.map(_hint_row_job, jobs) if pool is not None else [_hint_row_job(j) for j in jobs]
    return dict(zip(sel, vals))
