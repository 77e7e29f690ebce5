"""Pins for the oracle's PRG of the silent offline phase (Sec. 4.3, "Lowering offline
communication costs"): ChaCha20 against RFC 8439's printed vectors and against OpenSSL's
independent implementation, the rejection sampler against the uniform distribution on
Z_{N^2}, and a full-protocol round trip whose random keys come from a seed alone."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import workload as wl
from oracle import paillier, prg, protocol, server
from tests.instances import make_instance


def _golden(name):
    path = os.path.join(os.path.dirname(__file__), "golden", name)
    rows = []
    for line in open(path):
        line = line.split("#")[0].strip()
        if line:
            rows.append(line.split())
    return rows


def test_rfc8439_quarter_round_and_block():
    rows = _golden("chacha20_rfc8439.txt")
    kinds = [r[0] for r in rows]
    assert kinds.count("qr") == 1 and kinds.count("block") == 1
    for r in rows:
        if r[0] == "qr":
            a, b, c, d, *want = [int(x, 16) for x in r[1:]]
            assert list(prg.quarter_round(a, b, c, d)) == want
        else:
            key, counter, nonce, want = bytes.fromhex(r[1]), int(r[2]), bytes.fromhex(r[3]), r[4]
            assert prg.block(key, counter, nonce).hex() == want


@pytest.mark.skipif(shutil.which("openssl") is None, reason="openssl not installed")
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_keystream_matches_openssl(seed):
    # OpenSSL's chacha20 cipher takes a 16-byte IV = block counter (little-endian) || nonce;
    # encrypting zeros returns the keystream.  Several blocks, random key, nonce and counter.
    g = np.random.default_rng(seed)
    key = g.bytes(32)
    nonce = g.bytes(12)
    counter = int(g.integers(0, 1 << 20))
    nblocks = 5
    iv = counter.to_bytes(4, "little") + nonce
    out = subprocess.run(["openssl", "enc", "-chacha20", "-K", key.hex(), "-iv", iv.hex()],
                         input=bytes(64 * nblocks), capture_output=True, check=True).stdout
    mine = b"".join(prg.block(key, counter + i, nonce) for i in range(nblocks))
    assert out == mine


def test_keystream_words_are_consecutive_blocks():
    key = bytes(range(100, 132))
    nonce = prg.nonce_words(7, 8, 9)
    ws = prg.keystream_words(key, nonce, 40)
    want = prg.block_words(key, 0, nonce) + prg.block_words(key, 1, nonce) + prg.block_words(key, 2, nonce)
    assert ws == want[:40]
    assert nonce == bytes([7, 0, 0, 0, 8, 0, 0, 0, 9, 0, 0, 0])


def test_random_key_entries_are_residues_and_reproducible():
    pr = wl.paillier_primes(1200, 0, 256)
    N = pr.P * pr.Q
    seed = bytes(range(32))
    a = prg.random_key(seed, N, 6, query=0)
    assert a == prg.random_key(seed, N, 6, query=0)
    assert all(0 <= x < N * N for x in a)
    b = prg.random_key(seed, N, 6, query=1)
    c = prg.random_key(bytes(32), N, 6, query=0)
    assert len(set(a) | set(b) | set(c)) == 18          # queries and seeds give other keys
    assert a[:3] == prg.random_key(seed, N, 3, query=0)  # entry k does not depend on n


def test_random_key_rejects_candidates_at_or_above_N2():
    # N^2 just above a power of two: a candidate is rejected with probability close to 1/2,
    # and each rejected attempt's candidate is indeed >= N^2.
    N = 2 ** 64 + 13     # any odd N works for the sampler
    N2 = N * N
    bits = N2.bit_length()
    seed = bytes([5] * 32)
    rejected = 0
    for k in range(64):
        x = prg.random_key_entry(seed, N, 0, k)
        assert x < N2
        r = 0
        while True:
            ws = prg.keystream_words(seed, prg.nonce_words(0, k, r), (bits + 31) // 32)
            cand = sum(w << (32 * i) for i, w in enumerate(ws)) & ((1 << bits) - 1)
            if cand < N2:
                break
            r += 1
        assert cand == x
        rejected += r
    assert 20 < rejected < 120     # about one rejection per entry on average


def test_random_key_is_uniform_on_a_tiny_modulus():
    # N = 3, N^2 = 9: 4-bit candidates, accepted below 9; 9000 entries give each residue
    # about 1000 times (chi-square with 8 degrees of freedom below its 0.999 quantile, 26.1).
    seed = bytes(range(32, 64))
    xs = [prg.random_key_entry(seed, 3, q, k) for q in range(9) for k in range(1000)]
    counts = np.bincount(xs, minlength=9)
    assert len(counts) == 9
    chi2 = float(((counts - 1000.0) ** 2 / 1000.0).sum())
    assert chi2 < 26.1


def test_seeded_full_protocol_round_trip():
    # Alg. 5 with ck_r drawn from a seed (Sec. 4.3): the server needs only N and the seed; the
    # client derives the same ck_r, decrypts it at query time, and the extraction recovers
    # the column on every row, for two queries from one seed.
    inst = make_instance(cfg=1201, rows=12, cols=24, n=5, n_bits=256, encrypt_secret=False)
    cl = inst.clients[0]
    seed = bytes(range(200, 232))
    E = server.exponents(server.global_hint(inst.D, inst.A))
    b = server.answer(inst.D, cl.qu)
    for q in (0, 1):
        ckr = prg.random_key(seed, cl.N, inst.n, q)
        pt_r = protocol.random_key_plaintexts(cl.sk, ckr)
        cko = protocol.query_offset(cl.s, pt_r, cl.N)
        k = server.client_hint(ckr, E, cl.N)
        t = protocol.offset_answer(b, E, cko, cl.N)
        assert [protocol.extract(cl.sk, k[j], t[j]) for j in range(inst.rows)] == inst.D[:, cl.col].tolist()
        c = [protocol.combine_offset(k[j], t[j], cl.N) for j in range(inst.rows)]
        assert [protocol.extract_combined(cl.sk, x) for x in c] == inst.D[:, cl.col].tolist()


def test_mutation_wrong_rotation_is_caught(monkeypatch):
    # a plausible slip in the quarter round (rotating by 12 where 8 belongs) fails the
    # RFC vectors
    orig = prg._rotl

    def bad(x, n):
        return orig(x, 12 if n == 8 else n)
    monkeypatch.setattr(prg, "_rotl", bad)
    with pytest.raises(AssertionError):
        test_rfc8439_quarter_round_and_block()


def test_mutation_counter_in_nonce_slot_is_caught(monkeypatch):
    # placing the block counter after the nonce instead of before it fails the block vector
    def bad(key, counter, nonce):
        init = list(prg.CONSTANTS) + prg._words_le(key) + prg._words_le(nonce) + [counter]
        x = list(init)
        for _ in range(10):
            for i0, i1, i2, i3 in ((0, 4, 8, 12), (1, 5, 9, 13), (2, 6, 10, 14), (3, 7, 11, 15),
                                   (0, 5, 10, 15), (1, 6, 11, 12), (2, 7, 8, 13), (3, 4, 9, 14)):
                x[i0], x[i1], x[i2], x[i3] = prg.quarter_round(x[i0], x[i1], x[i2], x[i3])
        return [(a + b) & prg.MASK for a, b in zip(x, init)]
    monkeypatch.setattr(prg, "block_words", bad)
    with pytest.raises(AssertionError):
        test_rfc8439_quarter_round_and_block()
