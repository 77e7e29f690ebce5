"""GPU parity of standalone compression (Sec. 3): LWE ciphertexts (Alg. 2) at the Table 2
moduli, RLWE coefficients (Alg. 8) and packed compression keys (Alg. 6).

Every compressed ciphertext is compared bit for bit with ``oracle.compress`` on the same seeded
inputs, and the client's decryption recovers the encrypted message (Theorem 1 and its RLWE
and packed-key variants).
"""
from multiprocessing import Pool

import numpy as np
import pytest

import workload as wl
from oracle import compress, lwe, paillier, params
from tests.gpu_util import limbs_rows_to_ints, log, pool_size

pytestmark = pytest.mark.gpu

Q27 = 134217689          # a prime below 2^27 (an RLWE modulus of Table 2's size)


@pytest.fixture(scope="module")
def native():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_09190_amd import native as nat
    return nat


def _key(cfg, bits):
    pr = wl.paillier_primes(cfg, 0, bits)
    return paillier.keygen(pr.P, pr.Q)


def _enc_key(sk, s, cfg):
    rs = wl.paillier_randomness(cfg, 0, len(s), sk.pk.N)
    return [paillier.encrypt(sk.pk, int(s[i]) % sk.pk.N, rs[i]) for i in range(len(s))]


def _limbs(sk, bits):
    h = (bits + 31) // 32
    return wl.int_to_limbs(sk.pk.N, h), 2 * h


def _lwe_batch(g, s, q, p, rows):
    n = len(s)
    A = np.zeros((rows, n), np.uint64)
    B = np.zeros(rows, np.uint64)
    mu = g.integers(0, p, size=rows)
    for r in range(rows):
        a = [int(x) for x in g.integers(0, q, size=n, dtype=np.uint64)] if q < 1 << 64 else \
            [int(x) for x in g.integers(0, 1 << 64, size=n, dtype=np.uint64)]
        e = int(np.rint(6.4 * g.standard_normal()))
        A[r] = a
        B[r] = lwe.lwe_encrypt(s, a, int(mu[r]), e, q, p)
    return A, B, mu


def _compress_job(args):
    ck, a, b, q, N = args
    return compress.lwe_compress(ck, a, b, q, N)


@pytest.mark.parametrize("q_bits,n,N_bits,rows", [(64, 40, 1024, 5), (64, 24, 512, 300), (32, 16, 512, 64),
                                                  (11, 200, 256, 9), (27, 30, 512, 17)])
def test_lwe_compress_matches_oracle(native, q_bits, n, N_bits, rows):
    q = Q27 if q_bits == 27 else 1 << q_bits
    p = 16
    log(f"lwe compress: q 2^{q_bits} n {n} N {N_bits} rows {rows}")
    sk = _key(960 + q_bits, N_bits)
    assert sk.pk.N > params.compression_bound(n, q)
    g = np.random.default_rng(q_bits * 1000 + n)
    s = [int(x) for x in g.integers(0, q, size=n, dtype=np.uint64)]
    ck = _enc_key(sk, s, 960 + q_bits)
    A, B, mu = _lwe_batch(g, s, q, p, rows)
    N_limbs, L = _limbs(sk, N_bits)
    dt = np.uint32 if q <= 1 << 32 else np.uint64
    with native.Compressor(n, q, N_limbs, N_bits, ck=wl.ints_to_limbs(ck, L)) as cmp:
        assert cmp.L == L and cmp.windows == (q_bits + 7) // 8
        X = np.zeros((rows, L), np.uint32)
        cmp.compress_lwe(A.astype(dt), B.astype(dt), X)
    got = limbs_rows_to_ints(X)
    with Pool(pool_size()) as pool:
        want = pool.map(_compress_job, [(ck, [int(x) for x in A[r]], int(B[r]), q, sk.pk.N) for r in range(rows)])
    assert got == want
    assert [compress.modified_lwe_decrypt(sk, x, q, p) for x in got] == mu.tolist()


def test_lwe_compress_many_rows_one_wave_each(native):
    # 8192 ciphertexts: one wavefront per ciphertext, no partial products
    q, p, n, N_bits, rows = 1 << 64, 16, 6, 256, 8192
    sk = _key(970, N_bits)
    g = np.random.default_rng(970)
    s = [int(x) for x in g.integers(0, q, size=n, dtype=np.uint64)]
    ck = _enc_key(sk, s, 970)
    A = g.integers(0, 1 << 64, size=(rows, n), dtype=np.uint64)
    A[0] = 0                                   # exponent q - 0 -> 0 for every base
    B = g.integers(0, 1 << 64, size=rows, dtype=np.uint64)
    B[1] = 0
    N_limbs, L = _limbs(sk, N_bits)
    with native.Compressor(n, q, N_limbs, N_bits, ck=wl.ints_to_limbs(ck, L)) as cmp:
        X = np.zeros((rows, L), np.uint32)
        cmp.compress_lwe(A, B, X)
    got = limbs_rows_to_ints(X)
    idx = [0, 1, 2, 4095, rows - 1] + list(range(100, rows, 997))
    for r in idx:
        assert got[r] == compress.lwe_compress(ck, [int(x) for x in A[r]], int(B[r]), q, sk.pk.N), r
    assert got[0] == (1 + int(B[0]) * sk.pk.N) % sk.pk.N ** 2


@pytest.mark.parametrize("rows,n", [(16390, 6), (400, 400)])
def test_lwe_compress_four_items_per_wave(native, rows, n):
    # From 16384 work items (ciphertext x part) on, four share a wavefront (one per 16 lanes):
    # 16390 ciphertexts of one part each, and 400 ciphertexts cut into 41 parts of 9 or 10
    # bases (then reduced in a tree); every ciphertext matches the oracle.
    q, p, N_bits = 1 << 64, 16, 256
    log(f"lwe compress, four items per wave: rows {rows} n {n}")
    sk = _key(975 + n, N_bits)
    g = np.random.default_rng(975 + n)
    s = [int(x) for x in g.integers(0, q, size=n, dtype=np.uint64)]
    ck = _enc_key(sk, s, 975 + n)
    A = g.integers(0, 1 << 64, size=(rows, n), dtype=np.uint64)
    B = g.integers(0, 1 << 64, size=rows, dtype=np.uint64)
    A[0] = 0
    N_limbs, L = _limbs(sk, N_bits)
    with native.Compressor(n, q, N_limbs, N_bits, ck=wl.ints_to_limbs(ck, L)) as cmp:
        X = np.zeros((rows, L), np.uint32)
        cmp.compress_lwe(A, B, X)
    got = limbs_rows_to_ints(X)
    with Pool(pool_size()) as pool:
        want = pool.map(_compress_job, [(ck, [int(x) for x in A[r]], int(B[r]), q, sk.pk.N) for r in range(rows)],
                        chunksize=256)
    assert got == want


def test_table2_parameters(native):
    """Table 2's LWE parameter sets (n, q) = (630, 2^64) and (1305, 2^11) with a 3072-bit
    modulus: two ciphertexts each, bit-exact, and decryption recovers the message."""
    p = 16
    for n, q in ((630, 1 << 64), (1305, 1 << 11)):
        log(f"table 2: n {n} q {q.bit_length() - 1} bits")
        sk = _key(980 + n, 3072)
        g = np.random.default_rng(n)
        s = [int(x) for x in g.integers(0, q, size=n, dtype=np.uint64)]
        with Pool(pool_size()) as pool:
            rs = wl.paillier_randomness(980 + n, 0, n, sk.pk.N)
            ck = pool.starmap(paillier.encrypt, [(sk.pk, s[i], rs[i]) for i in range(n)])
            A, B, mu = _lwe_batch(g, s, q, p, 2)
            N_limbs, L = _limbs(sk, 3072)
            dt = np.uint32 if q <= 1 << 32 else np.uint64
            with native.Compressor(n, q, N_limbs, 3072, ck=wl.ints_to_limbs(ck, L)) as cmp:
                X = np.zeros((2, L), np.uint32)
                cmp.compress_lwe(A.astype(dt), B.astype(dt), X)
            got = limbs_rows_to_ints(X)
            want = pool.map(_compress_job, [(ck, [int(x) for x in A[r]], int(B[r]), q, sk.pk.N) for r in range(2)])
        assert got == want
        assert [compress.modified_lwe_decrypt(sk, x, q, p) for x in got] == mu.tolist()


def test_rlwe_coefficients_match_oracle(native):
    q, p, Nr, N_bits = Q27, 16, 64, 512
    sk = _key(990, N_bits)
    g = np.random.default_rng(990)
    S = [int(x) for x in g.integers(0, q, size=Nr)]
    A = [int(x) for x in g.integers(0, q, size=Nr)]
    E = [int(x) for x in np.rint(6.4 * g.standard_normal(Nr))]
    mu = [int(x) for x in g.integers(0, p, size=Nr)]
    B = compress.rlwe_encrypt(S, mu, A, E, q, p)
    ck = _enc_key(sk, S, 990)
    N_limbs, L = _limbs(sk, N_bits)
    ks = [0, 1, 2, 31, 62, 63, 17]
    with native.Compressor(Nr, q, N_limbs, N_bits, ck=wl.ints_to_limbs(ck, L)) as cmp:
        X = np.zeros((len(ks), L), np.uint32)
        cmp.compress_rlwe(np.array(A, np.uint32), np.array(B, np.uint32), ks, X)
        with pytest.raises(native.ZipPIRError) as ei:
            cmp.compress_rlwe(np.array(A, np.uint32), np.array(B, np.uint32), [Nr], X[:1])
        assert ei.value.status == native.PIR_EINVAL
    got = limbs_rows_to_ints(X)
    for j, k in enumerate(ks):
        assert got[j] == compress.rlwe_compress_coefficient(ck, A, B, k, q, sk.pk.N), k
        assert compress.modified_lwe_decrypt(sk, got[j], q, p) == mu[k]


def test_packed_key(native):
    # Alg. 6 with delta = 2^bitlen(q + n q^2): the device unpacks the key like the oracle, and
    # compression with it decrypts through the packed-key decryption.
    q, p, n, N_bits = 1 << 32, 16, 20, 1024
    sk = _key(995, N_bits)
    N = sk.pk.N
    dbits = params.compression_bound(n, q).bit_length()
    delta = 1 << dbits
    t = compress.packed_digits_per_key(N_bits, delta)
    g = np.random.default_rng(995)
    s = [int(x) for x in g.integers(0, q, size=n, dtype=np.uint64)]
    rs = wl.paillier_randomness(995, 0, -(-n // t), N)
    pck = compress.generate_packed_key(sk.pk, s, delta, t, rs)
    ck = compress.unpack_compression_key(pck, delta, t, n, N)
    N_limbs, L = _limbs(sk, N_bits)
    A, B, mu = _lwe_batch(g, s, q, p, 6)
    with native.Compressor(n, q, N_limbs, N_bits, packed=wl.ints_to_limbs(pck, L), t=t, delta_log2=dbits) as cmp:
        assert limbs_rows_to_ints(cmp.key()) == ck
        X = np.zeros((6, L), np.uint32)
        cmp.compress_lwe(A.astype(np.uint32), B.astype(np.uint32), X)
    got = limbs_rows_to_ints(X)
    assert got == [compress.lwe_compress(ck, [int(x) for x in A[r]], int(B[r]), q, N) for r in range(6)]
    assert [compress.modified_decrypt_packed_key(sk, x, delta, t, q, p) for x in got] == mu.tolist()


def _rlwe_job(args):
    ck, A, B, k, q, N = args
    return compress.rlwe_compress_coefficient(ck, A, B, k, q, N)


def test_rlwe_paper_size(native):
    """RLWE(1024, 27) of Table 2 with a 3072-bit modulus: coefficients 0, 1, N_r - 1 and a random
    one, bit-exact, and each decrypts to its message (Alg. 8 then the modified decryption)."""
    q, p, Nr, N_bits = Q27, 16, 1024, 3072
    log("rlwe paper size: N_r 1024, q 2^27, N 3072 bits")
    sk = _key(1024, N_bits)
    N, N2 = sk.pk.N, sk.pk.N2
    g = np.random.default_rng(1024)
    S = [int(x) for x in g.integers(0, q, size=Nr)]
    A = [int(x) for x in g.integers(0, q, size=Nr)]
    E = [int(x) for x in np.rint(6.4 * g.standard_normal(Nr))]
    mu = [int(x) for x in g.integers(0, p, size=Nr)]
    B = compress.rlwe_encrypt(S, mu, A, E, q, p)
    # Enc(S_i; r) for one r: (1 + S_i N) r^N mod N^2, so r^N is computed once
    r = wl.paillier_randomness(1024, 0, 1, N)[0]
    rN = pow(r, N, N2)
    ck = [(1 + s_i * N) * rN % N2 for s_i in S]
    assert ck[5] == paillier.encrypt(sk.pk, S[5], r)
    ks = [0, 1, Nr - 1, int(g.integers(2, Nr - 1))]
    N_limbs, L = _limbs(sk, N_bits)
    with native.Compressor(Nr, q, N_limbs, N_bits, ck=wl.ints_to_limbs(ck, L)) as cmp:
        X = np.zeros((len(ks), L), np.uint32)
        cmp.compress_rlwe(np.array(A, np.uint32), np.array(B, np.uint32), ks, X)
    got = limbs_rows_to_ints(X)
    with Pool(pool_size()) as pool:
        want = pool.map(_rlwe_job, [(ck, A, B, k, q, N) for k in ks])
    assert got == want
    assert [compress.modified_lwe_decrypt(sk, x, q, p) for x in got] == [mu[k] for k in ks]


def _packed_job(args):
    pk, digits, delta, t, r = args
    return compress.generate_packed_key(pk, digits, delta, t, [r])[0]


def _unpack_job(args):
    # the key entries of packed ciphertext i alone
    pck_i, delta, t, count, N = args
    return compress.unpack_compression_key([pck_i], delta, t, count, N)


@pytest.mark.parametrize("binary", [False, True])
def test_packed_key_table3_size(native, binary):
    """Alg. 6 at Table 3's (630, 2^64) with a 3072-bit modulus: the device's unpacked key equals
    the oracle's entry by entry, and two compressed ciphertexts match the oracle and decrypt
    (binary keys take delta above q + n q, others above q + n q^2)."""
    q, p, n, N_bits = 1 << 64, 16, 630, 3072
    log(f"packed key, table 3 size: n {n} q 2^64 N 3072 bits binary {binary}")
    sk = _key(1630, N_bits)
    N = sk.pk.N
    dbits = (q + n * q * (1 if binary else q)).bit_length()
    delta = 1 << dbits
    t = compress.packed_digits_per_key(N_bits, delta)
    keys = -(-n // t)
    g = np.random.default_rng(1630 + binary)
    s = [int(x) for x in g.integers(0, 2 if binary else q, size=n, dtype=np.uint64)]
    rs = wl.paillier_randomness(1630, int(binary), keys, N)
    N_limbs, L = _limbs(sk, N_bits)
    A, B, mu = _lwe_batch(g, s, q, p, 2)
    with Pool(pool_size()) as pool:
        pck = pool.map(_packed_job, [(sk.pk, s[i * t:(i + 1) * t], delta, t, rs[i]) for i in range(keys)])
        with native.Compressor(n, q, N_limbs, N_bits, packed=wl.ints_to_limbs(pck, L), t=t,
                               delta_log2=dbits) as cmp:
            assert cmp.setup_ms()["unpack_ms"] > 0
            dev_ck = limbs_rows_to_ints(cmp.key())
            X = np.zeros((2, L), np.uint32)
            cmp.compress_lwe(A, B, X)
        ck = sum(pool.map(_unpack_job, [(pck[i], delta, t, min(t, n - i * t), N) for i in range(keys)]), [])
        assert len(ck) == n and dev_ck == ck
        got = limbs_rows_to_ints(X)
        want = pool.map(_compress_job, [(ck, [int(x) for x in A[r]], int(B[r]), q, N) for r in range(2)])
    assert got == want
    assert [compress.modified_decrypt_packed_key(sk, x, delta, t, q, p) for x in got] == mu.tolist()


def test_compressor_errors(native):
    q, n = 1 << 64, 8
    sk = _key(996, 128)                         # 128 bits < q + n q^2
    N_limbs, L = _limbs(sk, 128)
    with pytest.raises(native.ZipPIRError) as ei:
        native.Compressor(n, q, N_limbs, 128, ck=np.ones((n, L), np.uint32))
    assert ei.value.status == native.PIR_EINVAL
    sk = _key(997, 512)
    N_limbs, L = _limbs(sk, 512)
    bad = np.full((n, L), 0xFFFFFFFF, np.uint32)  # not below N^2
    with pytest.raises(native.ZipPIRError) as ei:
        native.Compressor(n, q, N_limbs, 512, ck=bad)
    assert ei.value.status == native.PIR_EINVAL


@pytest.mark.parametrize("N_bits,n,dbits", [(1024, 5, 600), (1024, 130, 9), (2048, 77, 13),
                                            (3072, 30, 138), (4096, 205, 20)])
def test_unpack_chains_every_width(native, N_bits, n, dbits):
    """Alg. 6's unpacking alone, at every limb width of N^2 (64, 128, 192 and 256 words): the
    device's key equals the oracle's entry by entry for uniform packed elements of Z*_(N^2), with
    ragged last groups (n not a multiple of t) and one case of t = 1 (no squarings at all)."""
    sk = _key(2000 + N_bits, N_bits)
    N = sk.pk.N
    delta = 1 << dbits
    t = max(1, compress.packed_digits_per_key(N_bits, delta))
    keys = -(-n // t)
    log(f"unpack chains: N {N_bits} bits, n {n}, delta 2^{dbits}, t {t}, {keys} packed")
    pck = wl.uniform_ciphertexts(2000 + N_bits, dbits, keys, N)
    N_limbs, L = _limbs(sk, N_bits)
    with native.Compressor(n, 1 << 32, N_limbs, N_bits, packed=wl.ints_to_limbs(pck, L), t=t,
                           delta_log2=dbits) as cmp:
        dev_ck = limbs_rows_to_ints(cmp.key())
    with Pool(pool_size()) as pool:
        ck = sum(pool.map(_unpack_job, [(pck[i], delta, t, min(t, n - i * t), N) for i in range(keys)]), [])
    assert len(ck) == n and dev_ck == ck
