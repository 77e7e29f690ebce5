"""Pins for the CPU oracle: facts fixed by the paper and by arithmetic, not by the oracle itself.

Each test names what fixes the expected value.  Mutation tests at the end plant plausible
mistakes in the oracle (on the CPU) and check that a pin catches each one.
"""
import math

import numpy as np
import pytest

import workload as wl
from oracle import brute, compress, lwe, paillier, params, protocol, server
from tests.instances import make_instance, oracle_client_hint

Q = 1 << 32


# ----------------------------------------------------------------------------- LWE (Alg. 1)

def test_delta_closed_form():
    # Delta = round(q/p) (Sec. 2.1): q = 2^32, p = 256 gives exactly 2^24.
    assert lwe.delta(Q, 256) == 1 << 24
    assert lwe.delta(100, 8) == 13          # 12.5 rounds up
    assert lwe.delta(97, 8) == 12           # 12.125 rounds down


def test_lwe_round_trip():
    # Alg. 1: decrypting a fresh ciphertext with small error returns the message.
    g = np.random.default_rng(1)
    n, p = 32, 256
    sk = g.integers(0, Q, n)
    for _ in range(50):
        a = g.integers(0, Q, n)
        mu = int(g.integers(0, p))
        e = int(g.integers(-1000, 1000))
        b = lwe.lwe_encrypt(sk, a, mu, e, Q, p)
        assert lwe.lwe_decrypt(sk, a, b, Q, p) == mu
        # the phase is exactly Delta*mu + e mod q
        assert lwe.lwe_phase(sk, a, b, Q) == (lwe.delta(Q, p) * mu + e) % Q


def test_extract_rounding():
    # Alg. 5 Extract: f = round((mu mod q) p / q) mod p.
    D24 = 1 << 24
    for v in (0, 1, 77, 255):
        for e in (-(D24 // 2) + 1, -5, 0, 5, D24 // 2 - 1):
            mu = (v * D24 + e) % Q + 7 * Q         # the integer may exceed q; only mu mod q matters
            assert lwe.pir_extract_value(mu) == v


# ----------------------------------------------------------------------------- Paillier (Sec. 2.1)

def test_paillier_hand_example():
    # Textbook scheme by hand: P=3, Q=5 -> N=15, N^2=225, lambda=lcm(2,4)=4,
    # g^lambda = 16^4 = 65536 = 291*225 + 61, L(61) = 4, mu = 4^-1 mod 15 = 4.
    # Enc(7; 2) = 16^7 * 2^15 mod 225 = 106 * 143 mod 225 = 83.
    sk = paillier.keygen(3, 5)
    assert (sk.pk.N, sk.lam, sk.mu) == (15, 4, 4)
    c = paillier.encrypt(sk.pk, 7, 2)
    assert c == 83
    # Dec(83): 83^4 mod 225 = 196, L(196) = 13, 13*4 mod 15 = 7.
    assert paillier.decrypt(sk, 83) == 7


@pytest.fixture(scope="module")
def key512():
    pr = wl.paillier_primes(99, 0, 512)
    return paillier.keygen(pr.P, pr.Q)


def test_paillier_homomorphisms(key512):
    # Dec(Enc(m)) = m; Dec(c1 c2) = m1 + m2; Dec(c^k) = k m; Dec(c (N+1)^b) = m + b (mod N).
    sk = key512
    pk = sk.pk
    g = wl.rng(99, "paillier_r", 5)
    for _ in range(6):
        m1, m2 = wl.uniform_below(g, pk.N), wl.uniform_below(g, pk.N)
        r1, r2 = wl.uniform_unit(g, pk.N), wl.uniform_unit(g, pk.N)
        k = wl.uniform_below(g, 1 << 32)
        b = wl.uniform_below(g, 1 << 32)
        c1, c2 = paillier.encrypt(pk, m1, r1), paillier.encrypt(pk, m2, r2)
        assert paillier.decrypt(sk, c1) == m1
        assert paillier.decrypt(sk, paillier.add(pk, c1, c2)) == (m1 + m2) % pk.N
        assert paillier.decrypt(sk, paillier.scalar_mul(pk, k, c1)) == k * m1 % pk.N
        assert paillier.decrypt(sk, paillier.add_plain(pk, c1, b)) == (m1 + b) % pk.N


def test_generator_power_closed_form(key512):
    # Binomial theorem: (N+1)^b = 1 + bN mod N^2.
    pk = key512.pk
    for b in (0, 1, 2, 12345, (1 << 32) - 1):
        assert pow(pk.g, b, pk.N2) == (1 + b * pk.N) % pk.N2


def test_paillier_randomness_does_not_matter(key512):
    sk = key512
    pk = sk.pk
    g = wl.rng(99, "paillier_r", 6)
    m = wl.uniform_below(g, pk.N)
    cs = {paillier.encrypt(pk, m, wl.uniform_unit(g, pk.N)) for _ in range(3)}
    assert len(cs) == 3 and all(paillier.decrypt(sk, c) == m for c in cs)


# ----------------------------------------------------------------------------- answer b = D.qu

def test_answer_closed_forms():
    g = np.random.default_rng(3)
    rows, cols = 37, 53
    D = g.integers(0, 256, (rows, cols), dtype=np.uint8)
    # unit vector e_i selects column i
    for i in (0, 17, cols - 1):
        u = np.zeros(cols, np.uint32)
        u[i] = 1
        assert np.array_equal(server.answer(D, u), D[:, i].astype(np.uint32))
    # all-ones query gives the row sums
    assert np.array_equal(server.answer(D, np.ones(cols, np.uint32)), D.sum(axis=1).astype(np.uint32))
    # linearity mod 2^32
    x = g.integers(0, Q, cols, dtype=np.uint32)
    y = g.integers(0, Q, cols, dtype=np.uint32)
    lhs = server.answer(D, (x.astype(np.uint64) + y) .astype(np.uint32))
    rhs = (server.answer(D, x).astype(np.uint64) + server.answer(D, y)) % Q
    assert np.array_equal(lhs, rhs.astype(np.uint32))
    # D = 255, qu = 2^32 - 1 everywhere: b = -255 cols mod 2^32
    b = server.answer(np.full((3, cols), 255, np.uint8), np.full(cols, Q - 1, np.uint32))
    assert np.all(b == (-255 * cols) % Q)
    # qu = 2^31 everywhere: b = (rowsum mod 2) 2^31
    b = server.answer(D, np.full(cols, 1 << 31, np.uint32))
    assert np.array_equal(b, ((D.sum(axis=1) % 2) << 31).astype(np.uint32))


def test_answer_batch_is_columnwise():
    g = np.random.default_rng(4)
    D = g.integers(0, 256, (9, 11), dtype=np.uint8)
    Qm = g.integers(0, Q, (5, 11), dtype=np.uint32)
    B = server.answer_batch(D, Qm)
    for c in range(5):
        assert B[c].tolist() == brute.matvec(D.tolist(), Qm[c].tolist())


def test_answer_rows_vs_brute_and_full_answer():
    # answer_rows (the sampled-row form of b = D.qu that the full-size tests use) against a
    # pure-Python loop per listed row, and against the full answer, for rows listed out of
    # order, repeated, and at both ends; extreme values where every product wraps 2^32.
    g = np.random.default_rng(41)
    rows, cols = 23, 47
    D = g.integers(0, 256, (rows, cols), dtype=np.uint8)
    D[5] = 255
    qu = g.integers(0, Q, cols, dtype=np.uint32)
    qu[:7] = Q - 1
    sel = [22, 0, 5, 5, 13, 0, 22, 1]
    got = server.answer_rows(D, qu, sel)
    assert got.dtype == np.uint32 and got.shape == (len(sel),)
    assert got.tolist() == [brute.matvec([D[j].tolist()], qu.tolist())[0] for j in sel]
    assert np.array_equal(got, server.answer(D, qu)[sel])
    # a single row and the empty selection
    assert server.answer_rows(D, qu, [7]).tolist() == brute.matvec([D[7].tolist()], qu.tolist())
    assert server.answer_rows(D, qu, []).shape == (0,)


# ----------------------------------------------------------------------------- H and E

def test_global_hint_vs_brute_rectangular():
    g = np.random.default_rng(5)
    D = g.integers(0, 256, (7, 13), dtype=np.uint8)
    A = g.integers(0, Q, (13, 5), dtype=np.uint32)
    H = server.global_hint(D, A)
    assert H.shape == (7, 5)
    assert H.tolist() == brute.matmul(D.tolist(), A.tolist())
    assert np.array_equal(server.global_hint(D, A, rows=[6, 0, 3]), H[[6, 0, 3]])


def test_global_hint_identity():
    # A = identity (cols = n) gives H = D.
    g = np.random.default_rng(6)
    D = g.integers(0, 256, (10, 10), dtype=np.uint8)
    assert np.array_equal(server.global_hint(D, np.eye(10, dtype=np.uint32)), D.astype(np.uint32))


def test_exponents():
    H = np.array([[0, 1, 2, Q - 1, 1 << 31]], dtype=np.uint32)
    E = server.exponents(H)
    assert E.tolist() == [[0, Q - 1, Q - 2, 1, 1 << 31]]
    assert np.all((E.astype(np.uint64) + H) % Q == 0)


# ----------------------------------------------------------------------------- K and c

@pytest.fixture(scope="module")
def tiny():
    # rows=cols=8, n=4, N of 96 bits: N > q + n q^2 = 2^32 + 2^66 holds.
    return make_instance(cfg=900, rows=8, cols=8, n=4, n_bits=96, zero_row=5)


def test_tiny_bound(tiny):
    N = tiny.clients[0].N
    assert N.bit_length() == 96
    assert params.compression_ok(N, tiny.n)


def test_hint_matches_brute_force(tiny):
    cl = tiny.clients[0]
    H = server.global_hint(tiny.D, tiny.A)
    E = server.exponents(H)
    K = server.client_hint(cl.ck, E, cl.N)
    Hb = brute.matmul(tiny.D.tolist(), tiny.A.tolist())
    Eb = [[brute.negate(x) for x in row] for row in Hb]
    for j in range(tiny.rows):
        assert K[j] == brute.hint_row(cl.ck, Eb[j], cl.N)
    assert K[5] == 1                          # all-zero row: every exponent is 0


def test_hint_plaintext_is_the_integer_sum(tiny):
    # Proof of Theorem 1: the plaintext sum of E_jk s_k is below N, so Dec returns it exactly.
    cl = tiny.clients[0]
    E = server.exponents(server.global_hint(tiny.D, tiny.A))
    K = server.client_hint(cl.ck, E, cl.N)
    for j in range(tiny.rows):
        assert paillier.decrypt(cl.sk, K[j]) == server.hint_plaintext_row(E[j], cl.s)


def test_compress_closed_form_and_decrypt(tiny):
    cl = tiny.clients[0]
    E = server.exponents(server.global_hint(tiny.D, tiny.A))
    K = server.client_hint(cl.ck, E, cl.N)
    b = server.answer(tiny.D, cl.qu)
    c = server.compress(K, b, cl.N)
    N2 = cl.N * cl.N
    for j in range(tiny.rows):
        assert c[j] == K[j] * (1 + int(b[j]) * cl.N) % N2
        assert c[j] == brute.combine(K[j], int(b[j]), cl.N)
        assert paillier.decrypt(cl.sk, c[j]) == int(b[j]) + server.hint_plaintext_row(E[j], cl.s)


def _round_trip(inst, cl):
    E = server.exponents(server.global_hint(inst.D, inst.A))
    K = server.client_hint(cl.ck, E, cl.N)
    b = server.answer(inst.D, cl.qu)
    c = server.compress(K, b, cl.N)
    return [lwe.pir_extract_value(paillier.decrypt(cl.sk, x)) for x in c]


def test_pir_round_trip_tiny(tiny):
    # ZipPIR correctness (Sec. 4.2): the client recovers the selected column.
    cl = tiny.clients[0]
    assert _round_trip(tiny, cl) == tiny.D[:, cl.col].tolist()


def test_pir_round_trip_small():
    inst = make_instance(cfg=901, rows=24, cols=40, n=8, n_bits=160)
    cl = inst.clients[0]
    # the noise term D.e stays below Delta/2 = 2^23
    assert np.max(np.abs(inst.D.astype(np.int64) @ cl.e)) < 1 << 23
    assert _round_trip(inst, cl) == inst.D[:, cl.col].tolist()


def test_compression_bound_is_needed():
    # Theorem 1's bound: with N far below q + n q^2 the plaintext sum wraps mod N and the
    # client's value mod q is wrong for most rows.
    inst = make_instance(cfg=902, rows=16, cols=16, n=16, n_bits=64)
    cl = inst.clients[0]
    assert not params.compression_ok(cl.N, inst.n)
    got = _round_trip(inst, cl)
    assert sum(int(a != b) for a, b in zip(got, inst.D[:, cl.col].tolist())) >= 8


def test_noise_condition():
    # q/p > 2 p sigma sqrt(2 d0 ln(2/delta)): holds for every database side used here.
    for cols in (256, 16384, 32768, 65536, 131072):
        assert params.zippir_noise_ok(cols)
    assert not params.zippir_noise_ok(1 << 24)


def test_hint_pool_helper(tiny):
    cl = tiny.clients[0]
    E = server.exponents(server.global_hint(tiny.D, tiny.A))
    d = oracle_client_hint(cl.ck, E, cl.N, rows=[3, 1])
    assert d == {3: server.client_hint_row(cl.ck, E[3], cl.N), 1: server.client_hint_row(cl.ck, E[1], cl.N)}


# ----------------------------------------------------------------------------- mutations

def test_mutation_wrong_exponent_sign_is_caught(tiny, monkeypatch):
    # Planted mistake: E = H instead of -H.  The round trip (and Dec(K) identity) must fail.
    cl = tiny.clients[0]
    monkeypatch.setattr(server, "exponents", lambda H: H.copy())
    assert _round_trip(tiny, cl) != tiny.D[:, cl.col].tolist()


def test_mutation_transposed_database_is_caught(monkeypatch):
    g = np.random.default_rng(8)
    D = g.integers(0, 256, (6, 6), dtype=np.uint8)
    orig = server.answer
    monkeypatch.setattr(server, "answer", lambda D, qu, chunk_rows=1024: orig(np.ascontiguousarray(D.T), qu))
    u = np.zeros(6, np.uint32)
    u[2] = 1
    assert not np.array_equal(server.answer(D, u), D[:, 2].astype(np.uint32))


def test_mutation_dropped_plaintext_term_is_caught(tiny, monkeypatch):
    # Planted mistake: the combine forgets the (N+1)^b factor.
    cl = tiny.clients[0]
    monkeypatch.setattr(server, "compress", lambda K, b, N: [int(k) for k in K])
    assert _round_trip(tiny, cl) != tiny.D[:, cl.col].tolist()


def test_mutation_wrong_delta_is_caught(monkeypatch):
    monkeypatch.setattr(lwe, "delta", lambda q, p: q // p + 1)
    # the phase identity of Alg. 1 fails with the wrong scale
    sk = [3, 5]
    b = lwe.lwe_encrypt(sk, [7, 11], 200, 0, Q, 256)
    assert lwe.lwe_phase(sk, [7, 11], b, Q) != (200 << 24) % Q


# ----------------------------------------------------------------------------- workload draws

def test_workload_reproducible_and_primes():
    a = wl.database(7, 5, 9)
    b = wl.database(7, 5, 9)
    assert np.array_equal(a, b) and a.dtype == np.uint8
    pr = wl.paillier_primes(7, 0, 256)
    for p in (pr.P, pr.Q):
        # Fermat test with fixed bases (independent of the generator's Miller-Rabin)
        assert all(pow(base, p - 1, p) == 1 for base in (2, 3, 5, 7, 11, 13))
    assert (pr.P * pr.Q).bit_length() == 256
    idx, new = wl.update_rows(7, 32768, 4)
    assert len(idx) == 328 and len(set(idx.tolist())) == 328 and new.shape == (328, 4)
    cts = wl.uniform_ciphertexts(7, 0, 4, pr.P * pr.Q)
    N2 = (pr.P * pr.Q) ** 2
    assert all(0 < c < N2 and math.gcd(c, pr.P * pr.Q) == 1 for c in cts)


# ----------------------------------------------------------------------------- batched compression (Alg. 3)

@pytest.mark.parametrize("gamma_kind", ["paper", "pow2"])
def test_packed_round_trip(gamma_kind):
    # Theorem 2: with gamma >= q + n q^2 and N > gamma^ell the digits of Dec(c_g) are the
    # per-row plaintexts, and the client recovers the column from each digit.
    inst = make_instance(cfg=903, rows=11, cols=24, n=4, n_bits=384)
    cl = inst.clients[0]
    gmin = server.packing_scale_min(inst.n)
    gamma = gmin if gamma_kind == "paper" else 1 << (gmin - 1).bit_length()
    assert gamma >= gmin
    ell = 1
    while gamma ** (ell + 1) < cl.N:
        ell += 1
    assert ell >= 4 and gamma ** ell < cl.N
    E = server.exponents(server.global_hint(inst.D, inst.A))
    K = server.client_hint(cl.ck, E, cl.N)
    b = server.answer(inst.D, cl.qu)
    cg = server.compress_packed(K, b, cl.N, ell, gamma)
    assert len(cg) == -(-inst.rows // ell)
    rec = []
    for g, c in enumerate(cg):
        digits = server.packed_digits(paillier.decrypt(cl.sk, c), ell, gamma)
        for j in range(min(ell, inst.rows - g * ell)):
            r = g * ell + j
            assert digits[j] == int(b[r]) + server.hint_plaintext_row(E[r], cl.s)
            rec.append(lwe.pir_extract_value(digits[j]))
    assert rec == inst.D[:, cl.col].tolist()


def test_packed_needs_theorem2_bound():
    # gamma^ell >= N: the packed plaintext wraps modulo N and the digits are wrong.
    inst = make_instance(cfg=904, rows=6, cols=16, n=4, n_bits=256)
    cl = inst.clients[0]
    gamma = 1 << 70
    ell = 6                      # 2^420 > N
    E = server.exponents(server.global_hint(inst.D, inst.A))
    K = server.client_hint(cl.ck, E, cl.N)
    b = server.answer(inst.D, cl.qu)
    c = server.compress_packed(K, b, cl.N, ell, gamma)[0]
    digits = server.packed_digits(paillier.decrypt(cl.sk, c), ell, gamma)
    truth = [int(b[r]) + server.hint_plaintext_row(E[r], cl.s) for r in range(6)]
    assert digits != truth


def test_packed_is_power_product_closed_form():
    # With gamma = 2^t the group ciphertext is the Horner fold c = (...((c_last^{2^t}) c_.)^{2^t} ...) c_0.
    N = 1000003 * 1000033
    N2 = N * N
    g = np.random.default_rng(12)
    K = [int(g.integers(1, 1 << 62)) % N2 for _ in range(5)]
    b = [int(x) for x in g.integers(0, 1 << 32, 5)]
    t = 7
    got = server.compress_packed(K, b, N, 5, 1 << t)[0]
    acc = 1
    for j in reversed(range(5)):
        acc = pow(acc, 1 << t, N2) * server.compress_row(K[j], b[j], N) % N2
    assert got == acc


# ----------------------------------------------------------------------------- full protocol (Alg. 5)

def _full_protocol(inst, cl):
    """(E, b, k, pt_r, ck_o, t) for a client whose ck holds random ciphertexts (ck_r)."""
    E = server.exponents(server.global_hint(inst.D, inst.A))
    b = server.answer(inst.D, cl.qu)
    k = server.client_hint(cl.ck, E, cl.N)
    pt_r = protocol.random_key_plaintexts(cl.sk, cl.ck)
    cko = protocol.query_offset(cl.s, pt_r, cl.N)
    t = protocol.offset_answer(b, E, cko, cl.N)
    return E, b, k, pt_r, cko, t


@pytest.fixture(scope="module")
def full_small():
    # ck_r: uniform elements of Z*_{N^2} (Alg. 5 Setup samples the random key uniformly)
    return make_instance(cfg=905, rows=20, cols=32, n=6, n_bits=192, encrypt_secret=False)


def test_full_protocol_round_trip(full_small):
    # ZipPIR correctness theorem: from (k_j, t_j), and from the Sec. 4.3 combined ciphertext,
    # the client recovers the selected column on every row.
    inst = full_small
    cl = inst.clients[0]
    E, b, k, pt_r, cko, t = _full_protocol(inst, cl)
    want = inst.D[:, cl.col].tolist()
    assert [protocol.extract(cl.sk, k[j], t[j]) for j in range(inst.rows)] == want
    c = [protocol.combine_offset(k[j], t[j], cl.N) for j in range(inst.rows)]
    assert [protocol.extract_combined(cl.sk, x) for x in c] == want


def test_full_protocol_identity(full_small):
    # Appendix proof of correctness: t_j + Dec(k_j) = b_j + sum_k E_jk s_k mod N, and the
    # right side is an integer below N (Theorem 1's bound), so equality holds over Z.
    inst = full_small
    cl = inst.clients[0]
    E, b, k, pt_r, cko, t = _full_protocol(inst, cl)
    assert all(0 <= x < cl.N for x in cko)
    for j in range(inst.rows):
        lhs = (t[j] + paillier.decrypt(cl.sk, k[j])) % cl.N
        assert lhs == int(b[j]) + server.hint_plaintext_row(E[j], cl.s)
        # the combined form decrypts to the same value (Paillier addition, randomness 1)
        assert paillier.decrypt(cl.sk, protocol.combine_offset(k[j], t[j], cl.N)) == lhs
        assert protocol.combine_offset(k[j], t[j], cl.N) == brute.combine(k[j], t[j], cl.N)


def test_offset_answer_brute_and_closed_forms(full_small):
    inst = full_small
    cl = inst.clients[0]
    N = cl.N
    E = server.exponents(server.global_hint(inst.D, inst.A))
    b = server.answer(inst.D, cl.qu)
    g = np.random.default_rng(21)
    cko = [wl.uniform_below(g, N) for _ in range(inst.n)]
    t = protocol.offset_answer(b, E, cko, N)
    for j in range(inst.rows):
        assert t[j] == brute.offset_row(int(b[j]), E[j].tolist(), cko, N)
    # ck_o = 0: t = b; ck_o = unit vector at k: t_j = b_j + E_jk; ck_o = N - 1 everywhere:
    # t_j = b_j - sum_k E_jk mod N
    assert protocol.offset_answer(b, E, [0] * inst.n, N) == [int(x) for x in b]
    for kk in (0, inst.n - 1):
        u = [0] * inst.n
        u[kk] = 1
        assert protocol.offset_answer(b, E, u, N) == [int(b[j]) + int(E[j, kk]) for j in range(inst.rows)]
    assert protocol.offset_answer(b, E, [N - 1] * inst.n, N) == \
        [(int(b[j]) - int(E[j].astype(np.int64).sum())) % N for j in range(inst.rows)]
    # listed rows come back in the given order
    assert protocol.offset_answer(b, E, cko, N, rows=[7, 2]) == [t[7], t[2]]


def test_mutation_offset_sign_is_caught(full_small, monkeypatch):
    # Planted mistake: ck_o = s + pt_r instead of s - pt_r.
    inst = full_small
    cl = inst.clients[0]
    monkeypatch.setattr(protocol, "query_offset", lambda s, pt, N: [(int(x) + int(p)) % N for x, p in zip(s, pt)])
    E, b, k, pt_r, cko, t = _full_protocol(inst, cl)
    got = [protocol.extract(cl.sk, k[j], t[j]) for j in range(inst.rows)]
    assert got != inst.D[:, cl.col].tolist()


def test_mutation_offset_without_answer_is_caught(full_small, monkeypatch):
    # Planted mistake: the response drops the LWE answer b.
    inst = full_small
    cl = inst.clients[0]
    orig = protocol.offset_answer_row
    monkeypatch.setattr(protocol, "offset_answer_row", lambda b_j, e, c, N: orig(0, e, c, N))
    E, b, k, pt_r, cko, t = _full_protocol(inst, cl)
    got = [protocol.extract(cl.sk, k[j], t[j]) for j in range(inst.rows)]
    assert got != inst.D[:, cl.col].tolist()


# ----------------------------------------------------------------------------- sizes the paper prints

def _golden(name):
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", name)
    rows = []
    for line in open(path):
        line = line.split("#")[0].strip()
        if line:
            rows.append(line.split())
    return rows


def test_table2_single_compression_sizes():
    # Table 2: one 3072-bit Paillier ciphertext (768 B) against (n + 1) log2 q bits.
    rows = _golden("table2_single_compression.txt")
    assert len(rows) == 8
    for n, logq, comp, unc_kb, red in rows:
        n, logq = int(n), int(logq)
        assert params.additive_ciphertext_bits(3072) // 8 == int(comp)
        assert round(params.lwe_ciphertext_bits(n, logq) / 8 / 1000, 2) == float(unc_kb)
        assert abs(100 * params.size_reduction(n, logq, 3072) - float(red)) <= 0.01


def test_table3_packed_key_sizes():
    # Table 3: ceil(n / floor(3072 / log2 delta)) ciphertexts of 768 B, in KiB, rounded.
    rows = _golden("table3_packed_keys.txt")
    assert len(rows) == 4
    for n, logq, nb_kb, b_kb in rows:
        n, q = int(n), 1 << int(logq)
        for binary, want in ((False, int(nb_kb)), (True, int(b_kb))):
            kib = params.packed_key_ciphertexts(n, q, 3072, binary) * 768 / 1024
            assert abs(kib - want) <= 0.5, (n, binary, kib, want)


def test_packing_count_matches_sec_3_3():
    # Sec. 3.3: floor(log2 m / log2 (q + n q^2)) ciphertexts per additive plaintext; the power
    # of two used by the packed response never packs more than that.
    for n in (256, 1024, 1400):
        gmin = server.packing_scale_min(n)
        t = (gmin - 1).bit_length()
        for N_bits in (1024, 2048, 3072, 4096):
            assert (N_bits - 1) // t <= params.pack_count(N_bits, gmin)


# ----------------------------------------------------------------------------- standalone compression (Sec. 3)

def _key(cfg, bits):
    pr = wl.paillier_primes(cfg, 0, bits)
    return paillier.keygen(pr.P, pr.Q)


def _lwe_cts(g, s, q, p, count):
    n = len(s)
    cts = []
    for _ in range(count):
        a = [int(x) for x in g.integers(0, q, size=n, dtype=np.uint64)]
        mu = int(g.integers(0, p))
        e = int(np.rint(6.4 * g.standard_normal()))
        b = lwe.lwe_encrypt(s, a, mu, e, q, p)
        cts.append((a, b, mu))
    return cts


def test_lwe_compress_round_trip_q64():
    # Theorem 1 at the Table 2 modulus q = 2^64: Dec(x) is the integer b + sum (q - a_i) s_i
    # and ModifiedLWEDecrypt returns the LWE plaintext.
    q, p, n = 1 << 64, 16, 12
    sk = _key(950, 512)
    g = np.random.default_rng(50)
    s = [int(x) for x in g.integers(0, q, size=n, dtype=np.uint64)]
    rs = wl.paillier_randomness(950, 0, n, sk.pk.N)
    ck = [paillier.encrypt(sk.pk, s[i], rs[i]) for i in range(n)]
    assert sk.pk.N > params.compression_bound(n, q)
    for a, b, mu in _lwe_cts(g, s, q, p, 8):
        x = compress.lwe_compress(ck, a, b, q, sk.pk.N)
        assert paillier.decrypt(sk, x) == compress.lwe_phase_plaintext(a, b, s, q)
        assert compress.modified_lwe_decrypt(sk, x, q, p) == mu == lwe.lwe_decrypt(s, a, b, q, p)
        # the closed form of Alg. 2 by brute force
        assert x == brute.combine(1, b, sk.pk.N) * math.prod(
            brute.modexp(c, (q - ai) % q, sk.pk.N ** 2) for c, ai in zip(ck, a)) % sk.pk.N ** 2


def test_lwe_compress_binary_key_corollary():
    # Corollary of Theorem 1: a binary key needs only m > q + n q; with a uniform key the same
    # small modulus wraps and decryption fails.
    q, p, n = 1 << 64, 16, 12
    sk = _key(951, 96)
    N = sk.pk.N
    assert q + n * q < N < params.compression_bound(n, q)
    g = np.random.default_rng(51)
    s_bin = [int(x) for x in g.integers(0, 2, size=n)]
    rs = wl.paillier_randomness(951, 0, n, N)
    ck = [paillier.encrypt(sk.pk, s_bin[i], rs[i]) for i in range(n)]
    for a, b, mu in _lwe_cts(g, s_bin, q, p, 8):
        assert compress.modified_lwe_decrypt(sk, compress.lwe_compress(ck, a, b, q, N), q, p) == mu
    s_uni = [int(x) for x in g.integers(0, q, size=n, dtype=np.uint64)]
    ck_u = [paillier.encrypt(sk.pk, s_uni[i] % N, rs[i]) for i in range(n)]
    bad = sum(compress.modified_lwe_decrypt(sk, compress.lwe_compress(ck_u, a, b, q, N), q, p) != mu
              for a, b, mu in _lwe_cts(g, s_uni, q, p, 8))
    assert bad >= 4


def test_packed_key_round_trip():
    # Alg. 6: unpacked keys scale the phase by delta^(t-1); the packed-key decryption recovers
    # the plaintext when delta is a power of two above q + n q^2 (so q divides it) and
    # t = floor(0.5 log2 m / log2 delta).
    q, p, n = 1 << 32, 16, 20
    sk = _key(952, 1024)
    N = sk.pk.N
    delta = 1 << params.compression_bound(n, q).bit_length()
    t = compress.packed_digits_per_key(1024, delta)
    assert t == 7 and delta ** (2 * t - 1) < N
    g = np.random.default_rng(52)
    s = [int(x) for x in g.integers(0, q, size=n, dtype=np.uint64)]
    rs = wl.paillier_randomness(952, 0, -(-n // t), N)
    pck = compress.generate_packed_key(sk.pk, s, delta, t, rs)
    assert len(pck) == 3
    ck = compress.unpack_compression_key(pck, delta, t, n, N)
    # plaintext of ck[it+j] is delta^-j sum_l s[it+l] delta^l mod N
    for k in range(n):
        i, j = divmod(k, t)
        want = sum(s[i * t + l] * delta ** l for l in range(t) if i * t + l < n) * pow(delta, -j, N) % N
        assert paillier.decrypt(sk, ck[k]) == want
    ok = 0
    for a, b, mu in _lwe_cts(g, s, q, p, 10):
        x = compress.lwe_compress(ck, a, b, q, N)
        assert compress.modified_decrypt_packed_key(sk, x, delta, t, q, p) == mu
        ok += compress.modified_lwe_decrypt(sk, x, q, p) == mu
    assert ok <= 5, "the packed key must change the decryption"


def test_packed_key_needs_half_width():
    # With t twice as large (floor(log2 m / log2 delta)) the digits above delta^(t-1) wrap
    # modulo m and the packed-key decryption fails for most ciphertexts.
    q, p, n = 1 << 32, 16, 28
    sk = _key(953, 1024)
    N = sk.pk.N
    delta = 1 << params.compression_bound(n, q).bit_length()
    t = 2 * compress.packed_digits_per_key(1024, delta)
    assert delta ** (2 * t - 1) > N
    g = np.random.default_rng(53)
    s = [int(x) for x in g.integers(0, q, size=n, dtype=np.uint64)]
    rs = wl.paillier_randomness(953, 0, -(-n // t), N)
    ck = compress.unpack_compression_key(compress.generate_packed_key(sk.pk, s, delta, t, rs), delta, t, n, N)
    bad = sum(compress.modified_decrypt_packed_key(sk, compress.lwe_compress(ck, a, b, q, N), delta, t, q, p) != mu
              for a, b, mu in _lwe_cts(g, s, q, p, 10))
    assert bad >= 5


def test_negacyclic_product_closed_form():
    # X^Nr = -1: the product by X shifts and negates the top coefficient; numpy convolution
    # folded at Nr gives the same product.
    q, Nr = 1 << 32, 8
    g = np.random.default_rng(54)
    A = [int(x) for x in g.integers(0, q, size=Nr, dtype=np.uint64)]
    X = [0, 1] + [0] * (Nr - 2)
    assert compress.negacyclic_mul(A, X, q) == [(q - A[-1]) % q] + A[:-1]
    S = [int(x) for x in g.integers(0, q, size=Nr, dtype=np.uint64)]
    full = [0] * (2 * Nr - 1)
    for i in range(Nr):
        for j in range(Nr):
            full[i + j] += A[i] * S[j]
    folded = [(full[k] - (full[k + Nr] if k + Nr < 2 * Nr - 1 else 0)) % q for k in range(Nr)]
    assert compress.negacyclic_mul(A, S, q) == folded


def test_rlwe_coefficient_compression():
    # Alg. 8 and the extracted LWE ciphertext agree, and both decrypt to coefficient k of the
    # RLWE plaintext (Theorem of appendix B; needs m > q + Nr q^2).
    q, p, Nr = 1 << 32, 16, 16
    sk = _key(955, 512)
    N = sk.pk.N
    assert N > params.compression_bound(Nr, q)
    g = np.random.default_rng(55)
    S = [int(x) for x in g.integers(0, q, size=Nr, dtype=np.uint64)]
    A = [int(x) for x in g.integers(0, q, size=Nr, dtype=np.uint64)]
    E = [int(x) for x in np.rint(6.4 * g.standard_normal(Nr))]
    mu = [int(x) for x in g.integers(0, p, size=Nr)]
    B = compress.rlwe_encrypt(S, mu, A, E, q, p)
    rs = wl.paillier_randomness(955, 0, Nr, N)
    ck = [paillier.encrypt(sk.pk, S[i], rs[i]) for i in range(Nr)]
    for k in (0, 1, Nr // 2, Nr - 1):
        x = compress.rlwe_compress_coefficient(ck, A, B, k, q, N)
        a, b = compress.rlwe_extract_lwe(A, B, k, q)
        assert x == compress.lwe_compress(ck, a, b, q, N)
        assert lwe.lwe_phase(S, a, b, q) == (B[k] - compress.negacyclic_mul(A, S, q)[k]) % q
        assert compress.modified_lwe_decrypt(sk, x, q, p) == mu[k] == compress.rlwe_decrypt_coefficient(S, A, B, k, q, p)


@pytest.fixture(scope="module")
def full_wide():
    # 640-bit N: room for up to 9 packed rows of 67 bits
    return make_instance(cfg=906, rows=20, cols=32, n=6, n_bits=640, encrypt_secret=False)


@pytest.mark.parametrize("ell", [3, 7])
def test_full_protocol_packed_round_trip(full_wide, ell):
    # Batched compression in the full protocol: per group, t_g + Dec(k_g) is the base-gamma
    # number whose digits are the rows' plaintexts b_j + E_j.s (Theorem 2), so the client
    # recovers every row, the short last group included; the combined form decrypts the same.
    inst = full_wide
    cl = inst.clients[0]
    E, b, k, pt_r, cko, t = _full_protocol(inst, cl)
    gamma = 1 << (server.packing_scale_min(inst.n) - 1).bit_length()
    assert gamma ** ell < cl.N
    tg = protocol.offset_answer_packed(t, ell, gamma, cl.N)
    kg = protocol.packed_keys(k, ell, gamma, cl.N)
    assert len(tg) == len(kg) == -(-inst.rows // ell)
    got = []
    for g, (x, y) in enumerate(zip(kg, tg)):
        r0 = g * ell
        nj = min(ell, inst.rows - r0)
        mu = (y + paillier.decrypt(cl.sk, x)) % cl.N
        assert mu == sum(gamma ** j * (int(b[r0 + j]) + server.hint_plaintext_row(E[r0 + j], cl.s))
                         for j in range(nj))
        got += protocol.extract_packed(cl.sk, x, y, nj, gamma)
        c = protocol.combine_offset(x, y, cl.N)
        assert paillier.decrypt(cl.sk, c) == mu
    assert got == inst.D[:, cl.col].tolist()
