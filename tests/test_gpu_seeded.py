"""GPU parity of the silent offline phase (Sec. 4.3, "Lowering offline communication costs",
"Supporting multiple queries"): the server expands a 32-byte seed into each query's random
hint keys ck_r on the device (ChaCha20 of RFC 8439, rejection sampling in Z_{N^2}).  The
expanded keys equal ``oracle.prg`` bit for bit, and a full-protocol round trip that starts
from N and the seed alone recovers the selected column."""
import numpy as np
import pytest

import workload as wl
from oracle import prg, protocol, server
from tests.gpu_util import limbs_rows_to_ints, log
from tests.instances import make_instance

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def native():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_09190_amd import native as nat
    return nat


def _moduli():
    out = []
    for nb in (256, 1024, 2048, 4096):
        pr = wl.paillier_primes(1300, 0, nb)
        out.append((pr.P * pr.Q, nb))
    # N = 2^191 + 13 (not a Paillier modulus, but any odd N of the stated size is accepted): N^2
    # is just above 2^382, so about half the candidates are rejected
    out.append(((1 << 191) + 13, 192))
    return out


@pytest.mark.parametrize("idx", range(5))
def test_seeded_keys_match_oracle(native, idx):
    N, nb = _moduli()[idx]
    rows, cols, n = 8, 16, 7
    log(f"seeded keys: N {nb}-bit")
    g = np.random.default_rng(1301 + idx)
    D = g.integers(0, 256, (rows, cols), dtype=np.uint8)
    A = g.integers(0, 1 << 32, (cols, n), dtype=np.uint32)
    seed = g.bytes(32)
    h = (nb + 31) // 32
    L = 2 * h
    with native.Server(D, A) as srv:
        ids = srv.add_client_seeded(wl.int_to_limbs(N, h), nb, seed, first_query=5, count=3)
        assert len(set(ids)) == 3
        got = []
        for cid in ids:
            K = np.zeros((n, L), np.uint32)
            srv.client_key(cid, 0, n, K)
            got.append(limbs_rows_to_ints(K))
        part = np.zeros((2, L), np.uint32)
        srv.client_key(ids[1], 3, 2, part)
    for i, q in enumerate((5, 6, 7)):
        assert got[i] == prg.random_key(seed, N, n, q), f"query {q}"
    assert limbs_rows_to_ints(part) == got[1][3:5]


def test_seeded_rejects_bad_arguments(native):
    rows, cols, n = 4, 8, 2
    D = np.zeros((rows, cols), np.uint8)
    A = np.zeros((cols, n), np.uint32)
    pr = wl.paillier_primes(1310, 0, 256)
    N = pr.P * pr.Q
    with native.Server(D, A) as srv:
        for count in (0, 4097):
            with pytest.raises(native.ZipPIRError) as ei:
                srv.add_client_seeded(wl.int_to_limbs(N, 8), 256, bytes(32), 0, count)
            assert ei.value.status == native.PIR_EINVAL
        with pytest.raises(native.ZipPIRError) as ei:     # even N
            srv.add_client_seeded(wl.int_to_limbs(N + 1, 8), 256, bytes(32), 0, 1)
        assert ei.value.status == native.PIR_EINVAL
        with pytest.raises(native.ZipPIRError) as ei:     # key range beyond n
            cid = srv.add_client_seeded(wl.int_to_limbs(N, 8), 256, bytes(32), 0, 1)[0]
            srv.client_key(cid, 1, 2, np.zeros((2, 16), np.uint32))
        assert ei.value.status == native.PIR_EINVAL


@pytest.mark.parametrize("n_bits", [1024, 3072])
def test_seeded_full_protocol_round_trip(native, n_bits):
    """The offline message is N and a 32-byte seed (416 bytes at the paper's 3072-bit N); two
    queries from one seed: the hint k of each against the oracle on every row, the online
    offset answer and the Paillier-added response, and the client's extraction."""
    rows, cols, n = 21, 40, 9
    log(f"seeded full protocol: N {n_bits}")
    inst = make_instance(cfg=1320 + n_bits, rows=rows, cols=cols, n=n, n_bits=n_bits, encrypt_secret=False)
    cl = inst.clients[0]
    h = n_bits // 32
    L = 2 * h
    seed = np.random.default_rng(1321).bytes(32)
    N_limbs = wl.int_to_limbs(cl.N, h)
    assert N_limbs.nbytes + len(seed) == n_bits // 8 + 32
    E = server.exponents(server.global_hint(inst.D, inst.A))
    b = server.answer(inst.D, cl.qu)
    with native.Server(inst.D, inst.A) as srv:
        ids = srv.add_client_seeded(N_limbs, n_bits, seed, first_query=0, count=2)
        B = np.zeros((1, rows), np.uint32)
        srv.answer(cl.qu[None, :], B)
        assert np.array_equal(B[0], b)
        for q, cid in enumerate(ids):
            # client side: the same keys from the seed, decrypted at query time
            ckr = prg.random_key(seed, cl.N, n, q)
            pt_r = protocol.random_key_plaintexts(cl.sk, ckr)
            cko = protocol.query_offset(cl.s, pt_r, cl.N)
            srv.hint(cid)
            K = np.zeros((rows, L), np.uint32)
            srv.client_hint(cid, 0, rows, K)
            k_or = server.client_hint(ckr, E, cl.N)
            assert limbs_rows_to_ints(K) == k_or, f"hint of query {q}"
            T = np.zeros((1, rows, h), np.uint32)
            srv.offset_answer([cid], wl.ints_to_limbs(cko, h)[None], B, T)
            t_or = protocol.offset_answer(b, E, cko, cl.N)
            assert limbs_rows_to_ints(T[0]) == t_or
            C = np.zeros((1, rows, L), np.uint32)
            srv.compress_offset([cid], T, C)
            c_gpu = limbs_rows_to_ints(C[0])
            assert c_gpu == [protocol.combine_offset(k_or[j], t_or[j], cl.N) for j in range(rows)]
            assert [protocol.extract_combined(cl.sk, x) for x in c_gpu] == inst.D[:, cl.col].tolist()
