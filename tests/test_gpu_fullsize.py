"""GPU parity at the full sizes, with the launch configuration the benchmark uses.

* 1 GiB database, one query (32768 x 32768 uint8, n = 1024, N 2048-bit): full answer vs the
  oracle on every row; K and c on sampled rows (first, last, a planted zero row and seeded
  random rows) vs the oracle; the client's decryption recovers the column on those rows.
  Packed response at ell = 27 (gamma = 2^75): three groups (first, the zero row's, the short
  last one) vs the oracle, and their decryption recovers the column on every row.
* 1 GiB database, 32 clients: the int8-MFMA batch vs 32 matvecs on every row, vs the oracle
  on sampled rows; the batch-32 combine vs the oracle on sampled rows per client.
* Offline hint and 1% update: H on sampled rows vs the oracle; after replacing 328 rows,
  H and K equal a from-scratch server on the new database (every row), and the rows that
  did not change keep their bytes.
Integer path: all comparisons are bit-exact.
"""
from multiprocessing import Pool

import numpy as np
import pytest

import workload as wl
from oracle import lwe, paillier, server
from tests.gpu_util import client_arrays, limbs_rows_to_ints, log, pool_size
from tests.instances import _hint_row_job, make_client, oracle_client_hint

pytestmark = pytest.mark.gpu

SIDE, NLWE, NBITS = 32768, 1024, 2048
ZERO_ROW = 12345


@pytest.fixture(scope="module")
def native():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_09190_amd import native as nat
    return nat


@pytest.fixture(scope="module")
def big():
    log("fullsize: generating 1 GiB database and A")
    D = wl.database(1, SIDE, SIDE)
    D[ZERO_ROW] = 0
    A = wl.lwe_matrix(1, SIDE, NLWE)
    return D, A


def sample_rows(n_random=60, seed=7):
    g = np.random.default_rng(seed)
    rnd = g.choice(SIDE, size=n_random, replace=False)
    return sorted(set([0, SIDE - 1, ZERO_ROW, *rnd.tolist()]))


def test_c2_one_query_full(native, big):
    import torch
    D, A = big
    with Pool(pool_size()) as pool:
        log("fullsize c2: client keygen + Enc(s) (1024 encryptions)")
        cl = make_client(1, 0, A, NBITS, encrypt_secret=True, pool=pool)
        N_limbs, ck, L = client_arrays(cl, NBITS)
        dev = torch.device("cuda:0")
        with native.Server(torch.from_numpy(D).to(dev), torch.from_numpy(A.view(np.int32)).to(dev),
                           stream=torch.cuda.current_stream().cuda_stream) as srv:
            cid = srv.add_client(N_limbs, NBITS, ck)
            log("fullsize c2: pir_hint (all rows)")
            srv.hint(cid)
            q = torch.from_numpy(cl.qu.view(np.int32)[None, :].copy()).to(dev)
            B = torch.zeros((1, SIDE), dtype=torch.int32, device=dev)
            C = torch.zeros((1, SIDE, L), dtype=torch.int32, device=dev)
            log("fullsize c2: answer + compress")
            srv.answer(q, B, native.PATH_MATVEC)
            srv.compress([cid], B, C)
            srv.sync()
            b_gpu = B.cpu().numpy().view(np.uint32)[0]
            rows = sample_rows()
            K_gpu = np.zeros((SIDE, L), np.uint32)
            srv.client_hint(cid, 0, SIDE, K_gpu)
            C_gpu = C.cpu().numpy().view(np.uint32)[0]
            log("fullsize c2: packed response (ell = ell_max)")
            info = srv.packing_info(cid)
            ell, t = info["ell_max"], info["log2_gamma"]
            assert (t, ell) == (75, 27)
            srv.set_packing(cid, ell)
            G = srv.packing_info(cid)["groups"]
            Cp = torch.zeros((1, G, L), dtype=torch.int32, device=dev)
            srv.compress_packed([cid], B, Cp)
            srv.sync()
            Cp_gpu = Cp.cpu().numpy().view(np.uint32)[0]
            B2 = torch.zeros_like(B)
            srv.answer(q, B2, native.PATH_MFMA)
            srv.sync()
            assert torch.equal(B, B2), "MFMA path differs from the matvec at batch 1"
        log("fullsize c2: oracle answer (all rows)")
        b_or = server.answer(D, cl.qu)
        assert np.array_equal(b_gpu, b_or)
        # the sampled rows, and every row of the three checked packed groups (first, the zero
        # row's, the short last one): K from the oracle for all of them
        pgroups = (0, ZERO_ROW // ell, G - 1)
        grows = [j for g in pgroups for j in range(g * ell, min(SIDE, g * ell + ell))]
        krows = sorted(set(rows) | set(grows))
        log(f"fullsize c2: oracle hint on {len(krows)} rows")
        E = server.exponents(server.global_hint(D, A, rows=krows))
        K_list = oracle_client_hint(cl.ck, E, cl.N, rows=None, pool=pool)
        K_or = {j: K_list[i] for i, j in enumerate(krows)}
    for j in krows:
        assert wl.limbs_to_int(K_gpu[j]) == K_or[j], f"K row {j}"
    for j in rows:
        c_or = server.compress_row(K_or[j], int(b_or[j]), cl.N)
        assert wl.limbs_to_int(C_gpu[j]) == c_or, f"c row {j}"
        mu = paillier.decrypt(cl.sk, c_or)
        assert lwe.pir_extract_value(mu) == int(D[j, cl.col]), f"round trip row {j}"
    assert K_or[ZERO_ROW] == 1
    # packed groups from the oracle's K: every row's digit decrypts to D
    log("fullsize c2: packed groups vs oracle")
    gamma = 1 << t
    for g in pgroups:
        r0, r1 = g * ell, min(SIDE, g * ell + ell)
        Kg = [K_or[j] for j in range(r0, r1)]
        want = server.compress_packed(Kg, b_or[r0:r1], cl.N, ell, gamma)[0]
        assert wl.limbs_to_int(Cp_gpu[g]) == want, f"packed group {g}"
        digits = server.packed_digits(paillier.decrypt(cl.sk, want), r1 - r0, gamma)
        assert [lwe.pir_extract_value(m) for m in digits] == D[r0:r1, cl.col].tolist()


def test_c3_batch32_full(native, big):
    import torch
    D, A = big
    batch = 32
    log("fullsize c3: 32 clients (queries, keys)")
    clients = [make_client(3, c, A, NBITS, encrypt_secret=False) for c in range(batch)]
    Q = np.stack([c.qu for c in clients])
    dev = torch.device("cuda:0")
    with native.Server(torch.from_numpy(D).to(dev), torch.from_numpy(A.view(np.int32)).to(dev),
                       stream=torch.cuda.current_stream().cuda_stream) as srv:
        ids = []
        for c in clients:
            N_limbs, ck, L = client_arrays(c, NBITS)
            ids.append(srv.add_client(N_limbs, NBITS, ck))
        Qt = torch.from_numpy(Q.view(np.int32)).to(dev)
        Bm = torch.zeros((batch, SIDE), dtype=torch.int32, device=dev)
        Bv = torch.zeros_like(Bm)
        log("fullsize c3: MFMA batch and 32 matvecs")
        srv.answer(Qt, Bm, native.PATH_MFMA)
        srv.answer(Qt, Bv, native.PATH_MATVEC)
        srv.sync()
        assert torch.equal(Bm, Bv), "batched MFMA answer differs from 32 matvecs"
        log("fullsize c3: hints for 32 clients")
        for cid in ids:
            srv.hint(cid)
        C = torch.zeros((batch, SIDE, L), dtype=torch.int32, device=dev)
        srv.compress(ids, Bm, C)
        srv.sync()
        B = Bm.cpu().numpy().view(np.uint32)
        rows = sample_rows(n_random=13, seed=9)
        Cs = C.cpu().numpy().view(np.uint32)[:, rows]
        Ks = np.zeros((batch, len(rows), L), np.uint32)
        for ci, cid in enumerate(ids):
            for i, j in enumerate(rows):
                srv.client_hint(cid, j, 1, Ks[ci, i:i + 1])
    log("fullsize c3: oracle on sampled rows")
    B_or = np.stack([server.answer_rows(D, Q[c], rows) for c in range(batch)])
    assert np.array_equal(B[:, rows], B_or)
    H = server.global_hint(D, A, rows=rows)
    E = server.exponents(H)
    jobs = []
    for ci, c in enumerate(clients[:4]):  # Paillier rows of four clients (the others share the kernels)
        jobs.append((ci, c))
    # every sampled row of four clients, and two sampled rows (the first and one more) of each
    # other client: K and c from the oracle, all (client, row) pairs in one pool
    pairs = [(ci, i) for ci, _ in jobs for i in range(len(rows))]
    pairs += [(ci, i) for ci in range(4, batch) for i in (0, 1 + (ci * 7) % (len(rows) - 1))]
    with Pool(pool_size()) as pool:
        K_pairs = pool.map(_hint_row_job, [(clients[ci].ck, E[i], clients[ci].N) for ci, i in pairs])
    for (ci, i), k in zip(pairs, K_pairs):
        c = clients[ci]
        assert wl.limbs_to_int(Ks[ci, i]) == k, f"client {ci} K row {rows[i]}"
        assert wl.limbs_to_int(Cs[ci, i]) == server.compress_row(k, int(B_or[ci, i]), c.N)


def test_c5_hint_and_update(native, big):
    import torch
    D, A = big
    log("fullsize c5: client")
    cl = make_client(5, 0, A, NBITS, encrypt_secret=False)
    N_limbs, ck, L = client_arrays(cl, NBITS)
    upd_rows, upd_new = wl.update_rows(5, SIDE, SIDE, 0.01)
    assert len(upd_rows) == 328
    dev = torch.device("cuda:0")
    D2 = D.copy()
    D2[upd_rows] = upd_new
    with native.Server(torch.from_numpy(D).to(dev), torch.from_numpy(A.view(np.int32)).to(dev),
                       stream=torch.cuda.current_stream().cuda_stream) as srv:
        cid = srv.add_client(N_limbs, NBITS, ck)
        log("fullsize c5: full hint")
        srv.hint(cid)
        H0 = np.zeros((SIDE, NLWE), np.uint32)
        srv.global_hint(0, SIDE, H0)
        K0 = np.zeros((SIDE, L), np.uint32)
        srv.client_hint(cid, 0, SIDE, K0)
        log("fullsize c5: update 328 rows")
        srv.update_rows(upd_rows, upd_new)
        assert srv.stale_rows(cid) == 328
        srv.hint(cid, rows=upd_rows)
        H1 = np.zeros_like(H0)
        srv.global_hint(0, SIDE, H1)
        K1 = np.zeros_like(K0)
        srv.client_hint(cid, 0, SIDE, K1)
    log("fullsize c5: from-scratch server on the updated database")
    with native.Server(torch.from_numpy(D2).to(dev), torch.from_numpy(A.view(np.int32)).to(dev),
                       stream=torch.cuda.current_stream().cuda_stream) as srv2:
        cid2 = srv2.add_client(N_limbs, NBITS, ck)
        srv2.hint(cid2)
        H2 = np.zeros_like(H0)
        srv2.global_hint(0, SIDE, H2)
        K2 = np.zeros_like(K0)
        srv2.client_hint(cid2, 0, SIDE, K2)
    assert np.array_equal(H1, H2) and np.array_equal(K1, K2)
    keep = np.setdiff1d(np.arange(SIDE), upd_rows)
    assert np.array_equal(K1[keep], K0[keep]) and np.array_equal(H1[keep], H0[keep])
    log("fullsize c5: oracle on sampled rows (old and updated)")
    rows = sample_rows(n_random=24, seed=11)
    assert np.array_equal(H0[rows], server.global_hint(D, A, rows=rows))
    urows = sorted(upd_rows[:24].tolist())
    assert np.array_equal(H1[urows], server.global_hint(D2, A, rows=urows))
    E = server.exponents(server.global_hint(D2, A, rows=urows[:16]))
    with Pool(pool_size()) as pool:
        K_or = oracle_client_hint(cl.ck, E, cl.N, pool=pool)
    for i, j in enumerate(urows[:16]):
        assert wl.limbs_to_int(K1[j]) == K_or[i], f"updated K row {j}"


def test_database_above_one_launch(native):
    """A 40000 x 65536 database (2.4 GiB) is streamed in two row chunks per query; every row of
    the matvec and of the batched contraction agrees, and sampled rows on both sides of the
    chunk boundary (row 32768) match the oracle."""
    import torch
    rows, cols = 40000, 65536
    log("chunked: generating 2.4 GiB database")
    D = wl.database(6, rows, cols)
    A = wl.lwe_matrix(6, cols, 4)
    Q = wl.uniform_queries(6, 3, cols)
    dev = torch.device("cuda:0")
    with native.Server(torch.from_numpy(D).to(dev), torch.from_numpy(A.view(np.int32)).to(dev),
                       stream=torch.cuda.current_stream().cuda_stream) as srv:
        Qt = torch.from_numpy(Q.view(np.int32)).to(dev)
        Bm = torch.zeros((3, rows), dtype=torch.int32, device=dev)
        Bv = torch.zeros_like(Bm)
        srv.answer(Qt, Bv, native.PATH_MATVEC)
        srv.answer(Qt, Bm, native.PATH_MFMA)
        srv.sync()
        assert torch.equal(Bm, Bv)
        B = Bv.cpu().numpy().view(np.uint32)
    sample = [0, 1, 32766, 32767, 32768, 32769, 39998, 39999] + list(range(1000, 40000, 4111))
    ref = np.stack([server.answer_rows(D, Q[c], sample) for c in range(3)])
    assert np.array_equal(B[:, sample], ref)
