"""GPU parity of the paper's full protocol (Alg. 5 with random hint keys): the online offset
answer t = (b + E.ck_o) mod N and the Paillier-added response c = k (1 + t N) mod N^2.

Every comparison is bit-exact against ``oracle.protocol`` on the same seeded inputs, and the
client's extraction recovers the selected column (ZipPIR correctness theorem).
"""
from multiprocessing import Pool

import numpy as np
import pytest

import workload as wl
from oracle import protocol, server
from tests.gpu_util import client_arrays, limbs_rows_to_ints, log, pool_size
from tests.instances import make_client, make_instance, oracle_client_hint

pytestmark = pytest.mark.gpu

Q32 = 1 << 32


@pytest.fixture(scope="module")
def native():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_09190_amd import native as nat
    return nat


def _decrypt_one(args):
    sk, c = args
    return protocol.random_key_plaintexts(sk, [c])[0]


def _offsets(cl, pool=None):
    """ck_o for a client whose ck holds random ciphertexts (ck_r), and its limb array."""
    if pool is None:
        pt_r = protocol.random_key_plaintexts(cl.sk, cl.ck)
    else:
        pt_r = pool.map(_decrypt_one, [(cl.sk, int(c)) for c in cl.ck])
    cko = protocol.query_offset(cl.s, pt_r, cl.N)
    h = (cl.N.bit_length() + 31) // 32
    return cko, wl.ints_to_limbs(cko, h)


@pytest.mark.parametrize("n_bits,rows,cols,n", [(256, 13, 40, 6), (1024, 70, 96, 70), (2048, 33, 64, 16),
                                                (3072, 20, 48, 9), (4096, 17, 40, 8)])
def test_offset_answer_and_combine(native, n_bits, rows, cols, n):
    log(f"full protocol: N {n_bits} rows {rows} n {n}")
    inst = make_instance(cfg=970 + n_bits, rows=rows, cols=cols, n=n, n_bits=n_bits,
                         encrypt_secret=False, zero_row=rows // 3)
    cl = inst.clients[0]
    N_limbs, ckr, L = client_arrays(cl, n_bits)
    h = L // 2
    cko, CKO = _offsets(cl)
    E = server.exponents(server.global_hint(inst.D, inst.A))
    b = server.answer(inst.D, cl.qu)
    k_or = server.client_hint(cl.ck, E, cl.N)
    t_or = protocol.offset_answer(b, E, cko, cl.N)
    with native.Server(inst.D, inst.A) as srv:
        cid = srv.add_client(N_limbs, n_bits, ckr)
        B = np.zeros((1, rows), np.uint32)
        srv.answer(cl.qu[None, :], B)
        T = np.zeros((1, rows, h), np.uint32)
        srv.offset_answer([cid], CKO[None], B, T)   # computes H on first use
        t_gpu = limbs_rows_to_ints(T[0])
        srv.hint(cid)
        C = np.zeros((1, rows, L), np.uint32)
        srv.compress_offset([cid], T, C)
        c_gpu = limbs_rows_to_ints(C[0])
    assert t_gpu == t_or
    assert c_gpu == [protocol.combine_offset(k_or[j], t_or[j], cl.N) for j in range(rows)]
    want = inst.D[:, cl.col].tolist()
    assert [protocol.extract(cl.sk, k_or[j], t_gpu[j]) for j in range(rows)] == want
    assert [protocol.extract_combined(cl.sk, x) for x in c_gpu] == want


@pytest.mark.parametrize("n_bits", [256, 2048])
def test_offset_many_rows_four_per_wave(native, n_bits):
    # 16390 rows take the four-rows-per-wavefront kernels (one row per 16 lanes) for the hint
    # and the combine, the last wavefront holding two rows; every row matches the oracle.
    rows, cols, n = 16390, 24, 3
    log(f"full protocol, four rows per wavefront: N {n_bits} rows {rows}")
    inst = make_instance(cfg=975 + n_bits, rows=rows, cols=cols, n=n, n_bits=n_bits,
                         encrypt_secret=False, zero_row=rows - 1)
    cl = inst.clients[0]
    N_limbs, ckr, L = client_arrays(cl, n_bits)
    h = L // 2
    cko, CKO = _offsets(cl)
    E = server.exponents(server.global_hint(inst.D, inst.A))
    b = server.answer(inst.D, cl.qu)
    with Pool(pool_size()) as pool:
        k_or = oracle_client_hint(cl.ck, E, cl.N, pool=pool)
    t_or = protocol.offset_answer(b, E, cko, cl.N)
    with native.Server(inst.D, inst.A) as srv:
        cid = srv.add_client(N_limbs, n_bits, ckr)
        srv.hint(cid)
        B = np.zeros((1, rows), np.uint32)
        srv.answer(cl.qu[None, :], B)
        T = np.zeros((1, rows, h), np.uint32)
        srv.offset_answer([cid], CKO[None], B, T)
        C = np.zeros((1, rows, L), np.uint32)
        srv.compress_offset([cid], T, C)
        K = np.zeros((rows, L), np.uint32)
        srv.client_hint(cid, 0, rows, K)
    assert limbs_rows_to_ints(K) == [k_or[j] for j in range(rows)]
    assert limbs_rows_to_ints(T[0]) == t_or
    # combine_offset's (N+1)^t equals 1 + t N mod N^2 (binomial theorem); the closed form
    # keeps 16390 rows of 2048-bit exponents off the CPU, and a few rows use the oracle itself
    N2 = cl.N * cl.N
    c_gpu = limbs_rows_to_ints(C[0])
    assert c_gpu == [k_or[j] * (1 + t_or[j] * cl.N) % N2 for j in range(rows)]
    for j in (0, 1, rows // 2, rows - 2, rows - 1):
        assert c_gpu[j] == protocol.combine_offset(k_or[j], t_or[j], cl.N)


def test_offset_answer_extremes(native):
    # ck_o entries at 0, N - 1 and 2^(32h) - 1 (the largest the layout holds), E rows from an
    # all-zero and an all-255 database row, b at 0 and 2^32 - 1.
    n_bits, rows, cols, n = 2048, 8, 64, 12
    inst = make_instance(cfg=981, rows=rows, cols=cols, n=n, n_bits=n_bits, encrypt_secret=False)
    cl = inst.clients[0]
    N_limbs, ckr, L = client_arrays(cl, n_bits)
    h = L // 2
    D = inst.D.copy()
    D[0] = 0
    D[1] = 255
    E = server.exponents(server.global_hint(D, inst.A))
    cases = [[0] * n, [cl.N - 1] * n, [(1 << (32 * h)) - 1] * n,
             [(1 << (32 * h)) - 1 if k % 2 else cl.N - 1 for k in range(n)]]
    with native.Server(D, inst.A) as srv:
        cid = srv.add_client(N_limbs, n_bits, ckr)
        for cko in cases:
            for bval in (0, Q32 - 1):
                B = np.full((1, rows), bval, np.uint32)
                T = np.zeros((1, rows, h), np.uint32)
                srv.offset_answer([cid], wl.ints_to_limbs(cko, h)[None], B, T)
                assert limbs_rows_to_ints(T[0]) == protocol.offset_answer(B[0], E, cko, cl.N)


def test_offset_batch_of_clients_and_update(native):
    # three clients with their own keys in one call; after a row update the next call
    # rebuilds E from the refreshed H
    n_bits, rows, cols, n = 1024, 40, 80, 10
    inst = make_instance(cfg=982, rows=rows, cols=cols, n=n, n_bits=n_bits, nclients=3, encrypt_secret=False)
    offs = [_offsets(cl) for cl in inst.clients]
    h = (n_bits + 31) // 32
    CKO = np.stack([o[1] for o in offs])
    Q = np.stack([cl.qu for cl in inst.clients])
    idx = np.array([3, 39], np.uint32)
    new = np.random.default_rng(9).integers(0, 256, size=(2, cols), dtype=np.uint8)
    with native.Server(inst.D, inst.A) as srv:
        ids = []
        for cl in inst.clients:
            N_limbs, ckr, _ = client_arrays(cl, n_bits)
            ids.append(srv.add_client(N_limbs, n_bits, ckr))
        B = np.zeros((3, rows), np.uint32)
        srv.answer(Q, B)
        T = np.zeros((3, rows, h), np.uint32)
        srv.offset_answer(ids, CKO, B, T)
        E = server.exponents(server.global_hint(inst.D, inst.A))
        for i, cl in enumerate(inst.clients):
            assert limbs_rows_to_ints(T[i]) == protocol.offset_answer(B[i], E, offs[i][0], cl.N)
        srv.update_rows(idx, new)
        D2 = inst.D.copy()
        D2[idx] = new
        srv.answer(Q, B)
        srv.offset_answer(ids, CKO, B, T)
        E2 = server.exponents(server.global_hint(D2, inst.A))
        for i, cl in enumerate(inst.clients):
            assert limbs_rows_to_ints(T[i]) == protocol.offset_answer(B[i], E2, offs[i][0], cl.N)
        # the combined form needs each client's hint
        C = np.zeros((3, rows, 2 * h), np.uint32)
        with pytest.raises(native.ZipPIRError) as ei:
            srv.compress_offset(ids, T, C)
        assert ei.value.status == native.PIR_ESTALE


def test_offset_full_size(native):
    """1 GiB database, n = 1024, N 2048-bit: t on sampled rows vs the oracle, the combined
    response on the same rows, and the client's extraction of each."""
    import torch
    side, nlwe, nbits = 32768, 1024, 2048
    log("full protocol 1 GiB: database")
    D = wl.database(1, side, side)
    A = wl.lwe_matrix(1, side, nlwe)
    with Pool(pool_size()) as pool:
        log("full protocol 1 GiB: client (random key, 1024 decryptions)")
        cl = make_client(11, 0, A, nbits, encrypt_secret=False)
        cko, CKO = _offsets(cl, pool)
        N_limbs, ckr, L = client_arrays(cl, nbits)
        h = L // 2
        dev = torch.device("cuda:0")
        with native.Server(torch.from_numpy(D).to(dev), torch.from_numpy(A.view(np.int32)).to(dev),
                           stream=torch.cuda.current_stream().cuda_stream) as srv:
            cid = srv.add_client(N_limbs, nbits, ckr)
            log("full protocol 1 GiB: hint")
            srv.hint(cid)
            q = torch.from_numpy(cl.qu.view(np.int32)[None, :].copy()).to(dev)
            B = torch.zeros((1, side), dtype=torch.int32, device=dev)
            Kt = torch.from_numpy(CKO.view(np.int32)[None].copy()).to(dev)
            T = torch.zeros((1, side, h), dtype=torch.int32, device=dev)
            C = torch.zeros((1, side, L), dtype=torch.int32, device=dev)
            log("full protocol 1 GiB: answer, offset answer, combine")
            srv.answer(q, B, native.PATH_MATVEC)
            srv.offset_answer([cid], Kt, B, T)
            srv.compress_offset([cid], T, C)
            srv.sync()
            b = B.cpu().numpy().view(np.uint32)[0]
            Tn = T.cpu().numpy().view(np.uint32)[0]
            Cn = C.cpu().numpy().view(np.uint32)[0]
        g = np.random.default_rng(13)
        rows = sorted(set([0, side - 1, *g.choice(side, 40, replace=False).tolist()]))
        log(f"full protocol 1 GiB: oracle on {len(rows)} rows")
        E = server.exponents(server.global_hint(D, A, rows=rows))
        b_or = server.answer_rows(D, cl.qu, rows)
        assert np.array_equal(b[rows], b_or)
        k_or = oracle_client_hint(cl.ck, E, cl.N, pool=pool)
    for i, j in enumerate(rows):
        t_or = protocol.offset_answer_row(int(b_or[i]), E[i], cko, cl.N)
        assert wl.limbs_to_int(Tn[j]) == t_or, f"t row {j}"
        c_or = protocol.combine_offset(k_or[i], t_or, cl.N)
        assert wl.limbs_to_int(Cn[j]) == c_or, f"c row {j}"
        assert protocol.extract(cl.sk, k_or[i], t_or) == int(D[j, cl.col])
        assert protocol.extract_combined(cl.sk, c_or) == int(D[j, cl.col])


@pytest.mark.parametrize("n_bits,rows,ell", [(1024, 45, 13), (2048, 61, 29)])
def test_packed_full_protocol(native, n_bits, rows, ell):
    """Batched compression in the full protocol: packed offset answers and their Paillier-
    added form against the oracle on every group (ragged last group), and the client's digits
    recover the column on every row."""
    n = 16
    inst = make_instance(cfg=985 + n_bits, rows=rows, cols=48, n=n, n_bits=n_bits, encrypt_secret=False)
    cl = inst.clients[0]
    N_limbs, ckr, L = client_arrays(cl, n_bits)
    h = L // 2
    cko, CKO = _offsets(cl)
    E = server.exponents(server.global_hint(inst.D, inst.A))
    b = server.answer(inst.D, cl.qu)
    k_or = server.client_hint(cl.ck, E, cl.N)
    t_or = protocol.offset_answer(b, E, cko, cl.N)
    with native.Server(inst.D, inst.A) as srv:
        cid = srv.add_client(N_limbs, n_bits, ckr)
        srv.hint(cid)
        srv.set_packing(cid, ell)
        info = srv.packing_info(cid)
        G, gamma = info["groups"], 1 << info["log2_gamma"]
        B = np.zeros((1, rows), np.uint32)
        srv.answer(cl.qu[None, :], B)
        Tg = np.zeros((1, G, h), np.uint32)
        srv.offset_answer_packed([cid], CKO[None], B, Tg)
        Cg = np.zeros((1, G, L), np.uint32)
        srv.compress_offset_packed([cid], Tg, Cg)
        srv.set_packing(cid, 1)
        with pytest.raises(native.ZipPIRError) as ei:
            srv.offset_answer_packed([cid], CKO[None], B, Tg)
        assert ei.value.status == native.PIR_EINVAL
    tg_or = protocol.offset_answer_packed(t_or, ell, gamma, cl.N)
    kg_or = protocol.packed_keys(k_or, ell, gamma, cl.N)
    assert limbs_rows_to_ints(Tg[0]) == tg_or
    assert limbs_rows_to_ints(Cg[0]) == [protocol.combine_offset(x, y, cl.N) for x, y in zip(kg_or, tg_or)]
    got = []
    for g in range(G):
        got += protocol.extract_packed(cl.sk, kg_or[g], tg_or[g], min(ell, rows - g * ell), gamma)
    assert got == inst.D[:, cl.col].tolist()


def test_packed_offset_answer_many_rows(native):
    """16390 rows: the packed offset answer's terms 2^(tj) t mod N take four rows per
    wavefront; every group's t_g matches the oracle (the group keys are not needed for it)."""
    rows, cols, n, n_bits, ell = 16390, 24, 3, 1024, 13
    log(f"packed offset answer, four rows per wavefront: rows {rows}")
    inst = make_instance(cfg=988, rows=rows, cols=cols, n=n, n_bits=n_bits, encrypt_secret=False)
    cl = inst.clients[0]
    N_limbs, ckr, L = client_arrays(cl, n_bits)
    h = L // 2
    cko, CKO = _offsets(cl)
    E = server.exponents(server.global_hint(inst.D, inst.A))
    b = server.answer(inst.D, cl.qu)
    t_or = protocol.offset_answer(b, E, cko, cl.N)
    with native.Server(inst.D, inst.A) as srv:
        cid = srv.add_client(N_limbs, n_bits, ckr)
        srv.hint(cid)
        srv.set_packing(cid, ell)
        info = srv.packing_info(cid)
        G, gamma = info["groups"], 1 << info["log2_gamma"]
        B = np.zeros((1, rows), np.uint32)
        srv.answer(cl.qu[None, :], B)
        Tg = np.zeros((1, G, h), np.uint32)
        srv.offset_answer_packed([cid], CKO[None], B, Tg)
    assert limbs_rows_to_ints(Tg[0]) == protocol.offset_answer_packed(t_or, ell, gamma, cl.N)


@pytest.mark.parametrize("nclients,n_bits,on_device", [(1, 2048, False), (1, 1024, True), (3, 1024, True),
                                                     (2, 256, False)])
def test_answer_offset_one_call(native, nclients, n_bits, on_device):
    """pir_answer_offset: the answer and the offset answer in one call, the contraction on the
    server's second stream beside the answer; B and T equal the oracle on every row (and a row
    update between calls is seen by both). One client takes the one-query form (the matvec's
    per-segment partials summed in the reduction), several the batched answer."""
    rows, cols, n = 150, 300, 12
    log(f"answer_offset: {nclients} clients, N {n_bits}, device {on_device}")
    inst = make_instance(cfg=990 + nclients, rows=rows, cols=cols, n=n, n_bits=n_bits, nclients=nclients,
                         encrypt_secret=False, zero_row=7)
    offs = [_offsets(cl) for cl in inst.clients]
    h = (n_bits + 31) // 32
    CKO = np.ascontiguousarray(np.stack([o[1] for o in offs]))
    Q = np.ascontiguousarray(np.stack([cl.qu for cl in inst.clients]))
    upd = np.array([0, rows - 1], np.uint32)
    new = np.random.default_rng(991).integers(0, 256, size=(2, cols), dtype=np.uint8)
    with native.Server(inst.D, inst.A) as srv:
        ids = []
        for cl in inst.clients:
            N_limbs, ckr, _ = client_arrays(cl, n_bits)
            ids.append(srv.add_client(N_limbs, n_bits, ckr))
        for rnd, D in enumerate((inst.D, None)):
            if rnd == 1:
                srv.update_rows(upd, new)
                D = inst.D.copy()
                D[upd] = new
            if on_device:
                import torch
                dev = torch.device("cuda:0")
                Bt = torch.zeros((nclients, rows), dtype=torch.int32, device=dev)
                Tt = torch.zeros((nclients, rows, h), dtype=torch.int32, device=dev)
                srv.answer_offset(ids, torch.from_numpy(Q.view(np.int32)).to(dev),
                                  torch.from_numpy(CKO.view(np.int32)).to(dev), Bt, Tt)
                srv.sync()
                B = Bt.cpu().numpy().view(np.uint32)
                T = Tt.cpu().numpy().view(np.uint32)
            else:
                B = np.zeros((nclients, rows), np.uint32)
                T = np.zeros((nclients, rows, h), np.uint32)
                srv.answer_offset(ids, Q, CKO, B, T)
            E = server.exponents(server.global_hint(D, inst.A))
            for i, cl in enumerate(inst.clients):
                b = server.answer(D, cl.qu)
                assert np.array_equal(B[i], b), f"answer of client {i}, round {rnd}"
                assert limbs_rows_to_ints(T[i]) == protocol.offset_answer(b, E, offs[i][0], cl.N), \
                    f"offset answer of client {i}, round {rnd}"


@pytest.mark.parametrize("n_bits", [1024, 1100, 2048, 4096])
def test_answer_offset_carry_and_wrap(native, n_bits):
    """Offsets solved so that, before b is added, row j0's offset term is 2^96 - 1 (b's addition
    carries out of the low three limbs, across the lanes that hold them) and row j1's is N - 1
    (adding b wraps past N). Both call forms must still equal the oracle on every row. At 1100
    bits a row is 35 limbs, so rows start off 16-byte boundaries."""
    rows, cols, n = 40, 64, 10
    log(f"answer_offset carry and wrap: N {n_bits}")
    inst = make_instance(cfg=1990 + n_bits, rows=rows, cols=cols, n=n, n_bits=n_bits, encrypt_secret=False)
    cl = inst.clients[0]
    N = cl.N
    h = (n_bits + 31) // 32
    E = server.exponents(server.global_hint(inst.D, inst.A))
    b = server.answer(inst.D, cl.qu)
    j0, j1 = [int(j) for j in np.nonzero(b)[0][:2]]
    rng = np.random.default_rng(1991)
    cko = [int(x) % N for x in rng.integers(0, 1 << 62, size=n)]
    # solve E[j, 0] x0 + E[j, 1] x1 = target_j - sum_{k >= 2} E[j, k] cko_k (mod N) for j0, j1
    rest = [sum(int(E[j, k]) * cko[k] for k in range(2, n)) for j in (j0, j1)]
    r = [((1 << 96) - 1 - rest[0]) % N, (N - 1 - rest[1]) % N]
    a, bb, c, d = int(E[j0, 0]), int(E[j0, 1]), int(E[j1, 0]), int(E[j1, 1])
    inv = pow((a * d - bb * c) % N, -1, N)
    cko[0] = (d * r[0] - bb * r[1]) * inv % N
    cko[1] = (a * r[1] - c * r[0]) * inv % N
    assert sum(int(E[j0, k]) * cko[k] for k in range(n)) % N == (1 << 96) - 1
    assert sum(int(E[j1, k]) * cko[k] for k in range(n)) % N == N - 1
    CKO = wl.ints_to_limbs(cko, h)
    want = protocol.offset_answer(b, E, cko, N)
    assert want[j1] == int(b[j1]) - 1 and want[j0] == (1 << 96) - 1 + int(b[j0])
    with native.Server(inst.D, inst.A) as srv:
        N_limbs, ckr, _ = client_arrays(cl, n_bits)
        cid = srv.add_client(N_limbs, n_bits, ckr)
        B = np.zeros((1, rows), np.uint32)
        T = np.zeros((1, rows, h), np.uint32)
        srv.answer_offset([cid], cl.qu[None], CKO[None], B, T)
        assert np.array_equal(B[0], b)
        assert limbs_rows_to_ints(T[0]) == want, "one call"
        T2 = np.zeros((1, rows, h), np.uint32)
        srv.offset_answer([cid], CKO[None], B, T2)
        assert limbs_rows_to_ints(T2[0]) == want, "two calls"


def test_answer_offset_one_query_many_segments(native):
    """The one-query form of pir_answer_offset on a database of 70000 columns: 18 column
    segments of partial sums, more than one per lane of a row in the reduction that adds them
    into b. B and T equal the oracle on every row."""
    rows, cols, n, n_bits = 40, 70000, 6, 1024
    log(f"answer_offset one query, {cols} columns")
    inst = make_instance(cfg=2990, rows=rows, cols=cols, n=n, n_bits=n_bits, encrypt_secret=False, zero_row=5)
    cl = inst.clients[0]
    h = (n_bits + 31) // 32
    cko, CKO = _offsets(cl)
    E = server.exponents(server.global_hint(inst.D, inst.A))
    b = server.answer(inst.D, cl.qu)
    with native.Server(inst.D, inst.A) as srv:
        N_limbs, ckr, _ = client_arrays(cl, n_bits)
        cid = srv.add_client(N_limbs, n_bits, ckr)
        B = np.zeros((1, rows), np.uint32)
        T = np.zeros((1, rows, h), np.uint32)
        srv.answer_offset([cid], cl.qu[None], CKO[None], B, T)
    assert np.array_equal(B[0], b)
    assert limbs_rows_to_ints(T[0]) == protocol.offset_answer(b, E, cko, cl.N)
