"""GPU parity at the limits the C-ABI accepts, against the oracle, every compared element
bit-exact:

* pir_answer with batches of 33, 64, 100 and 1024 queries: more than one 32-query column block
  of the int8-MFMA contraction, with column-major answers, on a ragged database (every row);
* pir_offset_answer with batches of 4, 37 and 128 clients, including 4096-bit moduli, where
  the operand has 128 x 516 columns;
* the offset answer at its largest n (16384) and batch (128), where the operand spans more
  than 2^31 bytes;
* H = D.A with 4 n pitch above 2^31, where the contraction's operand offsets pass 2^31.
"""
import numpy as np
import pytest

import workload as wl
from oracle import protocol, server
from tests.gpu_util import client_arrays, limbs_rows_to_ints, log
from tests.instances import make_client, make_instance

pytestmark = pytest.mark.gpu

Q32 = 1 << 32


@pytest.fixture(scope="module")
def native():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_09190_amd import native as nat
    return nat


def _rand(seed, shape, hi, dtype):
    return np.random.default_rng(seed).integers(0, hi, size=shape, dtype=dtype)


@pytest.mark.parametrize("batch", [33, 64, 100, 1024])
def test_answer_large_batches(native, batch):
    rows, cols = 301, 700
    log(f"answer batch {batch}")
    D = _rand(100, (rows, cols), 256, np.uint8)
    A = _rand(101, (cols, 4), Q32, np.uint32)
    Qm = _rand(102 + batch, (batch, cols), Q32, np.uint32)
    Qm[0] = Q32 - 1      # extremes in the first and last query
    Qm[-1] = 0
    want = server.answer_batch(D, Qm)
    with native.Server(D, A) as srv:
        B = np.zeros((batch, rows), np.uint32)
        srv.answer(Qm, B)                       # PIR_PATH_AUTO: the contraction
        assert np.array_equal(B, want)
        B[:] = 0
        srv.answer(Qm, B, native.PATH_MATVEC)
        assert np.array_equal(B, want)
        if batch == 100:                        # row-major D as well as the tiled copy
            srv.set_tiled_copy(False)
            B[:] = 0
            srv.answer(Qm, B, native.PATH_MFMA)
            assert np.array_equal(B, want)


def _offsets(cl):
    pt_r = protocol.random_key_plaintexts(cl.sk, cl.ck)
    cko = protocol.query_offset(cl.s, pt_r, cl.N)
    h = (cl.N.bit_length() + 31) // 32
    return cko, wl.ints_to_limbs(cko, h)


@pytest.mark.parametrize("batch", [4, 37, 128])
def test_offset_answer_batches(native, batch):
    """batch clients with their own keys (256-bit N), one call: t of every row of every
    client against the oracle, and the extraction recovers each client's column."""
    rows, cols, n, nb = 45, 64, 6, 256
    log(f"offset answer batch {batch}")
    inst = make_instance(cfg=1100 + batch, rows=rows, cols=cols, n=n, n_bits=nb, nclients=batch,
                         encrypt_secret=False)
    offs = [_offsets(cl) for cl in inst.clients]
    h = (nb + 31) // 32
    CKO = np.stack([o[1] for o in offs])
    Q = np.stack([cl.qu for cl in inst.clients])
    E = server.exponents(server.global_hint(inst.D, inst.A))
    with native.Server(inst.D, inst.A) as srv:
        ids = []
        for cl in inst.clients:
            N_limbs, ckr, _ = client_arrays(cl, nb)
            ids.append(srv.add_client(N_limbs, nb, ckr))
        B = np.zeros((batch, rows), np.uint32)
        srv.answer(Q, B)
        T = np.zeros((batch, rows, h), np.uint32)
        srv.offset_answer(ids, CKO, B, T)
    B_or = server.answer_batch(inst.D, Q)
    assert np.array_equal(B, B_or)
    for i, cl in enumerate(inst.clients):
        t_or = protocol.offset_answer(B_or[i], E, offs[i][0], cl.N)
        assert limbs_rows_to_ints(T[i]) == t_or, f"client {i}"
    k_or = server.client_hint(inst.clients[-1].ck, E, inst.clients[-1].N)
    t_last = limbs_rows_to_ints(T[-1])
    assert [protocol.extract(inst.clients[-1].sk, k_or[j], t_last[j]) for j in range(rows)] == \
        inst.D[:, inst.clients[-1].col].tolist()


def test_offset_answer_batch_128_wide_moduli(native):
    """128 offset vectors of a 4096-bit modulus in one call (the packed operand has 66048
    columns): t of every row of every client against the oracle.  The offsets are uniform
    below 2^(32 h), the largest values the layout takes."""
    rows, cols, n, nb, batch = 20, 48, 4, 4096, 128
    log("offset answer batch 128, N 4096")
    inst = make_instance(cfg=1130, rows=rows, cols=cols, n=n, n_bits=nb, encrypt_secret=False)
    cl = inst.clients[0]
    h = nb // 32
    g = np.random.default_rng(1131)
    CKO = g.integers(0, Q32, size=(batch, n, h), dtype=np.uint32)
    B = g.integers(0, Q32, size=(batch, rows), dtype=np.uint32)
    E = server.exponents(server.global_hint(inst.D, inst.A))
    N_limbs, ckr, _ = client_arrays(cl, nb)
    with native.Server(inst.D, inst.A) as srv:
        cid = srv.add_client(N_limbs, nb, ckr)
        T = np.zeros((batch, rows, h), np.uint32)
        srv.offset_answer([cid] * batch, CKO, B, T)
    for i in range(batch):
        cko = [wl.limbs_to_int(CKO[i, k]) for k in range(n)]
        assert limbs_rows_to_ints(T[i]) == protocol.offset_answer(B[i], E, cko, cl.N), f"vector {i}"


def test_offset_answer_largest_n_and_batch(native):
    """n = 16384 and 128 offset vectors of a 2048-bit modulus: the packed operand holds
    128 x 260 columns of 65536 bytes (2.2 GB, offsets past 2^31).  Vectors 0, 63, 126 and 127
    (the last two start beyond byte 2^31 of the operand) against the oracle on every row."""
    import torch
    rows, cols, n, nb, batch = 16, 16, 16384, 2048, 128
    log("offset answer n 16384 batch 128: instance")
    D = _rand(1140, (rows, cols), 256, np.uint8)
    A = _rand(1141, (cols, n), Q32, np.uint32)
    pr = wl.paillier_primes(1142, 0, nb)
    N = pr.P * pr.Q
    h = nb // 32
    ckr = wl.ints_to_limbs(wl.uniform_ciphertexts(1142, 0, n, N), 2 * h)
    g = np.random.default_rng(1143)
    CKO = g.integers(0, Q32, size=(batch, n, h), dtype=np.uint32)
    B = g.integers(0, Q32, size=(batch, rows), dtype=np.uint32)
    dev = torch.device("cuda:0")
    with native.Server(D, A) as srv:
        cid = srv.add_client(wl.int_to_limbs(N, h), nb, ckr)
        Kt = torch.from_numpy(CKO.view(np.int32)).to(dev)
        Bt = torch.from_numpy(B.view(np.int32)).to(dev)
        Tt = torch.zeros((batch, rows, h), dtype=torch.int32, device=dev)
        log("offset answer n 16384 batch 128: GPU")
        srv.offset_answer([cid] * batch, Kt, Bt, Tt)
        srv.sync()
        T = Tt.cpu().numpy().view(np.uint32)
    E = server.exponents(server.global_hint(D, A))
    for i in (0, 63, 126, 127):
        cko = [wl.limbs_to_int(CKO[i, k]) for k in range(n)]
        assert limbs_rows_to_ints(T[i]) == protocol.offset_answer(B[i], E, cko, N), f"vector {i}"


def test_global_hint_operand_beyond_2gib(native):
    """H = D.A with cols 65536 and n 8256: the four byte planes of A take 4 n pitch = 2.16 GB,
    so plane offsets of the last columns pass 2^31.  Rows 0, 9, 19 on sampled columns
    (the first, the last 64 and seeded ones) against the oracle."""
    rows, cols, n, nb = 20, 65536, 8256, 256
    log("global hint beyond 2 GiB: instance")
    D = _rand(1150, (rows, cols), 256, np.uint8)
    A = wl.lwe_matrix(1150, cols, n)
    pr = wl.paillier_primes(1151, 0, nb)
    N = pr.P * pr.Q
    ck = wl.ints_to_limbs(wl.uniform_ciphertexts(1151, 0, n, N), 16)
    with native.Server(D, A) as srv:
        cid = srv.add_client(wl.int_to_limbs(N, 8), nb, ck)
        log("global hint beyond 2 GiB: GPU")
        srv.hint(cid, rows=[0])          # brings every row of H up to date
        H = np.zeros((rows, n), np.uint32)
        srv.global_hint(0, rows, H)
    ks = sorted(set([0, 1, *range(n - 64, n), *np.random.default_rng(1152).choice(n, 32, replace=False).tolist()]))
    sel = [0, 9, 19]
    want = server.global_hint(D, np.ascontiguousarray(A[:, ks]), rows=sel)
    assert np.array_equal(H[np.ix_(sel, ks)], want)
