"""GPU parity of the packed response (batched compression, Alg. 3 in the combined form of
Sec. 4.3, with gamma = 2^t, t = 64 + bitlen(n)).

Each group of ell rows becomes one ciphertext C_g = prod_j c_{g ell + j}^(gamma^j) mod N^2.
The GPU result is compared bit for bit with ``oracle.server.compress_packed`` on every group
(ragged last group included), and the client's decryption of each C_g splits into base-gamma
digits that recover the selected column of every row (Theorem 2).
"""
import numpy as np
import pytest

import workload as wl
from oracle import lwe, paillier, server
from tests.gpu_util import client_arrays, limbs_rows_to_ints, log
from tests.instances import make_instance

pytestmark = pytest.mark.gpu

Q32 = 1 << 32


@pytest.fixture(scope="module")
def native():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_09190_amd import native as nat
    return nat


def _t_for(n):
    return 64 + int(n).bit_length()


def _check_groups(cl, D, K_or, b, ell, t, got):
    gamma = 1 << t
    assert got == server.compress_packed(K_or, b, cl.N, ell, gamma)
    for g, c in enumerate(got):
        r0 = g * ell
        nj = min(ell, D.shape[0] - r0)
        digits = server.packed_digits(paillier.decrypt(cl.sk, c), nj, gamma)
        assert [lwe.pir_extract_value(m) for m in digits] == D[r0:r0 + nj, cl.col].tolist(), f"group {g}"


@pytest.mark.parametrize("n_bits,rows,ell", [(256, 13, 3), (1024, 50, 7), (2048, 100, 29),
                                             (3072, 90, 44), (4096, 61, 59)])
def test_packed_matches_oracle(native, n_bits, rows, ell):
    n = 16
    log(f"packed: N {n_bits} rows {rows} ell {ell}")
    inst = make_instance(cfg=950 + n_bits, rows=rows, cols=72, n=n, n_bits=n_bits, zero_row=rows // 2)
    cl = inst.clients[0]
    N_limbs, ck, L = client_arrays(cl, n_bits)
    t = _t_for(n)
    assert (1 << t) >= server.packing_scale_min(n)
    E = server.exponents(server.global_hint(inst.D, inst.A))
    K_or = server.client_hint(cl.ck, E, cl.N)
    b = server.answer(inst.D, cl.qu)
    with native.Server(inst.D, inst.A) as srv:
        cid = srv.add_client(N_limbs, n_bits, ck)
        info = srv.packing_info(cid)
        assert info["log2_gamma"] == t and info["ell"] == 1
        assert info["ell_max"] == (n_bits - 1) // t
        assert ell <= info["ell_max"]
        srv.hint(cid)
        srv.set_packing(cid, ell)
        G = srv.packing_info(cid)["groups"]
        assert G == -(-rows // ell)
        B = np.zeros((1, rows), np.uint32)
        srv.answer(cl.qu[None, :], B)
        C = np.zeros((1, G, L), np.uint32)
        srv.compress_packed([cid], B, C)
        got = limbs_rows_to_ints(C[0])
    _check_groups(cl, inst.D, K_or, b, ell, t, got)


def test_packed_edge_answers(native):
    # b in {0, 2^32 - 1, mixed}: every digit boundary of beta_g is exercised.
    n_bits, rows, n = 2048, 40, 8
    inst = make_instance(cfg=961, rows=rows, cols=48, n=n, n_bits=n_bits, encrypt_secret=False)
    cl = inst.clients[0]
    N_limbs, ck, L = client_arrays(cl, n_bits)
    t = _t_for(n)
    E = server.exponents(server.global_hint(inst.D, inst.A))
    K_or = server.client_hint(cl.ck, E, cl.N)
    with native.Server(inst.D, inst.A) as srv:
        cid = srv.add_client(N_limbs, n_bits, ck)
        ell = srv.packing_info(cid)["ell_max"]
        srv.set_packing(cid, ell)   # before the hint: groups are built by pir_hint
        srv.hint(cid)
        G = srv.packing_info(cid)["groups"]
        for bvals in ([0] * rows, [Q32 - 1] * rows, [(Q32 - 1) if j % 2 else 1 for j in range(rows)]):
            B = np.array([bvals], np.uint32)
            C = np.zeros((1, G, L), np.uint32)
            srv.compress_packed([cid], B, C)
            assert limbs_rows_to_ints(C[0]) == server.compress_packed(K_or, bvals, cl.N, ell, 1 << t)


def test_packed_errors_stale_and_update(native):
    n_bits, rows, n = 512, 30, 4
    inst = make_instance(cfg=962, rows=rows, cols=40, n=n, n_bits=n_bits)
    cl = inst.clients[0]
    N_limbs, ck, L = client_arrays(cl, n_bits)
    t = _t_for(n)
    with native.Server(inst.D, inst.A) as srv:
        cid = srv.add_client(N_limbs, n_bits, ck)
        ell_max = srv.packing_info(cid)["ell_max"]
        assert ell_max == (n_bits - 1) // t
        for bad in (0, ell_max + 1):
            with pytest.raises(native.ZipPIRError) as ei:
                srv.set_packing(cid, bad)
            assert ei.value.status == native.PIR_EINVAL
        B = np.zeros((1, rows), np.uint32)
        srv.answer(cl.qu[None, :], B)
        C = np.zeros((1, rows, L), np.uint32)
        with pytest.raises(native.ZipPIRError) as ei:   # no packing set
            srv.compress_packed([cid], B, C)
        assert ei.value.status == native.PIR_EINVAL
        ell = 4
        srv.set_packing(cid, ell)
        G = srv.packing_info(cid)["groups"]
        C = np.zeros((1, G, L), np.uint32)
        with pytest.raises(native.ZipPIRError) as ei:   # hint not built yet
            srv.compress_packed([cid], B, C)
        assert ei.value.status == native.PIR_ESTALE
        srv.hint(cid)
        srv.compress_packed([cid], B, C)
        # update two rows in different groups: those groups go stale until pir_hint
        idx = np.array([5, 29], np.uint32)
        new = np.random.default_rng(5).integers(0, 256, size=(2, inst.cols), dtype=np.uint8)
        srv.update_rows(idx, new)
        with pytest.raises(native.ZipPIRError) as ei:
            srv.compress_packed([cid], B, C)
        assert ei.value.status == native.PIR_ESTALE
        srv.hint(cid, rows=idx)
        D2 = inst.D.copy()
        D2[idx] = new
        srv.answer(cl.qu[None, :], B)
        srv.compress_packed([cid], B, C)
        got = limbs_rows_to_ints(C[0])
        # back to one ciphertext per row
        srv.set_packing(cid, 1)
        C1 = np.zeros((1, rows, L), np.uint32)
        srv.compress([cid], B, C1)
    E2 = server.exponents(server.global_hint(D2, inst.A))
    K_or = server.client_hint(cl.ck, E2, cl.N)
    b2 = server.answer(D2, cl.qu)
    _check_groups(cl, D2, K_or, b2, ell, t, got)
    assert limbs_rows_to_ints(C1[0]) == server.compress(K_or, b2, cl.N)


def test_packed_batch_of_clients(native):
    # three clients with their own keys, one call; each slice equals that client's own call
    n_bits, rows, n = 1024, 37, 8
    inst = make_instance(cfg=963, rows=rows, cols=64, n=n, n_bits=n_bits, nclients=3, encrypt_secret=False)
    t = _t_for(n)
    ell = 9
    with native.Server(inst.D, inst.A) as srv:
        ids = []
        for cl in inst.clients:
            N_limbs, ck, L = client_arrays(cl, n_bits)
            cid = srv.add_client(N_limbs, n_bits, ck)
            srv.hint(cid)
            srv.set_packing(cid, ell)
            ids.append(cid)
        G = srv.packing_info(ids[0])["groups"]
        Q = np.stack([cl.qu for cl in inst.clients])
        B = np.zeros((3, rows), np.uint32)
        srv.answer(Q, B)
        C = np.zeros((3, G, L), np.uint32)
        srv.compress_packed(ids, B, C)
    E = server.exponents(server.global_hint(inst.D, inst.A))
    for i, cl in enumerate(inst.clients):
        K_or = server.client_hint(cl.ck, E, cl.N)
        assert limbs_rows_to_ints(C[i]) == server.compress_packed(K_or, B[i], cl.N, ell, 1 << t)
