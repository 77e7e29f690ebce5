"""pir_answer_compress_noalloc (the one-call online step with its segment partials in the
library's static per-device scratch array, for callers that cannot allocate) gives the same
bits as pir_answer_compress, which the oracle fixes (Alg. 5 Response, first line; Sec. 4.3
Paillier addition): two calls in a row on the shared array, the second on a smaller database,
then a database whose partials would exceed the array (rejected before any launch)."""
import numpy as np
import pytest

import workload as wl
from oracle import server
from tests.gpu_util import client_arrays, limbs_rows_to_ints, log
from tests.instances import make_instance

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_native():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_09190_amd import native as nat
    return torch, nat


def _one_case(torch, native, cfg, rows, cols, n, n_bits):
    inst = make_instance(cfg=cfg, rows=rows, cols=cols, n=n, n_bits=n_bits, encrypt_secret=False)
    cl = inst.clients[0]
    N_limbs, ck, L = client_arrays(cl, n_bits)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev).cuda_stream
    Dt = torch.from_numpy(inst.D).to(dev)
    At = torch.from_numpy(inst.A.view(np.int32)).to(dev)
    with native.Server(Dt, At, device=0, stream=stream) as srv:
        cid = srv.add_client(N_limbs, n_bits, ck)
        srv.hint(cid)
        q = torch.from_numpy(cl.qu.view(np.int32).copy()).to(dev)
        B1 = torch.zeros(rows, dtype=torch.int32, device=dev)
        C1 = torch.zeros((rows, L), dtype=torch.int32, device=dev)
        srv.answer_compress(q, cid, B1, C1)
        # outputs start from garbage: the entry point must write every element
        B2 = torch.full((rows,), -1, dtype=torch.int32, device=dev)
        C2 = torch.full((rows, L), 0x5A5A5A5A, dtype=torch.int32, device=dev)
        srv.answer_compress_noalloc(q, cid, B2, C2)
        srv.sync()
        Kh = np.zeros((rows, L), np.uint32)
        srv.client_hint(cid, 0, rows, Kh)
    b1, b2 = B1.cpu().numpy().view(np.uint32), B2.cpu().numpy().view(np.uint32)
    c1, c2 = C1.cpu().numpy().view(np.uint32), C2.cpu().numpy().view(np.uint32)
    assert np.array_equal(b2, b1), "answer differs from pir_answer_compress"
    assert np.array_equal(c2, c1), "combined response differs from pir_answer_compress"
    # and both equal the oracle (answer on every row; the combine from oracle K on sampled rows)
    want_b = server.answer(inst.D, cl.qu)
    assert np.array_equal(b2, want_b)
    sel = sorted({0, rows - 1, rows // 2, 1 % rows, (7 * rows) // 9})
    E = server.exponents(server.global_hint(inst.D[sel], inst.A))
    K = server.client_hint(cl.ck, E, cl.N)
    assert limbs_rows_to_ints(Kh[sel]) == K
    want_c = server.compress(K, want_b[sel], cl.N)
    assert limbs_rows_to_ints(c2[sel]) == want_c


def test_noalloc_matches_answer_compress_twice(torch_native):
    torch, native = torch_native
    # first call: 9 column segments; second: fewer rows and one segment on the same array
    for cfg, rows, cols, n, nb in ((2101, 1500, 33000, 8, 256), (2102, 77, 300, 5, 1024)):
        log(f"noalloc step: rows {rows} cols {cols} N {nb}")
        _one_case(torch, native, cfg, rows, cols, n, nb)


def test_noalloc_rejects_beyond_its_scratch(torch_native):
    torch, native = torch_native
    rows, cols, n = (4 << 20) + 1, 1, 1   # 4 Mi + 1 rows of one segment: one word above the limit
    log("noalloc limit")
    dev = torch.device("cuda:0")
    D = torch.zeros((rows, cols), dtype=torch.uint8, device=dev)
    A = torch.zeros((cols, n), dtype=torch.int32, device=dev)
    pr = wl.paillier_primes(2103, 0, 256)
    N = pr.P * pr.Q
    ck = wl.ints_to_limbs(wl.uniform_ciphertexts(2103, 0, n, N), 16)
    with native.Server(D, A, device=0, stream=torch.cuda.current_stream(dev).cuda_stream) as srv:
        cid = srv.add_client(wl.int_to_limbs(N, 8), 256, ck)
        q = torch.zeros(cols + 3, dtype=torch.int32, device=dev)   # 16-byte aligned allocation
        B = torch.zeros(rows, dtype=torch.int32, device=dev)
        C = torch.zeros((rows, 16), dtype=torch.int32, device=dev)
        with pytest.raises(native.ZipPIRError) as ei:
            srv.answer_compress_noalloc(q, cid, B, C)
        assert ei.value.status == native.PIR_EINVAL
        assert "limit" in str(ei.value)
        with pytest.raises(native.ZipPIRError) as ei:   # a misaligned query
            srv.answer_compress_noalloc(q[1:], cid, B, C)
        assert ei.value.status == native.PIR_EINVAL
