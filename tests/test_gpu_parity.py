"""GPU parity at small sizes: every server step through the C-ABI against the CPU oracle.

Integer path: every comparison is bit-exact.  Sizes span several tiles and ragged tails
(rows and cols that are not multiples of the kernels' tile sizes).
"""
from multiprocessing import Pool

import numpy as np
import pytest

import workload as wl
from oracle import lwe, paillier, server
from tests.gpu_util import client_arrays, limbs_rows_to_ints, log, pool_size
from tests.instances import make_instance, oracle_client_hint

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


# ----------------------------------------------------------------------------- answer

@pytest.mark.parametrize("rows,cols", [(200, 1000), (33, 256), (1, 17), (513, 4100)])
def test_matvec_matches_oracle(native, rows, cols):
    log(f"matvec rows={rows} cols={cols}")
    D = _rand(1, (rows, cols), 256, np.uint8)
    A = _rand(2, (cols, 8), Q32, np.uint32)
    qu = _rand(3, (1, cols), Q32, np.uint32)
    with native.Server(D, A) as srv:
        B = np.zeros((1, rows), np.uint32)
        srv.answer(qu, B, native.PATH_MATVEC)
        assert np.array_equal(B[0], server.answer(D, qu[0]))
        # closed forms: a unit vector selects a column, all-ones gives row sums
        u = np.zeros((1, cols), np.uint32)
        u[0, cols // 2] = 1
        srv.answer(u, B, native.PATH_MATVEC)
        assert np.array_equal(B[0], D[:, cols // 2].astype(np.uint32))


def test_matvec_extremes(native):
    rows, cols = 64, 768
    D = np.full((rows, cols), 255, np.uint8)
    A = np.zeros((cols, 4), np.uint32)
    with native.Server(D, A) as srv:
        B = np.zeros((1, rows), np.uint32)
        srv.answer(np.full((1, cols), Q32 - 1, np.uint32), B, native.PATH_MATVEC)
        assert np.all(B == (-255 * cols) % Q32)


@pytest.mark.parametrize("batch", [2, 5, 16, 32])
def test_mfma_batch_matches_oracle(native, batch):
    rows, cols = 300, 700
    log(f"mfma batch={batch}")
    D = _rand(4, (rows, cols), 256, np.uint8)
    A = _rand(5, (cols, 4), Q32, np.uint32)
    Qm = _rand(6 + batch, (batch, cols), Q32, np.uint32)
    with native.Server(D, A) as srv:
        B = np.zeros((batch, rows), np.uint32)
        srv.answer(Qm, B, native.PATH_MFMA)
        assert np.array_equal(B, server.answer_batch(D, Qm))
        B2 = np.zeros_like(B)
        srv.answer(Qm, B2, native.PATH_MATVEC)
        assert np.array_equal(B2, B)


@pytest.mark.parametrize("cols", [1, 300, 700, 1100, 2200, 70000])
def test_mfma_k_lengths(native, cols):
    # From one K step per block to several, and a K range beyond 64 KiB (split over blocks that
    # add into the output).  The first contraction of each problem shape also runs every
    # candidate launch shape, and the library checks each one's output against the first.
    rows, batch = 37, 3
    log(f"mfma cols={cols}")
    D = _rand(40 + cols, (rows, cols), 256, np.uint8)
    A = _rand(41, (cols, 4), Q32, np.uint32)
    Qm = _rand(42 + cols, (batch, cols), Q32, np.uint32)
    with native.Server(D, A) as srv:
        B = np.zeros((batch, rows), np.uint32)
        srv.answer(Qm, B, native.PATH_MFMA)
        assert np.array_equal(B, server.answer_batch(D, Qm))


@pytest.mark.parametrize("dval,qval", [(0, 0), (255, Q32 - 1), (0, Q32 - 1), (255, 0), (128, 0x80808080)])
def test_mfma_extreme_values(native, dval, qval):
    # D = 0 and Q = 0 both shift to -128 in every plane: the largest MFMA partial sums.
    rows, cols = 130, 512
    D = np.full((rows, cols), dval, np.uint8)
    A = np.zeros((cols, 4), np.uint32)
    Qm = np.full((3, cols), qval, np.uint32)
    with native.Server(D, A) as srv:
        B = np.zeros((3, rows), np.uint32)
        srv.answer(Qm, B, native.PATH_MFMA)
        assert np.all(B == (dval * qval * cols) % Q32)


def test_answer_device_tensors(native):
    import torch
    rows, cols = 96, 512
    D = _rand(7, (rows, cols), 256, np.uint8)
    A = _rand(8, (cols, 4), Q32, np.uint32)
    Qm = _rand(9, (4, cols), Q32, np.uint32)
    Dt = torch.from_numpy(D).cuda()
    At = torch.from_numpy(A.view(np.int32)).cuda()
    with native.Server(Dt, At) as srv:
        Qt = torch.from_numpy(Qm.view(np.int32)).cuda()
        Bt = torch.zeros((4, rows), dtype=torch.int32, device="cuda")
        srv.answer(Qt, Bt)
        srv.sync()
        assert np.array_equal(Bt.cpu().numpy().view(np.uint32), server.answer_batch(D, Qm))


# ----------------------------------------------------------------------------- global hint

@pytest.mark.parametrize("rows,cols,n", [(100, 300, 40), (257, 256, 33)])
def test_global_hint_matches_oracle(native, rows, cols, n):
    log(f"global hint rows={rows} cols={cols} n={n}")
    inst = make_instance(cfg=910, rows=rows, cols=cols, n=n, n_bits=256, encrypt_secret=False)
    cl = inst.clients[0]
    N_limbs, ck, L = client_arrays(cl, 256)
    with native.Server(inst.D, inst.A) as srv:
        cid = srv.add_client(N_limbs, 256, ck)
        srv.hint(cid, rows=[0])
        H = np.zeros((rows, n), np.uint32)
        srv.global_hint(0, rows, H)
        assert np.array_equal(H, server.global_hint(inst.D, inst.A))


# ----------------------------------------------------------------------------- Paillier

def test_small_hint_and_compress_match_oracle(native):
    # rows 12 (ragged), n 8, 256-bit N: K, c and the client round trip, all rows.
    inst = make_instance(cfg=911, rows=12, cols=40, n=8, n_bits=256, zero_row=3)
    cl = inst.clients[0]
    N_limbs, ck, L = client_arrays(cl, 256)
    E = server.exponents(server.global_hint(inst.D, inst.A))
    K_or = server.client_hint(cl.ck, E, cl.N)
    b_or = server.answer(inst.D, cl.qu)
    c_or = server.compress(K_or, b_or, cl.N)
    with native.Server(inst.D, inst.A) as srv:
        cid = srv.add_client(N_limbs, 256, ck)
        assert srv.limbs(cid) == L
        srv.hint(cid)
        K = np.zeros((inst.rows, L), np.uint32)
        srv.client_hint(cid, 0, inst.rows, K)
        assert limbs_rows_to_ints(K) == K_or
        assert K_or[3] == 1
        B = np.zeros((1, inst.rows), np.uint32)
        srv.answer(cl.qu[None, :], B)
        assert np.array_equal(B[0], b_or)
        C = np.zeros((1, inst.rows, L), np.uint32)
        srv.compress([cid], B, C)
        got = limbs_rows_to_ints(C[0])
        assert got == c_or
    f = [lwe.pir_extract_value(paillier.decrypt(cl.sk, x)) for x in got]
    assert f == inst.D[:, cl.col].tolist()


@pytest.mark.parametrize("n_bits", [1024, 2048, 3072, 4096])
def test_compress_edge_values(native, n_bits):
    # b in {0, 1, 2^32-1}; K in {1, N^2-1, random}: c must equal K (1 + bN) mod N^2.
    rows, cols, n = 9, 256, 4
    inst = make_instance(cfg=912, rows=rows, cols=cols, n=n, n_bits=n_bits, encrypt_secret=False)
    cl = inst.clients[0]
    N = cl.N
    N2 = N * N
    # choose ck so that K rows take edge values: with all-zero D rows, K_j = 1
    D = inst.D.copy()
    D[0] = 0
    N_limbs, ck, L = client_arrays(cl, n_bits)
    E = server.exponents(server.global_hint(D, inst.A))
    K_or = server.client_hint(cl.ck, E, N)
    with native.Server(D, inst.A) as srv:
        cid = srv.add_client(N_limbs, n_bits, ck)
        srv.hint(cid)
        for bvals in ([0] * rows, [Q32 - 1] * rows, list(range(rows)), [1] * rows):
            B = np.array([bvals], np.uint32)
            C = np.zeros((1, rows, L), np.uint32)
            srv.compress([cid], B, C)
            got = limbs_rows_to_ints(C[0])
            assert got == [K_or[j] * (1 + int(bvals[j]) * N) % N2 for j in range(rows)]
            assert got[0] == (1 + int(bvals[0]) * N) % N2


def test_stale_and_update(native):
    inst = make_instance(cfg=913, rows=40, cols=64, n=6, n_bits=256, encrypt_secret=False)
    cl = inst.clients[0]
    N_limbs, ck, L = client_arrays(cl, 256)
    with native.Server(inst.D, inst.A) as srv:
        cid = srv.add_client(N_limbs, 256, ck)
        B = np.zeros((1, inst.rows), np.uint32)
        srv.answer(cl.qu[None, :], B)
        C = np.zeros((1, inst.rows, L), np.uint32)
        with pytest.raises(native.ZipPIRError) as ei:
            srv.compress([cid], B, C)
        assert ei.value.status == native.PIR_ESTALE
        srv.hint(cid)
        K0 = np.zeros((inst.rows, L), np.uint32)
        srv.client_hint(cid, 0, inst.rows, K0)
        # update three rows
        idx = np.array([2, 17, 39], np.uint32)
        new = _rand(55, (3, inst.cols), 256, np.uint8)
        srv.update_rows(idx, new)
        assert srv.stale_rows(cid) == 3 and srv.stale_rows() == 3
        with pytest.raises(native.ZipPIRError):
            srv.compress([cid], B, C)
        srv.hint(cid, rows=idx)
        assert srv.stale_rows(cid) == 0 and srv.stale_rows() == 0
        D2 = inst.D.copy()
        D2[idx] = new
        K1 = np.zeros_like(K0)
        srv.client_hint(cid, 0, inst.rows, K1)
        E2 = server.exponents(server.global_hint(D2, inst.A))
        K_or = server.client_hint(cl.ck, E2, cl.N)
        assert limbs_rows_to_ints(K1) == K_or
        untouched = np.setdiff1d(np.arange(inst.rows), idx)
        assert np.array_equal(K1[untouched], K0[untouched])
        H = np.zeros((inst.rows, inst.n), np.uint32)
        srv.global_hint(0, inst.rows, H)
        assert np.array_equal(H, server.global_hint(D2, inst.A))
        srv.answer(cl.qu[None, :], B)
        assert np.array_equal(B[0], server.answer(D2, cl.qu))


def test_rejects_small_modulus(native):
    # Theorem 1: N must exceed q + n q^2 = 2^32 + n 2^64.
    rows, cols, n = 8, 16, 16
    D = _rand(60, (rows, cols), 256, np.uint8)
    A = _rand(61, (cols, n), Q32, np.uint32)
    N = (1 << 67) + 1   # 68 bits < 2^32 + 16 * 2^64 = 2^68 + 2^32
    with native.Server(D, A) as srv:
        with pytest.raises(native.ZipPIRError) as ei:
            srv.add_client(wl.int_to_limbs(N, 3), 68, np.ones((n, 6), np.uint32))
        assert ei.value.status == native.PIR_EINVAL


# ----------------------------------------------------------------------------- toy end to end

def test_toy_config_end_to_end(native):
    """Toy PIR: D 256x256, n = 256, N 1024-bit, every row of K and c checked, and the
    client's decryption recovers the selected column."""
    log("toy: building instance")
    with Pool(pool_size()) as pool:
        inst = make_instance(cfg=0, rows=256, cols=256, n=256, n_bits=1024, pool=pool)
        cl = inst.clients[0]
        E = server.exponents(server.global_hint(inst.D, inst.A))
        log("toy: oracle hint")
        K_or = oracle_client_hint(cl.ck, E, cl.N, pool=pool)
    N_limbs, ck, L = client_arrays(cl, 1024)
    log("toy: GPU")
    with native.Server(inst.D, inst.A) as srv:
        cid = srv.add_client(N_limbs, 1024, ck)
        srv.hint(cid)
        K = np.zeros((256, L), np.uint32)
        srv.client_hint(cid, 0, 256, K)
        assert limbs_rows_to_ints(K) == [K_or[j] for j in range(256)]
        B = np.zeros((1, 256), np.uint32)
        srv.answer(cl.qu[None, :], B)
        assert np.array_equal(B[0], server.answer(inst.D, cl.qu))
        C = np.zeros((1, 256, L), np.uint32)
        srv.compress([cid], B, C)
        got = limbs_rows_to_ints(C[0])
    assert got == server.compress([K_or[j] for j in range(256)], B[0], cl.N)
    f = [lwe.pir_extract_value(paillier.decrypt(cl.sk, x)) for x in got]
    assert f == inst.D[:, cl.col].tolist()


@pytest.mark.parametrize("n_bits", [1536, 3072, 4096])
def test_hint_and_combine_other_moduli(native, n_bits):
    """Every limbs-per-lane instantiation of the Montgomery kernels (N of 1536, 3072 -- the
    paper's Paillier size -- and 4096 bits): K on every row, the combine, and the client's
    decryption of every compressed row."""
    rows, cols, n = 20, 96, 6
    log(f"modulus {n_bits}: instance")
    inst = make_instance(cfg=930 + n_bits, rows=rows, cols=cols, n=n, n_bits=n_bits, zero_row=7)
    cl = inst.clients[0]
    N_limbs, ck, L = client_arrays(cl, n_bits)
    E = server.exponents(server.global_hint(inst.D, inst.A))
    K_or = server.client_hint(cl.ck, E, cl.N)
    b_or = server.answer(inst.D, cl.qu)
    with native.Server(inst.D, inst.A) as srv:
        cid = srv.add_client(N_limbs, n_bits, ck)
        srv.hint(cid)
        K = np.zeros((rows, L), np.uint32)
        srv.client_hint(cid, 0, rows, K)
        assert limbs_rows_to_ints(K) == K_or
        B = np.zeros((1, rows), np.uint32)
        srv.answer(cl.qu[None, :], B)
        C = np.zeros((1, rows, L), np.uint32)
        srv.compress([cid], B, C)
    got = limbs_rows_to_ints(C[0])
    assert got == server.compress(K_or, b_or, cl.N)
    f = [lwe.pir_extract_value(paillier.decrypt(cl.sk, x)) for x in got]
    assert f == inst.D[:, cl.col].tolist()


def test_autotuned_shape_is_persisted(native, tmp_path, monkeypatch):
    # The first batched contraction of a new shape times the candidate launch shapes and
    # records the winner; every candidate computes the same bits.  On the tiled copy the fused
    # batched kernel is tuned (a "batch" line keyed by rows, pitch and 32-query groups); on
    # row-major D the byte-plane contraction (its own line layout, tiled flag 0).
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("ZIPPIR_TUNE_CACHE", str(cache))
    rows, cols, batch = 77, 1280, 3
    D = _rand(70, (rows, cols), 256, np.uint8)
    A = _rand(71, (cols, 4), Q32, np.uint32)
    Qm = _rand(72, (batch, cols), Q32, np.uint32)
    with native.Server(D, A) as srv:
        assert srv.tiled_copy()
        B = np.zeros((batch, rows), np.uint32)
        srv.answer(Qm, B, native.PATH_MFMA)
        assert np.array_equal(B, server.answer_batch(D, Qm))
        srv.set_tiled_copy(False)  # the row-major layout is tuned under its own key
        B[:] = 0
        srv.answer(Qm, B, native.PATH_MFMA)
        assert np.array_equal(B, server.answer_batch(D, Qm))
    lines = [l.split() for l in cache.read_text().splitlines()]
    pitch = str(cols + (-cols) % 256)
    mine = [l for l in lines if l[:5] == [str(rows), pitch, str(batch), "0", "4"]]
    assert [l[5] for l in mine] == ["0"] and all(len(l) == 12 for l in mine)
    fused = [l for l in lines if l[:4] == ["batch", str(rows), pitch, "1"]]
    assert len(fused) == 1 and len(fused[0]) == 8


@pytest.mark.parametrize("rows,cols", [(1000, 3000), (16, 256), (4099, 700)])
def test_tiled_copy_layouts(native, rows, cols):
    # The contraction reads the tiled copy of D by default (so do the hint tests' H = D.A):
    # batched answers equal the oracle for row counts that are not multiples of 16, after row
    # updates (which rewrite the tiled rows too), with the copy freed (row-major D) and after it
    # is made again.
    log(f"tiled copy rows {rows} cols {cols}")
    batch = 5
    D = _rand(80 + rows, (rows, cols), 256, np.uint8)
    A = _rand(81, (cols, 4), Q32, np.uint32)
    Qm = _rand(82, (batch, cols), Q32, np.uint32)
    upd = np.array(sorted({0, rows // 2, rows - 1}), np.uint32)
    new = _rand(83, (len(upd), cols), 256, np.uint8)
    with native.Server(D, A) as srv:
        assert srv.tiled_copy()
        B = np.zeros((batch, rows), np.uint32)
        srv.answer(Qm, B, native.PATH_MFMA)
        assert np.array_equal(B, server.answer_batch(D, Qm))
        srv.update_rows(upd, new)
        D2 = D.copy()
        D2[upd] = new
        want = server.answer_batch(D2, Qm)
        B[:] = 0
        srv.answer(Qm, B, native.PATH_MFMA)
        assert np.array_equal(B, want)
        srv.set_tiled_copy(False)
        assert not srv.tiled_copy()
        B[:] = 0
        srv.answer(Qm, B, native.PATH_MFMA)
        assert np.array_equal(B, want)
        srv.set_tiled_copy(True)
        assert srv.tiled_copy()
        B[:] = 0
        srv.answer(Qm, B, native.PATH_MFMA)
        assert np.array_equal(B, want)


def test_read_probe(native):
    # measurement helper: reads the buffer once (the xor of the per-block words is the xor of
    # every word read); a misaligned buffer is rejected
    import torch
    dev = torch.device("cuda:0")
    src = torch.arange(1 << 20, dtype=torch.int32, device=dev)
    sink = torch.zeros(64, dtype=torch.int32, device=dev)
    native.read_probe(src, sink, 64)
    torch.cuda.synchronize()
    want = int(np.bitwise_xor.reduce(src.cpu().numpy().view(np.uint32)))
    assert int(np.bitwise_xor.reduce(sink.cpu().numpy().view(np.uint32))) == want
    # ragged: 262139 words are 65534 whole 16-byte units plus 12 bytes that are not read, over
    # 7 workgroups whose chunks do not divide the units evenly
    part = src[:262139]
    sink7 = torch.zeros(7, dtype=torch.int32, device=dev)
    native.read_probe(part, sink7, 7)
    torch.cuda.synchronize()
    want7 = int(np.bitwise_xor.reduce(src.cpu().numpy().view(np.uint32)[:65534 * 4]))
    assert int(np.bitwise_xor.reduce(sink7.cpu().numpy().view(np.uint32))) == want7
    st = native.lib().pir_read_probe(src.data_ptr() + 4, 1024, sink.data_ptr(), 64, None)
    assert st == native.PIR_EINVAL


def test_hint_four_rows_per_wave_ragged_count(native):
    # 16385 rows take the four-rows-per-wavefront hint kernel (one row per 16 lanes), the last
    # wavefront holding a single row, and the 11-bit window table (a pir_hint over few rows
    # takes the one-row kernel and 8-bit windows); every row of K matches the oracle.
    rows, cols, n, n_bits = 16385, 64, 4, 256
    inst = make_instance(cfg=931, rows=rows, cols=cols, n=n, n_bits=n_bits, encrypt_secret=False, zero_row=rows - 1)
    cl = inst.clients[0]
    N_limbs, ck, L = client_arrays(cl, n_bits)
    E = server.exponents(server.global_hint(inst.D, inst.A))
    with native.Server(inst.D, inst.A) as srv:
        cid = srv.add_client(N_limbs, n_bits, ck)
        assert srv.hint_window_bits(cid) == 0
        srv.hint(cid)
        assert srv.hint_window_bits(cid) == 11
        K = np.zeros((rows, L), np.uint32)
        srv.client_hint(cid, 0, rows, K)
        K8 = K.copy()
        srv.hint(cid, rows=[0, 5, rows - 1])
        assert srv.hint_window_bits(cid) == 8
        srv.client_hint(cid, 0, rows, K8)
    with Pool(pool_size()) as pool:
        K_or = oracle_client_hint(cl.ck, E, cl.N, pool=pool)
    assert limbs_rows_to_ints(K) == [K_or[j] for j in range(rows)]
    assert np.array_equal(K8, K)
    assert K_or[rows - 1] == 1


@pytest.mark.parametrize("rows,n", [(1101, 250), (300, 250), (1, 64)])
def test_hint_split_rows(native, rows, n):
    # Under 4096 rows each row's product over its n bases is split into parts, one wavefront
    # per (row, part), and the parts are joined: 1101 rows x 15 parts of 17 bases (the last
    # part 12), 300 rows x 50 parts of 5, a single row 64 parts of one base.  K equals the
    # oracle on every row, and a re-hint of a few rows after an update equals it too.
    log(f"hint split rows {rows} n {n}")
    cols, n_bits = 64, 256
    inst = make_instance(cfg=960 + rows, rows=rows, cols=cols, n=n, n_bits=n_bits, encrypt_secret=False)
    cl = inst.clients[0]
    N_limbs, ck, L = client_arrays(cl, n_bits)
    upd = np.array(sorted({0, rows // 2, rows - 1}), np.uint32)
    new = _rand(961, (len(upd), cols), 256, np.uint8)
    D2 = inst.D.copy()
    D2[upd] = new
    with native.Server(inst.D, inst.A) as srv:
        cid = srv.add_client(N_limbs, n_bits, ck)
        srv.hint(cid)
        K = np.zeros((rows, L), np.uint32)
        srv.client_hint(cid, 0, rows, K)
        srv.update_rows(upd, new)
        srv.hint(cid, rows=upd)
        K2 = np.zeros((rows, L), np.uint32)
        srv.client_hint(cid, 0, rows, K2)
    with Pool(pool_size()) as pool:
        K_or = oracle_client_hint(cl.ck, server.exponents(server.global_hint(inst.D, inst.A)), cl.N, pool=pool)
        K2_or = oracle_client_hint(cl.ck, server.exponents(server.global_hint(D2, inst.A, rows=upd)), cl.N, pool=pool)
    assert limbs_rows_to_ints(K) == [K_or[j] for j in range(rows)]
    got2 = limbs_rows_to_ints(K2[upd])
    assert got2 == [K2_or[j] for j in range(len(upd))]
    keep = np.setdiff1d(np.arange(rows), upd)
    assert np.array_equal(K2[keep], K[keep])


def test_empty_and_degenerate_inputs(native):
    # empty shapes are rejected; a 1 x 1 database answers and compresses; empty row lists
    # of an update are a no-op; an empty compressor batch does nothing
    for shape in ((0, 64), (8, 0)):
        D = np.zeros(shape, np.uint8)
        A = np.zeros((shape[1], 4), np.uint32)
        with pytest.raises(native.ZipPIRError) as ei:
            native.Server(D, A)
        assert ei.value.status == native.PIR_EINVAL
    with pytest.raises(native.ZipPIRError) as ei:
        native.Server(np.zeros((8, 8), np.uint8), np.zeros((8, 0), np.uint32))
    assert ei.value.status == native.PIR_EINVAL
    inst = make_instance(cfg=933, rows=1, cols=1, n=2, n_bits=256)
    cl = inst.clients[0]
    N_limbs, ck, L = client_arrays(cl, 256)
    E = server.exponents(server.global_hint(inst.D, inst.A))
    K_or = server.client_hint(cl.ck, E, cl.N)
    with native.Server(inst.D, inst.A) as srv:
        B = np.zeros((1, 1), np.uint32)
        with pytest.raises(native.ZipPIRError) as ei:
            srv.answer(np.zeros((0, 1), np.uint32), np.zeros((0, 1), np.uint32))
        assert ei.value.status == native.PIR_EINVAL
        srv.answer(cl.qu[None, :], B)
        assert np.array_equal(B[0], server.answer(inst.D, cl.qu))
        cid = srv.add_client(N_limbs, 256, ck)
        srv.hint(cid)
        srv.update_rows(np.zeros(0, np.uint32), np.zeros((0, 1), np.uint8))
        assert srv.stale_rows(cid) == 0
        C = np.zeros((1, 1, L), np.uint32)
        srv.compress([cid], B, C)
        assert limbs_rows_to_ints(C[0]) == server.compress(K_or, B[0], cl.N)
    sk_pr = wl.paillier_primes(934, 0, 256)
    N = sk_pr.P * sk_pr.Q
    with native.Compressor(4, 1 << 16, wl.int_to_limbs(N, 8), 256,
                           ck=wl.ints_to_limbs(wl.uniform_ciphertexts(934, 0, 4, N), 16)) as cmp:
        X = np.zeros((0, 16), np.uint32)
        cmp.compress_lwe(np.zeros((0, 4), np.uint32), np.zeros(0, np.uint32), X)


def test_hint_wide_table_against_narrow(native):
    # n = 1024 bases: over 16385 rows the hint builds the 11-bit table with four bases per
    # wavefront and takes four rows per wavefront; in chunks of 4096 rows it takes the 8-bit
    # table, one base and one row per wavefront.  The two K agree on every row, and sampled rows
    # match the oracle.
    rows, cols, n, n_bits = 16385, 16, 1024, 256
    inst = make_instance(cfg=932, rows=rows, cols=cols, n=n, n_bits=n_bits, encrypt_secret=False, zero_row=7)
    cl = inst.clients[0]
    N_limbs, ck, L = client_arrays(cl, n_bits)
    with native.Server(inst.D, inst.A) as srv:
        cid = srv.add_client(N_limbs, n_bits, ck)
        srv.hint(cid)
        assert srv.hint_window_bits(cid) == 11
        K11 = np.zeros((rows, L), np.uint32)
        srv.client_hint(cid, 0, rows, K11)
        for r0 in range(0, rows, 4096):
            srv.hint(cid, rows=np.arange(r0, min(rows, r0 + 4096), dtype=np.uint32))
            assert srv.hint_window_bits(cid) == 8
        K8 = np.zeros((rows, L), np.uint32)
        srv.client_hint(cid, 0, rows, K8)
    assert np.array_equal(K11, K8)
    sample = [0, 7, 1, 4095, 4096, 8191, 12345, rows - 1]
    E = server.exponents(server.global_hint(inst.D, inst.A, rows=sample))
    with Pool(pool_size()) as pool:
        K_or = oracle_client_hint(cl.ck, E, cl.N, pool=pool)
    assert [wl.limbs_to_int(K11[j]) for j in sample] == [K_or[i] for i in range(len(sample))]
    assert K_or[1] == 1


@pytest.mark.parametrize("rows,cols,n_bits", [(1, 1, 256), (37, 300, 256), (300, 5000, 1024), (257, 8193, 256),
                                              (130, 70000, 2048)])
def test_answer_compress_two_launches(native, rows, cols, n_bits):
    # pir_answer_compress (query planes built in the matvec, per-segment partials added up by
    # the combine) gives the bits of pir_answer + pir_compress and of the oracle, for one to 18
    # column segments, ragged rows and columns, and queries at their extremes.
    log(f"answer_compress rows {rows} cols {cols} N {n_bits}")
    n = 4
    inst = make_instance(cfg=940 + rows, rows=rows, cols=cols, n=n, n_bits=n_bits, encrypt_secret=False)
    cl = inst.clients[0]
    N_limbs, ck, L = client_arrays(cl, n_bits)
    g = np.random.default_rng(941 + rows)
    queries = [cl.qu, np.full(cols, Q32 - 1, np.uint32), g.integers(0, Q32, size=cols, dtype=np.uint32)]
    # the expected responses use the oracle's K, never the library's
    K_int = server.client_hint(cl.ck, server.exponents(server.global_hint(inst.D, inst.A)), cl.N)
    with native.Server(inst.D, inst.A) as srv:
        cid = srv.add_client(N_limbs, n_bits, ck)
        srv.hint(cid)
        K = np.zeros((rows, L), np.uint32)
        srv.client_hint(cid, 0, rows, K)
        assert limbs_rows_to_ints(K) == K_int
        for q in queries:
            B1 = np.zeros((1, rows), np.uint32)
            C1 = np.zeros((1, rows, L), np.uint32)
            srv.answer(q[None, :], B1)
            srv.compress([cid], B1, C1)
            B2 = np.full(rows, 0xDEADBEEF, np.uint32)
            C2 = np.full((rows, L), 0xDEADBEEF, np.uint32)
            srv.answer_compress(q, cid, B2, C2)
            assert np.array_equal(B2, B1[0])
            assert np.array_equal(C2, C1[0])
            b_or = server.answer(inst.D, q)
            assert np.array_equal(B2, b_or)
            assert limbs_rows_to_ints(C2) == server.compress(K_int, b_or, cl.N)
        with pytest.raises(native.ZipPIRError) as ei:
            srv.answer_compress(queries[0], cid + 7, B2, C2)
        assert ei.value.status == native.PIR_EINVAL


@pytest.mark.parametrize("rows,cols,n_bits,misalign", [(16387, 300, 256, False), (16390, 520, 2048, False),
                                                       (16390, 520, 2048, True), (16385, 70000, 256, False)])
def test_answer_compress_four_rows_per_wave(native, rows, cols, n_bits, misalign):
    # from 16384 rows the combine takes four rows per wavefront: rows that fill all 16 lanes'
    # limbs (N 2048-bit) move in 16-byte pieces unless an array is not 16-byte aligned (a
    # response buffer 4 bytes off), shorter rows (N 256-bit) take clamped loads, and 70000
    # columns give 18 segment partials per row (more than one per lane of a row).  Ragged row
    # counts leave part of the last wavefront empty.
    import torch
    log(f"answer_compress four rows per wave: rows {rows} cols {cols} N {n_bits} misaligned {misalign}")
    n = 4
    inst = make_instance(cfg=950 + cols, rows=rows, cols=cols, n=n, n_bits=n_bits, encrypt_secret=False)
    cl = inst.clients[0]
    N_limbs, ck, L = client_arrays(cl, n_bits)
    g = np.random.default_rng(951 + rows)
    q = g.integers(0, Q32, size=cols, dtype=np.uint32)
    with native.Server(inst.D, inst.A) as srv:
        cid = srv.add_client(N_limbs, n_bits, ck)
        srv.hint(cid)
        B1 = np.zeros((1, rows), np.uint32)
        C1 = np.zeros((1, rows, L), np.uint32)
        srv.answer(q[None, :], B1)
        srv.compress([cid], B1, C1)
        qd = torch.from_numpy(q.view(np.int32).copy()).cuda()
        B2 = torch.full((rows,), -1, dtype=torch.int32, device="cuda")
        Cbig = torch.full((rows * L + 4,), -1, dtype=torch.int32, device="cuda")
        C2 = Cbig[1:1 + rows * L].view(rows, L) if misalign else Cbig[:rows * L].view(rows, L)
        assert (C2.data_ptr() % 16 != 0) == misalign
        srv.answer_compress(qd, cid, B2, C2)
        srv.sync()
        b = B2.cpu().numpy().view(np.uint32)
        c = C2.cpu().numpy().view(np.uint32)
        assert np.array_equal(b, B1[0])
        assert np.array_equal(c, C1[0])
        K = np.zeros((rows, L), np.uint32)
        srv.client_hint(cid, 0, rows, K)
    sample = np.unique(np.concatenate([np.arange(8), np.arange(rows - 8, rows), g.integers(0, rows, 24)]))
    b_or = server.answer_rows(inst.D, q, sample)
    assert np.array_equal(b[sample], b_or)
    # K on the sampled rows from the oracle: the expected responses use no library output
    K_or = server.client_hint(cl.ck, server.exponents(server.global_hint(inst.D, inst.A, rows=sample)), cl.N)
    assert limbs_rows_to_ints(K[sample]) == K_or
    assert limbs_rows_to_ints(c[sample]) == server.compress(K_or, b_or, cl.N)


def test_answer_compress_device_and_stale(native):
    import torch
    rows, cols, n, n_bits = 96, 4200, 4, 256
    inst = make_instance(cfg=945, rows=rows, cols=cols, n=n, n_bits=n_bits, encrypt_secret=False)
    cl = inst.clients[0]
    N_limbs, ck, L = client_arrays(cl, n_bits)
    with native.Server(inst.D, inst.A) as srv:
        cid = srv.add_client(N_limbs, n_bits, ck)
        srv.hint(cid)
        q = torch.from_numpy(cl.qu.view(np.int32).copy()).cuda()
        B = torch.zeros(rows, dtype=torch.int32, device="cuda")
        C = torch.zeros((rows, L), dtype=torch.int32, device="cuda")
        for _ in range(2):
            srv.answer_compress(q, cid, B, C)
        srv.sync()
        b = B.cpu().numpy().view(np.uint32)
        assert np.array_equal(b, server.answer(inst.D, cl.qu))
        K = np.zeros((rows, L), np.uint32)
        srv.client_hint(cid, 0, rows, K)
        assert limbs_rows_to_ints(C.cpu().numpy().view(np.uint32)) == server.compress(limbs_rows_to_ints(K), b, cl.N)
        srv.update_rows([5], np.zeros((1, cols), np.uint8))
        with pytest.raises(native.ZipPIRError) as ei:
            srv.answer_compress(q, cid, B, C)
        assert ei.value.status == native.PIR_ESTALE
