"""Serving engine on the GPU: every response is the same alone and in a concurrent mix
(bit-exact, tolerance 0 on an integer path), under memory pressure too, and equals the
oracle's compressed row."""
import numpy as np
import pytest

import workload as wl
from oracle import server
from tests.gpu_util import client_arrays, limbs_rows_to_ints, log
from tests.instances import make_instance

pytestmark = pytest.mark.gpu

# (rows, cols, client modulus sizes)
DBS = [(300, 1000, (512, 512)), (512, 512, (512, 1024)), (1100, 768, (1024,))]
N_LWE = 8


@pytest.fixture(scope="module")
def native():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_09190_amd import native as nat
    return nat


@pytest.fixture(scope="module")
def setup(native):
    import torch
    streams, servers, infos = [], [], []
    for i, (rows, cols, sizes) in enumerate(DBS):
        inst = make_instance(cfg=920 + i, rows=rows, cols=cols, n=N_LWE, n_bits=sizes[0], encrypt_secret=False)
        st = torch.cuda.Stream()
        streams.append(st)
        srv = native.Server(inst.D, inst.A, stream=st.cuda_stream)
        clients = []
        for k, nb in enumerate(sizes):
            from tests.instances import make_client
            cl = make_client(920 + i, k, inst.A, nb, encrypt_secret=False)
            N_limbs, ck, L = client_arrays(cl, nb)
            cid = srv.add_client(N_limbs, nb, ck)
            srv.hint(cid)
            clients.append((cid, cl, L))
        servers.append(srv)
        infos.append((inst, clients))
    yield servers, infos, streams
    for s in servers:
        s.close()


def _requests(infos, count, seed):
    g = np.random.default_rng(seed)
    reqs = []
    for _ in range(count):
        db = int(g.integers(0, len(infos)))
        inst, clients = infos[db]
        ci = int(g.integers(0, len(clients)))
        q = g.integers(0, 1 << 32, size=inst.cols, dtype=np.uint32)
        reqs.append((db, ci, q))
    return reqs


def _run(native, servers, infos, reqs, max_batch=32, budget=0, together=True, steps=None):
    outs = []
    with native.Engine(max_batch=max_batch, hbm_budget=budget) as eng:
        if steps:
            eng.set_steps(*steps)
        for s in servers:
            eng.add_db(s)
        bufs = []
        for db, ci, q in reqs:
            inst, clients = infos[db]
            cid, cl, L = clients[ci]
            buf = native.PinnedArray((inst.rows, L))
            bufs.append(buf)
        comps = []
        for (db, ci, q), buf in zip(reqs, bufs):
            cid = infos[db][1][ci][0]
            eng.submit(db, cid, q, buf.array)
            if not together:
                eng.drain()
        eng.drain()
        comps = eng.poll(max_items=len(reqs) + 8)
        stats = eng.stats()
        outs = [b.array.copy() for b in bufs]
        for b in bufs:
            b.close()
    return outs, comps, stats


def test_alone_equals_mix(native, setup):
    servers, infos, _ = setup
    reqs = _requests(infos, 48, seed=1)
    log("serve: alone")
    alone, comps_a, _ = _run(native, servers, infos, reqs, together=False)
    log("serve: mix")
    mix, comps_m, stats = _run(native, servers, infos, reqs, together=True)
    assert len(comps_m) == len(reqs) and all(c["status"] == 0 for c in comps_m)
    assert all(c["batch"] == 1 for c in comps_a)
    assert stats["mean_batch"] > 1.0, "the mix never formed a batch"
    for a, m in zip(alone, mix):
        assert np.array_equal(a, m)
    # the oracle on three requests, every row
    for idx in (0, 1, 2):
        db, ci, q = reqs[idx]
        inst, clients = infos[db]
        cid, cl, L = clients[ci]
        E = server.exponents(server.global_hint(inst.D, inst.A))
        K = server.client_hint(cl.ck, E, cl.N)
        b = server.answer(inst.D, q)
        assert limbs_rows_to_ints(mix[idx]) == server.compress(K, b, cl.N)
    assert stats["p99_ms"] >= stats["p50_ms"] > 0


def test_stepped_batches_equal_alone(native, setup):
    # Small steps: the answer in ranges of 256 rows (pitch 1024 and 768) or 512 rows (pitch
    # 512), ragged at the end, and each response downloaded in pieces of 10000 bytes; with three
    # databases registered at most two steps of a batch are queued at a time.  Every response
    # equals the one-at-a-time run with default steps, and the oracle's on two requests.
    servers, infos, _ = setup
    reqs = _requests(infos, 40, seed=4)
    alone, _, _ = _run(native, servers, infos, reqs, together=False)
    log("serve: stepped mix")
    mix, comps, stats = _run(native, servers, infos, reqs, steps=(256 * 1024, 10000))
    assert all(c["status"] == 0 for c in comps) and stats["mean_batch"] > 1.0
    for a, m in zip(alone, mix):
        assert np.array_equal(a, m)
    for idx in (3, 4):
        db, ci, q = reqs[idx]
        inst, clients = infos[db]
        cid, cl, L = clients[ci]
        K = server.client_hint(cl.ck, server.exponents(server.global_hint(inst.D, inst.A)), cl.N)
        assert limbs_rows_to_ints(mix[idx]) == server.compress(K, server.answer(inst.D, q), cl.N)


def test_memory_pressure_still_exact(native, setup):
    servers, infos, _ = setup
    reqs = _requests(infos, 24, seed=2)
    free, _, _ = _run(native, servers, infos, reqs)
    # budget for one request of the largest database: its batches hold one request, and no
    # batch's buffers exceed the budget
    def per_request(db, L):
        rows, cols, _ = DBS[db]
        return 4 * cols + 4 * rows + 4 * rows * L

    rows, cols, sizes = DBS[2]
    budget = per_request(2, 2 * ((max(sizes) + 31) // 32)) + 1024
    tight, comps, stats = _run(native, servers, infos, reqs, budget=budget)
    assert all(c["status"] == 0 for c in comps)
    assert all(c["batch"] == 1 for c in comps if c["db"] == 2)
    limbs = {r: infos[db][1][ci][2] for r, (db, ci, q) in enumerate(reqs, start=1)}
    for c in comps:
        assert c["batch"] * per_request(c["db"], limbs[c["request_id"]]) <= budget
    assert stats["device_bytes_peak"] <= budget
    for a, b in zip(free, tight):
        assert np.array_equal(a, b)


def test_arrival_times_are_respected(native, setup):
    servers, infos, _ = setup
    inst, clients = infos[0]
    cid, cl, L = clients[0]
    with native.Engine() as eng:
        for s in servers:
            eng.add_db(s)
        bufs = [native.PinnedArray((inst.rows, L)) for _ in range(5)]
        t0 = eng.now_ms()
        for k, b in enumerate(bufs):
            eng.submit(0, cid, np.full(inst.cols, k, np.uint32), b.array, arrival_ms=t0 + 20.0 + 10.0 * k)
        eng.drain()
        comps = sorted(eng.poll(16), key=lambda c: c["request_id"])
        for k, c in enumerate(comps):
            assert c["start_ms"] >= t0 + 20.0 + 10.0 * k - 1e-6
            assert c["done_ms"] >= c["start_ms"]
        for b in bufs:
            b.close()


def test_engine_errors(native, setup):
    servers, infos, _ = setup
    inst, clients = infos[0]
    cid, cl, L = clients[0]
    with native.Engine() as eng:
        eng.add_db(servers[0])
        buf = native.PinnedArray((inst.rows, L))
        with pytest.raises(native.ZipPIRError):
            eng.submit(5, cid, np.zeros(inst.cols, np.uint32), buf.array)           # unknown database
        with pytest.raises(native.ZipPIRError):
            eng.submit(0, 999, np.zeros(inst.cols, np.uint32), buf.array)           # unknown client
        with pytest.raises(native.ZipPIRError):
            eng.submit(0, cid, np.zeros(inst.cols, np.uint32), np.zeros((inst.rows, L), np.uint32))  # pageable
        buf.close()
    # a client whose hint is stale completes with PIR_ESTALE and the engine keeps serving
    srv = servers[1]
    inst1, clients1 = infos[1]
    cid1, cl1, L1 = clients1[0]
    row = np.array([3], np.uint32)
    srv_new = np.random.default_rng(3).integers(0, 256, (1, inst1.cols), dtype=np.uint8)
    srv.update_rows(row, srv_new)   # no engine holds the server during the update
    with native.Engine() as eng:
        eng.add_db(srv)
        b1 = native.PinnedArray((inst1.rows, L1))
        eng.submit(0, cid1, np.zeros(inst1.cols, np.uint32), b1.array)
        eng.drain()
        c = eng.poll(4)
        assert c[0]["status"] == native.PIR_ESTALE
        b1.close()
    srv.hint(cid1, rows=row)
    inst1.D[3] = srv_new[0]
    with native.Engine() as eng:
        eng.add_db(srv)
        b1 = native.PinnedArray((inst1.rows, L1))
        q = np.arange(inst1.cols, dtype=np.uint32)
        eng.submit(0, cid1, q, b1.array)
        eng.drain()
        assert eng.poll(4)[0]["status"] == 0
        E = server.exponents(server.global_hint(inst1.D, inst1.A))
        K = server.client_hint(cl1.ck, E, cl1.N)
        assert limbs_rows_to_ints(b1.array) == server.compress(K, server.answer(inst1.D, q), cl1.N)
        b1.close()


def test_packed_clients_in_the_mix(native):
    """A database with one packed client (ell = 5) and one plain client: requests of the two
    kinds never share a batch, every response equals the library's own packed or plain
    combine of that request's answer, and one request of each kind equals the oracle."""
    import torch
    rows, cols, nb = 203, 320, 512
    inst = make_instance(cfg=940, rows=rows, cols=cols, n=N_LWE, n_bits=nb, nclients=2, encrypt_secret=False)
    st = torch.cuda.Stream()
    g = np.random.default_rng(4)
    with native.Server(inst.D, inst.A, stream=st.cuda_stream) as srv:
        ids = []
        for cl in inst.clients:
            N_limbs, ck, L = client_arrays(cl, nb)
            cid = srv.add_client(N_limbs, nb, ck)
            srv.hint(cid)
            ids.append(cid)
        srv.set_packing(ids[0], 5)
        groups = srv.packing_info(ids[0])["groups"]
        assert groups == -(-rows // 5)
        reqs = [(int(g.integers(0, 2)), g.integers(0, 1 << 32, size=cols, dtype=np.uint32)) for _ in range(40)]
        with native.Engine(max_batch=8) as eng:
            eng.add_db(srv)
            bufs = [native.PinnedArray((groups if k == 0 else rows, L)) for k, _ in reqs]
            for (k, q), buf in zip(reqs, bufs):
                eng.submit(0, ids[k], q, buf.array)
            eng.drain()
            comps = eng.poll(max_items=64)
            got = [b.array.copy() for b in bufs]
            for b in bufs:
                b.close()
        assert len(comps) == len(reqs) and all(c["status"] == 0 for c in comps)
        by_id = {c["request_id"]: c for c in comps}
        for i, ((k, q), out) in enumerate(zip(reqs, got), start=1):
            B = np.zeros((1, rows), np.uint32)
            srv.answer(q[None, :], B)
            if k == 0:
                C = np.zeros((1, groups, L), np.uint32)
                srv.compress_packed([ids[0]], B, C)
            else:
                C = np.zeros((1, rows, L), np.uint32)
                srv.compress([ids[1]], B, C)
            assert np.array_equal(out, C[0]), f"request {i}"
            assert by_id[i]["batch"] >= 1
    # the first packed and the first plain request against the oracle, every group and row
    E = server.exponents(server.global_hint(inst.D, inst.A))
    t = 64 + N_LWE.bit_length()
    for kind in (0, 1):
        i = next(i for i, (k, _) in enumerate(reqs) if k == kind)
        q = reqs[i][1]
        cl = inst.clients[kind]
        K = server.client_hint(cl.ck, E, cl.N)
        b = server.answer(inst.D, q)
        want = server.compress_packed(K, b, cl.N, 5, 1 << t) if kind == 0 else server.compress(K, b, cl.N)
        assert limbs_rows_to_ints(got[i]) == want, f"request {i + 1} vs the oracle"


def _hint_row(args):
    ck, e_row, N = args
    return server.client_hint_row(ck, e_row, N)


def test_mix_at_serving_scale_sampled(native):
    """The 256 MiB (16384 x 16384) and 1 GiB (32768 x 32768) databases of the serving mix,
    n = 1024, 2048-bit N, default steps (the 1 GiB answer in four 256 MiB steps, paced beside
    the other database): every response of a 24-request mix with staggered arrivals equals
    the one-at-a-time run, and sampled rows of three 256 MiB responses equal the oracle's."""
    import torch
    from multiprocessing import Pool
    from tests.gpu_util import pool_size
    from tests.instances import make_client
    n, nb, sides = 1024, 2048, (16384, 32768)
    servers, clients, Ds, streams = [], [], [], []
    for i, side in enumerate(sides):
        log(f"serve scale: database {side}x{side}")
        D = wl.database(60 + i, side, side, threads=16)
        A = wl.lwe_matrix(60 + i, side, n)
        st = torch.cuda.Stream()
        srv = native.Server(D, A, stream=st.cuda_stream)
        cl = make_client(60 + i, 0, A, nb, encrypt_secret=False)
        N_limbs, ck, L = client_arrays(cl, nb)
        cid = srv.add_client(N_limbs, nb, ck)
        srv.hint(cid)
        servers.append(srv)
        streams.append(st)
        clients.append((cid, cl, L, A))
        Ds.append(D)
    g = np.random.default_rng(61)
    which = [int(x) for x in g.integers(0, 2, size=24)]
    which[:3] = [0, 0, 0]
    qs = [g.integers(0, 1 << 32, size=sides[w], dtype=np.uint32) for w in which]

    def run(together):
        with native.Engine(max_batch=32) as eng:
            for s in servers:
                eng.add_db(s)
            bufs = [native.PinnedArray((sides[w], clients[w][2])) for w in which]
            t0 = eng.now_ms()
            for k, (w, q, b) in enumerate(zip(which, qs, bufs)):
                eng.submit(w, clients[w][0], q, b.array, arrival_ms=t0 + 0.3 * k if together else -1.0)
                if not together:
                    eng.drain()
            eng.drain()
            comps = eng.poll(64)
            outs = [b.array.copy() for b in bufs]
            for b in bufs:
                b.close()
        return outs, comps

    log("serve scale: one at a time")
    alone, _ = run(False)
    log("serve scale: mix")
    mix, comps = run(True)
    assert len(comps) == 24 and all(c["status"] == 0 for c in comps)
    for a, m in zip(alone, mix):
        assert np.array_equal(a, m)
    cid, cl, L, A = clients[0]
    rows = [0, 1, sides[0] - 1] + [int(x) for x in g.integers(2, sides[0] - 1, size=5)]
    E = server.exponents(server.global_hint(Ds[0], A, rows=rows))
    with Pool(pool_size()) as pool:
        K = pool.map(_hint_row, [(cl.ck, E[j], cl.N) for j in range(len(rows))])
    for k in range(3):
        b = server.answer(Ds[0][rows], qs[k])
        assert limbs_rows_to_ints(mix[k][rows]) == server.compress(K, b, cl.N), k
    for s in servers:
        s.close()
