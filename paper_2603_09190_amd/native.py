"""ctypes binding of libzippir.so (include/zippir.h), argument marshalling only.

Arrays may be numpy arrays (host memory) or torch tensors on the server's GPU; one call's
arrays must all live on the same side.  Every computation happens in the HIP library:
if libzippir.so is missing this module raises on import.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libzippir.so")

PIR_OK, PIR_EINVAL, PIR_ENOMEM, PIR_EDEVICE, PIR_ESTALE, PIR_EBUSY = 0, -1, -2, -3, -4, -5
PIR_PTR_HOST, PIR_PTR_DEVICE = 0, 1
PATH_AUTO, PATH_MATVEC, PATH_MFMA = 0, 1, 2
KERNELS = {"matvec": 0, "gemm": 1, "compress": 2, "hint": 3, "table": 4, "key": 5, "offset_gemm": 6,
           "offset": 7, "step_matvec": 8, "step_combine": 9}


class ZipPIRError(RuntimeError):
    def __init__(self, status: int, func: str, detail: str):
        super().__init__(f"{func}: status {status} ({detail})")
        self.status = status


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2603_09190_amd.build`")

_lib = ctypes.CDLL(LIB_PATH)

_c_u32p = ctypes.c_void_p
_sig = {
    "pir_setup": (ctypes.c_int32, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32,
                                   ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32]),
    "pir_destroy": (None, [ctypes.c_void_p]),
    "pir_add_client": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32,
                                        ctypes.c_void_p, ctypes.c_uint32,
                                        ctypes.POINTER(ctypes.c_uint32)]),
    "pir_add_client_seeded": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32,
                                               ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32,
                                               ctypes.c_uint32, ctypes.c_void_p]),
    "pir_get_client_key": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                            ctypes.c_void_p, ctypes.c_uint32]),
    "pir_remove_client": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_uint32]),
    "pir_hint": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_uint32]),
    "pir_update_rows": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32,
                                         ctypes.c_void_p, ctypes.c_uint32]),
    "pir_answer": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32,
                                    ctypes.c_void_p, ctypes.c_uint32]),
    "pir_answer_path": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32,
                                         ctypes.c_void_p, ctypes.c_uint32, ctypes.c_int32]),
    "pir_compress": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32]),
    "pir_answer_compress": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32,
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32]),
    "pir_answer_compress_noalloc": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32,
                                                     ctypes.c_void_p, ctypes.c_void_p]),
    "pir_set_packing": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32]),
    "pir_packing_info": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint32),
                                          ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint32),
                                          ctypes.POINTER(ctypes.c_uint32)]),
    "pir_compress_packed": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32,
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32]),
    "pir_offset_answer": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32]),
    "pir_answer_offset": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32]),
    "pir_compressor_setup_ms": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_float),
                                                 ctypes.POINTER(ctypes.c_float)]),
    "pir_compress_offset": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32,
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32]),
    "pir_offset_answer_packed": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32,
                                                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                                  ctypes.c_uint32]),
    "pir_compress_offset_packed": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32,
                                                    ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32]),
    "pir_get_global_hint": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32,
                                             ctypes.c_void_p, ctypes.c_uint32]),
    "pir_get_client_hint": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32,
                                             ctypes.c_uint32, ctypes.c_void_p, ctypes.c_uint32]),
    "pir_client_limbs": (ctypes.c_uint32, [ctypes.c_void_p, ctypes.c_uint32]),
    "pir_stale_rows": (ctypes.c_int64, [ctypes.c_void_p, ctypes.c_uint32]),
    "pir_hint_window_bits": (ctypes.c_uint32, [ctypes.c_void_p, ctypes.c_uint32]),
    "pir_set_tiled_copy": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32]),
    "pir_tiled_copy": (ctypes.c_int32, [ctypes.c_void_p]),
    "pir_shape": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint32),
                                   ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint32),
                                   ctypes.POINTER(ctypes.c_uint64)]),
    "pir_profile": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32]),
    "pir_profile_read": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(ctypes.c_uint64)]),
    "pir_sync": (ctypes.c_int32, [ctypes.c_void_p]),
    "pir_engine_create": (ctypes.c_int32, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_uint32, ctypes.c_uint64]),
    "pir_engine_set_steps": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64]),
    "pir_engine_add_db": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint32)]),
    "pir_engine_submit": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_double, ctypes.POINTER(ctypes.c_uint64)]),
    "pir_engine_poll": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32,
                                         ctypes.POINTER(ctypes.c_uint32), ctypes.c_int32]),
    "pir_engine_drain": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32]),
    "pir_engine_stats_get": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p]),
    "pir_engine_now_ms": (ctypes.c_double, [ctypes.c_void_p]),
    "pir_engine_destroy": (None, [ctypes.c_void_p]),
    "pir_engine_capacity": (ctypes.c_uint32, [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32]),
    "pir_engine_plan": (ctypes.c_uint32, [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32]),
    "pir_compressor_create": (ctypes.c_int32, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.c_void_p,
                                               ctypes.c_uint32, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_uint32,
                                               ctypes.c_void_p, ctypes.c_uint32]),
    "pir_compressor_create_packed": (ctypes.c_int32, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int,
                                                      ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64,
                                                      ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p,
                                                      ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32]),
    "pir_compressor_destroy": (None, [ctypes.c_void_p]),
    "pir_compressor_key": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_void_p,
                                            ctypes.c_uint32]),
    "pir_compressor_info": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint32),
                                             ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint64)]),
    "pir_compress_lwe": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32,
                                          ctypes.c_void_p, ctypes.c_uint32]),
    "pir_compress_rlwe": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_uint32, ctypes.c_void_p, ctypes.c_uint32]),
    "pir_read_probe": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_uint32,
                                        ctypes.c_void_p]),
    "pir_host_alloc": (ctypes.c_void_p, [ctypes.c_uint64]),
    "pir_host_free": (None, [ctypes.c_void_p]),
    "pir_strerror": (ctypes.c_char_p, [ctypes.c_int32]),
    "pir_last_error": (ctypes.c_char_p, []),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_sig)


def lib() -> ctypes.CDLL:
    return _lib


def _check(st: int, func: str) -> None:
    if st != PIR_OK:
        raise ZipPIRError(st, func, _lib.pir_last_error().decode(errors="replace"))


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


def _ptr(x, want_device: bool | None = None):
    """(pointer, is_device) of a contiguous numpy array or torch tensor."""
    if x is None:
        return None, None
    if _is_torch(x):
        if not x.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return ctypes.c_void_p(x.data_ptr()), bool(x.is_cuda)
    a = np.asarray(x)
    if not a.flags.c_contiguous:
        raise ValueError("array must be C-contiguous")
    return ctypes.c_void_p(a.ctypes.data), False


def _flags(*arrays) -> int:
    kinds = {_ptr(a)[1] for a in arrays if a is not None}
    if len(kinds) != 1:
        raise ValueError("all arrays of one call must be on the host or all on the device")
    return PIR_PTR_DEVICE if kinds.pop() else PIR_PTR_HOST


def _rows_arg(rows):
    if rows is None:
        return None, 0, None
    r = np.ascontiguousarray(np.asarray(rows, dtype=np.uint32))
    return ctypes.c_void_p(r.ctypes.data), len(r), r


def _nbytes(x) -> int:
    if _is_torch(x):
        return x.numel() * x.element_size()
    return np.asarray(x).nbytes


class Server:
    """One database (rows x cols uint8) with its public LWE matrix A (cols x n uint32)."""

    def __init__(self, D, A, device: int = 0, stream=None):
        rows, cols = D.shape
        cols2, n = A.shape
        if cols2 != cols:
            raise ValueError("A must have one row per database column")
        h = ctypes.c_void_p()
        st = ctypes.c_void_p(stream) if stream is not None else None
        fl = _flags(D, A)
        if _nbytes(D) != rows * cols or _nbytes(A) != cols * n * 4:
            raise ValueError("D must be uint8 and A 32-bit")
        _check(_lib.pir_setup(ctypes.byref(h), device, st, _ptr(D)[0], rows, cols, _ptr(A)[0], n, fl),
               "pir_setup")
        self._h = h
        self.rows, self.cols, self.n = rows, cols, n

    def close(self) -> None:
        if getattr(self, "_h", None):
            _lib.pir_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- clients
    def add_client(self, N_limbs, N_bits: int, ck) -> int:
        cid = ctypes.c_uint32()
        _check(_lib.pir_add_client(self._h, _ptr(N_limbs)[0], N_bits, _ptr(ck)[0], _flags(N_limbs, ck),
                                   ctypes.byref(cid)), "pir_add_client")
        return cid.value

    def add_client_seeded(self, N_limbs, N_bits: int, seed: bytes, first_query: int, count: int) -> list:
        """Clients for queries first_query .. first_query+count-1 whose keys the device expands
        from the 32-byte seed (pir_add_client_seeded); returns their ids."""
        if len(seed) != 32:
            raise ValueError("seed must be 32 bytes")
        sb = ctypes.create_string_buffer(bytes(seed), 32)
        ids = np.zeros(count, np.uint32)
        _check(_lib.pir_add_client_seeded(self._h, _ptr(N_limbs)[0], N_bits, ctypes.cast(sb, ctypes.c_void_p),
                                          first_query, count, _flags(N_limbs), ctypes.c_void_p(ids.ctypes.data)),
               "pir_add_client_seeded")
        return [int(x) for x in ids]

    def client_key(self, cid: int, k0: int, nk: int, out) -> None:
        _check(_lib.pir_get_client_key(self._h, cid, k0, nk, _ptr(out)[0], _flags(out)), "pir_get_client_key")

    def remove_client(self, cid: int) -> None:
        _check(_lib.pir_remove_client(self._h, cid), "pir_remove_client")

    def limbs(self, cid: int) -> int:
        return _lib.pir_client_limbs(self._h, cid)

    def stale_rows(self, cid: int | None = None) -> int:
        return _lib.pir_stale_rows(self._h, 0xFFFFFFFF if cid is None else cid)

    def set_tiled_copy(self, enable: bool) -> None:
        """Make (True) or free (False) the contraction's tiled copy of D (see pir_set_tiled_copy)."""
        _check(_lib.pir_set_tiled_copy(self._h, 1 if enable else 0), "pir_set_tiled_copy")

    def tiled_copy(self) -> bool:
        return bool(_lib.pir_tiled_copy(self._h))

    def hint_window_bits(self, cid: int) -> int:
        """Window width of the fixed-base table the client's last hint used (8 or 11)."""
        return _lib.pir_hint_window_bits(self._h, cid)

    def hint(self, cid: int, rows=None) -> None:
        p, n, _keep = _rows_arg(rows)
        _check(_lib.pir_hint(self._h, cid, p, n), "pir_hint")

    def update_rows(self, rows, new_rows) -> None:
        p, n, _keep = _rows_arg(rows)
        _check(_lib.pir_update_rows(self._h, p, n, _ptr(new_rows)[0], _flags(new_rows)), "pir_update_rows")

    # -- online
    def answer(self, Q, B, path: int = PATH_AUTO) -> None:
        batch = Q.shape[0] if len(Q.shape) == 2 else 1
        _check(_lib.pir_answer_path(self._h, _ptr(Q)[0], batch, _ptr(B)[0], _flags(Q, B), path),
               "pir_answer_path")

    def compress(self, ids, B, C) -> None:
        ids_a = np.ascontiguousarray(np.asarray(ids, dtype=np.uint32))
        _check(_lib.pir_compress(self._h, ctypes.c_void_p(ids_a.ctypes.data), len(ids_a), _ptr(B)[0],
                                 _ptr(C)[0], _flags(B, C)), "pir_compress")

    def answer_compress(self, q, cid: int, B, C) -> None:
        """One query of one client: B = D.q mod 2^32 and C = K (1 + B N) mod N^2 in one call."""
        _check(_lib.pir_answer_compress(self._h, _ptr(q)[0], cid, _ptr(B)[0], _ptr(C)[0], _flags(q, B, C)),
               "pir_answer_compress")

    def answer_compress_noalloc(self, q, cid: int, B, C) -> None:
        """pir_answer_compress on device arrays with no device allocation: the matvec's segment
        partials go to the library's static per-device scratch array."""
        for x in (q, B, C):
            if _ptr(x)[1] is not True:
                raise ValueError("pir_answer_compress_noalloc takes device arrays only")
        _check(_lib.pir_answer_compress_noalloc(self._h, _ptr(q)[0], cid, _ptr(B)[0], _ptr(C)[0]),
               "pir_answer_compress_noalloc")

    # -- packed responses
    def set_packing(self, cid: int, ell: int) -> None:
        _check(_lib.pir_set_packing(self._h, cid, ell), "pir_set_packing")

    def packing_info(self, cid: int) -> dict:
        v = [ctypes.c_uint32() for _ in range(4)]
        _check(_lib.pir_packing_info(self._h, cid, *[ctypes.byref(x) for x in v]), "pir_packing_info")
        return dict(zip(("ell", "ell_max", "log2_gamma", "groups"), (x.value for x in v)))

    def compress_packed(self, ids, B, C) -> None:
        ids_a = np.ascontiguousarray(np.asarray(ids, dtype=np.uint32))
        _check(_lib.pir_compress_packed(self._h, ctypes.c_void_p(ids_a.ctypes.data), len(ids_a), _ptr(B)[0],
                                        _ptr(C)[0], _flags(B, C)), "pir_compress_packed")

    # -- full protocol (offset answer)
    def offset_answer(self, ids, CKO, B, T) -> None:
        ids_a = np.ascontiguousarray(np.asarray(ids, dtype=np.uint32))
        _check(_lib.pir_offset_answer(self._h, ctypes.c_void_p(ids_a.ctypes.data), len(ids_a), _ptr(CKO)[0],
                                      _ptr(B)[0], _ptr(T)[0], _flags(CKO, B, T)), "pir_offset_answer")

    def answer_offset(self, ids, Q, CKO, B, T) -> None:
        """B = D.Q and T = (B + E.CKO) mod N in one call (the contraction beside the answer)."""
        ids_a = np.ascontiguousarray(np.asarray(ids, dtype=np.uint32))
        _check(_lib.pir_answer_offset(self._h, ctypes.c_void_p(ids_a.ctypes.data), len(ids_a), _ptr(Q)[0],
                                      _ptr(CKO)[0], _ptr(B)[0], _ptr(T)[0], _flags(Q, CKO, B, T)),
               "pir_answer_offset")

    def compress_offset(self, ids, T, C) -> None:
        ids_a = np.ascontiguousarray(np.asarray(ids, dtype=np.uint32))
        _check(_lib.pir_compress_offset(self._h, ctypes.c_void_p(ids_a.ctypes.data), len(ids_a), _ptr(T)[0],
                                        _ptr(C)[0], _flags(T, C)), "pir_compress_offset")

    def offset_answer_packed(self, ids, CKO, B, Tg) -> None:
        ids_a = np.ascontiguousarray(np.asarray(ids, dtype=np.uint32))
        _check(_lib.pir_offset_answer_packed(self._h, ctypes.c_void_p(ids_a.ctypes.data), len(ids_a), _ptr(CKO)[0],
                                             _ptr(B)[0], _ptr(Tg)[0], _flags(CKO, B, Tg)), "pir_offset_answer_packed")

    def compress_offset_packed(self, ids, Tg, Cg) -> None:
        ids_a = np.ascontiguousarray(np.asarray(ids, dtype=np.uint32))
        _check(_lib.pir_compress_offset_packed(self._h, ctypes.c_void_p(ids_a.ctypes.data), len(ids_a),
                                               _ptr(Tg)[0], _ptr(Cg)[0], _flags(Tg, Cg)), "pir_compress_offset_packed")

    # -- introspection
    def global_hint(self, row0: int, nrows: int, out) -> None:
        _check(_lib.pir_get_global_hint(self._h, row0, nrows, _ptr(out)[0], _flags(out)),
               "pir_get_global_hint")

    def client_hint(self, cid: int, row0: int, nrows: int, out) -> None:
        _check(_lib.pir_get_client_hint(self._h, cid, row0, nrows, _ptr(out)[0], _flags(out)),
               "pir_get_client_hint")

    def device_bytes(self) -> int:
        r, c, n, b = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint64()
        _check(_lib.pir_shape(self._h, ctypes.byref(r), ctypes.byref(c), ctypes.byref(n), ctypes.byref(b)),
               "pir_shape")
        return b.value

    def profile(self, enable: bool) -> None:
        _check(_lib.pir_profile(self._h, 1 if enable else 0), "pir_profile")

    def profile_read(self, kernel: str):
        """(total milliseconds, launches) of one kernel since profiling started."""
        ms, cnt = ctypes.c_double(), ctypes.c_uint64()
        _check(_lib.pir_profile_read(self._h, KERNELS[kernel], ctypes.byref(ms), ctypes.byref(cnt)),
               "pir_profile_read")
        return ms.value, cnt.value

    def sync(self) -> None:
        _check(_lib.pir_sync(self._h), "pir_sync")


# ----------------------------------------------------------------------------- serving engine

class Completion(ctypes.Structure):
    _fields_ = [("request_id", ctypes.c_uint64), ("db", ctypes.c_uint32), ("client_id", ctypes.c_uint32),
                ("status", ctypes.c_int32), ("batch", ctypes.c_uint32), ("arrival_ms", ctypes.c_double),
                ("start_ms", ctypes.c_double), ("done_ms", ctypes.c_double)]


class EngineStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("failed", ctypes.c_uint64),
                ("batches", ctypes.c_uint64), ("admission_waits", ctypes.c_uint64),
                ("device_bytes_peak", ctypes.c_uint64), ("p50_ms", ctypes.c_double),
                ("p99_ms", ctypes.c_double), ("mean_batch", ctypes.c_double)]


class Compressor:
    """Standalone LWE / RLWE ciphertext compressor with a resident compression key.

    ``q`` is the LWE modulus (2 <= q <= 2^64).  Arrays of LWE entries are uint32 when
    q <= 2^32 and uint64 otherwise; keys and outputs are uint32 limb arrays (L limbs each).
    """

    def __init__(self, n: int, q: int, N_limbs, N_bits: int, ck=None, packed=None, t: int = 0,
                 delta_log2: int = 0, device: int = 0, stream=None):
        if not (2 <= q <= 1 << 64):
            raise ValueError("q must be in [2, 2^64]")
        h = ctypes.c_void_p()
        st = ctypes.c_void_p(stream) if stream is not None else None
        qarg = q % (1 << 64)
        N_limbs = np.ascontiguousarray(N_limbs, dtype=np.uint32)
        if packed is None:
            key = np.ascontiguousarray(ck, dtype=np.uint32)
            _check(_lib.pir_compressor_create(ctypes.byref(h), device, st, n, qarg, _ptr(N_limbs)[0], N_bits,
                                              _ptr(key)[0], PIR_PTR_HOST), "pir_compressor_create")
        else:
            key = np.ascontiguousarray(packed, dtype=np.uint32)
            _check(_lib.pir_compressor_create_packed(ctypes.byref(h), device, st, n, qarg, _ptr(N_limbs)[0],
                                                     N_bits, _ptr(key)[0], t, delta_log2, PIR_PTR_HOST),
                   "pir_compressor_create_packed")
        self._h = h
        self.n, self.q = n, q
        self.dtype = np.uint32 if q <= 1 << 32 else np.uint64
        L, w, b = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint64()
        _check(_lib.pir_compressor_info(self._h, ctypes.byref(L), ctypes.byref(w), ctypes.byref(b)),
               "pir_compressor_info")
        self.L, self.windows = L.value, w.value

    def setup_ms(self) -> dict:
        """Device milliseconds of the setup: key unpacking (packed keys) and table build."""
        u, t = ctypes.c_float(), ctypes.c_float()
        _check(_lib.pir_compressor_setup_ms(self._h, ctypes.byref(u), ctypes.byref(t)), "pir_compressor_setup_ms")
        return {"unpack_ms": u.value, "table_ms": t.value}

    def info(self) -> dict:
        L, w, b = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint64()
        _check(_lib.pir_compressor_info(self._h, ctypes.byref(L), ctypes.byref(w), ctypes.byref(b)),
               "pir_compressor_info")
        return {"L": L.value, "windows": w.value, "device_bytes": b.value}

    def key(self, k0: int = 0, nk: int | None = None) -> np.ndarray:
        nk = self.n - k0 if nk is None else nk
        out = np.zeros((nk, self.L), np.uint32)
        _check(_lib.pir_compressor_key(self._h, k0, nk, _ptr(out)[0], PIR_PTR_HOST), "pir_compressor_key")
        return out

    def compress_lwe(self, A, B, X) -> None:
        """A: rows x n, B: rows (entries of self.dtype); X: rows x L uint32 (host or device)."""
        rows = int(np.shape(B)[0])
        _check(_lib.pir_compress_lwe(self._h, _ptr(A)[0], _ptr(B)[0], rows, _ptr(X)[0], _flags(A, B, X)),
               "pir_compress_lwe")

    def compress_rlwe(self, A, B, ks, X) -> None:
        """A, B: the n coefficients of an RLWE ciphertext; ks: coefficient indices; X: len(ks) x L."""
        k = np.ascontiguousarray(np.asarray(ks, dtype=np.uint32))
        _check(_lib.pir_compress_rlwe(self._h, _ptr(A)[0], _ptr(B)[0], ctypes.c_void_p(k.ctypes.data), len(k),
                                      _ptr(X)[0], _flags(A, B, X)), "pir_compress_rlwe")

    def close(self) -> None:
        if getattr(self, "_h", None):
            _lib.pir_compressor_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def read_probe(buf, sink, blocks: int = 8192, stream=None) -> None:
    """One streaming read of the device tensor ``buf`` (measurement only; see pir_read_probe)."""
    st = ctypes.c_void_p(stream) if stream is not None else None
    _check(_lib.pir_read_probe(_ptr(buf)[0], _nbytes(buf), _ptr(sink)[0], blocks, st), "pir_read_probe")


class PinnedArray:
    """A numpy view of pinned host memory from pir_host_alloc."""

    def __init__(self, shape, dtype=np.uint32):
        self.nbytes = int(np.prod(shape)) * np.dtype(dtype).itemsize
        self._p = _lib.pir_host_alloc(self.nbytes)
        if not self._p:
            raise MemoryError("pir_host_alloc failed")
        buf = (ctypes.c_char * self.nbytes).from_address(self._p)
        self.array = np.frombuffer(buf, dtype=dtype).reshape(shape)

    def close(self):
        if getattr(self, "_p", None):
            self.array = None
            _lib.pir_host_free(self._p)
            self._p = None

    def __del__(self):
        self.close()


def engine_capacity(budget_free: int, bytes_per_request: int, max_batch: int) -> int:
    return _lib.pir_engine_capacity(budget_free, bytes_per_request, max_batch)


def engine_plan(queued_limbs, capacity: int) -> int:
    a = np.ascontiguousarray(np.asarray(queued_limbs, dtype=np.uint32))
    return _lib.pir_engine_plan(ctypes.c_void_p(a.ctypes.data), len(a), capacity)


class Engine:
    """Continuous-batching serving engine over several Servers (each with its own stream)."""

    def __init__(self, max_batch: int = 32, hbm_budget: int = 0):
        h = ctypes.c_void_p()
        _check(_lib.pir_engine_create(ctypes.byref(h), max_batch, hbm_budget), "pir_engine_create")
        self._h = h
        self._servers = []

    def set_steps(self, step_bytes: int, copy_bytes: int) -> None:
        """Bytes of D per answer step and response bytes per download step (before add_db)."""
        _check(_lib.pir_engine_set_steps(self._h, step_bytes, copy_bytes), "pir_engine_set_steps")

    def add_db(self, server: Server) -> int:
        idx = ctypes.c_uint32()
        _check(_lib.pir_engine_add_db(self._h, server._h, ctypes.byref(idx)), "pir_engine_add_db")
        self._servers.append(server)
        return idx.value

    def submit(self, db: int, client: int, query, result, arrival_ms: float = -1.0) -> int:
        q = np.ascontiguousarray(np.asarray(query, dtype=np.uint32))
        rid = ctypes.c_uint64()
        _check(_lib.pir_engine_submit(self._h, db, client, ctypes.c_void_p(q.ctypes.data), _ptr(result)[0],
                                      float(arrival_ms), ctypes.byref(rid)), "pir_engine_submit")
        return rid.value

    def poll(self, max_items: int = 256, timeout_ms: int = 0):
        arr = (Completion * max_items)()
        cnt = ctypes.c_uint32()
        _check(_lib.pir_engine_poll(self._h, arr, max_items, ctypes.byref(cnt), timeout_ms), "pir_engine_poll")
        return [{f: getattr(arr[i], f) for f, _ in Completion._fields_} for i in range(cnt.value)]

    def drain(self, timeout_ms: int = -1) -> None:
        _check(_lib.pir_engine_drain(self._h, timeout_ms), "pir_engine_drain")

    def stats(self) -> dict:
        st = EngineStats()
        _check(_lib.pir_engine_stats_get(self._h, ctypes.byref(st)), "pir_engine_stats_get")
        return {f: getattr(st, f) for f, _ in EngineStats._fields_}

    def now_ms(self) -> float:
        return _lib.pir_engine_now_ms(self._h)

    def close(self) -> None:
        if getattr(self, "_h", None):
            _lib.pir_engine_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
