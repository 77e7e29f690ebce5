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
KERNELS = {"matvec": 0, "gemm": 1, "compress": 2, "hint": 3, "table": 4, "kappa": 5}


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
    "pir_get_global_hint": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32,
                                             ctypes.c_void_p, ctypes.c_uint32]),
    "pir_get_client_hint": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32,
                                             ctypes.c_uint32, ctypes.c_void_p, ctypes.c_uint32]),
    "pir_client_limbs": (ctypes.c_uint32, [ctypes.c_void_p, ctypes.c_uint32]),
    "pir_stale_rows": (ctypes.c_int64, [ctypes.c_void_p, ctypes.c_uint32]),
    "pir_shape": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint32),
                                   ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint32),
                                   ctypes.POINTER(ctypes.c_uint64)]),
    "pir_profile": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32]),
    "pir_profile_read": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(ctypes.c_uint64)]),
    "pir_sync": (ctypes.c_int32, [ctypes.c_void_p]),
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

    def remove_client(self, cid: int) -> None:
        _check(_lib.pir_remove_client(self._h, cid), "pir_remove_client")

    def limbs(self, cid: int) -> int:
        return _lib.pir_client_limbs(self._h, cid)

    def stale_rows(self, cid: int | None = None) -> int:
        return _lib.pir_stale_rows(self._h, 0xFFFFFFFF if cid is None else cid)

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
