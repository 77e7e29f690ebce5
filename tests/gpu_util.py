"""Helpers for GPU tests: the HIP server built from a test instance."""
from __future__ import annotations

import os
import sys

import numpy as np

import workload as wl


def log(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


def client_arrays(cl, n_bits: int):
    """N limbs and ck limbs (n x L) for the C-ABI."""
    h = (n_bits + 31) // 32
    L = 2 * h
    N_limbs = wl.int_to_limbs(cl.N, h)
    ck = wl.ints_to_limbs([int(x) for x in cl.ck], L)
    return N_limbs, ck, L


def limbs_rows_to_ints(arr: np.ndarray) -> list:
    return [wl.limbs_to_int(arr[i]) for i in range(arr.shape[0])]


def pool_size() -> int:
    return max(1, min(16, os.cpu_count() or 1))
