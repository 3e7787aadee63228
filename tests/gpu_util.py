"""Shared helpers for the GPU tests (inputs and comparisons only)."""

import sys

import numpy as np
import scipy.sparse as sp


def announce(*args):
    """Print what the next GPU step is about, flushed before it runs."""
    print("[gpu]", *args, flush=True)
    sys.stdout.flush()


def random_csr(rows, cols, lengths, seed):
    """CSR with the given row lengths, sorted distinct columns, values in [-1, 1)."""
    rng = np.random.default_rng(seed)
    lengths = np.minimum(np.asarray(lengths, dtype=np.int64), cols)
    row_ptr = np.zeros(rows + 1, dtype=np.int64)
    np.cumsum(lengths, out=row_ptr[1:])
    col = np.empty(row_ptr[-1], dtype=np.int32)
    for i in range(rows):
        k = int(lengths[i])
        if k:
            col[row_ptr[i]:row_ptr[i + 1]] = np.sort(rng.choice(cols, size=k, replace=False))
    val = rng.uniform(-1.0, 1.0, size=row_ptr[-1])
    return row_ptr, col, val


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def true_rel_residual(A, x, f):
    S = A.to_scipy() if hasattr(A, "to_scipy") else A
    return np.linalg.norm(f - S @ x) / np.linalg.norm(f)


def scipy_of(row_ptr, col, val, rows, cols):
    return sp.csr_matrix((val, col, row_ptr), shape=(rows, cols))
