"""Python binding of the C ABI in ``include/amg.h`` (ctypes; marshalling only).

Every step of the solve runs in the library's HIP kernels; this module only
converts arguments.  PyTorch supplies device memory (through the caching
allocator, handed to the library as its allocator hook) and the current HIP
stream.  The shared library is built in-tree by ``paper_1811_05704_amd.build``;
if it is missing, loading raises instead of falling back to anything else.
"""

from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libamg.so")

AMG_OK = 0
AMG_NOT_CONVERGED = 1
AMG_ERR = {
    -1: "AMG_ERR_INVALID_ARG", -2: "AMG_ERR_BAD_CSR", -3: "AMG_ERR_ZERO_DIAG",
    -4: "AMG_ERR_SINGULAR_COARSE", -5: "AMG_ERR_OOM", -6: "AMG_ERR_HIP",
    -7: "AMG_ERR_BREAKDOWN", -8: "AMG_ERR_TOO_LARGE", -9: "AMG_ERR_NAN",
}
SOLVERS = {"cg": 0, "bicgstab": 1, "gmres": 2}
RELAX = {"spai0": 0, "jacobi": 1, "chebyshev": 2}
PRECISION = {"fp64": 0, "mixed": 1}


class AmgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{AMG_ERR.get(code, code)}: {msg}")
        self.code = code


class Params(C.Structure):
    _fields_ = [
        ("solver", C.c_int32), ("relax", C.c_int32), ("precision", C.c_int32),
        ("npre", C.c_int32), ("npost", C.c_int32), ("coarse_enough", C.c_int32),
        ("max_levels", C.c_int32), ("max_iter", C.c_int32),
        ("eps_strong", C.c_double), ("jacobi_omega", C.c_double), ("tol", C.c_double),
        ("use_graph", C.c_int32), ("check_every", C.c_int32),
        ("cheb_degree", C.c_int32), ("cheb_ratio", C.c_double), ("gmres_m", C.c_int32),
        ("fuse_coarse", C.c_int32),
    ]


class Info(C.Structure):
    _fields_ = [
        ("iters", C.c_int32), ("levels", C.c_int32), ("restarts", C.c_int32), ("status", C.c_int32),
        ("rel_resid", C.c_double), ("true_rel_resid", C.c_double), ("setup_s", C.c_double),
        ("solve_s", C.c_double), ("op_complexity", C.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class Allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", C.c_void_p)]


_lib = None


def lib():
    """Load ``libamg.so``; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} not found: build it with `python -m paper_1811_05704_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    P64, P32, PD = C.POINTER(C.c_int64), C.POINTER(C.c_int32), C.POINTER(C.c_double)
    sig = {
        "amg_params_default": (None, [C.POINTER(Params)]),
        "amg_setup": (i32, [i64, P64, P32, PD, C.POINTER(Params), C.POINTER(Allocator), vp, C.POINTER(vp)]),
        "amg_setup_host": (i32, [i64, P64, P32, PD, C.POINTER(Params), C.POINTER(vp)]),
        "amg_setup_block": (i32, [i64, i32, P64, P32, PD, C.POINTER(Params), C.POINTER(Allocator), vp,
                                  C.POINTER(vp)]),
        "amg_setup_block_host": (i32, [i64, i32, P64, P32, PD, C.POINTER(Params), C.POINTER(vp)]),
        "amg_setup_schur": (i32, [i64, P64, P32, PD, i64, C.POINTER(Params), C.POINTER(Allocator), vp,
                                  C.POINTER(vp)]),
        "amg_setup_schur_host": (i32, [i64, P64, P32, PD, i64, C.POINTER(Params), C.POINTER(vp)]),
        "amg_setup_schur_masked": (i32, [i64, P64, P32, PD, C.POINTER(C.c_uint8), C.POINTER(Params),
                                         C.POINTER(Allocator), vp, C.POINTER(vp)]),
        "amg_get_level_bsr": (i32, [vp, i32, i32, P64, P32, PD]),
        "amg_get_smoother_blocks": (i32, [vp, i32, PD, PD]),
        "amg_solve": (i32, [vp, vp, vp, vp, C.POINTER(Info)]),
        "amg_release": (None, [vp]),
        "amg_last_error": (C.c_char_p, []),
        "amg_vcycle": (i32, [vp, vp, vp, vp]),
        "amg_num_levels": (i32, [vp]),
        "amg_level_info": (i32, [vp, i32, P64, P64, P64]),
        "amg_get_aggregates": (i32, [vp, i32, P32]),
        "amg_get_level_csr": (i32, [vp, i32, i32, P64, P32, PD]),
        "amg_get_smoother": (i32, [vp, i32, PD, PD, PD]),
        "amg_level_kernel_info": (i32, [vp, i32, i32, i32, P32, P32, P32, P32]),
        "amg_csr_upload": (i32, [i64, i64, P64, P32, PD, i32, vp, C.POINTER(vp)]),
        "amg_csr_spmv": (i32, [vp, vp, vp, vp]),
        "amg_csr_kernel_info": (i32, [vp, P32, P32, P32, P32]),
        "amg_csr_column_bytes": (i32, [vp, P32]),
        "amg_csr_release": (None, [vp]),
        "amg_time_kernel": (i32, [vp, i32, i32, vp, PD, PD]),
        "amg_tail_info": (i32, [vp, P32, P32]),
        "amg_setup_profile": (i32, [vp, PD]),
        "amg_vcycle_noalloc": (i32, [vp, vp, vp, vp]),
        "amg_tail_set_wait": (i32, [vp, dbl]),
        "amg_server_create": (i32, [C.POINTER(Params), C.c_size_t, i32, i32, vp, C.POINTER(vp)]),
        "amg_server_submit": (i32, [vp, C.c_uint64, i64, P64, P32, PD, PD]),
        "amg_server_step": (i32, [vp, P32, P32]),
        "amg_server_wait_ready": (i32, [vp, i32, C.c_double, P32]),
        "amg_server_poll": (i32, [vp, C.POINTER(C.c_uint64), P64]),
        "amg_server_fetch": (i32, [vp, C.c_uint64, PD, C.POINTER(Info), PD]),
        "amg_server_destroy": (None, [vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def exported_symbols():
    return [
        "amg_params_default", "amg_setup", "amg_setup_host", "amg_setup_block", "amg_setup_block_host",
        "amg_setup_schur", "amg_setup_schur_host", "amg_setup_schur_masked",
        "amg_get_level_bsr", "amg_get_smoother_blocks", "amg_solve", "amg_release",
        "amg_last_error", "amg_vcycle", "amg_num_levels", "amg_level_info", "amg_get_aggregates",
        "amg_get_level_csr", "amg_get_smoother", "amg_level_kernel_info", "amg_csr_upload", "amg_csr_spmv",
        "amg_csr_kernel_info", "amg_csr_column_bytes", "amg_csr_release", "amg_time_kernel", "amg_tail_info", "amg_tail_set_wait",
        "amg_setup_profile", "amg_vcycle_noalloc",
        "amg_server_create", "amg_server_submit", "amg_server_step", "amg_server_wait_ready", "amg_server_poll",
        "amg_server_fetch", "amg_server_destroy",
    ]


def _check(code):
    if code < 0:
        raise AmgError(code, lib().amg_last_error().decode())
    return code


def make_params(**kw) -> Params:
    """Defaults of ``amg_params_default`` overridden by keyword arguments.

    Accepts the names of the struct fields and string values for ``solver``
    ("cg" | "bicgstab" | "gmres"), ``relax`` ("spai0" | "jacobi" | "chebyshev") and ``precision``
    ("fp64" | "mixed").
    """
    p = Params()
    lib().amg_params_default(C.byref(p))
    for k, v in kw.items():
        if k == "solver" and isinstance(v, str):
            v = SOLVERS[v]
        elif k == "relax" and isinstance(v, str):
            v = RELAX[v]
        elif k == "precision" and isinstance(v, str):
            v = PRECISION[v]
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def _csr_arrays(A):
    row_ptr = np.ascontiguousarray(A.row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(A.col, dtype=np.int32)
    val = np.ascontiguousarray(A.val, dtype=np.float64)
    return row_ptr, col, val


def _is_block(A):
    return hasattr(A, "nb") and hasattr(A, "b")


def _bsr_arrays(A):
    row_ptr = np.ascontiguousarray(A.row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(A.col, dtype=np.int32)
    val = np.ascontiguousarray(A.val, dtype=np.float64)
    return row_ptr, col, val


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


class _Handle:
    """Queries shared by device and host-only handles."""

    _h = None

    @property
    def nlevels(self) -> int:
        return int(lib().amg_num_levels(self._h))

    def level_info(self, level):
        n, na, npp = C.c_int64(), C.c_int64(), C.c_int64()
        _check(lib().amg_level_info(self._h, level, C.byref(n), C.byref(na), C.byref(npp)))
        return n.value, na.value, npp.value

    def aggregates(self, level) -> np.ndarray:
        n, _, _ = self.level_info(level)
        out = np.empty(n, dtype=np.int32)
        _check(lib().amg_get_aggregates(self._h, level, _ptr(out, C.c_int32)))
        return out

    def level_csr(self, level, which="A"):
        """(rows, cols, row_ptr, col, val) of A_l, P_l or R_l."""
        w = {"A": 0, "P": 1, "R": 2}[which]
        n, na, npp = self.level_info(level)
        if w == 0:
            rows, nnz = n, na
            cols = n
        else:
            nc = self.level_info(level + 1)[0]
            rows, cols = (n, nc) if w == 1 else (nc, n)
            nnz = npp
        rp = np.empty(rows + 1, dtype=np.int64)
        c = np.empty(nnz, dtype=np.int32)
        v = np.empty(nnz, dtype=np.float64)
        _check(lib().amg_get_level_csr(self._h, level, w, _ptr(rp, C.c_int64), _ptr(c, C.c_int32),
                                       _ptr(v, C.c_double)))
        return rows, cols, rp, c, v

    def level_scipy(self, level, which="A"):
        import scipy.sparse as sp

        rows, cols, rp, c, v = self.level_csr(level, which)
        return sp.csr_matrix((v, c, rp), shape=(rows, cols))

    def smoother(self, level):
        n, _, _ = self.level_info(level)
        m = np.empty(n, dtype=np.float64)
        om = C.c_double()
        hi = C.c_double()
        _check(lib().amg_get_smoother(self._h, level, _ptr(m, C.c_double), C.byref(om), C.byref(hi)))
        return m, om.value, hi.value

    SETUP_PHASES = ("input", "strength", "aggregate", "prolongator", "transpose", "smoother", "galerkin",
                    "upload", "coarse_inverse", "other")

    def setup_profile(self):
        """Seconds of the setup by step (names in SETUP_PHASES)."""
        out = (C.c_double * len(self.SETUP_PHASES))()
        _check(lib().amg_setup_profile(self._h, out))
        return dict(zip(self.SETUP_PHASES, list(out)))

    def level_bsr(self, level, which="A", b=4):
        """(block rows, block cols, row_ptr, col, blocks[nnzb, b, b]) of a block level matrix."""
        w = {"A": 0, "P": 1, "R": 2}[which]
        n, na, npp = self.level_info(level)
        if w == 0:
            rows, cols, nnzb = n, n, na
        else:
            nc = self.level_info(level + 1)[0]
            rows, cols = (n, nc) if w == 1 else (nc, n)
            nnzb = npp
        rp = np.empty(rows + 1, dtype=np.int64)
        c = np.empty(nnzb, dtype=np.int32)
        v = np.empty(nnzb * b * b, dtype=np.float64)
        _check(lib().amg_get_level_bsr(self._h, level, w, _ptr(rp, C.c_int64), _ptr(c, C.c_int32),
                                       _ptr(v, C.c_double)))
        return rows, cols, rp, c, v.reshape(nnzb, b, b)

    def smoother_blocks(self, level, b=4):
        n, _, _ = self.level_info(level)
        M = np.empty(n * b * b, dtype=np.float64)
        om = C.c_double()
        _check(lib().amg_get_smoother_blocks(self._h, level, _ptr(M, C.c_double), C.byref(om)))
        return M.reshape(n, b, b), om.value

    def level_kernel_info(self, level, which="A", precision="fp64"):
        """SpMV schedule of A_l, P_l or R_l in the given value type (host query)."""
        w = {"A": 0, "P": 1, "R": 2}[which]
        p = PRECISION[precision] if isinstance(precision, str) else int(precision)
        k, l, b, nb = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib().amg_level_kernel_info(self._h, level, w, p, C.byref(k), C.byref(l), C.byref(b), C.byref(nb)))
        return {"kind": ("stream", "vector")[k.value], "lanes": l.value, "blocks": b.value,
                "block_bytes": nb.value}

    def release(self):
        if self._h:
            lib().amg_release(self._h)
            self._h = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass


class HostHierarchy(_Handle):
    """Hierarchy built on the host only (``amg_setup_host``, or
    ``amg_setup_block_host`` for a block matrix, or ``amg_setup_schur_host``
    for a field split with ``n_u`` velocity unknowns); no device needed."""

    def __init__(self, A, n_u=None, **params):
        self.params = make_params(**params)
        h = C.c_void_p()
        if n_u is not None:
            rp, c, v = _csr_arrays(A)
            _check(lib().amg_setup_schur_host(int(A.n), _ptr(rp, C.c_int64), _ptr(c, C.c_int32),
                                              _ptr(v, C.c_double), int(n_u), C.byref(self.params), C.byref(h)))
        elif _is_block(A):
            rp, c, v = _bsr_arrays(A)
            _check(lib().amg_setup_block_host(int(A.nb), int(A.b), _ptr(rp, C.c_int64), _ptr(c, C.c_int32),
                                              _ptr(v, C.c_double), C.byref(self.params), C.byref(h)))
        else:
            rp, c, v = _csr_arrays(A)
            _check(lib().amg_setup_host(int(A.n), _ptr(rp, C.c_int64), _ptr(c, C.c_int32), _ptr(v, C.c_double),
                                        C.byref(self.params), C.byref(h)))
        self._h = h


def _torch_stream():
    import torch

    return torch.cuda.current_stream()


class Solver(_Handle):
    """AMG-preconditioned Krylov solver resident on the current HIP device.

    ``A`` has ``n``, ``row_ptr``, ``col``, ``val`` (host arrays); keyword
    arguments are :class:`Params` fields.  With ``torch_alloc`` (default) the
    library's device memory comes from PyTorch's caching allocator.  With
    ``n_u`` the Schur-complement field split (``amg_setup_schur``): A is the
    whole velocity/pressure system, velocity unknowns first; with ``pmask``
    (one byte per unknown, 1 = pressure) the same split in any order
    (``amg_setup_schur_masked``).
    """

    def __init__(self, A, torch_alloc: bool = True, alloc_limit=None, n_u=None, pmask=None, **params):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("amg.Solver needs a HIP device")
        self.params = make_params(**params)
        self.n = int(A.n)
        self.device = torch.cuda.current_device()
        stream = _torch_stream()
        self._alloc = None
        alloc_p = None
        # alloc_limit (bytes, with torch_alloc): requests that would take the
        # library's live device memory past it are refused (the library then
        # runs that setup step on the host, or reports AMG_ERR_OOM)
        self.peak_bytes = 0
        if torch_alloc:
            dev = self.device
            self._live = {}
            live_bytes = [0]

            def _a(size, strm, ctx):
                size = int(size)
                if alloc_limit is not None and live_bytes[0] + size > alloc_limit:
                    return None
                try:
                    ptr = torch.cuda.caching_allocator_alloc(size, dev, stream)
                except Exception:
                    return None
                self._live[ptr] = size
                live_bytes[0] += size
                self.peak_bytes = max(self.peak_bytes, live_bytes[0])
                return ptr

            def _f(ptr, strm, ctx):
                if ptr in self._live:
                    live_bytes[0] -= self._live.pop(ptr)
                    torch.cuda.caching_allocator_delete(ptr)

            self._alloc = Allocator(ALLOC_FN(_a), FREE_FN(_f), None)
            alloc_p = C.byref(self._alloc)
        h = C.c_void_p()
        if pmask is not None:
            rp, c, v = _csr_arrays(A)
            self._pmask = np.ascontiguousarray(pmask, dtype=np.uint8)
            assert self._pmask.size == self.n
            _check(lib().amg_setup_schur_masked(self.n, _ptr(rp, C.c_int64), _ptr(c, C.c_int32),
                                                _ptr(v, C.c_double), _ptr(self._pmask, C.c_uint8),
                                                C.byref(self.params), alloc_p, C.c_void_p(stream.cuda_stream),
                                                C.byref(h)))
        elif n_u is not None:
            rp, c, v = _csr_arrays(A)
            _check(lib().amg_setup_schur(self.n, _ptr(rp, C.c_int64), _ptr(c, C.c_int32), _ptr(v, C.c_double),
                                         int(n_u), C.byref(self.params), alloc_p, C.c_void_p(stream.cuda_stream),
                                         C.byref(h)))
        elif _is_block(A):
            rp, c, v = _bsr_arrays(A)
            _check(lib().amg_setup_block(int(A.nb), int(A.b), _ptr(rp, C.c_int64), _ptr(c, C.c_int32),
                                         _ptr(v, C.c_double), C.byref(self.params), alloc_p,
                                         C.c_void_p(stream.cuda_stream), C.byref(h)))
        else:
            rp, c, v = _csr_arrays(A)
            _check(lib().amg_setup(self.n, _ptr(rp, C.c_int64), _ptr(c, C.c_int32), _ptr(v, C.c_double),
                                   C.byref(self.params), alloc_p, C.c_void_p(stream.cuda_stream), C.byref(h)))
        self._h = h

    def solve(self, f, x0=None, raise_on_error: bool = True):
        """Solve A x = f; f (and x0) are float64 device tensors of length n.

        Returns (x, info dict).  info["status"] is AMG_OK (0) or
        AMG_NOT_CONVERGED (1); errors raise.
        """
        import torch

        assert f.dtype == torch.float64 and f.is_cuda and f.numel() == self.n
        f = f.contiguous()
        x = torch.zeros_like(f) if x0 is None else x0.clone().contiguous()
        info = Info()
        code = lib().amg_solve(self._h, C.c_void_p(f.data_ptr()), C.c_void_p(x.data_ptr()),
                               C.c_void_p(_torch_stream().cuda_stream), C.byref(info))
        if raise_on_error:
            _check(code)
        d = info.as_dict()
        d["status"] = code
        return x, d

    KERNELS = ("outer_spmv_dot", "pre_smooth_residual", "post_smooth_dot", "restrict", "prolong", "vcycle",
               "split_outer_spmv_dot", "split_precond")

    def time_kernel(self, which, reps=50):
        """(mean microseconds per launch, algorithmic bytes per launch) of one hot kernel."""
        k = self.KERNELS.index(which) if isinstance(which, str) else int(which)
        us, by = C.c_double(), C.c_double()
        _check(lib().amg_time_kernel(self._h, k, reps, C.c_void_p(_torch_stream().cuda_stream),
                                     C.byref(us), C.byref(by)))
        return us.value, by.value

    def vcycle_noalloc(self, r, z=None):
        """z = V(r) with the work vectors in the library's fixed device array
        (no device allocation by the library; enqueued on the current stream,
        no wait)."""
        import torch

        assert r.dtype == torch.float64 and r.is_cuda and r.numel() == self.n
        r = r.contiguous()
        if z is None:
            z = torch.empty_like(r)
        _check(lib().amg_vcycle_noalloc(self._h, C.c_void_p(r.data_ptr()), C.c_void_p(z.data_ptr()),
                                        C.c_void_p(_torch_stream().cuda_stream)))
        return z

    def tail_info(self):
        """(first fused level or -1, workgroups of the fused launch)."""
        first, grid = C.c_int32(), C.c_int32()
        _check(lib().amg_tail_info(self._h, C.byref(first), C.byref(grid)))
        return first.value, grid.value

    def set_tail_wait(self, seconds):
        """Test hook: longest grid-barrier wait of the fused launch."""
        _check(lib().amg_tail_set_wait(self._h, float(seconds)))

    def vcycle(self, r):
        """z = V(r): one V-cycle on a float64 device tensor."""
        import torch

        assert r.dtype == torch.float64 and r.is_cuda and r.numel() == self.n
        r = r.contiguous()
        z = torch.empty_like(r)
        _check(lib().amg_vcycle(self._h, C.c_void_p(r.data_ptr()), C.c_void_p(z.data_ptr()),
                                C.c_void_p(_torch_stream().cuda_stream)))
        return z


class DeviceMatrix:
    """Standalone device CSR matrix for y = A x (kernel tests and measurement)."""

    def __init__(self, rows, cols, row_ptr, col, val, precision="fp64"):
        self.rows, self.cols = int(rows), int(cols)
        self.precision = PRECISION[precision] if isinstance(precision, str) else int(precision)
        rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
        c = np.ascontiguousarray(col, dtype=np.int32)
        v = np.ascontiguousarray(val, dtype=np.float64)
        h = C.c_void_p()
        _check(lib().amg_csr_upload(self.rows, self.cols, _ptr(rp, C.c_int64), _ptr(c, C.c_int32),
                                    _ptr(v, C.c_double), self.precision,
                                    C.c_void_p(_torch_stream().cuda_stream), C.byref(h)))
        self._h = h

    def kernel_info(self):
        k, l, b, nb = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib().amg_csr_kernel_info(self._h, C.byref(k), C.byref(l), C.byref(b), C.byref(nb)))
        cb = C.c_int32()
        _check(lib().amg_csr_column_bytes(self._h, C.byref(cb)))
        return {"kind": ("stream", "vector")[k.value], "lanes": l.value, "blocks": b.value,
                "block_bytes": nb.value, "column_bytes": cb.value}

    def spmv(self, x, y=None):
        import torch

        dt = torch.float64 if self.precision == 0 else torch.float32
        assert x.dtype == dt and x.is_cuda and x.numel() == self.cols
        x = x.contiguous()
        if y is None:
            y = torch.empty(self.rows, dtype=dt, device=x.device)
        _check(lib().amg_csr_spmv(self._h, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()),
                                  C.c_void_p(_torch_stream().cuda_stream)))
        return y

    def release(self):
        if self._h:
            lib().amg_csr_release(self._h)
            self._h = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass


class Server:
    """Continuous-batching request loop (``amg_server_*``).

    ``submit`` copies a system in; ``step`` admits ready requests, runs
    ``check_every`` batched PCG iterations of every live solve and retires
    finished ones; ``results`` drains finished requests as
    ``(request_id, x, info, status, times)`` with times = (submit, setup done,
    admitted, finished) on the library's monotonic clock.
    """

    def __init__(self, hbm_budget_bytes, max_slots=32, setup_threads=8, **params):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("amg.Server needs a HIP device")
        params.setdefault("precision", "mixed")
        self.params = make_params(**params)
        h = C.c_void_p()
        _check(lib().amg_server_create(C.byref(self.params), int(hbm_budget_bytes), int(max_slots),
                                       int(setup_threads), C.c_void_p(_torch_stream().cuda_stream), C.byref(h)))
        self._h = h

    def submit(self, request_id, A, f):
        rp, c, v = _csr_arrays(A)
        f = np.ascontiguousarray(f, dtype=np.float64)
        _check(lib().amg_server_submit(self._h, int(request_id), int(A.n), _ptr(rp, C.c_int64),
                                       _ptr(c, C.c_int32), _ptr(v, C.c_double), _ptr(f, C.c_double)))

    def wait_ready(self, count, timeout=60.0):
        """Block until ``count`` requests are set up (True) or timeout / nothing left (False)."""
        r = C.c_int32()
        return _check(lib().amg_server_wait_ready(self._h, int(count), float(timeout), C.byref(r))) == AMG_OK

    def step(self):
        live, waiting = C.c_int32(), C.c_int32()
        _check(lib().amg_server_step(self._h, C.byref(live), C.byref(waiting)))
        return live.value, waiting.value

    def results(self):
        out = []
        while True:
            rid, n = C.c_uint64(), C.c_int64()
            code = _check(lib().amg_server_poll(self._h, C.byref(rid), C.byref(n)))
            if code == AMG_NOT_CONVERGED:
                return out
            x = np.empty(n.value, dtype=np.float64)
            info = Info()
            times = np.zeros(4, dtype=np.float64)
            status = lib().amg_server_fetch(self._h, rid.value, _ptr(x, C.c_double), C.byref(info),
                                            _ptr(times, C.c_double))
            d = info.as_dict()
            d["status"] = status
            if status < 0:
                d["error"] = lib().amg_last_error().decode()
            out.append((rid.value, x, d, status, tuple(times)))

    def release(self):
        if self._h:
            lib().amg_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass
