"""Device SpMV kernels vs a plain CPU product (GPU).

Covers the SpMV variants the library selects by mean row length (LDS-staged
stream blocks of 4 KB or, for matrices with at least 32 MiB of values, 8 or 16 KB,
whose rows are reduced by G = 1, 4, 16 or 64 lanes, including rows longer
than one LDS block; 64 lanes per row straight from memory for
very long rows), empty rows, a ragged tail, rectangular shapes, FP64 and
FP32, and sampled rows of the full-size 150^3 Poisson operator.
"""

import zlib

import numpy as np
import pytest

from tests.gpu_util import announce, random_csr, scipy_of

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

from paper_1811_05704_amd import amg  # noqa: E402

import problems  # noqa: E402


def _run(rows, cols, rp, col, val, precision, seed=0):
    M = amg.DeviceMatrix(rows, cols, rp, col, val, precision=precision)
    info = M.kernel_info()
    x = np.random.default_rng(seed + 1).uniform(-1, 1, cols)
    dt = torch.float64 if precision == "fp64" else torch.float32
    xd = torch.tensor(x, dtype=dt, device="cuda")
    announce("spmv", rows, cols, int(rp[-1]), precision, info)
    y = M.spmv(xd).cpu().numpy().astype(np.float64)
    M.release()
    return x, y, info


def _ref(rp, col, val, rows, cols, x, precision):
    S = scipy_of(rp, col, val, rows, cols)
    if precision == "fp64":
        return S @ x, abs(S) @ np.abs(x)
    S32 = S.astype(np.float32).astype(np.float64)
    x32 = x.astype(np.float32).astype(np.float64)
    return S32 @ x32, abs(S32) @ np.abs(x32)


CASES = [
    # name, rows, cols, row-length generator
    ("short_ragged", 10007, 10007, lambda r: r.integers(0, 13, 10007)),
    ("with_empty_rows", 5000, 5000, lambda r: np.where(r.random(5000) < 0.3, 0, r.integers(1, 9, 5000))),
    ("one_row", 1, 50, lambda r: np.array([7])),
    ("long_row_in_stream", 3000, 6000, lambda r: np.where(np.arange(3000) == 1234, 5000, r.integers(1, 8, 3000))),
    ("rectangular_tall", 20000, 3000, lambda r: r.integers(1, 5, 20000)),
    ("stream_g4_13", 4001, 4001, lambda r: r.integers(10, 17, 4001)),
    ("stream_g4_30", 3001, 5000, lambda r: r.integers(20, 41, 3001)),
    ("stream_g16_100", 1003, 5000, lambda r: r.integers(60, 141, 1003)),
    ("stream_g64_300", 503, 5000, lambda r: r.integers(200, 401, 503)),
    ("stream_g64_mixed_long", 203, 20000, lambda r: np.where(np.arange(203) % 50 == 7, 6000, r.integers(200, 400, 203))),
    ("vector_long_rows", 300, 20000, lambda r: r.integers(1000, 9000, 300)),
    # at least 32 MiB of values in both precisions: 16 KB stream blocks
    ("large_blocks_g1", 1400000, 1400000, lambda r: r.integers(1, 13, 1400000)),
    ("large_blocks_g4", 300000, 300000, lambda r: r.integers(20, 41, 300000)),
    ("large_blocks_g16", 150000, 150000, lambda r: r.integers(50, 71, 150000)),  # FP32: 8 KB blocks
]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("name,rows,cols,gen", CASES, ids=[c[0] for c in CASES])
def test_spmv_matches_cpu(name, rows, cols, gen, precision):
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    lengths = gen(rng)
    rp, col, val = random_csr(rows, cols, lengths, seed=3)
    prec = "fp64" if precision == "fp64" else "mixed"
    x, y, info = _run(rows, cols, rp, col, val, prec)
    yr, scale = _ref(rp, col, val, rows, cols, x, precision)
    mean = rp[-1] / max(rows, 1)
    assert info["kind"] == ("stream" if mean <= 512 else "vector")
    if info["kind"] == "stream":
        expect = 1 if mean <= 12 else 4 if mean <= 48 else 16 if mean <= 192 else 64
        assert info["lanes"] == expect
        sz = 8 if precision == "fp64" else 4
        vbytes = int(rp[-1]) * sz
        one_pass = (2 if expect == 16 else 1) * (256 // expect) * mean  # entries of the reduction passes
        if vbytes < 32 << 20:
            assert info["block_bytes"] == 4096
        elif expect == 1 and precision == "fp64":
            assert info["block_bytes"] == 8192
        elif one_pass <= 4096 // sz:
            assert info["block_bytes"] == 4096
        elif expect <= 16 and one_pass <= 8192 // sz:
            assert info["block_bytes"] == 8192
        else:
            assert info["block_bytes"] == 16384
    # 2-byte column offsets unless a stream block spans more than 65536 columns
    if info["kind"] == "stream" and cols <= 65536:
        assert info["column_bytes"] == 2
    if info["kind"] == "vector" or name.startswith("large_blocks"):  # random columns over > 65536: int32
        assert info["column_bytes"] == 4
    # worst case grows with the row length (per-lane partial sums + a tree)
    tol = 5e-14 if precision == "fp64" else 2e-5
    err = np.abs(y - yr)
    assert np.all(err <= tol * np.maximum(scale, 1e-300) + 1e-300), (name, err.max())
    assert np.all(y[np.diff(rp) == 0] == 0.0)


def test_spmv_stream_fp64_bit_exact_row_order():
    # the stream variant sums each row in column order from LDS, the same
    # order as a sequential CPU loop
    rp, col, val = random_csr(7777, 7777, np.random.default_rng(4).integers(1, 8, 7777), seed=5)
    x, y, info = _run(7777, 7777, rp, col, val, "fp64")
    assert info["kind"] == "stream"
    yr = np.zeros(7777)
    for i in range(7777):
        s = 0.0
        for e in range(rp[i], rp[i + 1]):
            s += val[e] * x[col[e]]
        yr[i] = s
    assert np.array_equal(y, yr)


@pytest.mark.timeout(600)
def test_spmv_full_size_poisson150_sampled_rows():
    A = problems.poisson3d(150)
    M = amg.DeviceMatrix(A.n, A.n, A.row_ptr, A.col, A.val, precision="fp64")
    assert M.kernel_info()["kind"] == "stream"
    assert M.kernel_info()["column_bytes"] == 2  # a block of rows spans at most 2 N^2 + 1 columns
    x = np.random.default_rng(9).random(A.n)
    announce("spmv poisson 150^3 full size")
    y = M.spmv(torch.tensor(x, device="cuda")).cpu().numpy()
    rows = np.random.default_rng(10).choice(A.n, size=20000, replace=False)
    rows = np.concatenate([rows, [0, 1, A.n - 1, A.n - 2, 150 * 150 - 1]])
    for i in rows:
        s = 0.0
        for e in range(A.row_ptr[i], A.row_ptr[i + 1]):
            s += A.val[e] * x[A.col[e]]
        assert y[i] == s
    M.release()
