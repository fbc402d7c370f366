"""GPU tests at a size where element offsets pass 2^31: n = 48 000, so A has
2.3e9 entries (36.9 GB in complex128, 18.4 GB in complex64).  Every product
entry point is checked bit for bit on sampled rows against exact integer
sums on the host (A and the vectors are small Gaussian integers, so every
partial sum of every product is an exact integer, in FP32 too); a BiCGSTAB
solve on the shifted matrix is checked by its confirmed true residual and its
forward error."""
import numpy as np
import pytest

from paper_1208_4869_amd import ccg

pytestmark = pytest.mark.gpu

N = 48000
SHIFT = 2000.0  # diagonal shift of the solve: A + SHIFT I is well conditioned


@pytest.fixture(scope="module")
def big():
    """A with entries re, im in {-1, 0, 1}, generated on the device."""
    import torch
    g = torch.Generator(device="cuda").manual_seed(4800)
    A = torch.empty((N, N), dtype=torch.complex128, device="cuda")
    rows = 4000
    for r0 in range(0, N, rows):
        re = torch.randint(-1, 2, (rows, N), generator=g, device="cuda", dtype=torch.int8)
        im = torch.randint(-1, 2, (rows, N), generator=g, device="cuda", dtype=torch.int8)
        A[r0:r0 + rows] = torch.complex(re.double(), im.double())
    torch.cuda.synchronize()
    yield A
    del A
    torch.cuda.empty_cache()


def int_vec(n, k, seed, bound=3):
    rng = np.random.default_rng(seed)
    shape = (n,) if k is None else (n, k)
    return (rng.integers(-bound, bound + 1, shape)
            + 1j * rng.integers(-bound, bound + 1, shape)).astype(np.complex128)


def exact_dot(a, x):
    """sum_j a_j x_j in Python-exact int64 arithmetic (a, x Gaussian integers)."""
    ar, ai = a.real.astype(np.int64), a.imag.astype(np.int64)
    xr, xi = x.real.astype(np.int64), x.imag.astype(np.int64)
    return complex(int(ar @ xr - ai @ xi), int(ar @ xi + ai @ xr))


def sample_rows():
    rng = np.random.default_rng(48)
    return sorted(set([0, 1, N // 2, N - 2, N - 1] + list(rng.integers(0, N, 12))))


def test_large_products_exact(big):
    import torch
    A = big
    x = int_vec(N, None, 1)
    xd = torch.from_numpy(x).cuda()
    yn = ccg.ccg_matvec(ccg.OP_N, A, xd).cpu().numpy()
    yc = ccg.ccg_matvec(ccg.OP_C, A, xd).cpu().numpy()
    ys = ccg.ccg_matvec(ccg.OP_S, A, xd).cpu().numpy()
    for i in sample_rows():
        row = A[i].cpu().numpy()
        col = A[:, i].cpu().numpy()
        assert yn[i] == exact_dot(row, x), ("A x", i)
        assert yc[i] == exact_dot(np.conj(col), x), ("A^H x", i)
        # upper triangle: column i above the diagonal, row i from the diagonal on
        want = exact_dot(col[:i], x[:i]) + exact_dot(row[i:], x[i:])
        assert ys[i] == want, ("upper-triangle A x", i)


def test_large_block_and_c64_products_exact(big):
    import torch
    A = big
    k = 8
    B = int_vec(N, k, 2)
    Z = ccg.ccg_matmat(A, torch.from_numpy(B).cuda()).cpu().numpy()
    A32 = ccg.ccg_round_c64(A)
    x = int_vec(N, None, 3)
    y32 = ccg.ccg_matvec_c64(A32, torch.from_numpy(x.astype(np.complex64)).cuda())
    y32 = y32.cpu().numpy()
    Z32 = ccg.ccg_matmat_c64(A32, torch.from_numpy(B).cuda()).cpu().numpy()
    del A32
    torch.cuda.empty_cache()
    for i in sample_rows():
        row = A[i].cpu().numpy()
        for c in range(k):
            assert Z[i, c] == exact_dot(row, B[:, c]), ("A B", i, c)
            assert Z32[i, c] == exact_dot(row, B[:, c]), ("A32 B", i, c)
        assert complex(y32[i]) == exact_dot(row, x), ("A32 x", i)


def exact_row_residual(row, shift, i, x, yi):
    """y_i - sum_j (A + shift I)_ij x_j for a Gaussian-integer row, each term
    (+-x_j components) exact and the sums correctly rounded (math.fsum)."""
    import math
    xr, xi = x.real, x.imag
    ar, ai = row.real.astype(np.int64), row.imag.astype(np.int64)
    re_terms = np.concatenate([xr[ar == 1], -xr[ar == -1], -xi[ai == 1], xi[ai == -1],
                               [shift * xr[i], -yi.real]])
    im_terms = np.concatenate([xi[ar == 1], -xi[ar == -1], xr[ai == 1], -xr[ai == -1],
                               [shift * xi[i], -yi.imag]])
    return -complex(math.fsum(re_terms), math.fsum(im_terms))


def test_large_solve(big):
    """BiCGSTAB on (A + SHIFT I) x = y.  x_true is a Gaussian-integer vector,
    so y = (A + SHIFT I) x_true has integer partial sums below 2^53 and torch's
    own product (rocBLAS, outside this library) forms it exactly.  Checks: info
    0; the true relative residual recomputed with torch's product (FP64,
    rounding far below 1e-10 here) within 1e-10; the residual of 17 sampled
    rows evaluated exactly on the host, within 1e-10 ||y|| / sqrt(n) each
    times a safety factor of 10; forward error within 1e-8."""
    import torch
    A = big
    A.diagonal().add_(SHIFT)
    try:
        xt_h = int_vec(N, None, 5)
        xt = torch.from_numpy(xt_h).cuda()
        y = A @ xt  # exact: integer sums below 2^53
        y_h = y.cpu().numpy()
        assert np.array_equal(y_h.real, np.round(y_h.real))  # integers, as they must be
        x = torch.empty_like(xt)
        res = ccg.ccg_bicgstab_ex(A, y, x, 1e-10, 200, flags=ccg.X0_ZERO)
        torch.cuda.synchronize()
        assert res.info == 0, res
        rel = float(torch.linalg.norm(y - A @ x) / torch.linalg.norm(y))
        assert rel <= 1e-10, rel
        x_h = x.cpu().numpy()
        ny = np.linalg.norm(y_h)
        for i in sample_rows():
            ri = exact_row_residual(A[i].cpu().numpy() - SHIFT * (np.arange(N) == i),
                                    SHIFT, i, x_h, y_h[i])
            assert abs(ri) <= 10 * 1e-10 * ny / np.sqrt(N), (i, abs(ri))
        fe = np.linalg.norm(x_h - xt_h) / np.linalg.norm(xt_h)
        assert fe <= 1e-8, fe
    finally:
        A.diagonal().sub_(SHIFT)
