"""GPU parity of the block entry points: Z = A B on FP64 matrix cores
(ccg_matmat) and block BiCGSTAB (ccg_bicgstab_block), against the oracle run
column by column on the same inputs."""
import numpy as np
import pytest

from gpu_util import dev, gamma, host_relres
from paper_1208_4869_amd import ccg, inputs

pytestmark = pytest.mark.gpu


def int_block(n, k, seed, bound=1024):
    rng = np.random.default_rng(seed)
    return (rng.integers(-bound, bound + 1, (n, k))
            + 1j * rng.integers(-bound, bound + 1, (n, k))).astype(np.complex128)


@pytest.mark.parametrize("n,k", [(1, 1), (5, 3), (64, 16), (65, 17), (130, 64),
                                 (257, 33), (200, 70), (1000, 64),
                                 (67, 5), (130, 8), (1000, 6), (3, 7)])
def test_matmat_integer_bitwise(orc, n, k):
    """Gaussian-integer inputs: exact in any summation order, so the matrix-core
    product equals the oracle's column products bit for bit (this also fixes
    the MFMA operand and result lane layout; 5 to 8 columns take the packed
    form, real and imaginary parts of B in one 16-wide tile)."""
    A = inputs.gaussian_integer_matrix(n, n, bound=1024)
    B = int_block(n, k, n + k)
    Z = ccg.ccg_matmat(dev(A), dev(B)).cpu().numpy()
    assert np.array_equal(Z, orc.matmat(A, B))


@pytest.mark.parametrize("n,k", [(7, 5), (300, 64), (1031, 40), (513, 8), (100, 12),
                                 (257, 20)])
def test_matmat_random_bound_and_layout(orc, n, k):
    """Random inputs against the oracle within 4 gamma_{n+2} |A| |B| (the
    three-real-product form's bound is about 3 u |A| |B| per element for the
    imaginary part), every column-tile count: 5 and 8 columns packed, 12, 20,
    40 and 64 on one to four tiles."""
    rng = np.random.default_rng(n)
    A = inputs.cn01(rng, (n, n))
    Bbig = inputs.cn01(rng, (n, k + 3))
    B = np.ascontiguousarray(Bbig[:, :k])
    Bd = dev(Bbig)[:, :k]  # ldb = k + 3
    Zbig = np.zeros((n, k + 5), dtype=np.complex128)
    Zd = dev(Zbig)
    ccg.ccg_matmat(dev(A), Bd, Zd[:, :k])
    Zg = Zd.cpu().numpy()
    assert np.all(Zg[:, k:] == 0)  # nothing written past column k
    ref = orc.matmat(A, B)
    bound = 4 * gamma(n + 2) * (np.abs(A) @ np.abs(B))
    assert np.all(np.abs(Zg[:, :k] - ref) <= bound)
    Z2 = ccg.ccg_matmat(dev(A), Bd).cpu().numpy()
    assert np.array_equal(Z2, Zg[:, :k])  # fixed summation order


@pytest.mark.parametrize("k", [12, 64])
def test_matmat_cancellation_bound(orc, k):
    """Real parts six orders above the imaginary ones: the three-real-product
    form recovers Im Z as (P3 - P1) - P2 from terms of the size of the real
    parts, so its error is bounded normwise (by |A| |B|) and not relative to
    |Im Z|; the elementwise bound of the other product tests still holds."""
    rng = np.random.default_rng(99 + k)
    n = 700
    A = rng.standard_normal((n, n)) + 1e-6j * rng.standard_normal((n, n))
    B = rng.standard_normal((n, k)) + 1e-6j * rng.standard_normal((n, k))
    Z = ccg.ccg_matmat(dev(A), dev(B)).cpu().numpy()
    ref = orc.matmat(A, B)
    bound = 4 * gamma(n + 2) * (np.abs(A) @ np.abs(B))
    assert np.all(np.abs(Z - ref) <= bound)


def check_block(orc, A, Xt, Y, cols_oracle=None, tol=1e-10, maxit=1000):
    n, k = Y.shape
    Ad, Yd = dev(A), dev(Y)
    import torch
    Xd = torch.full((n, k), float("nan"), dtype=torch.complex128, device="cuda")
    res = ccg.ccg_bicgstab_block_ex(Ad, Yd, Xd, tol, maxit, flags=ccg.X0_ZERO)
    X = Xd.cpu().numpy()
    cols = range(k) if cols_oracle is None else cols_oracle
    refs = dict(zip(cols, orc.bicgstab_block(A, Y, tol=tol, maxit=maxit, cols=cols)))
    fes = []
    for c in range(k):
        rel, slack = host_relres(A, X[:, c], Y[:, c])
        assert res[c].info == 0, (c, res[c])
        assert rel <= tol + slack, (c, rel)
        fe = np.linalg.norm(X[:, c] - Xt[:, c]) / np.linalg.norm(Xt[:, c])
        fes.append(fe)
        if c in refs:
            r = refs[c]
            fe_ref = np.linalg.norm(r.x - Xt[:, c]) / np.linalg.norm(Xt[:, c])
            assert r.info == 0
            assert abs(res[c].iters - r.iters) <= 1, (c, res[c].iters, r.iters)
            assert fe <= 100 * max(fe_ref, 1e-13), (c, fe, fe_ref)
    return res, np.array(fes)


@pytest.mark.parametrize("k", [1, 5, 16, 64])
def test_block_dense_n256(orc, k):
    A = inputs.dense_matrix(256, 11)
    Xt = inputs.cn01(np.random.default_rng(12), (256, k))
    Y = A @ Xt
    check_block(orc, A, Xt, Y)


def test_block_lattice_20_k64(orc):
    """The 20^3 lattice with 64 right-hand sides (X_true seed 5): every column
    converged with its host-recomputed residual <= 1e-10; four sampled columns
    against the oracle one by one."""
    A, Xt, Y = inputs.lattice_system(20, 5, nrhs=64)
    res, fes = check_block(orc, A, Xt, Y, cols_oracle=[0, 21, 42, 63])
    assert np.max(fes) < 1e-9


def test_block_edge_columns(orc):
    """A zero column (x = 0, no work), a non-finite column (info 4, x left
    untouched), a column held to a tiny budget, next to ordinary columns."""
    import torch
    n, k = 96, 6
    A = inputs.dense_matrix(n, 3)
    Xt = inputs.cn01(np.random.default_rng(4), (n, k))
    Y = A @ Xt
    Y[:, 1] = 0
    Y[5, 2] = np.nan
    X0 = np.full((n, k), 0.25 + 0.5j)
    Xd = dev(X0).clone()
    res = ccg.ccg_bicgstab_block_ex(dev(A), dev(Y), Xd, 1e-10, 1000, flags=0)
    X = Xd.cpu().numpy()
    assert res[1].info == 0 and res[1].iters == 0 and np.all(X[:, 1] == 0)
    assert res[2].info == 4 and np.array_equal(X[:, 2], X0[:, 2])
    for c in (0, 3, 4, 5):
        ref = orc.bicgstab(A, Y[:, c], x0=X0[:, c])
        assert res[c].info == 0 and abs(res[c].iters - ref.iters) <= 1
        assert res[c].matvecs - ref.matvecs in (-2, -1, 0, 1, 2)
        assert host_relres(A, X[:, c], Y[:, c])[0] <= 1.01e-10
    # budget: maxit = 2 for every column
    Xd = dev(X0).clone()
    res = ccg.ccg_bicgstab_block_ex(dev(A), dev(Y), Xd, 1e-10, 2, flags=0)
    for c in (0, 3, 4, 5):
        ref = orc.bicgstab(A, Y[:, c], x0=X0[:, c], maxit=2)
        assert (res[c].info, res[c].iters) == (ref.info, ref.iters) == (1, 2)
    # short form
    Xd = torch.zeros((n, 3), dtype=torch.complex128, device="cuda")
    info = ccg.ccg_bicgstab_block(dev(A), dev(np.ascontiguousarray(Y[:, 3:])), Xd)
    assert info == [0, 0, 0]
