"""GPU tests of the complex64 block product on FP32 matrix cores
(ccg_matmat_c64) and of the mixed-precision block solver
(ccg_bicgstab_block_mixed_ex): against the oracle's products and solvers on
the same inputs."""
import numpy as np
import pytest

from gpu_util import dev, host_relres
from paper_1208_4869_amd import ccg, inputs

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def int_block(n, k, seed, bound):
    rng = np.random.default_rng(seed)
    return (rng.integers(-bound, bound + 1, (n, k))
            + 1j * rng.integers(-bound, bound + 1, (n, k))).astype(np.complex128)


@pytest.mark.parametrize("n,k", [(1, 1), (5, 3), (64, 16), (65, 17), (130, 64),
                                 (257, 33), (200, 70), (1000, 64)])
def test_matmat_c64_integer_bitwise(orc, n, k):
    """Small Gaussian integers: exact in complex64 and in every FP32 partial
    sum, so the product equals the oracle's bit for bit (this also fixes the
    FP32 matrix-core lane layout)."""
    A = inputs.gaussian_integer_matrix(n, n, bound=16)
    B = int_block(n, k, n + 3 * k, 16)
    import torch
    A32 = torch.from_numpy(A.astype(np.complex64)).cuda()
    Z = ccg.ccg_matmat_c64(A32, dev(B)).cpu().numpy()
    assert np.array_equal(Z, orc.matmat(A, B))


@pytest.mark.parametrize("n,k", [(7, 5), (300, 64), (1031, 40)])
def test_matmat_c64_random_bound(orc, n, k):
    """Random inputs: within the FP32 accumulation bound of the exact product
    of the complex64-rounded operands; padded leading dimensions; nothing
    written past column k; repeatable bit for bit."""
    import torch
    rng = np.random.default_rng(n)
    A = inputs.cn01(rng, (n, n))
    A32h = A.astype(np.complex64)
    Bbig = inputs.cn01(rng, (n, k + 3))
    B32 = Bbig[:, :k].astype(np.complex64).astype(np.complex128)
    ref = orc.matmat(A32h.astype(np.complex128), np.ascontiguousarray(B32))
    A32 = torch.from_numpy(A32h).cuda()
    Zbig = torch.zeros((n, k + 5), dtype=torch.complex128, device="cuda")
    ccg.ccg_matmat_c64(A32, dev(Bbig)[:, :k], Zbig[:, :k])
    Z = Zbig.cpu().numpy()
    assert np.all(Z[:, k:] == 0)
    bound = 4 * (n / 8 + 2) * U32 * (np.abs(A32h) @ np.abs(B32)) + 1e-300
    assert np.all(np.abs(Z[:, :k] - ref) <= bound)
    Z2 = ccg.ccg_matmat_c64(A32, dev(Bbig)[:, :k]).cpu().numpy()
    assert np.array_equal(Z2, Z[:, :k])


def run_block_mixed(A, Y, X0=None, **kw):
    import torch
    n, k = Y.shape
    Ad = dev(A)
    A32 = ccg.ccg_round_c64(Ad)
    if X0 is None:
        X = torch.full((n, k), float("nan"), dtype=torch.complex128, device="cuda")
        flags = ccg.X0_ZERO
    else:
        X = dev(X0)
        flags = 0
    res = ccg.ccg_bicgstab_block_mixed_ex(Ad, A32, dev(Y), X, flags=flags, **kw)
    torch.cuda.synchronize()
    return X.cpu().numpy(), res


def check_against_wide_oracle(orc, A, y, res, label=""):
    """One column against the oracle of the same refinement (complex64
    products, complex128 inner vectors, FP64 scalars and refinement): same
    info, outer steps within one, inner iterations within one per outer step,
    and the outer residual history ||r_j|| / ||y|| within a factor of two at
    every check both made while it was above 1e-13 (FP32 rounding moves the
    inner iterates, so the values agree to a few percent, not bitwise)."""
    ref = orc.bicgstab_mixed_wide(A, y)
    msg = "%s: gpu info %d outer %d inner %d | oracle info %d outer %d inner %d" % (
        label, res.info, res.outer, res.inner_iters, ref.info, ref.outer, ref.inner_iters)
    assert res.info == ref.info, msg
    assert abs(res.outer - ref.outer) <= 1, msg
    assert abs(res.inner_iters - ref.inner_iters) <= max(res.outer, ref.outer), msg
    g, o = res.outer_res, ref.outer_res
    both = ~np.isnan(g) & ~np.isnan(o)
    assert both[0] and g[0] == o[0] == 1.0, msg  # x0 = 0: the first check is ||y|| / ||y||
    for j in np.nonzero(both)[0]:
        if min(g[j], o[j]) <= 1e-13:
            break
        assert 0.5 <= g[j] / o[j] <= 2.0, msg + " check %d: %.3e vs %.3e" % (j, g[j], o[j])
    return ref


@pytest.mark.parametrize("kind,size,k,cols", [("lattice", 6, 8, None),
                                              ("dense", 256, 16, (0, 7, 15)),
                                              ("lattice", 20, 64, (0, 31, 63))])
def test_block_mixed_solves(orc, kind, size, k, cols):
    """Every column: true residual <= 1e-10 (host, FP64); sampled columns:
    forward error within 100x the FP64 oracle's, and info, outer steps, inner
    iterations and the outer residual history against the oracle of the same
    refinement."""
    if kind == "lattice":
        A, Xt, Y = inputs.lattice_system(size, 5, nrhs=k)
    else:
        A = inputs.dense_matrix(size, 21)
        Xt = inputs.cn01(np.random.default_rng(22), (size, k))
        Y = A @ Xt
    X, res = run_block_mixed(A, Y)
    for c in range(k):
        rel, slack = host_relres(A, X[:, c], Y[:, c])
        assert res[c].info == 0 and rel <= 1e-10 + slack, (c, res[c], rel)
        assert res[c].outer >= 1 and res[c].matvecs32 >= 1
        assert res[c].matvecs64 == res[c].outer  # x0 = 0: one FP64 residual per step
    for c in (range(k) if cols is None else cols):
        ref64 = orc.bicgstab(A, Y[:, c], tol=1e-10, maxit=1000)
        check_against_wide_oracle(orc, A, Y[:, c], res[c], label="%s col %d" % (kind, c))
        fe = np.linalg.norm(X[:, c] - Xt[:, c]) / np.linalg.norm(Xt[:, c])
        fe64 = np.linalg.norm(ref64.x - Xt[:, c]) / np.linalg.norm(Xt[:, c])
        assert fe <= 100 * max(fe64, 1e-13), (c, fe, fe64)


def test_block_mixed_inner_breakdown_ends_the_column(orc):
    """A column whose inner solve breaks down before its first update (the
    rotation [[0, 1], [-1, 0]] with y = e1: sigma = 0 exactly) ends after
    one outer step with the inner info 2 and x = 0, as in the oracle, while
    the other column (y = e1 + i e2 / 3, for which sigma is not zero)
    converges."""
    A = np.array([[0, 1], [-1, 0]], dtype=np.complex128)
    Y = np.array([[1, 1], [0, 1j / 3.0]], dtype=np.complex128)
    X, res = run_block_mixed(A, Y)
    ref = orc.bicgstab_mixed_wide(A, Y[:, 0])
    assert (ref.info, ref.outer, ref.inner_iters) == (2, 1, 0)
    assert (res[0].info, res[0].outer, res[0].inner_iters) == (2, 1, 0)
    assert res[0].matvecs64 == 0 and np.all(X[:, 0] == 0)
    assert res[1].info == 0 and host_relres(A, X[:, 1], Y[:, 1])[0] <= 1.01e-10


def test_block_mixed_edges():
    m = 5
    A, Xt, Y = inputs.lattice_system(m, 6, nrhs=4)
    n = m ** 3
    Y = Y.copy()
    Y[:, 1] = 0
    Y[7, 2] = np.inf
    X0 = np.full((n, 4), 0.5 - 0.25j)
    X, res = run_block_mixed(A, Y, X0=X0)
    assert res[0].info == 0 and res[3].info == 0
    assert res[1].info == 0 and np.all(X[:, 1] == 0) and res[1].outer == 0
    assert res[2].info == 4 and np.array_equal(X[:, 2], X0[:, 2])
    # outer budget 0: info 1, x = 0 from the x0 = 0 start
    X, res = run_block_mixed(A, Y[:, [0, 3]], maxit=0)
    assert all(r.info == 1 and r.outer == 0 for r in res) and np.all(X == 0)
    # warm start from the exact solution: at most one refinement step
    xs = np.linalg.solve(A, Y[:, [0, 3]])
    X, res = run_block_mixed(A, Y[:, [0, 3]], X0=xs)
    assert all(r.info == 0 and r.outer <= 1 for r in res)
