"""GPU parity of the mixed-precision solver (ccg_bicgstab_mixed_ex: FP64
refinement around complex64 BiCGSTAB) against the mixed oracle and the FP64
oracle on the same inputs."""
import numpy as np
import pytest

from gpu_util import dev, host_relres
from paper_1208_4869_amd import ccg, inputs

pytestmark = pytest.mark.gpu


def run_mixed(A, y, x0=None, **kw):
    import torch
    Ad = dev(A)
    A32 = ccg.ccg_round_c64(Ad)
    n = A.shape[0]
    if x0 is None:
        x = torch.full((n,), float("nan"), dtype=torch.complex128, device="cuda")
        flags = ccg.X0_ZERO
    else:
        x = dev(np.asarray(x0, dtype=np.complex128)).clone()
        flags = 0
    res = ccg.ccg_bicgstab_mixed_ex(Ad, A32, dev(y), x, flags=flags, **kw)
    torch.cuda.synchronize()
    return x.cpu().numpy(), res


@pytest.mark.parametrize("n", [1, 63, 64, 65, 500, 1031])
def test_matvec_c64_integer_exact(orc, n):
    """complex64 product on small Gaussian integers: all partial sums are
    integers below 2^24, so GPU and oracle agree bit for bit."""
    A = inputs.gaussian_integer_matrix(n, n, bound=8).astype(np.complex64)
    x = inputs.gaussian_integer_vector(n, n + 1, bound=8).astype(np.complex64)
    got = ccg.ccg_matvec_c64(dev(A), dev(x)).cpu().numpy()
    assert np.array_equal(got, orc.matvec_c64(A, x))


def test_matvec_c64_rounding_bound(orc):
    n = 777
    rng = np.random.default_rng(8)
    A = inputs.cn01(rng, (n, n)).astype(np.complex64)
    x = inputs.cn01(rng, n).astype(np.complex64)
    got = ccg.ccg_matvec_c64(dev(A), dev(x)).cpu().numpy().astype(np.complex128)
    exact = A.astype(np.complex128) @ x.astype(np.complex128)
    u32 = 2.0 ** -24
    bound = 2 * (n + 4) * u32 * (np.abs(A).astype(np.float64) @ np.abs(x).astype(np.float64))
    assert np.all(np.abs(got - exact) <= bound + 2 * u32 * np.abs(exact))


def test_round_c64_matches_numpy():
    rng = np.random.default_rng(3)
    A = inputs.cn01(rng, (37, 53)) * 1e3
    got = ccg.ccg_round_c64(dev(A)).cpu().numpy()
    assert np.array_equal(got, A.astype(np.complex64))


@pytest.mark.parametrize("kind,size", [("lattice", 6), ("dense", 256), ("lattice", 20),
                                       ("dense", 1029)])
def test_mixed_parity(orc, kind, size):
    if kind == "lattice":
        A, xt, y = inputs.lattice_system(size, 2)
    else:
        A, xt, y = inputs.dense_system(size, 60 + size)
    ref = orc.bicgstab_mixed(A, y)
    ref64 = orc.bicgstab(A, y)
    x, res = run_mixed(A, y)
    rel, slack = host_relres(A, x, y)
    fe = np.linalg.norm(x - xt) / np.linalg.norm(xt)
    fe64 = np.linalg.norm(ref64.x - xt) / np.linalg.norm(xt)
    msg = "%s %d: gpu %s | oracle outer %d inner %d" % (kind, size, res, ref.outer,
                                                        ref.inner_iters)
    assert ref.info == 0 and res.info == 0, msg
    assert rel <= 1e-10 + slack, msg
    assert abs(res.outer - ref.outer) <= 1, msg
    assert abs(res.inner_iters - ref.inner_iters) <= 2 * max(res.outer, 1), msg
    assert fe <= 100 * max(fe64, 1e-13), msg + " fe %.3e vs FP64 oracle %.3e" % (fe, fe64)


def test_mixed_26_lattice(orc):
    """The 26^3 lattice (n = 17576): complex64 inner solves, FP64 refinement."""
    A, xt, y = inputs.lattice_system(26, 2)
    x, res = run_mixed(A, y)
    rel, slack = host_relres(A, x, y)
    assert res.info == 0 and rel <= 1e-10 + slack
    ref = orc.bicgstab_mixed(A, y)
    assert abs(res.outer - ref.outer) <= 1
    fe = np.linalg.norm(x - xt) / np.linalg.norm(xt)
    fe_ref = np.linalg.norm(ref.x - xt) / np.linalg.norm(xt)
    assert fe <= 100 * max(fe_ref, 1e-13)


def test_mixed_edges(orc):
    A, _, y = inputs.dense_system(80, 4)
    x0 = np.full(80, 0.5 + 0.25j)
    ybad = y.copy()
    ybad[9] = np.inf
    x, res = run_mixed(A, ybad, x0=x0)
    assert res.info == 4 and np.array_equal(x, x0)
    x, res = run_mixed(A, np.zeros(80, dtype=np.complex128), x0=x0)
    assert res.info == 0 and np.all(x == 0) and res.outer == 0
    x, res = run_mixed(A, y, maxit=0)
    assert res.info == 1 and res.outer == 0 and np.all(x == 0)
    # warm start from the FP64 solution: converges with at most one step
    xs = np.linalg.solve(A, y)
    x, res = run_mixed(A, y, x0=xs)
    assert res.info == 0 and res.outer <= 1
    # a tighter inner tolerance needs fewer outer steps
    x1, r1 = run_mixed(A, y, tol_inner=1e-3)
    x2, r2 = run_mixed(A, y, tol_inner=1e-6)
    assert r1.info == 0 and r2.info == 0 and r2.outer <= r1.outer
    ref = orc.bicgstab_mixed(A, y, tol_inner=1e-3)
    assert abs(r1.outer - ref.outer) <= 1


def test_mixed_inner_breakdown_ends_the_refinement(orc):
    """An inner breakdown before the first inner update (the rotation
    [[0, 1], [-1, 0]] with y = e1, and from x0 = (1/2, 1/2): sigma = 0
    exactly) ends the refinement with info 2 after one step, x as it was --
    as in the oracle -- instead of repeating the step until the budget."""
    A = np.array([[0, 1], [-1, 0]], dtype=np.complex128)
    y = np.array([1, 0], dtype=np.complex128)
    for x0 in (None, np.array([0.5, 0.5], dtype=np.complex128)):
        ref = orc.bicgstab_mixed(A, y, x0=x0)
        x, res = run_mixed(A, y, x0=x0)
        assert (ref.info, ref.outer, ref.inner_iters) == (2, 1, 0)
        assert (res.info, res.outer, res.inner_iters) == (2, 1, 0)
        assert np.array_equal(x, ref.x)


@pytest.mark.parametrize("kind,size", [("lattice", 6), ("dense", 256)])
def test_mixed_outer_history(orc, kind, size):
    """The outer residual history ||r_j|| / ||y|| against the oracle's: the
    same number of checks within one, each value within a factor of two while
    above 1e-13 (FP32 rounding moves the inner iterates a little)."""
    if kind == "lattice":
        A, xt, y = inputs.lattice_system(size, 2)
    else:
        A, xt, y = inputs.dense_system(size, 61)
    ref = orc.bicgstab_mixed(A, y)
    x, res = run_mixed(A, y)
    g, o = res.outer_res, ref.outer_res
    assert g[0] == o[0] == 1.0
    assert abs(int(np.sum(~np.isnan(g))) - int(np.sum(~np.isnan(o)))) <= 1
    for j in range(len(g)):
        if np.isnan(g[j]) or np.isnan(o[j]) or min(g[j], o[j]) <= 1e-13:
            break
        assert 0.5 <= g[j] / o[j] <= 2.0, (j, g[j], o[j])
    assert g[res.outer] == res.relres_true
