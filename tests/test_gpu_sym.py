"""GPU tests of the upper-triangle product of a complex symmetric matrix
(ccg_matvec with CCG_OP_S) and of BiCGSTAB / CGNR / COCG / COCR run with it
(flag CCG_A_SYM_UPPER; CGNR's A^H r is then conj(A) r from the same
triangle), against the oracle on the same inputs.

Every device matrix here holds NaN below the diagonal: a single read there
would make a result non-finite, so finite results that match the oracle also
show that nothing below the diagonal is read."""
import numpy as np
import pytest

from gpu_util import assert_parity, dev, gamma, gpu_solve, host_relres
from paper_1208_4869_amd import ccg, inputs

pytestmark = pytest.mark.gpu

NANC = complex(np.nan, np.nan)


def stored_upper(A):
    """Copy of A with NaN below the diagonal (the part the product skips)."""
    S = np.array(A, dtype=np.complex128, copy=True)
    n = S.shape[0]
    S[np.tril_indices(n, -1)] = NANC
    return S


def full_from_upper(S):
    """The complex symmetric matrix whose upper triangle S stores."""
    up = np.triu(np.nan_to_num(S, nan=0.0))
    return up + np.triu(up, 1).T


@pytest.mark.parametrize("n", [1, 2, 5, 63, 64, 65, 130, 1000, 4095, 4096, 4100, 8000])
def test_product_integer_bitwise(orc, n):
    """Gaussian integers small enough that every partial sum is an exact
    integer: the product equals the oracle's bit for bit whatever the order
    of the sums.  Covers one tile, several tiles, ragged last tiles, the
    three tile edges (64 up to n = 3968, 128 up to 7936, 256 beyond) and the
    benchmark's n."""
    A = inputs.gaussian_integer_matrix(n, 300 + n, bound=32)
    x = inputs.gaussian_integer_vector(n, 400 + n, bound=32)
    S = stored_upper(A)
    y = ccg.ccg_matvec(ccg.OP_S, dev(S), dev(x)).cpu().numpy()
    assert np.array_equal(y, orc.matvec_sym_upper(S, x)), n


@pytest.mark.parametrize("n,pad", [(7, 0), (300, 5), (4100, 3)])
def test_product_random_bound_padded_repeatable(orc, n, pad):
    """Random inputs, padded leading dimension: componentwise within
    2 gamma_(n+2) (|A| |x|) of the oracle (each is within gamma_(n+2) of the
    exact product); the same bits on a second call and through
    ccg_matvec_ex with a caller workspace."""
    import torch
    rng = np.random.default_rng(n + pad)
    B = inputs.cn01(rng, (n, n + pad))
    B[:, :n][np.tril_indices(n, -1)] = NANC
    S = B[:, :n]
    x = inputs.cn01(rng, n)
    Bd = dev(B)
    Sd = Bd[:, :n]
    y = ccg.ccg_matvec(ccg.OP_S, Sd, dev(x)).cpu().numpy()
    ref = orc.matvec_sym_upper(S, x)
    bound = 2 * gamma(n + 2) * (np.abs(full_from_upper(S)) @ np.abs(x))
    assert np.all(np.abs(y - ref) <= bound + 1e-300)
    y2 = ccg.ccg_matvec(ccg.OP_S, Sd, dev(x)).cpu().numpy()
    assert np.array_equal(y, y2)
    ws = ccg.workspace(ccg.WS_MATVEC_S, n)
    y3 = torch.empty(n, dtype=torch.complex128, device="cuda")
    ccg.ccg_matvec_ex(ccg.OP_S, Sd, dev(x), y3, ws)
    assert np.array_equal(y, y3.cpu().numpy())


def test_product_lattice_matches_dense(orc):
    """The 20^3 lattice matrix (complex symmetric in full): the
    upper-triangle product with NaN below the diagonal agrees with the dense
    GPU product and the oracle's dense product within the rounding bound."""
    A = inputs.lattice_matrix(20)
    n = A.shape[0]
    x = inputs.cn01(np.random.default_rng(31), n)
    ys = ccg.ccg_matvec(ccg.OP_S, dev(stored_upper(A)), dev(x)).cpu().numpy()
    yd = ccg.ccg_matvec(ccg.OP_N, dev(A), dev(x)).cpu().numpy()
    ref = orc.matvec(A, x)
    bound = 2 * gamma(n + 2) * (np.abs(A) @ np.abs(x))
    assert np.all(np.abs(ys - ref) <= bound)
    assert np.all(np.abs(ys - yd) <= 2 * bound)


@pytest.mark.parametrize("method", ["bicgstab", "cgnr", "cocg", "cocr"])
@pytest.mark.parametrize("m", [6, 12, 20])
def test_solvers_lattice(orc, method, m):
    """Solves with the upper-triangle product (NaN below the diagonal on the
    device) against the oracle's dense solves of the full matrix: true
    residual <= tol, iterations within 1, forward error within 100x the
    oracle's, scalar histories within 1e-6."""
    A, xt, y = inputs.lattice_system(m, 8)
    assert_parity(orc, method, A, y, xt, Ad=dev(stored_upper(A)),
                  label="lattice %d^3, upper triangle" % m, flags=ccg.A_SYM_UPPER)


@pytest.mark.parametrize("method", ["cocg", "cocr", "bicgstab", "cgnr"])
@pytest.mark.parametrize("n", [1, 3, 65, 700])
def test_solvers_dense_symmetric(orc, method, n):
    rng = np.random.default_rng(900 + n)
    G = inputs.cn01(rng, (n, n))
    A = (G + G.T) / np.sqrt(2 * n) + (4.0 + 1.0j) * np.eye(n)
    xt = inputs.cn01(rng, n)
    y = A @ xt
    assert_parity(orc, method, A, y, xt, Ad=dev(stored_upper(A)),
                  label="symmetric dense, upper triangle", flags=ccg.A_SYM_UPPER)


def test_solver_edges(orc):
    """Warm start (set-up product from x0), y = 0, NaN in y, budget, and
    bitwise repeatability, all with the upper-triangle product."""
    import torch
    m = 5
    A, xt, y = inputs.lattice_system(m, 9)
    n = m ** 3
    Sd = dev(stored_upper(A))
    x0 = inputs.cn01(np.random.default_rng(10), n)
    for method in ("bicgstab", "cgnr", "cocg", "cocr"):
        fn = getattr(ccg, "ccg_%s_ex" % method)
        x = dev(x0)
        res = fn(Sd, dev(y), x, flags=ccg.A_SYM_UPPER)
        rel, slack = host_relres(A, x.cpu().numpy(), y)
        ref = getattr(orc, method)(A, y, x0=x0)
        assert res.info == 0 and rel <= 1e-10 + slack, (method, res)
        assert abs(res.iters - ref.iters) <= 1
        x = dev(x0)
        res = fn(Sd, dev(np.zeros(n, np.complex128)), x, flags=ccg.A_SYM_UPPER)
        assert res.info == 0 and np.all(x.cpu().numpy() == 0)
        ybad = y.copy()
        ybad[4] = np.nan
        x = dev(x0)
        res = fn(Sd, dev(ybad), x, flags=ccg.A_SYM_UPPER)
        assert res.info == 4 and np.array_equal(x.cpu().numpy(), x0)
        x = torch.zeros(n, dtype=torch.complex128, device="cuda")
        res = fn(Sd, dev(y), x, maxit=1, flags=ccg.A_SYM_UPPER | ccg.X0_ZERO)
        ref = getattr(orc, method)(A, y, maxit=1)
        assert res.info == ref.info == 1 and res.matvecs == ref.matvecs
        xa, ra, _ = gpu_solve(method, Sd, y, flags=ccg.A_SYM_UPPER)
        xb, rb, _ = gpu_solve(method, Sd, y, flags=ccg.A_SYM_UPPER)
        assert np.array_equal(xa, xb) and ra == rb


def test_small_workspace_is_rejected():
    A, _, y = inputs.lattice_system(4, 1)
    Sd = dev(stored_upper(A))
    import torch
    x = torch.zeros(A.shape[0], dtype=torch.complex128, device="cuda")
    for method, ws in (("cgnr", ccg.WS_CGNR), ("cocg", ccg.WS_COCG)):
        small = ccg.workspace(ws, A.shape[0])  # without the tile partials
        with pytest.raises(ValueError, match="argument 10"):
            getattr(ccg, "ccg_%s_ex" % method)(Sd, dev(y), x, flags=ccg.A_SYM_UPPER,
                                               work=small)


def test_cgnr_adjoint_product_matches_oracle(orc):
    """CGNR's A^H product from the upper triangle: one iteration from x0 = 0
    gives z = A^H y; compare the first iteration's alpha with the oracle's
    (its A^H comes from the full matrix)."""
    A, _, y = inputs.lattice_system(6, 3)
    x, res, h = gpu_solve("cgnr", dev(stored_upper(A)), y, maxit=1, flags=ccg.A_SYM_UPPER)
    ref = orc.cgnr(A, y, maxit=1)
    assert res.info == ref.info == 1
    assert abs(h[0, 0] - ref.hist[0, 0]) <= 1e-12 * abs(ref.hist[0, 0])
    assert np.linalg.norm(x - ref.x) <= 1e-12 * np.linalg.norm(ref.x)
