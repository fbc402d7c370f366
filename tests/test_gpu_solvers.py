"""GPU parity of ccg_bicgstab / ccg_cgnr against the oracle on the same
seeded inputs: every workload family, ragged sizes, and the degenerate cases
of the method (breakdowns, budget, non-finite input, zero right-hand side,
restarts after a failed confirmation)."""
import numpy as np
import pytest

import pins
from gpu_util import assert_parity, dev, gpu_solve, host_relres
from paper_1208_4869_amd import ccg, inputs

pytestmark = pytest.mark.gpu
METHODS = ("bicgstab", "cgnr")


@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("seed", range(10))
def test_dense_n256(orc, method, seed):
    """Dense family A = 4 I + G / sqrt(n), n = 256, seeds 0-9."""
    A, xt, y = inputs.dense_system(256, seed)
    assert_parity(orc, method, A, y, xt, label="dense seed %d" % seed)


@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("n", [1, 2, 3, 17, 64, 65, 257, 1000, 1029])
def test_ragged_sizes(orc, method, n):
    A, xt, y = inputs.dense_system(n, 1000 + n)
    assert_parity(orc, method, A, y, xt, label="ragged")


@pytest.fixture(scope="module")
def lattice20():
    A, xt, y = inputs.lattice_system(20, 1)
    return A, xt, y, dev(A), dev(y)


@pytest.mark.parametrize("method", METHODS)
def test_lattice_20(orc, method, lattice20):
    """Dipole-lattice family, 20^3 lattice (n = 8000), x_true seed 1."""
    A, xt, y, Ad, yd = lattice20
    assert_parity(orc, method, A, y, xt, Ad=Ad, yd=yd, label="lattice 20^3")


def test_lattice_26_bicgstab(orc):
    """26^3 lattice (n = 17576, 4.9 GB complex128), plain FP64 BiCGSTAB."""
    A, xt, y = inputs.lattice_system(26, 2)
    assert_parity(orc, "bicgstab", A, y, xt, label="lattice 26^3")


@pytest.mark.parametrize("method", METHODS)
def test_deterministic(method):
    A, _, y = inputs.dense_system(300, 3)
    x1, r1, _ = gpu_solve(method, A, y)
    x2, r2, _ = gpu_solve(method, A, y)
    assert np.array_equal(x1, x2) and r1.iters == r2.iters


@pytest.mark.parametrize("method", METHODS)
def test_warm_start_and_short_form(orc, method):
    import torch
    A, xt, y = inputs.dense_system(128, 4)
    x0 = xt + 1e-6
    ref = getattr(orc, method)(A, y, x0=x0)
    x, res, _ = gpu_solve(method, A, y, x0=x0)
    assert res.info == 0 and ref.info == 0 and abs(res.iters - ref.iters) <= 1
    assert res.matvecs - ref.matvecs in (-2, -1, 0, 1, 2)
    assert host_relres(A, x, y)[0] <= 1.01e-10
    # short form: explicit zero initial guess
    Ad, yd = dev(A), dev(y)
    xd = torch.zeros(128, dtype=torch.complex128, device="cuda")
    info = getattr(ccg, "ccg_" + method)(Ad, yd, xd)
    assert info == 0
    assert host_relres(A, xd.cpu().numpy(), y)[0] <= 1.01e-10


@pytest.mark.parametrize("method", METHODS)
def test_closed_forms(orc, method):
    c = 2.0 - 3.0j
    A = c * np.eye(40, dtype=np.complex128)
    y = inputs.cn01(np.random.default_rng(1), 40)
    x, res, _ = gpu_solve(method, A, y)
    assert res.info == 0 and res.iters == 1
    assert np.linalg.norm(x - y / c) <= 8 * pins.U * np.linalg.norm(y / c)
    D = pins.dft_matrix(16)
    y = inputs.cn01(np.random.default_rng(2), 16)
    x, res, _ = gpu_solve(method, D, y)
    ref = getattr(orc, method)(D, y)
    assert res.info == 0 and abs(res.iters - ref.iters) <= 1
    if method == "cgnr":
        assert res.iters == 1


def test_breakdowns_match_oracle(orc):
    A = np.array([[0, 1], [-1, 0]], dtype=np.complex128)
    y = np.array([1, 0], dtype=np.complex128)
    x, res, _ = gpu_solve("bicgstab", A, y)
    assert res.info == 2 and res.iters == 0 and np.all(x == 0)
    x, res, _ = gpu_solve("cgnr", A, y)
    assert res.info == 0 and res.iters == 1
    A3, y3 = pins.find_omega_zero_case()
    assert orc.bicgstab(A3, y3).info == 3
    x, res, _ = gpu_solve("bicgstab", A3, y3)
    assert res.info == 3 and res.iters == 0


@pytest.mark.parametrize("method", METHODS)
def test_budget_nonfinite_zero(orc, method):
    A, _, y = inputs.dense_system(96, 5)
    for maxit in (0, 1, 3):
        ref = getattr(orc, method)(A, y, maxit=maxit)
        x, res, _ = gpu_solve(method, A, y, maxit=maxit)
        assert (res.info, res.iters) == (ref.info, ref.iters) == (1, maxit)
        assert res.matvecs == ref.matvecs
    ybad = y.copy()
    ybad[7] = np.nan
    x0 = np.full(96, 0.5 + 0.5j)
    x, res, _ = gpu_solve(method, A, ybad, x0=x0)
    assert res.info == 4 and np.array_equal(x, x0)
    Abad = A.copy()
    Abad[10, 3] = np.inf
    x, res, _ = gpu_solve(method, Abad, y)
    assert res.info == 4 == getattr(orc, method)(Abad, y).info
    x, res, _ = gpu_solve(method, A, np.zeros(96, dtype=np.complex128), x0=x0)
    assert res.info == 0 and res.iters == 0 and res.matvecs == 0 and np.all(x == 0)
    x, res, _ = gpu_solve(method, A, np.zeros(96, dtype=np.complex128))
    assert res.info == 0 and np.all(x == 0)


@pytest.mark.parametrize("method", METHODS)
def test_restart_after_failed_confirmation(orc, method):
    """tol below round-off: the recursive residual falls while the true one
    stalls; confirmations fail, the true residual replaces r, and the budget
    ends the solve -- on the GPU as in the oracle."""
    A, _, y = inputs.dense_system(48, 2)
    ref = getattr(orc, method)(A, y, tol=1e-18, maxit=120)
    x, res, _ = gpu_solve(method, A, y, tol=1e-18, maxit=120)
    assert ref.info == 1 and res.info == 1 and res.iters == 120
    assert res.confirms >= 2
    assert res.relres_true <= 1e-14 and host_relres(A, x, y)[0] <= 1e-14


@pytest.mark.parametrize("method", METHODS)
def test_hist_and_result_fields(orc, method):
    A, _, y = inputs.dense_system(200, 8)
    ref = getattr(orc, method)(A, y)
    x, res, h = gpu_solve(method, A, y)
    assert res.matvecs == ref.matvecs and res.confirms == ref.confirms == 1
    assert res.relres_true <= 1e-10 and abs(res.relres_true - ref.relres_true) <= 1e-12
    k = res.iters
    finite_g = ~np.isnan(h[:k])
    finite_o = ~np.isnan(ref.hist[:k])
    assert np.array_equal(finite_g, finite_o)  # same fields produced


@pytest.mark.parametrize("method", ["bicgstab", "cgnr", "cocg", "cocr"])
def test_x0_zero_with_special_y(orc, method):
    """With the x0 = 0 flag the first kernel zeroes x, copies y and forms
    ||y||^2: a non-finite y ends with info 4 at x = 0 (the last finite
    iterate), y = 0 with info 0 and x = 0; neither spends a product."""
    A, _, y = inputs.dense_system(96, 5)
    ybad = y.copy()
    ybad[11] = complex(np.inf, 0.0)
    x, res, _ = gpu_solve(method, A, ybad)
    assert res.info == 4 and res.iters == 0 and res.matvecs == 0 and np.all(x == 0)
    assert getattr(orc, method)(A, ybad).info == 4
    x, res, _ = gpu_solve(method, A, np.zeros(96, dtype=np.complex128))
    assert res.info == 0 and res.iters == 0 and res.matvecs == 0 and np.all(x == 0)
