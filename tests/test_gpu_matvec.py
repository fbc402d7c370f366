"""GPU parity of ccg_matvec (A x and A^H x) against the oracle's products."""
import numpy as np
import pytest

from gpu_util import dev, gamma
from paper_1208_4869_amd import ccg, inputs

pytestmark = pytest.mark.gpu

SIZES = [1, 2, 63, 64, 65, 127, 200, 257, 1000, 1029]


@pytest.mark.parametrize("n", SIZES)
def test_integer_inputs_bitwise(orc, n):
    """Gaussian-integer A, x with |parts| <= 1024: every partial sum is an
    integer below 2^53, so GPU and oracle agree bit for bit."""
    A = inputs.gaussian_integer_matrix(n, n, bound=1024)
    x = inputs.gaussian_integer_vector(n, n + 1, bound=1024)
    Ad, xd = dev(A), dev(x)
    y = ccg.ccg_matvec(ccg.OP_N, Ad, xd).cpu().numpy()
    yh = ccg.ccg_matvec(ccg.OP_C, Ad, xd).cpu().numpy()
    assert np.array_equal(y, orc.matvec(A, x))
    assert np.array_equal(yh, orc.matvec_h(A, x))


@pytest.mark.parametrize("n", [5, 300, 1031])
def test_random_inputs_within_rounding_bound(orc, n):
    rng = np.random.default_rng(n)
    A = inputs.cn01(rng, (n, n))
    x = inputs.cn01(rng, n)
    Ad, xd = dev(A), dev(x)
    y = ccg.ccg_matvec(ccg.OP_N, Ad, xd).cpu().numpy()
    yh = ccg.ccg_matvec(ccg.OP_C, Ad, xd).cpu().numpy()
    b = 4 * gamma(n + 2)
    assert np.all(np.abs(y - orc.matvec(A, x)) <= b * (np.abs(A) @ np.abs(x)))
    assert np.all(np.abs(yh - orc.matvec_h(A, x)) <= b * (np.abs(A).T @ np.abs(x)))


def test_leading_dimension_and_determinism(orc):
    import torch
    n, lda = 100, 131
    rng = np.random.default_rng(2)
    big = inputs.cn01(rng, (n, lda))
    x = inputs.cn01(rng, n)
    Ad = dev(big)[:, :n]
    assert Ad.stride(0) == lda
    xd = dev(x)
    A = np.ascontiguousarray(big[:, :n])
    for op, ref in ((ccg.OP_N, orc.matvec(A, x)), (ccg.OP_C, orc.matvec_h(A, x))):
        y1 = ccg.ccg_matvec(op, Ad, xd).cpu().numpy()
        y2 = ccg.ccg_matvec(op, Ad, xd).cpu().numpy()
        assert np.array_equal(y1, y2)  # fixed summation order
        bnd = 4 * gamma(n + 2) * ((np.abs(A) if op == 0 else np.abs(A).T) @ np.abs(x))
        assert np.all(np.abs(y1 - ref) <= bnd)
    # caller-provided scratch for A^H x
    ws = torch.empty(ccg.ccg_workspace_bytes(ccg.WS_MATVEC_C, n), dtype=torch.uint8,
                     device="cuda")
    y3 = torch.empty_like(xd)
    ccg.ccg_matvec_ex(ccg.OP_C, Ad, xd, y3, ws)
    assert np.array_equal(y3.cpu().numpy(), ccg.ccg_matvec(ccg.OP_C, Ad, xd).cpu().numpy())


def test_empty_and_errors():
    import torch
    A = torch.zeros((0, 0), dtype=torch.complex128, device="cuda")
    x = torch.zeros(0, dtype=torch.complex128, device="cuda")
    assert ccg.ccg_matvec(ccg.OP_N, A, x).numel() == 0
    A1 = torch.ones((3, 3), dtype=torch.complex128, device="cuda")
    x1 = torch.ones(3, dtype=torch.complex128, device="cuda")
    with pytest.raises(ValueError):
        ccg.ccg_matvec(7, A1, x1)
    with pytest.raises(ValueError):  # y aliases x
        ccg.ccg_matvec(ccg.OP_N, A1, x1, x1)


@pytest.mark.parametrize("m", [20, 26])
def test_full_size_lattice(orc, m):
    """The 20^3 (n = 8000) and 26^3 (n = 17576) lattice matrices in the launch
    configuration the solvers and the benchmark use: every output against the
    oracle within the rounding bound, and the complex-symmetry identity
    A^H x = conj(A conj(x))."""
    A = inputs.lattice_matrix(m)
    n = A.shape[0]
    x = inputs.cn01(np.random.default_rng(m), n)
    Ad, xd = dev(A), dev(x)
    y = ccg.ccg_matvec(ccg.OP_N, Ad, xd).cpu().numpy()
    yh = ccg.ccg_matvec(ccg.OP_C, Ad, xd).cpu().numpy()
    absAx = np.abs(A) @ np.abs(x)
    b = 4 * gamma(n + 2)
    assert np.all(np.abs(y - orc.matvec(A, x)) <= b * absAx)
    assert np.all(np.abs(yh - orc.matvec_h(A, x)) <= b * absAx)  # |A| symmetric
    yc = np.conj(ccg.ccg_matvec(ccg.OP_N, Ad, dev(np.conj(x))).cpu().numpy())
    assert np.all(np.abs(yh - yc) <= 2 * b * absAx)
