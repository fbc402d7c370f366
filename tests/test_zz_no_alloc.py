"""ccg_matvec_noalloc (the allocation-free form of ccg_matvec, partial sums
in the library's fixed device array) against ccg_matvec_ex with a caller
workspace: bitwise equal results, for A x, A^H x and the upper-triangle
product, on two calls in a row with the second one smaller (the array keeps
the first call's partials, which the second must not see)."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _case(n, seed, sym=False):
    import torch
    rng = np.random.default_rng(seed)
    A = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(2 * n)
    if sym:
        A = A + A.T
        A[np.tril_indices(n, -1)] = np.nan  # never read by the upper-triangle product
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    return torch.from_numpy(A).cuda(), torch.from_numpy(x).cuda()


@pytest.mark.parametrize("op,sizes", [(0, (2000, 257)), (1, (3000, 1029)),
                                      (2, (4100, 700))])
def test_noalloc_matches_the_workspace_form(op, sizes):
    import torch

    from paper_1208_4869_amd import ccg
    lib = ccg.load()
    for k, n in enumerate(sizes):
        print("noalloc op=%d n=%d (call %d)" % (op, n, k + 1), flush=True)
        A, x = _case(n, 100 + 10 * op + k, sym=(op == ccg.OP_S))
        y_ref = torch.empty_like(x)
        ws = {ccg.OP_C: ccg.WS_MATVEC_C, ccg.OP_S: ccg.WS_MATVEC_S}.get(op)
        work = None
        if ws is not None:
            work = torch.empty(ccg.ccg_workspace_bytes(ws, n), dtype=torch.uint8,
                               device="cuda")
        ccg.ccg_matvec_ex(op, A, x, y_ref, work)
        y = torch.full_like(x, float("nan"))
        stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        rc = lib.ccg_matvec_noalloc(op, n, A.data_ptr(), n, x.data_ptr(), y.data_ptr(),
                                    stream)
        assert rc == 0
        torch.cuda.synchronize()
        assert torch.equal(y, y_ref), (op, n)
        # and the product itself: within the FP64 rounding bound of A x / A^H x
        An = A.cpu().numpy()
        if op == ccg.OP_S:
            An = np.triu(An) + np.triu(An, 1).T
        M = An.conj().T if op == ccg.OP_C else An
        xn = x.cpu().numpy()
        bound = 4 * (n + 2) * 2.0 ** -53 * (np.abs(M) @ np.abs(xn))
        assert np.all(np.abs(y.cpu().numpy() - M @ xn) <= bound)
