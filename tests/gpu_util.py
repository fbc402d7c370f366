"""Helpers of the GPU parity tests: move inputs to the device, run a solver
through the C ABI, and compare it with the oracle on the same inputs."""
import numpy as np

U = 2.0 ** -53


def gamma(k):
    return k * U / (1 - k * U)


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host_relres(A, x, y):
    """||y - A x|| / ||y|| in FP64 on the host (NumPy), and the rounding bound
    of that evaluation relative to ||y||."""
    r = y - A @ x
    ny = np.linalg.norm(y)
    bound = gamma(A.shape[0] + 2) * np.linalg.norm(np.abs(y) + np.abs(A) @ np.abs(x))
    return np.linalg.norm(r) / ny, bound / ny


def gpu_solve(method, A, y, tol=1e-10, maxit=1000, x0=None, hist=True, flags=0):
    """Run ccg_<method>_ex on the device copies of A and y.  x0 None means the
    x0 = 0 flag; flags are added to it.  Returns (x on the host, Result, hist
    array or None)."""
    import torch

    from paper_1208_4869_amd import ccg
    n = A.shape[0]
    Ad = A if isinstance(A, torch.Tensor) else dev(A)
    yd = y if isinstance(y, torch.Tensor) else dev(y)
    if x0 is None:
        x = torch.full((n,), float("nan"), dtype=torch.complex128, device="cuda")
        flags |= ccg.X0_ZERO
    else:
        x = dev(np.asarray(x0, dtype=np.complex128)).clone()
    h = ccg.new_hist(maxit) if hist else None
    fn = getattr(ccg, "ccg_%s_ex" % method)
    res = fn(Ad, yd, x, tol, maxit, flags=flags, hist=h)
    torch.cuda.synchronize()
    return x.cpu().numpy(), res, (h.cpu().numpy() if h is not None else None)


def assert_parity(orc, method, A, y, x_true=None, tol=1e-10, maxit=1000,
                  Ad=None, yd=None, label="", flags=0):
    """GPU vs oracle on the same realised A, y:
      * both converge (info 0);
      * the GPU's true relative residual, recomputed on the host in FP64, is
        <= tol (plus the rounding bound of that recomputation);
      * forward error <= 100 x max(oracle forward error, 1e-13);
      * iteration counts within 1;
      * the scalar histories (alpha, omega, beta) agree to 1e-6 relative while the
        residual is above 1e-8."""
    ref = getattr(orc, method)(A, y, tol=tol, maxit=maxit)
    x, res, h = gpu_solve(method, Ad if Ad is not None else A,
                          yd if yd is not None else y, tol, maxit, flags=flags)
    rel, slack = host_relres(A, x, y)
    msg = "%s %s n=%d: gpu info %d iters %d relres %.3e | oracle info %d iters %d" % (
        label, method, A.shape[0], res.info, res.iters, rel, ref.info, ref.iters)
    assert ref.info == 0, msg
    assert res.info == 0, msg
    assert rel <= tol + slack, msg
    assert abs(res.iters - ref.iters) <= 1, msg
    if x_true is not None:
        fe = np.linalg.norm(x - x_true) / np.linalg.norm(x_true)
        fe_ref = np.linalg.norm(ref.x - x_true) / np.linalg.norm(x_true)
        assert fe <= 100 * max(fe_ref, 1e-13), msg + " fe %.3e vs %.3e" % (fe, fe_ref)
    k = min(res.iters, ref.iters)
    for it in range(k):
        if not (ref.hist[it, 7] > 1e-8 or np.isnan(ref.hist[it, 7])):
            break
        for col in (0, 2, 4):  # alpha, omega, beta
            a = h[it, col] + 1j * h[it, col + 1]
            b = ref.hist[it, col] + 1j * ref.hist[it, col + 1]
            if np.isnan(b):
                continue
            assert abs(a - b) <= 1e-6 * abs(b), msg + " hist it %d col %d" % (it, col)
        if ref.hist[it, 6] <= 1e-8:
            break
    return x, res, ref
