"""GPU tests of the serving loop (ccg_server_*): independent block systems of
the dense n = 256 family at several sizes, batched across requests.

Every request's arithmetic (block partition, reduction order, product
slices) is that of the request solved alone, so its x and per-column records
must equal those of ccg_bicgstab_block_ex (x0 = 0) on the same inputs bit for
bit, whatever else shares the batch; the block solver itself is checked
against the oracle in the block tests, and a few columns here are checked
against the oracle again."""
import numpy as np
import pytest

from gpu_util import dev, host_relres
from paper_1208_4869_amd import ccg, inputs

pytestmark = pytest.mark.gpu


def make_request(n, k, seed):
    A = inputs.dense_matrix(n, seed) if n > 0 else np.zeros((0, 0), np.complex128)
    Xt = inputs.cn01(np.random.default_rng(seed + 7), (n, k))
    return A, A @ Xt, Xt


def alone(A, Y, tol=1e-10, maxit=1000, X0=None):
    import torch
    n, k = Y.shape
    X = dev(X0) if X0 is not None else torch.full(
        (n, k), float("nan"), dtype=torch.complex128, device="cuda")
    res = ccg.ccg_bicgstab_block_ex(dev(A), dev(Y), X, tol, maxit,
                                    flags=ccg.X0_ZERO)
    return X.cpu().numpy(), res


def same_result(a, b):
    return (a.info, a.iters, a.matvecs, a.confirms) == \
        (b.info, b.iters, b.matvecs, b.confirms) and \
        np.array_equal(np.array([a.relres_rec, a.relres_true]),
                       np.array([b.relres_rec, b.relres_true]), equal_nan=True)


def serve(reqs, pool_bytes=None, max_active=64, tol=1e-10, maxit=1000,
          steps_between=0, host=False):
    """Submit reqs (list of (A, Y)) to a fresh server, steps_between steps
    apart, then run to completion.  Returns ([(X, results)], stats)."""
    import torch
    if pool_bytes is None:
        pool_bytes = 64 * 2 ** 20 + sum(
            ccg.ccg_server_request_bytes(A.shape[0], Y.shape[1]) for A, Y in reqs)
    out = {}
    with ccg.Server(pool_bytes, max_active=max_active) as srv:
        tickets = []
        held = []
        for A, Y in reqs:
            n, k = Y.shape
            if host:
                Ad = torch.from_numpy(np.ascontiguousarray(A))
                Yd = torch.from_numpy(np.ascontiguousarray(Y))
                Xd = torch.full((n, k), float("nan"), dtype=torch.complex128)
            else:
                Ad, Yd = dev(A), dev(Y)
                Xd = torch.full((n, k), float("nan"), dtype=torch.complex128,
                                device="cuda")
            tickets.append(srv.submit(Ad, Yd, Xd, tol, maxit))
            held.append(Xd)
            for _ in range(steps_between):
                srv.step()
        res = srv.run_all(tickets)
        torch.cuda.synchronize()
        stats = srv.stats()
    for t, Xd in zip(tickets, held):
        out[t] = (Xd.cpu().numpy(), res[t])
    return [out[t] for t in tickets], stats


SIZES = [(1, 1), (7, 3), (64, 16), (100, 5), (256, 8), (300, 1), (513, 4),
         (1024, 2), (130, 16), (2048, 1)]


@pytest.fixture(scope="module")
def mix():
    return [make_request(n, k, 100 + i) for i, (n, k) in enumerate(SIZES)]


@pytest.fixture(scope="module")
def mix_alone(mix):
    return [alone(A, Y) for A, Y, _ in mix]


def check_equal(got, ref):
    for i, ((X, res), (Xr, resr)) in enumerate(zip(got, ref)):
        assert np.array_equal(X, Xr, equal_nan=True), i
        assert len(res) == len(resr)
        for a, b in zip(res, resr):
            assert same_result(a, b), (i, a, b)


def test_serve_mix_equals_alone(mix, mix_alone, orc):
    got, stats = serve([(A, Y) for A, Y, _ in mix])
    check_equal(got, mix_alone)
    assert stats["completed"] == len(mix)
    assert stats["peak_active"] == len(mix)  # all in one batch
    assert stats["pool_used"] == 0
    for (A, Y, Xt), (X, res) in zip(mix, got):
        for c in range(Y.shape[1]):
            assert res[c].info == 0
            rel, slack = host_relres(A, X[:, c], Y[:, c])
            assert rel <= 1e-10 + slack
    # the oracle on the first column of a few requests
    for i in (2, 4, 6):
        A, Y, Xt = mix[i]
        ref = orc.bicgstab(A, Y[:, 0], tol=1e-10, maxit=1000)
        X, res = got[i]
        assert ref.info == 0
        assert abs(res[0].iters - ref.iters) <= 1
        fe = np.linalg.norm(X[:, 0] - Xt[:, 0]) / np.linalg.norm(Xt[:, 0])
        fe_ref = np.linalg.norm(ref.x - Xt[:, 0]) / np.linalg.norm(Xt[:, 0])
        assert fe <= 100 * max(fe_ref, 1e-13)


def test_serve_staggered_arrivals_and_slot_limit(mix, mix_alone):
    """Requests arrive while others iterate, at most 3 at a time."""
    got, stats = serve([(A, Y) for A, Y, _ in mix], max_active=3,
                       steps_between=2)
    check_equal(got, mix_alone)
    assert stats["peak_active"] <= 3


def test_serve_small_pool_waits(mix, mix_alone):
    """A pool that holds the largest request and little else: admission
    waits for retirements, results are unchanged."""
    need = max(ccg.ccg_server_request_bytes(A.shape[0], Y.shape[1])
               for A, Y, _ in mix)
    got, stats = serve([(A, Y) for A, Y, _ in mix], pool_bytes=need + 2 ** 20)
    check_equal(got, mix_alone)
    assert stats["admission_waits"] > 0
    assert stats["pool_peak"] <= need + 2 ** 20


def test_serve_rejects_what_never_fits():
    import torch
    A, Y, _ = make_request(512, 2, 5)
    small = ccg.ccg_server_request_bytes(64, 1) + 2 ** 20
    with ccg.Server(small) as srv:
        X = torch.zeros((512, 2), dtype=torch.complex128, device="cuda")
        with pytest.raises(ccg.Rejected):
            srv.submit(dev(A), dev(Y), X)
        A2, Y2, _ = make_request(64, 1, 6)
        X2 = torch.zeros((64, 1), dtype=torch.complex128, device="cuda")
        t = srv.submit(dev(A2), dev(Y2), X2)
        res = srv.run_all([t])[t]
        assert srv.stats()["rejected"] == 1
    Xr, resr = alone(A2, Y2, X0=np.zeros((64, 1), np.complex128))
    assert np.array_equal(X2.cpu().numpy(), Xr)
    assert same_result(res[0], resr[0])


def test_serve_special_columns_and_budget():
    """maxit = 1 (budget spent), a zero right-hand side, a NaN right-hand
    side (x left as given), and n = 0."""
    import torch
    A, Y, _ = make_request(200, 4, 9)
    Y = Y.copy()
    Y[:, 1] = 0
    Y[3, 2] = np.nan
    X0 = np.full((200, 4), 2.5 + 1j, np.complex128)
    reqs = [(A, Y, 1), (A, Y, 1000)]
    with ccg.Server(4 * ccg.ccg_server_request_bytes(200, 4)) as srv:
        held, tickets = [], []
        for A_, Y_, mi in reqs:
            X = dev(X0)
            tickets.append(srv.submit(dev(A_), dev(Y_), X, 1e-10, mi))
            held.append(X)
        empty = torch.zeros((0, 2), dtype=torch.complex128, device="cuda")
        A0 = torch.zeros((0, 0), dtype=torch.complex128, device="cuda")
        t0 = srv.submit(A0, empty, empty.clone())
        st, res0 = srv.poll(t0)
        assert st == ccg.REQ_DONE and [r.info for r in res0] == [0, 0]
        out = srv.run_all(tickets)
    for (A_, Y_, mi), X, t in zip(reqs, held, tickets):
        Xr, resr = alone(A_, Y_, maxit=mi, X0=X0)
        assert np.array_equal(X.cpu().numpy(), Xr, equal_nan=True)
        for a, b in zip(out[t], resr):
            assert same_result(a, b), (a, b)
    infos = [r.info for r in out[tickets[1]]]
    assert infos[1] == 0 and infos[2] == 4
    assert [r.info for r in out[tickets[0]]][0] == 1


def test_serve_host_memory_sources(mix, mix_alone):
    """A, Y and X in host memory: the same results."""
    sub = [0, 3, 4]
    got, _ = serve([(mix[i][0], mix[i][1]) for i in sub], host=True)
    check_equal(got, [mix_alone[i] for i in sub])


def test_serve_strided_and_mixed_residency_sources(mix, mix_alone):
    """Sources given as views with padded leading dimensions: a device A is
    read in place, device Y and X are copied into the pool by the batched
    set-up; requests whose X is in host memory take the copy path.  Results
    equal the solves alone and the padding of the caller's X is untouched."""
    import torch
    sub = [1, 3, 4, 6]
    pad = complex(3.0, 4.0)
    pool = 64 * 2 ** 20 + sum(ccg.ccg_server_request_bytes(mix[i][0].shape[0],
                                                           mix[i][1].shape[1]) for i in sub)
    with ccg.Server(pool, max_active=8) as srv:
        tickets, held = [], []
        for j, i in enumerate(sub):
            A, Y, _ = mix[i]
            n, k = Y.shape
            Ab = torch.full((n, n + 3), pad, dtype=torch.complex128, device="cuda")
            Ab[:, :n] = dev(A)
            Yb = torch.full((n, k + 2), pad, dtype=torch.complex128, device="cuda")
            Yb[:, :k] = dev(Y)
            Xb = torch.full((n, k + 5), pad, dtype=torch.complex128,
                            device="cuda" if j % 2 == 0 else "cpu")
            Xb[:, :k] = float("nan")
            tickets.append(srv.submit(Ab[:, :n], Yb[:, :k], Xb[:, :k], 1e-10, 1000))
            held.append((Ab, Yb, Xb))
        res = srv.run_all(tickets)
        torch.cuda.synchronize()
    for t, i, (_, _, Xb) in zip(tickets, sub, held):
        Xr, resr = mix_alone[i]
        k = Xr.shape[1]
        X = Xb.cpu().numpy()
        assert np.array_equal(X[:, :k], Xr, equal_nan=True), i
        assert np.all(X[:, k:] == pad), i
        assert all(same_result(a, b) for a, b in zip(res[t], resr)), i


def test_serve_server_reuse_many_rounds():
    """Slots and pool blocks are reused across many requests (more requests
    than slots, several waves), results as alone."""
    reqs = [make_request(n, k, 300 + i) for i, (n, k) in
            enumerate([(96, 2), (33, 1), (160, 3)] * 4)]
    got, stats = serve([(A, Y) for A, Y, _ in reqs], max_active=2,
                       steps_between=1)
    check_equal(got, [alone(A, Y) for A, Y, _ in reqs])
    assert stats["admitted"] == len(reqs)
    assert stats["peak_active"] <= 2


def test_serve_full_size_mix(orc):
    """The benchmark's request distribution (n in {512, 1024, 2048, 4096},
    k in 1..8, dense family; 24 requests from one seed), arriving while
    others iterate under a pool that cannot hold them all: every request
    equals the block solver alone bit for bit, every column meets the
    tolerance on the host, and sampled columns match the oracle."""
    import torch
    rng = np.random.default_rng(2024)
    ns = rng.choice([512, 1024, 2048, 4096], 24)
    ks = rng.integers(1, 9, 24)
    reqs = [make_request(int(n), int(k), 500 + i) for i, (n, k) in enumerate(zip(ns, ks))]
    pool = 3 * ccg.ccg_server_request_bytes(4096, 8)
    got, stats = serve([(A, Y) for A, Y, _ in reqs], pool_bytes=pool, steps_between=1)
    assert stats["completed"] == len(reqs) and stats["admission_waits"] > 0
    for i, ((A, Y, Xt), (X, res)) in enumerate(zip(reqs, got)):
        Xr, resr = alone(A, Y)
        assert np.array_equal(X, Xr), i
        for c in range(Y.shape[1]):
            assert res[c].info == 0 and same_result(res[c], resr[c])
            rel, slack = host_relres(A, X[:, c], Y[:, c])
            assert rel <= 1e-10 + slack, (i, c, rel)
        torch.cuda.empty_cache()
    for i in (int(np.argmax(ns)), int(np.argmin(ns))):
        A, Y, Xt = reqs[i]
        ref = orc.bicgstab(A, Y[:, 0], tol=1e-10, maxit=1000)
        X, res = got[i]
        assert ref.info == 0 and abs(res[0].iters - ref.iters) <= 1
        fe = np.linalg.norm(X[:, 0] - Xt[:, 0]) / np.linalg.norm(Xt[:, 0])
        fe_ref = np.linalg.norm(ref.x - Xt[:, 0]) / np.linalg.norm(Xt[:, 0])
        assert fe <= 100 * max(fe_ref, 1e-13)


def alone_mixed(A, Y, maxit=10, tol_inner=1e-5):
    import torch
    n, k = Y.shape
    Ad = dev(A)
    X = torch.full((n, k), float("nan"), dtype=torch.complex128, device="cuda")
    res = ccg.ccg_bicgstab_block_mixed_ex(Ad, ccg.ccg_round_c64(Ad), dev(Y), X, 1e-10, maxit,
                                          tol_inner, 1000, flags=ccg.X0_ZERO)
    return X.cpu().numpy(), res


def test_serve_mixed_and_fp64_in_one_mix():
    """Mixed-precision requests (FP64 refinement, inner solves on complex64
    products) and FP64 requests share the batched iterations: each mixed
    request equals ccg_bicgstab_block_mixed_ex alone bit for bit, each FP64
    request the block solver alone; a small pool forces waits."""
    import torch
    specs = [(1024, 2, False), (1024, 4, True), (300, 3, True), (64, 1, False),
             (513, 8, True), (200, 16, True), (100, 5, False), (7, 2, True)]
    reqs = [make_request(n, k, 700 + i) for i, (n, k, _) in enumerate(specs)]
    need = max(ccg.ccg_server_request_bytes(A.shape[0], Y.shape[1], mixed=mx)
               for (A, Y, _), (_, _, mx) in zip(reqs, specs))
    out, held = {}, []
    with ccg.Server(need + need // 4, max_active=4) as srv:
        tickets = []
        for (A, Y, _), (_, _, mx) in zip(reqs, specs):
            n, k = Y.shape
            X = torch.full((n, k), float("nan"), dtype=torch.complex128, device="cuda")
            tickets.append(srv.submit(dev(A), dev(Y), X, 1e-10, 10 if mx else 1000,
                                      mixed=mx))
            held.append(X)
        # all queued first; the largest request (1024, 4, mixed) fits the pool
        # only beside small ones, so it waits for the 1024-row FP64 request
        # admitted before it
        res = srv.run_all(tickets)
        stats = srv.stats()
    assert stats["completed"] == len(reqs) and stats["admission_waits"] > 0
    for i, ((A, Y, Xt), (n, k, mx)) in enumerate(zip(reqs, specs)):
        X = held[i].cpu().numpy()
        got = res[tickets[i]]
        if mx:
            Xr, rr = alone_mixed(A, Y)
            assert np.array_equal(X, Xr), i
            for a, b in zip(got, rr):
                assert (a.info, a.iters, a.matvecs, a.confirms) == \
                    (b.info, b.inner_iters, b.matvecs32, b.matvecs64), (i, a, b)
                assert a.relres_true == b.relres_true
        else:
            Xr, rr = alone(A, Y)
            assert np.array_equal(X, Xr), i
            for a, b in zip(got, rr):
                assert same_result(a, b)
        for c in range(k):
            rel, slack = host_relres(A, X[:, c], Y[:, c])
            assert got[c].info == 0 and rel <= 1e-10 + slack, (i, c, rel)


def test_serve_mixed_special_columns():
    """A mixed request with a zero and a non-finite column, and outer budget 0."""
    import torch
    A, Y, _ = make_request(150, 3, 77)
    Y = Y.copy()
    Y[:, 1] = 0
    Y[5, 2] = np.nan
    X0 = np.full((150, 3), 1.5 - 2j)
    with ccg.Server(4 * ccg.ccg_server_request_bytes(150, 3, mixed=True)) as srv:
        X = dev(X0)
        t = srv.submit(dev(A), dev(Y), X, 1e-10, 10, mixed=True)
        X2 = dev(X0)
        t2 = srv.submit(dev(A), dev(Y), X2, 1e-10, 0, mixed=True)
        res = srv.run_all([t, t2])
    Xg = X.cpu().numpy()
    assert [r.info for r in res[t]] == [0, 0, 4]
    assert np.all(Xg[:, 1] == 0) and np.array_equal(Xg[:, 2], X0[:, 2])
    rel, slack = host_relres(A, Xg[:, 0], Y[:, 0])
    assert rel <= 1e-10 + slack
    assert res[t2][0].info == 1 and np.all(X2.cpu().numpy()[:, 0] == 0)
