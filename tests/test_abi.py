"""The C-ABI library loads and exports every entry point include/ccg.h
declares, and its host-side argument checks reject illegal arguments before
any GPU work (these calls make no HIP call, so they run without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ccg.h")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ccg_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1208_4869_amd import build, ccg
    if not os.path.exists(build.LIB):
        build.build()
    return ccg.load()


def test_header_declares_the_abi():
    names = declared()
    for want in ("ccg_matvec", "ccg_bicgstab", "ccg_cgnr", "ccg_bicgstab_ex",
                 "ccg_cgnr_ex", "ccg_workspace_bytes", "ccg_matvec_ex"):
        assert want in names


def test_library_exports_every_declared_symbol(lib):
    for name in declared():
        assert hasattr(lib, name), name


def test_workspace_sizes(lib):
    from paper_1208_4869_amd import ccg
    for n in (1, 256, 8000, 17576):
        b = ccg.ccg_workspace_bytes(ccg.WS_BICGSTAB, n)
        c = ccg.ccg_workspace_bytes(ccg.WS_CGNR, n)
        assert b >= 6 * 16 * n and c >= 4 * 16 * n
        assert ccg.ccg_workspace_bytes(ccg.WS_MATVEC_C, n) >= 16 * n
    assert ccg.ccg_workspace_bytes(99, 10) == 0
    assert ccg.ccg_workspace_bytes(ccg.WS_BICGSTAB, -1) == 0


def test_argument_errors_are_rejected_on_the_host(lib):
    P = ctypes.c_void_p
    dummy = P(256)  # never dereferenced: the checks fail first
    info = ctypes.c_int32(-7)
    for fn in (lib.ccg_bicgstab, lib.ccg_cgnr):
        assert fn(-1, dummy, 1, dummy, dummy, 1e-10, 10, ctypes.byref(info), None) == -1
        assert fn(4, None, 4, dummy, dummy, 1e-10, 10, ctypes.byref(info), None) == -2
        assert fn(4, dummy, 3, dummy, dummy, 1e-10, 10, ctypes.byref(info), None) == -3
        assert fn(4, dummy, 4, None, dummy, 1e-10, 10, ctypes.byref(info), None) == -4
        assert fn(4, dummy, 4, dummy, None, 1e-10, 10, ctypes.byref(info), None) == -5
        for tol in (0.0, -1.0, float("nan"), float("inf")):
            assert fn(4, dummy, 4, dummy, dummy, tol, 10, ctypes.byref(info), None) == -6
        assert fn(4, dummy, 4, dummy, dummy, 1e-10, -1, ctypes.byref(info), None) == -7
        assert fn(4, dummy, 4, dummy, dummy, 1e-10, 10, None, None) == -8
        # n = 0 is a no-op with info 0
        assert fn(0, None, 1, None, None, 1e-10, 10, ctypes.byref(info), None) == 0
        assert info.value == 0
    from paper_1208_4869_amd.ccg import _Result
    res = _Result()
    for fn in (lib.ccg_bicgstab_ex, lib.ccg_cgnr_ex):
        args = [4, dummy, 4, dummy, dummy, 1e-10, 10]
        assert fn(*args, 4, dummy, 1 << 20, ctypes.byref(res), None, None) == -8
        assert fn(*args, 0, None, 1 << 20, ctypes.byref(res), None, None) == -9
        assert fn(*args, 0, P(257), 1 << 20, ctypes.byref(res), None, None) == -9
        assert fn(*args, 0, dummy, 16, ctypes.byref(res), None, None) == -10
        assert fn(*args, 0, dummy, 1 << 20, None, None, None) == -11
    # the upper-triangle flag needs the larger workspace (checked on the host
    # before anything is enqueued)
    args = [4, dummy, 4, dummy, dummy, 1e-10, 10]
    for fn, ws in ((lib.ccg_bicgstab_ex, 2), (lib.ccg_cgnr_ex, 3), (lib.ccg_cocg_ex, 6),
                   (lib.ccg_cocr_ex, 7)):
        assert fn(*args, 4, dummy, 1 << 20, ctypes.byref(res), None, None) == -8
        n = 5000
        plain = lib.ccg_workspace_bytes(ws, n, 1)
        sym = lib.ccg_workspace_bytes(ws | 0x100, n, 1)
        assert sym >= plain + n * 16 * ((n + 127) // 128)
        big = [n, dummy, n, dummy, dummy, 1e-10, 10]
        assert fn(*big, 2, dummy, plain, ctypes.byref(res), None, None) == -10
    assert lib.ccg_workspace_bytes(12, 5000, 1) == 16 * 5000 * 40
    assert lib.ccg_workspace_bytes(1 | 0x100, 5000, 1) == 0  # no such form
    for op, code in ((3, -1), (-1, -1)):
        assert lib.ccg_matvec(op, 4, dummy, 4, dummy, P(4096), None) == code
    assert lib.ccg_matvec(0, -3, dummy, 4, dummy, P(4096), None) == -2
    assert lib.ccg_matvec(0, 4, None, 4, dummy, P(4096), None) == -3
    assert lib.ccg_matvec(0, 4, dummy, 2, dummy, P(4096), None) == -4
    assert lib.ccg_matvec(0, 4, dummy, 4, None, P(4096), None) == -5
    assert lib.ccg_matvec(0, 4, dummy, 4, dummy, None, None) == -6
    assert lib.ccg_matvec(0, 4, dummy, 4, dummy, P(256 + 16), None) == -6  # overlap
    assert lib.ccg_matvec(1, 0, None, 1, None, None, None) == 0
    assert lib.ccg_matvec_ex(1, 4, dummy, 4, dummy, P(4096), None, 0, None) == -7
    assert lib.ccg_matvec_ex(1, 4, dummy, 4, dummy, P(4096), dummy, 8, None) == -8


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_1208_4869_amd import ccg
    monkeypatch.setattr(ccg, "_lib", None)
    monkeypatch.setattr(ccg, "lib_path", lambda: str(tmp_path / "missing.so"))
    with pytest.raises(ccg.CcgError):
        ccg.load()


def test_server_argument_errors_are_rejected_on_the_host(lib):
    from paper_1208_4869_amd import ccg
    P = ctypes.c_void_p
    out = P()
    big = 1 << 30
    assert lib.ccg_server_create(None, big, 4, None, ctypes.byref(out)) == -1
    assert lib.ccg_server_create(P(256 + 8), big, 4, None, ctypes.byref(out)) == -1
    assert lib.ccg_server_create(P(256), 100, 4, None, ctypes.byref(out)) == -2
    assert lib.ccg_server_create(P(256), big, 0, None, ctypes.byref(out)) == -3
    assert lib.ccg_server_create(P(256), big, 129, None, ctypes.byref(out)) == -3
    assert lib.ccg_server_create(P(256), big, 4, None, None) == -5
    t = ctypes.c_int64()
    assert lib.ccg_server_submit(None, 4, 1, P(256), 4, P(256), 1, P(256), 1,
                                 1e-10, 10, ctypes.byref(t)) == -1
    assert lib.ccg_server_step(None, None, None) == -1
    st = ctypes.c_int32()
    assert lib.ccg_server_poll(None, 1, ctypes.byref(st), None) == -1
    assert lib.ccg_server_destroy(None) == -1
    assert lib.ccg_server_get_stats(None, None) == -1
    # footprints: A, Y, X and the block workspace; k limited to 16
    assert ccg.ccg_server_request_bytes(0, 1) == 0
    assert ccg.ccg_server_request_bytes(-1, 1) == 0
    assert ccg.ccg_server_request_bytes(10, 0) == 0
    assert ccg.ccg_server_request_bytes(10, 17) == 0
    for n, k in ((512, 1), (4096, 8), (1000, 16)):
        b = ccg.ccg_server_request_bytes(n, k)
        assert b >= 16 * n * n + 2 * 16 * n * k + 15 * 16 * n * k
        assert b % 256 == 0


def test_structured_argument_errors_are_rejected_on_the_host(lib):
    from paper_1208_4869_amd import ccg
    from paper_1208_4869_amd.ccg import _Result
    P = ctypes.c_void_p
    d = P(256)
    assert ccg.ccg_t3_op_bytes(0) == 0 and ccg.ccg_t3_op_bytes(129) == 0
    M = 64  # padded edge at m = 20
    assert ccg.ccg_t3_op_bytes(20) >= 2 * 16 * M ** 3
    assert ccg.ccg_t3_workspace_bytes(ccg.WS_T3_MATVEC, 20) >= 16 * (M * 400 + M * M * 20)
    assert ccg.ccg_t3_workspace_bytes(ccg.WS_CGNR, 20) == 0  # no structured CGNR
    big = 1 << 30
    assert lib.ccg_t3_setup(0, d, d, big, None) == -1
    assert lib.ccg_t3_setup(129, d, d, big, None) == -1
    assert lib.ccg_t3_setup(4, None, d, big, None) == -2
    assert lib.ccg_t3_setup(4, d, P(264), big, None) == -3
    assert lib.ccg_t3_setup(4, d, d, 64, None) == -4
    assert lib.ccg_t3_matvec(0, None, None, None, None, 0, None) == 0
    assert lib.ccg_t3_matvec(4, None, d, d, d, big, None) == -2
    assert lib.ccg_t3_matvec(4, d, None, d, d, big, None) == -3
    assert lib.ccg_t3_matvec(4, d, d, None, d, big, None) == -4
    assert lib.ccg_t3_matvec(4, d, d, d, P(300), big, None) == -5
    assert lib.ccg_t3_matvec(4, d, d, d, d, 16, None) == -6
    res = _Result()
    for fn in (lib.ccg_t3_bicgstab_ex, lib.ccg_t3_cocg_ex, lib.ccg_t3_cocr_ex):
        ok = [4, d, d, d, 1e-10, 10, 0, d, big, ctypes.byref(res), None, None]
        for pos, bad in ((0, -1), (0, 129), (1, None), (2, None), (3, None), (4, 0.0),
                         (5, -1), (6, 2), (7, None), (8, 16), (9, None)):
            args = list(ok)
            args[pos] = bad
            assert fn(*args) == -(pos + 1), (fn, pos)
        args = list(ok)
        args[0] = 0
        assert fn(*args) == 0 and res.info == 0


def test_build_flags_kernels_with_scratch():
    from paper_1208_4869_amd import build
    remarks = "\n".join([
        "a.hip:1:1: remark: Function Name: _Z3fooPi [-Rpass-analysis=kernel-resource-usage]",
        "a.hip:1:1: remark:     ScratchSize [bytes/lane]: 0 [-Rpass-analysis=kernel-resource-usage]",
        "a.hip:9:1: remark: Function Name: _Z3barPi [-Rpass-analysis=kernel-resource-usage]",
        "a.hip:9:1: remark:     ScratchSize [bytes/lane]: 48 [-Rpass-analysis=kernel-resource-usage]",
    ])
    assert build.scratch_kernels(remarks) == [("_Z3barPi", 48)]


def test_block_mixed_argument_errors_are_rejected_on_the_host(lib):
    from paper_1208_4869_amd import ccg
    from paper_1208_4869_amd.ccg import _MixedResult
    P = ctypes.c_void_p
    d = P(256)
    big = 1 << 30
    assert ccg.ccg_workspace_bytes(ccg.WS_MATMAT_C64, 100, 8) >= 8 * 100 * 8 * 16
    assert ccg.ccg_workspace_bytes(ccg.WS_BICGSTAB_BLOCK_MIXED, 100, 8) > \
        ccg.ccg_workspace_bytes(ccg.WS_BICGSTAB_BLOCK, 100, 8)
    assert ccg.ccg_workspace_bytes(ccg.WS_BICGSTAB_BLOCK_MIXED, 100, 65) == 0
    assert lib.ccg_matmat_c64(4, 2, None, 4, d, 2, d, 2, d, big, None) == -3
    assert lib.ccg_matmat_c64(4, 2, d, 3, d, 2, d, 2, d, big, None) == -4
    assert lib.ccg_matmat_c64(4, 2, d, 4, d, 2, d, 2, P(300), big, None) == -9
    assert lib.ccg_matmat_c64(4, 2, d, 4, d, 2, d, 2, d, 8, None) == -10
    assert lib.ccg_matmat_c64(0, 2, None, 1, None, 2, None, 2, None, 0, None) == 0
    res = (_MixedResult * 2)()
    ok = [4, 2, d, 4, d, 4, d, 2, d, 2, 1e-10, 10, 1e-5, 100, 0, d, big, res, None, None]
    for pos, bad in ((0, -1), (1, 0), (1, 65), (2, None), (3, 3), (4, None), (5, 3),
                     (6, None), (7, 1), (8, None), (9, 1), (10, 0.0), (11, -1),
                     (12, 1.0), (13, 0), (14, 2), (15, None), (16, 8), (17, None)):
        args = list(ok)
        args[pos] = bad
        want = -(pos + 1) if pos != 1 else -2
        assert lib.ccg_bicgstab_block_mixed_ex(*args) == want, (pos, bad)


def test_server_mixed_argument_errors_are_rejected_on_the_host(lib):
    from paper_1208_4869_amd import ccg
    P = ctypes.c_void_p
    t = ctypes.c_int64()
    assert lib.ccg_server_submit_mixed(None, 4, 1, P(256), 4, P(256), 1, P(256), 1, 1e-10, 10,
                                       1e-5, 100, ctypes.byref(t)) == -1
    for n, k in ((512, 1), (4096, 8)):
        b = ccg.ccg_server_request_bytes(n, k)
        bm = ccg.ccg_server_request_bytes(n, k, mixed=True)
        assert bm >= b + 8 * n * n  # the complex64 copy of A on top
    assert ccg.ccg_server_request_bytes(10, 17, mixed=True) == 0


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: --gpus 2 exits with status 2 and says so,
    before touching any device."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    proc = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                          capture_output=True, text=True, timeout=120)
    assert proc.returncode == 2
    assert "one GPU" in proc.stderr


def test_noalloc_product_rejects_sizes_beyond_its_array_on_the_host(lib):
    """ccg_matvec_noalloc refuses, before any HIP call, a product whose
    partial sums would not fit its fixed device array (CCG_OP_S beyond
    n = 16384, CCG_OP_C from n = 2^20 on), an unknown op and a negative n."""
    P = ctypes.c_void_p
    dummy = P(256)  # never dereferenced: the checks fail first
    fn = lib.ccg_matvec_noalloc
    assert fn(7, 4, dummy, 4, dummy, P(512), None) == -1
    assert fn(0, -1, dummy, 4, dummy, P(512), None) == -2
    assert fn(2, 16385, dummy, 16385, dummy, P(512), None) == -2
    assert fn(2, 40000, dummy, 40000, dummy, P(512), None) == -2
    assert fn(1, 1 << 21, dummy, 1 << 21, dummy, P(512), None) == -2
    assert fn(1, (1 << 30) + 1, dummy, (1 << 30) + 1, dummy, P(512), None) == -2
    # n = 0 is a no-op
    assert fn(1, 0, None, 1, None, None, None) == 0


def test_small_batched_argument_errors_on_the_host(lib):
    """ccg_solve_small_batched rejects every illegal argument before any HIP
    call (these calls return before touching the device)."""
    P = ctypes.c_void_p
    d = P(256)  # never dereferenced
    fn = lib.ccg_solve_small_batched

    def call(method=2, n=8, batch=3, A=d, lda=8, sA=64, Y=d, sY=8, X=P(4096), sX=8,
             tol=1e-10, maxit=10, flags=0, res=d):
        return fn(method, n, batch, A, lda, sA, Y, sY, X, sX, tol, maxit, flags, res, None)

    assert call(method=5) == -1
    assert call(n=-1) == -2 and call(n=1025, lda=1025, sA=1025 * 1025) == -2
    assert call(batch=-1) == -3
    assert call(A=None) == -4
    assert call(lda=7) == -5
    assert call(sA=63) == -6
    assert call(Y=None) == -7
    assert call(sY=7) == -8
    assert call(X=None) == -9
    assert call(sX=7) == -10
    for tol in (0.0, -1.0, float("nan"), float("inf")):
        assert call(tol=tol) == -11
    assert call(maxit=-1) == -12
    assert call(flags=2) == -13
    assert call(res=None) == -14
    assert call(batch=0, A=None, Y=None, X=None, res=None) == 0
    # one system: its strides are not checked
    assert call(method=3, batch=1, sA=0, sY=0, sX=0, res=None) == -14


def test_read_stream_and_event_log_argument_errors_on_the_host(lib):
    """The measurement aids reject bad arguments before any HIP call."""
    from paper_1208_4869_amd.ccg import _EventLog
    P = ctypes.c_void_p
    assert lib.ccg_read_stream(None, 16, P(256), 16, None) == -1
    assert lib.ccg_read_stream(P(256), 24, P(256), 16, None) == -2
    assert lib.ccg_read_stream(P(264), 16, P(256), 16, None) == -2
    assert lib.ccg_read_stream(P(256), 16, None, 16, None) == -3
    assert lib.ccg_read_stream(P(256), 262144 + 16, P(256), 16, None) == -4
    assert lib.ccg_read_stream(None, 0, None, 0, None) == 0
    bad = _EventLog(None, 4, 0, 1, 0, 0, 0)
    assert lib.ccg_set_event_log(ctypes.byref(bad)) == -1
    neg = _EventLog(None, -1, 0, 1, 0, 0, 0)
    assert lib.ccg_set_event_log(ctypes.byref(neg)) == -1
    empty = _EventLog(None, 0, 0, 1, 0, 0, 0)
    assert lib.ccg_set_event_log(ctypes.byref(empty)) == 0
    assert lib.ccg_set_event_log(None) == 0
