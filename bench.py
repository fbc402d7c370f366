"""Benchmark of the complex Krylov hot path on one MI355X.

Workload (the headline): the dipole-lattice system on a 20^3 cubic lattice,
n = 8000, dense complex128 A (1.024 GB, resident in HBM before timing), x_true
iid CN(0,1) from seed 1, y = A x_true, BiCGSTAB from x0 = 0 to a relative
residual of 1e-10 (maxit 1000).  One step = one complete BiCGSTAB solve through
the C ABI (set-up, iterations with their products, fused reductions and device
scalar steps, confirmation), ending when the host holds info.

Printed: one JSON line with solves/s, p50/p99 latency, the roofline of the
dominant kernel (A x, HBM-bound: algorithmic bytes 16 n^2 + 32 n per launch over
its average launch time from HIP events on the stream it runs on), CGNR on the
same system, and the CPU oracle timed on a bounded sample on the host.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
    python bench.py --profile-kernels     # short kernel mix for rocprofv3
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "BiCGSTAB solves/s at 1e-10 residual; matvec HBM GB/s; p50/p99 latency"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3
BLOCK_RHS = 64
BLOCK_SEED = 5
LATTICE_M = 20
X_SEED = 1
TOL = 1e-10
MAXIT = 1000


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_lattice20.md")


def measured_traffic(which="kernel"):
    """HBM bytes per launch from the committed FETCH_SIZE / WRITE_SIZE record
    (which = "role": the A x role kernels inside the solvers; "kernel": the
    plain products; "sym": the upper-triangle product), or None when that
    group's hashed kernel sources changed since it was taken."""
    import hashlib
    try:
        line = [ln for ln in open(TRAFFIC_FILE) if ln.startswith("traffic-json:")][0]
        rec = json.loads(line.split(":", 1)[1])
        h = hashlib.sha256()
        for p in rec[which + "_sources"]:
            h.update(open(os.path.join(ROOT, p), "rb").read())
        if h.hexdigest() != rec[which + "_sources_sha256"]:
            return None
        return rec
    except (OSError, IndexError, KeyError, ValueError):
        return None


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=30)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=15.0,
                   help="bound on the oracle's timed sample")
    p.add_argument("--no-mixed", action="store_true",
                   help="skip the 26^3 mixed-precision leg")
    p.add_argument("--no-block", action="store_true",
                   help="skip the 64 right-hand-side block leg")
    p.add_argument("--no-structured", action="store_true",
                   help="skip the structured (FFT) lattice product leg")
    p.add_argument("--no-serve", action="store_true",
                   help="skip the continuous-batching serving leg")
    p.add_argument("--serve-requests", type=int, default=512)
    p.add_argument("--serve-rate", type=float, default=None,
                   help="Poisson arrival rate (requests/s) of the serving leg")
    p.add_argument("--no-sym", action="store_true",
                   help="skip the upper-triangle (complex symmetric) leg")
    p.add_argument("--no-config0", action="store_true",
                   help="skip the n = 256 single-solve and 1024-system batch leg")
    p.add_argument("--headline-only", action="store_true",
                   help="only the headline BiCGSTAB solves and their product timing "
                        "(for kernel traces of the headline)")
    p.add_argument("--profile-kernels", action="store_true",
                   help="run a short mix of the kernels for rocprofv3 and exit")
    return p.parse_args()


def make_inputs():
    from paper_1208_4869_amd import inputs
    t = time.time()
    A = inputs.lattice_matrix(LATTICE_M)
    rng = np.random.default_rng(X_SEED)
    x_true = inputs.cn01(rng, A.shape[0])
    y = A @ x_true
    log("built the %d^3 lattice system (n=%d) in %.1fs" % (LATTICE_M, A.shape[0],
                                                         time.time() - t))
    return A, x_true, y


def time_solves(fn, A, y, x, work, steps, warmup, hist=None, flags=1, event_log=None):
    """Solves from x0 = 0 (flag 1) plus `flags`; host clock per solve.
    event_log: a ccg.EventLog attached over the timed solves (it samples
    their product launches with HIP events on the stream they run on)."""
    import contextlib

    import torch
    res = None
    flags |= 1
    for _ in range(warmup):
        res = fn(A, y, x, TOL, MAXIT, flags=flags, work=work, hist=hist)
    torch.cuda.synchronize()
    lat = []
    with (event_log if event_log is not None else contextlib.nullcontext()):
        t0 = time.perf_counter()
        for _ in range(steps):
            ts = time.perf_counter()
            res = fn(A, y, x, TOL, MAXIT, flags=flags, work=work, hist=hist)
            lat.append(time.perf_counter() - ts)
        torch.cuda.synchronize()
        total = time.perf_counter() - t0
    return total, np.array(lat), res


def time_kernel(launch, reps):
    """Average duration of one launch from HIP events recorded on torch's
    current stream, the stream the library launches on."""
    import torch
    launch()
    torch.cuda.synchronize()
    s = torch.cuda.Event(enable_timing=True)
    e = torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        launch()
    e.record()
    e.synchronize()
    return s.elapsed_time(e) / 1e3 / reps


def _time_oracle(orc, A, y, budget_s):
    """Complete oracle BiCGSTAB solves of (A, y) until budget_s has passed
    (at least one, at most 50): (solves/s, count, seconds, last result)."""
    t0 = time.perf_counter()
    k = 0
    res = None
    while True:
        res = orc.bicgstab(A, y, tol=TOL, maxit=MAXIT)
        k += 1
        el = time.perf_counter() - t0
        if el >= budget_s or k >= 50:
            break
    return k / el, k, el, res


PRODUCT_SAMPLE_STRIDE = 7


def headline_record(args, total, lat, res, n, relres, fwd):
    """The contract fields of the JSON line for the headline solves."""
    return {
        "metric": METRIC,
        "value": args.steps / total,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * total / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128",
        "data": "synthetic",
        "config": {"workload": "dipole-lattice 20^3, n=8000, dense complex128 "
                               "A resident in HBM, BiCGSTAB tol 1e-10 from x0=0",
                   "n": n, "tol": TOL, "maxit": MAXIT, "method": "bicgstab",
                   "x_seed": X_SEED},
        "p50_ms": float(np.percentile(lat, 50) * 1e3),
        "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "iters": res.iters,
        "matvecs": res.matvecs,
        "relres_true": relres,
        "fwd_err": fwd,
    }


READ_STREAM_BYTES = 4 << 30


def read_stream_peak():
    """The HBM read rate the chip delivers to a plain streaming read of 4 GiB
    with the products' 16-byte nontemporal loads (ccg_read_stream), best of
    10 launches timed with HIP events: the achievable ceiling the product
    rates are also set against."""
    import torch

    from paper_1208_4869_amd import ccg
    buf = torch.ones(READ_STREAM_BYTES // 8, dtype=torch.float64, device="cuda")
    out = ccg.ccg_read_stream(buf)
    torch.cuda.synchronize()
    best = None
    for _ in range(10):
        s = torch.cuda.Event(enable_timing=True)
        e = torch.cuda.Event(enable_timing=True)
        s.record()
        ccg.ccg_read_stream(buf, out)
        e.record()
        e.synchronize()
        t = s.elapsed_time(e) / 1e3
        best = t if best is None else min(best, t)
    del buf
    torch.cuda.empty_cache()
    gbs = READ_STREAM_BYTES / best / 1e9
    log("read stream: %.0f GB/s (%.1f%% of %.0f)" % (gbs, 100 * gbs / HBM_PEAK_GBS,
                                                    HBM_PEAK_GBS))
    return gbs


def cpu_baseline(A, y, budget_s):
    """The oracle timed on the host: the one-thread build pinned to one core
    (taskset-style affinity of this process, restored afterwards), and the
    OpenMP build of the same source on every core this process may use (the
    rows of the dense product shared out; the same results bit for bit).
    Half the budget each."""
    import oracle
    allowed = sorted(os.sched_getaffinity(0))
    core = allowed[0]
    os.sched_setaffinity(0, {core})
    try:
        v1, k1, el1, res = _time_oracle(oracle.get(), A, y, budget_s / 2)
    finally:
        os.sched_setaffinity(0, set(allowed))
    omp = oracle.get_omp()
    threads = omp.threads(len(allowed))
    vn, kn, eln, resn = _time_oracle(omp, A, y, budget_s / 2)
    same = bool(np.array_equal(res.x, resn.x))
    common = {"host_cpu": host_cpu(), "host_threads": os.cpu_count(),
              "allowed_cpus": len(allowed)}
    one = {"value": v1, "unit": "solves/s", "cores": 1, "kind": "oracle",
           "sample": "%d complete BiCGSTAB solve(s) of the same 20^3 lattice system "
                     "(n=8000) by the one-thread C oracle pinned to cpu %d, %.1f s"
                     % (k1, core, el1),
           "iters": res.iters, "relres_true": res.relres_true, **common}
    alln = {"value": vn, "unit": "solves/s", "cores": threads, "kind": "oracle (OpenMP build)",
            "sample": "%d complete solve(s) of the same system by the OpenMP build of the "
                      "same oracle source on %d threads, %.1f s; solution bit for bit "
                      "equal to the one-thread build's: %s" % (kn, threads, eln, same),
            "bitwise_equal_to_one_thread": same, **common}
    return one, alln


def host_cpu():
    """The host CPU's model name (Linux), or None."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def mixed_leg(steps):
    """The 26^3 lattice (n = 17576, 4.94 GB complex128 + 2.47 GB complex64
    copy): plain FP64 BiCGSTAB against FP64 refinement around complex64
    BiCGSTAB (inner tolerance 1e-5), both to 1e-10 on the FP64 true residual.
    The matrix is gathered on the device from the host displacement table
    (bitwise the host matrix); y = A x_true (x_true seed 2) by ccg_matvec."""
    import torch

    from paper_1208_4869_amd import ccg, inputs
    m = 26
    t0 = time.time()
    A = inputs.lattice_matrix_torch(m, "cuda")
    n = A.shape[0]
    xt = torch.from_numpy(inputs.cn01(np.random.default_rng(2), n)).cuda()
    y = ccg.ccg_matvec(ccg.OP_N, A, xt)
    A32 = ccg.ccg_round_c64(A)
    torch.cuda.synchronize()
    log("built the 26^3 system on the device in %.1fs" % (time.time() - t0))
    x64 = torch.empty_like(y)
    w64 = ccg.workspace(ccg.WS_BICGSTAB, n)
    t64, lat64, r64 = time_solves(ccg.ccg_bicgstab_ex, A, y, x64, w64, steps, 1)
    xm = torch.empty_like(y)
    wm = torch.empty(ccg.ccg_workspace_bytes(ccg.WS_BICGSTAB_MIXED, n), dtype=torch.uint8,
                     device="cuda")
    rm = ccg.ccg_bicgstab_mixed_ex(A, A32, y, xm, TOL, 10, 1e-5, MAXIT, flags=1, work=wm)
    torch.cuda.synchronize()
    ts = time.perf_counter()
    for _ in range(steps):
        rm = ccg.ccg_bicgstab_mixed_ex(A, A32, y, xm, TOL, 10, 1e-5, MAXIT, flags=1, work=wm)
    torch.cuda.synchronize()
    tm = (time.perf_counter() - ts) / steps
    # complex64 product (the inner kernel) timed with HIP events
    x32 = xt.to(torch.complex64)
    y32 = torch.empty_like(x32)
    tc = time_kernel(lambda: ccg.ccg_matvec_c64(A32, x32, y32), 20)
    tz = time_kernel(lambda: ccg.ccg_matvec(ccg.OP_N, A, xt, y), 20)
    diff = float(torch.linalg.norm(xm - x64) / torch.linalg.norm(x64))
    fe_m = float(torch.linalg.norm(xm - xt) / torch.linalg.norm(xt))
    fe_64 = float(torch.linalg.norm(x64 - xt) / torch.linalg.norm(xt))
    log("26^3: FP64 %.2f ms, mixed %.2f ms (%d outer, %d inner its)" % (
        t64 / steps * 1e3, tm * 1e3, rm.outer, rm.inner_iters))
    out = {"workload": "dipole-lattice 26^3, n=17576",
           "fp64": {"solves_per_s": steps / t64, "ms": t64 / steps * 1e3,
                    "iters": r64.iters, "matvecs": r64.matvecs,
                    "relres_true": r64.relres_true, "fwd_err": fe_64},
           "mixed": {"solves_per_s": 1.0 / tm, "ms": tm * 1e3, "outer": rm.outer,
                     "inner_iters": rm.inner_iters, "matvecs64": rm.matvecs64,
                     "matvecs32": rm.matvecs32, "relres_true": rm.relres_true,
                     "fwd_err": fe_m, "rel_diff_vs_fp64_solution": diff,
                     "tol_inner": 1e-5},
           "speedup": (t64 / steps) / tm,
           "matvec_c128_us": tz * 1e6, "matvec_c128_gbs": 16.0 * n * n / tz / 1e9,
           "matvec_c64_us": tc * 1e6, "matvec_c64_gbs": 8.0 * n * n / tc / 1e9}
    del A, A32
    torch.cuda.empty_cache()
    return out


def block_leg(A, A_h, steps):
    """The 20^3 lattice with 64 right-hand sides (X_true seed 5): the product
    A P on FP64 matrix cores timed with HIP events (8 n^2 k algorithmic flops
    per launch, of which the matrix cores execute 6 n^2 k: three real products
    per complex one), and complete block BiCGSTAB solves of all 64 columns."""
    import torch

    from paper_1208_4869_amd import ccg, inputs
    n = A.shape[0]
    k = BLOCK_RHS
    Xt = inputs.cn01(np.random.default_rng(BLOCK_SEED), (n, k))
    Y_h = A_h @ Xt
    Y = torch.from_numpy(Y_h).cuda()
    P = torch.from_numpy(Xt).cuda()
    Z = torch.empty_like(P)
    wmm = torch.empty(ccg.ccg_workspace_bytes(ccg.WS_MATMAT, n, k), dtype=torch.uint8,
                      device="cuda")
    tg = time_kernel(lambda: ccg.ccg_matmat(A, P, Z, work=wmm), 20)
    flops = 8.0 * n * n * k
    work = torch.empty(ccg.ccg_workspace_bytes(ccg.WS_BICGSTAB_BLOCK, n, k),
                       dtype=torch.uint8, device="cuda")
    X = torch.empty_like(P)
    res = ccg.ccg_bicgstab_block_ex(A, Y, X, TOL, MAXIT, flags=1, work=work)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        res = ccg.ccg_bicgstab_block_ex(A, Y, X, TOL, MAXIT, flags=1, work=work)
    torch.cuda.synchronize()
    tb = (time.perf_counter() - t0) / steps
    Xg = X.cpu().numpy()
    rel = np.linalg.norm(Y_h - A_h @ Xg, axis=0) / np.linalg.norm(Y_h, axis=0)
    log("block: A P %.1f us (%.1f TFLOP/s); 64-column solve %.2f ms" % (
        tg * 1e6, flops / tg / 1e12, tb * 1e3))
    # mixed precision: complex64 product on FP32 matrix cores + FP64 refinement
    A32 = ccg.ccg_round_c64(A)
    w32 = torch.empty(ccg.ccg_workspace_bytes(ccg.WS_MATMAT_C64, n, k), dtype=torch.uint8,
                      device="cuda")
    t32 = time_kernel(lambda: ccg.ccg_matmat_c64(A32, P, Z, work=w32), 20)
    wm = torch.empty(ccg.ccg_workspace_bytes(ccg.WS_BICGSTAB_BLOCK_MIXED, n, k),
                     dtype=torch.uint8, device="cuda")
    Xm = torch.empty_like(P)
    rm = ccg.ccg_bicgstab_block_mixed_ex(A, A32, Y, Xm, TOL, 10, 1e-5, MAXIT, flags=1, work=wm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        rm = ccg.ccg_bicgstab_block_mixed_ex(A, A32, Y, Xm, TOL, 10, 1e-5, MAXIT, flags=1,
                                             work=wm)
    torch.cuda.synchronize()
    tmix = (time.perf_counter() - t0) / steps
    Xmg = Xm.cpu().numpy()
    relm = np.linalg.norm(Y_h - A_h @ Xmg, axis=0) / np.linalg.norm(Y_h, axis=0)
    fem = np.linalg.norm(Xmg - Xt, axis=0) / np.linalg.norm(Xt, axis=0)
    fe64 = np.linalg.norm(Xg - Xt, axis=0) / np.linalg.norm(Xt, axis=0)
    log("block mixed: complex64 A P %.1f us (%.1f TFLOP/s); 64-column solve %.2f ms" % (
        t32 * 1e6, flops / t32 / 1e12, tmix * 1e3))
    del A32
    return {"rhs": k, "solves_per_s": k / tb, "ms_per_block_solve": tb * 1e3,
            "mixed": {"solves_per_s": k / tmix, "ms_per_block_solve": tmix * 1e3,
                      "speedup_vs_fp64_block": tb / tmix,
                      "max_outer": max(r.outer for r in rm),
                      "max_inner_iters": max(r.inner_iters for r in rm),
                      "all_converged": all(r.info == 0 for r in rm),
                      "max_relres_true": float(relm.max()),
                      "max_fwd_err": float(fem.max()),
                      "max_fwd_err_fp64_block": float(fe64.max()),
                      "gemm_c64": {"kernel": "k_cgemm (A32 P, FP32 MFMA)",
                                   "launch_us": t32 * 1e6, "achieved": flops / t32 / 1e12,
                                   "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                                   "frac": flops / t32 / 1e12 / FP32_PEAK_TFLOPS}},
            "max_iters": max(r.iters for r in res),
            "all_converged": all(r.info == 0 for r in res),
            "max_relres_true": float(rel.max()),
            "gemm": {"kernel": "k_zgemm (A P, FP64 MFMA)", "launch_us": tg * 1e6,
                     "flops_per_launch": flops, "achieved": flops / tg / 1e12,
                     "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": flops / tg / 1e12 / FP64_PEAK_TFLOPS,
                     # each complex product on the matrix cores takes three real
                     # products (the 3M form): 6 n^2 k flops executed per launch
                     "matrix_core_flops_per_launch": 0.75 * flops,
                     "matrix_core_achieved": 0.75 * flops / tg / 1e12,
                     "matrix_core_frac": 0.75 * flops / tg / 1e12 / FP64_PEAK_TFLOPS}}


CONFIG0_N = 256
CONFIG0_BATCH = 1024


def config0_leg(steps):
    """The dense n = 256 family (A = 4 I + G / sqrt(n), x_true iid CN(0,1),
    y = A x_true; seeds 0..1023): single-solve latency of one system (seed 0)
    through ccg_bicgstab_ex / ccg_cgnr_ex (one kernel per step of the method)
    and through ccg_solve_small_batched with a batch of one (one workgroup,
    one launch); then the 1024 seeds solved concurrently by one
    ccg_solve_small_batched launch per method, timed with HIP events, its
    algorithmic bytes (16 n^2 per product of every system) against the HBM
    peak."""
    import torch

    from paper_1208_4869_amd import ccg, inputs
    n, B = CONFIG0_N, CONFIG0_BATCH
    t = time.time()
    sys_ = [inputs.dense_system(n, s) for s in range(B)]
    A = torch.from_numpy(np.stack([a for a, _, _ in sys_])).cuda()
    Y = torch.from_numpy(np.stack([y for _, _, y in sys_])).cuda()
    Xt = np.stack([xt for _, xt, _ in sys_])
    torch.cuda.synchronize()
    log("built %d n=%d systems (%.2f GB of A) in %.1fs" % (B, n, A.numel() * 16 / 1e9,
                                                          time.time() - t))
    out = {"workload": "dense n=256 (A = 4I + G/sqrt(n)), seeds 0..%d, tol 1e-10, "
                       "x0 = 0" % (B - 1), "n": n}
    A0, y0 = A[0].contiguous(), Y[0].contiguous()
    # one system through the multi-kernel entry points
    for name, fn, wsid in (("bicgstab", ccg.ccg_bicgstab_ex, ccg.WS_BICGSTAB),
                           ("cgnr", ccg.ccg_cgnr_ex, ccg.WS_CGNR)):
        w = ccg.workspace(wsid, n)
        x = torch.empty_like(y0)
        tot, lat, res = time_solves(fn, A0, y0, x, w, steps, 3)
        out[name + "_single"] = {"entry": "ccg_%s_ex" % name, "solves_per_s": steps / tot,
                                 "p50_ms": float(np.percentile(lat, 50) * 1e3),
                                 "p99_ms": float(np.percentile(lat, 99) * 1e3),
                                 "iters": res.iters, "matvecs": res.matvecs, "info": res.info}
    method_ids = (("bicgstab", ccg.WS_BICGSTAB), ("cgnr", ccg.WS_CGNR))
    # one system, one workgroup: launch + wait per solve
    res_d = torch.empty(B * 32, dtype=torch.uint8, device="cuda")
    for name, wsid in method_ids:
        X1 = torch.empty_like(Y[:1])
        for _ in range(3):
            ccg.ccg_solve_small_batched(wsid, A[:1], Y[:1], X1, TOL, MAXIT, ccg.X0_ZERO, res_d)
        torch.cuda.synchronize()
        lat = []
        for _ in range(steps):
            ts = time.perf_counter()
            ccg.ccg_solve_small_batched(wsid, A[:1], Y[:1], X1, TOL, MAXIT, ccg.X0_ZERO, res_d)
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - ts)
        lat = np.array(lat)
        r1 = ccg.small_results(res_d, 1)[0]
        out[name + "_single_small"] = {"entry": "ccg_solve_small_batched, batch 1",
                                       "solves_per_s": 1.0 / lat.mean(),
                                       "p50_ms": float(np.percentile(lat, 50) * 1e3),
                                       "p99_ms": float(np.percentile(lat, 99) * 1e3),
                                       "iters": r1.iters, "matvecs": r1.matvecs,
                                       "info": r1.info}
    # the whole batch in one launch
    for name, wsid in method_ids:
        X = torch.empty_like(Y)
        ccg.ccg_solve_small_batched(wsid, A, Y, X, TOL, MAXIT, ccg.X0_ZERO, res_d)
        torch.cuda.synchronize()
        reps = max(steps // 10, 3)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(reps)]
        wall = []
        for a, b in ev:
            ts = time.perf_counter()
            a.record()
            ccg.ccg_solve_small_batched(wsid, A, Y, X, TOL, MAXIT, ccg.X0_ZERO, res_d)
            b.record()
            b.synchronize()
            wall.append(time.perf_counter() - ts)
        dur = np.array([a.elapsed_time(b) / 1e3 for a, b in ev])
        rs = ccg.small_results(res_d, B)
        mv = np.array([r.matvecs for r in rs])
        abytes = float(16.0 * n * n * mv.sum())
        tk = float(np.median(dur))
        Xh = X.cpu().numpy()
        sample = (0, 1, B // 2, B - 1)
        rel = [float(np.linalg.norm(sys_[b][2] - sys_[b][0] @ Xh[b]) / np.linalg.norm(sys_[b][2]))
               for b in sample]
        fe = [float(np.linalg.norm(Xh[b] - Xt[b]) / np.linalg.norm(Xt[b])) for b in sample]
        out[name + "_batch"] = {
            "entry": "ccg_solve_small_batched", "batch": B,
            "kernel": "k_small_%s (one workgroup per system, one launch)" % name,
            "launch_ms": tk * 1e3, "wall_ms_p50": float(np.percentile(wall, 50) * 1e3),
            "solves_per_s": B / tk, "solves_per_s_wall": B / float(np.median(wall)),
            "products": int(mv.sum()), "algorithmic_bytes": abytes,
            "achieved_gbs": abytes / tk / 1e9, "hbm_frac": abytes / tk / 1e9 / HBM_PEAK_GBS,
            "all_converged": all(r.info == 0 and r.relres_true <= TOL for r in rs),
            "iters_range": [int(min(r.iters for r in rs)), int(max(r.iters for r in rs))],
            "host_relres_sampled_max": max(rel), "fwd_err_sampled_max": max(fe)}
        log("config 0 %s: batch of %d in %.2f ms (%.0f solves/s, %.0f GB/s of A)" % (
            name, B, tk * 1e3, B / tk, abytes / tk / 1e9))
    del A, Y
    torch.cuda.empty_cache()
    return out


SERVE_SIZES = (512, 1024, 2048, 4096)
SERVE_SEED = 2024
SERVE_POOL_BYTES = 16 << 30
SERVE_BUDGET_BYTES = 6 << 30  # a pool that binds: the 128 slots would need ~11 GB
SERVE_TOL_INNER = 1e-5


def serve_inputs(nreq):
    """Requests of the dense family (A = 4 I + G / sqrt(n), G iid CN(0,1);
    X_true iid CN(0,1); Y = A X_true), n uniform over SERVE_SIZES and k
    uniform over 1..8, drawn from SERVE_SEED; each request's matrices come
    from its own seed on the device."""
    import torch
    rng = np.random.default_rng(SERVE_SEED)
    ns = rng.choice(SERVE_SIZES, nreq)
    ks = rng.integers(1, 9, nreq)
    g = torch.Generator(device="cuda")
    reqs = []
    for i in range(nreq):
        n, k = int(ns[i]), int(ks[i])
        g.manual_seed(SERVE_SEED * 1000 + i)
        A = torch.randn((n, n), dtype=torch.complex128, device="cuda", generator=g)
        A /= float(np.sqrt(n))
        A.diagonal().add_(4.0)
        Xt = torch.randn((n, k), dtype=torch.complex128, device="cuda", generator=g)
        Y = A @ Xt
        X = torch.empty((n, k), dtype=torch.complex128, device="cuda")
        reqs.append((A, Y, X))
    torch.cuda.synchronize()
    return reqs


def run_server(reqs, arrivals, mixed=False, tol_inner=SERVE_TOL_INNER,
               pool_bytes=SERVE_POOL_BYTES):
    """Feed reqs to a server at the given arrival times (seconds from the
    start); mixed: FP64 refinement around complex64 inner solves.  Returns
    (makespan, latencies, results, stats)."""
    from paper_1208_4869_amd import ccg
    N = len(reqs)
    lat = np.zeros(N)
    results = [None] * N
    index = {}
    done = 0
    i = 0
    with ccg.Server(pool_bytes, max_active=128) as srv:
        t0 = time.perf_counter()
        while done < N:
            now = time.perf_counter() - t0
            while i < N and arrivals[i] <= now:
                A, Y, X = reqs[i]
                if mixed:
                    index[srv.submit(A, Y, X, TOL, 10, mixed=True, tol_inner=tol_inner)] = i
                else:
                    index[srv.submit(A, Y, X, TOL, MAXIT)] = i
                i += 1
            act, q = srv.step()
            while True:
                t = srv.next_done()
                if not t:
                    break
                j = index.pop(t)
                results[j] = srv.poll(t)[1]
                lat[j] = time.perf_counter() - t0 - arrivals[j]
                done += 1
            if act == 0 and q == 0 and i < N:
                wait = arrivals[i] - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(wait)
        makespan = time.perf_counter() - t0
        stats = srv.stats()
    return makespan, lat, results, stats


def serve_leg(nreq, rate):
    """Continuous batching: nreq requests, first all at once (capacity), then
    with Poisson arrivals at `rate` requests/s (or 70% of the capacity when
    rate is None); against the same requests solved one at a time with
    ccg_bicgstab_block_ex."""
    import torch

    from paper_1208_4869_amd import ccg
    t = time.time()
    reqs = serve_inputs(nreq)
    rhs = sum(Y.shape[1] for _, Y, _ in reqs)
    log("built %d serving requests (%d right-hand sides, %.1f GB of A) in %.1fs" % (
        nreq, rhs, sum(A.numel() * 16 for A, _, _ in reqs) / 1e9, time.time() - t))
    # one at a time (warm the kernels first)
    ref = []
    A, Y, X = reqs[0]
    ccg.ccg_bicgstab_block_ex(A, Y, X, TOL, MAXIT, flags=1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for A, Y, X in reqs:
        ref.append(ccg.ccg_bicgstab_block_ex(A, Y, X, TOL, MAXIT, flags=1))
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    X_ref = [X.clone() for _, _, X in reqs]
    # capacity: everything arrives at t = 0
    run_server(reqs[:8], np.zeros(8))  # warm-up
    mk_c, lat_c, res_c, st_c = run_server(reqs, np.zeros(nreq))
    cap = nreq / mk_c
    if rate is None:
        rate = 0.7 * cap
    gaps = np.random.default_rng(SERVE_SEED + 1).exponential(1.0 / rate, nreq)
    arrivals = np.cumsum(gaps) - gaps[0]
    mk_p, lat_p, res_p, st_p = run_server(reqs, arrivals)
    # every request as alone: bitwise equal x and records
    same = all(torch.equal(X, Xr) for (_, _, X), Xr in zip(reqs, X_ref))
    same = same and all(
        [(a.info, a.iters) for a in r] == [(b.info, b.iters) for b in rr]
        for r, rr in zip(res_p, ref))
    ok = all(a.info == 0 and a.relres_true <= TOL for r in res_p for a in r)
    # algorithmic HBM bytes: one pass over A per product the slowest column
    # of a request needs (the other columns share it)
    a_bytes = sum(16.0 * A.shape[0] ** 2 * max(c.matvecs for c in r)
                  for (A, _, _), r in zip(reqs, res_c))
    log("serving: capacity %.0f req/s, Poisson %.0f req/s: p50 %.2f ms p99 %.2f ms; "
        "one at a time %.0f req/s" % (cap, rate, np.percentile(lat_p, 50) * 1e3,
                                      np.percentile(lat_p, 99) * 1e3, nreq / t_seq))
    # latency against offered load: Poisson arrivals at 50%, 90% and 120% of
    # the measured capacity (above 100% the queue grows over the run)
    sweep = []
    for i, load in enumerate((0.5, 0.9, 1.2)):
        g = np.random.default_rng(SERVE_SEED + 10 + i).exponential(1.0 / (load * cap), nreq)
        mk_s, lat_s, res_s, _ = run_server(reqs, np.cumsum(g) - g[0])
        ok = ok and all(a.info == 0 and a.relres_true <= TOL for r in res_s for a in r)
        sweep.append({"load": load, "rate_per_s": load * cap, "requests_per_s": nreq / mk_s,
                      "p50_ms": float(np.percentile(lat_s, 50) * 1e3),
                      "p99_ms": float(np.percentile(lat_s, 99) * 1e3)})
        log("serving at %.0f%% of capacity: p50 %.2f ms p99 %.2f ms" % (
            100 * load, sweep[-1]["p50_ms"], sweep[-1]["p99_ms"]))
    # a pool that binds: 6 GiB, so admission waits for pool bytes, not for
    # slots; capacity and Poisson arrivals at 70% of that capacity
    mk_b, lat_b, res_b, st_b = run_server(reqs, np.zeros(nreq), pool_bytes=SERVE_BUDGET_BYTES)
    cap_b = nreq / mk_b
    gb = np.random.default_rng(SERVE_SEED + 20).exponential(1.0 / (0.7 * cap_b), nreq)
    mk_bp, lat_bp, res_bp, st_bp = run_server(reqs, np.cumsum(gb) - gb[0],
                                              pool_bytes=SERVE_BUDGET_BYTES)
    ok = ok and all(a.info == 0 and a.relres_true <= TOL for r in res_bp for a in r)
    same_b = all(torch.equal(X, Xr) for (_, _, X), Xr in zip(reqs, X_ref))
    budget = {"pool_bytes": SERVE_BUDGET_BYTES,
              "capacity_requests_per_s": cap_b,
              "capacity_admission_waits": st_b["admission_waits"],
              "capacity_peak_active": st_b["peak_active"],
              "capacity_pool_peak_bytes": st_b["pool_peak"],
              "poisson_rate_per_s": 0.7 * cap_b,
              "poisson_requests_per_s": nreq / mk_bp,
              "poisson_p50_ms": float(np.percentile(lat_bp, 50) * 1e3),
              "poisson_p99_ms": float(np.percentile(lat_bp, 99) * 1e3),
              "poisson_admission_waits": st_bp["admission_waits"],
              "poisson_peak_active": st_bp["peak_active"],
              "bitwise_equal_to_alone": bool(same_b)}
    log("serving in a %d GiB pool: capacity %.0f req/s (%d admission waits); Poisson at "
        "70%%: p50 %.2f ms p99 %.2f ms" % (SERVE_BUDGET_BYTES >> 30, cap_b,
                                           st_b["admission_waits"], budget["poisson_p50_ms"],
                                           budget["poisson_p99_ms"]))
    # nonsingularity of the realised matrices: sigma_min of the first request
    # of every size (Gershgorin fails for this family)
    certs = []
    for size in SERVE_SIZES:
        j = next(k for k, (A, _, _) in enumerate(reqs) if A.shape[0] == size)
        sv = torch.linalg.svdvals(reqs[j][0])
        certs.append({"request": j, "n": size, "sigma_min": float(sv[-1]),
                      "sigma_max": float(sv[0])})
    # the mixed-precision variant on the same requests and arrivals
    X64 = [X.clone() for _, _, X in reqs]
    run_server(reqs[:8], np.zeros(8), mixed=True)  # warm-up
    mk_mc, lat_mc, res_mc, st_mc = run_server(reqs, np.zeros(nreq), mixed=True)
    mk_mp, lat_mp, res_mp, st_mp = run_server(reqs, arrivals, mixed=True)
    ok_m = all(a.info == 0 and a.relres_true <= TOL for r in res_mp for a in r)
    dmax = max(float(torch.linalg.norm(X - Xr) / torch.linalg.norm(Xr))
               for (_, _, X), Xr in zip(reqs, X64))
    log("serving, mixed: capacity %.0f req/s; Poisson p50 %.2f ms p99 %.2f ms" % (
        nreq / mk_mc, np.percentile(lat_mp, 50) * 1e3, np.percentile(lat_mp, 99) * 1e3))
    return {"workload": "%d requests, dense n in %s (A = 4I + G/sqrt(n)), k in 1..8, "
                        "tol 1e-10, FP64" % (nreq, list(SERVE_SIZES)),
            "rhs_total": rhs,
            "capacity": {"requests_per_s": cap, "rhs_solves_per_s": rhs / mk_c,
                         "a_bytes": a_bytes, "a_gbs": a_bytes / mk_c / 1e9,
                         "hbm_frac": a_bytes / mk_c / 1e9 / HBM_PEAK_GBS,
                         "makespan_s": mk_c, "ticks": st_c["ticks"],
                         "peak_active": st_c["peak_active"],
                         "admission_waits": st_c["admission_waits"],
                         "p50_ms": float(np.percentile(lat_c, 50) * 1e3),
                         "p99_ms": float(np.percentile(lat_c, 99) * 1e3)},
            "poisson": {"rate_per_s": rate, "requests_per_s": nreq / mk_p,
                        "rhs_solves_per_s": rhs / mk_p, "makespan_s": mk_p,
                        "p50_ms": float(np.percentile(lat_p, 50) * 1e3),
                        "p99_ms": float(np.percentile(lat_p, 99) * 1e3),
                        "ticks": st_p["ticks"], "peak_active": st_p["peak_active"]},
            "load_sweep": sweep,
            "one_at_a_time": {"requests_per_s": nreq / t_seq,
                              "rhs_solves_per_s": rhs / t_seq},
            "mixed": {"capacity_requests_per_s": nreq / mk_mc,
                      "capacity_rhs_solves_per_s": rhs / mk_mc,
                      "capacity_speedup_vs_fp64": mk_c / mk_mc,
                      "poisson_p50_ms": float(np.percentile(lat_mp, 50) * 1e3),
                      "poisson_p99_ms": float(np.percentile(lat_mp, 99) * 1e3),
                      "poisson_requests_per_s": nreq / mk_mp,
                      "all_converged": ok_m,
                      "max_rel_diff_vs_fp64_solution": dmax,
                      "ticks_capacity": st_mc["ticks"]},
            "pool_bytes": SERVE_POOL_BYTES,
            "budget_pool": budget,
            "sigma_min_certificates": certs,
            "all_converged": ok, "bitwise_equal_to_alone": bool(same)}


def t3_bytes(m, even=True):
    """Algorithmic HBM bytes of one structured product: x and y, the kernel
    transform (M^3 points; (M/2 + 1)^2 M for a kernel even in x and y, as
    the lattice kernel, whose rows of frequencies |kx|, |ky| <= M/2 are the
    only distinct ones), and the two intermediate grids, each written once
    and read once per direction (G1: M m^2, G2: M^2 m)."""
    M = 16
    while M < 2 * m - 1:
        M *= 2
    k = (M // 2 + 1) ** 2 * M if even else M ** 3
    return 16.0 * (2 * m ** 3 + k + 4 * M * m * m + 4 * M * M * m), M


def structured_leg(steps):
    """The lattice systems with the structured product (zero-padded 3-D FFT
    convolution, ccg_t3_*): product time per lattice edge, and BiCGSTAB /
    COCG / COCR solves of the 20^3, 26^3 and 64^3 lattices (x_true seeds 1,
    2, 3 as in the dense legs; y = A x_true by the structured product)."""
    import torch

    from paper_1208_4869_amd import ccg, inputs
    out = {"products": [], "solves": []}
    for m, kind in ((20, "lattice"), (26, "lattice"), (64, "lattice"), (100, "lattice"),
                    (100, "general")):
        if kind == "lattice":  # even in x and y: the folded kernel transform
            table = inputs.lattice_table(m)
        else:  # no symmetry: the full kernel transform
            table = inputs.cn01(np.random.default_rng(100 + m), (2 * m - 1) ** 3)
        op = ccg.T3Operator(m, table)
        x = torch.from_numpy(inputs.cn01(np.random.default_rng(m), m ** 3)).cuda()
        y = torch.empty_like(x)
        work = op.workspace(ccg.WS_T3_MATVEC)
        t = time_kernel(lambda: op.matvec(x, y, work), 20)
        b, M = t3_bytes(m, even=kind == "lattice")
        out["products"].append({"m": m, "n": m ** 3, "M": M, "table": kind, "us": t * 1e6,
                                "bytes": b, "gbs": b / t / 1e9, "frac": b / t / 1e9 / HBM_PEAK_GBS,
                                "dense_bytes": 16.0 * m ** 6})
        log("structured product m=%d (n=%d, M=%d, %s kernel): %.1f us, %.0f GB/s of %.3g bytes"
            % (m, m ** 3, M, kind, t * 1e6, b / t / 1e9, b))
        del op, work
    for m, seed in ((LATTICE_M, X_SEED), (26, 2), (64, 3)):
        op = ccg.T3Operator(m, inputs.lattice_table(m))
        n = m ** 3
        xt = torch.from_numpy(inputs.cn01(np.random.default_rng(seed), n)).cuda()
        yv = op.matvec(xt)
        for name in ("bicgstab", "cocg", "cocr"):
            meth = {"bicgstab": ccg.WS_BICGSTAB, "cocg": ccg.WS_COCG,
                    "cocr": ccg.WS_COCR}[name]
            work = op.workspace(meth)
            xs = torch.empty_like(xt)
            fn = getattr(op, name)
            fn(yv, xs, TOL, MAXIT, flags=1, work=work)
            torch.cuda.synchronize()
            lat = []
            for _ in range(steps):
                t0 = time.perf_counter()
                r = fn(yv, xs, TOL, MAXIT, flags=1, work=work)
                lat.append(time.perf_counter() - t0)
            fe = float(torch.linalg.norm(xs - xt) / torch.linalg.norm(xt))
            out["solves"].append({"m": m, "n": n, "method": name,
                                  "solves_per_s": 1.0 / np.mean(lat),
                                  "p50_ms": float(np.percentile(lat, 50) * 1e3),
                                  "iters": r.iters, "matvecs": r.matvecs, "info": r.info,
                                  "relres_true_device": r.relres_true, "fwd_err": fe})
            log("structured %s m=%d: %.0f solves/s (%d its)" % (name, m, 1.0 / np.mean(lat),
                                                               r.iters))
        del op
    torch.cuda.empty_cache()
    return out


def sym_leg(A, A_h, y, y_h, steps):
    """The lattice matrix is complex symmetric: the upper-triangle product
    (CCG_OP_S, half the bytes of A x) timed with HIP events, and BiCGSTAB,
    CGNR, COCG and COCR run with it (flag A_SYM_UPPER) on the same system."""
    import torch

    from paper_1208_4869_amd import ccg
    n = A.shape[0]
    xin = torch.from_numpy(inputs_cn01(n)).cuda()
    yout = torch.empty_like(xin)
    ws = ccg.workspace(ccg.WS_MATVEC_S, n)
    ts = time_kernel(lambda: ccg.ccg_matvec_ex(ccg.OP_S, A, xin, yout, ws), 50)
    tri = 16.0 * n * (n + 1) / 2 + 32.0 * n
    log("upper-triangle product: %.1f us (%.0f GB/s of triangle bytes)"
        % (ts * 1e6, tri / ts / 1e9))
    trec = measured_traffic("sym")
    out = {"product": {"kernel": "k_symv (tiles) + gather", "launch_us": ts * 1e6,
                       "bytes_per_launch": tri, "achieved_gbs": tri / ts / 1e9,
                       "frac": tri / ts / 1e9 / HBM_PEAK_GBS,
                       "partials_bytes": float(ccg.ccg_workspace_bytes(ccg.WS_MATVEC_S, n)),
                       "traffic": trec["k_symv_traffic_bytes"] if trec else None}}
    for name, fn, wsid in (("bicgstab", ccg.ccg_bicgstab_ex, ccg.WS_BICGSTAB),
                           ("cgnr", ccg.ccg_cgnr_ex, ccg.WS_CGNR),
                           ("cocg", ccg.ccg_cocg_ex, ccg.WS_COCG),
                           ("cocr", ccg.ccg_cocr_ex, ccg.WS_COCR)):
        wk = ccg.workspace(wsid | ccg.WS_SYM, n)
        xs = torch.empty(n, dtype=torch.complex128, device="cuda")
        log("timing %d %s solves with the upper-triangle product" % (steps, name.upper()))
        stot, slat, sres = time_solves(fn, A, y, xs, wk, steps, 1, flags=ccg.A_SYM_UPPER)
        xsg = xs.cpu().numpy()
        out[name] = {"solves_per_s": steps / stot,
                     "p50_ms": float(np.percentile(slat, 50) * 1e3),
                     "iters": sres.iters, "matvecs": sres.matvecs, "info": sres.info,
                     "relres_true": float(np.linalg.norm(y_h - A_h @ xsg)
                                          / np.linalg.norm(y_h))}
    return out


def inputs_cn01(n):
    from paper_1208_4869_amd import inputs
    return inputs.cn01(np.random.default_rng(X_SEED + 1), n)


def profile_kernels(A, y):
    """A short, fixed mix for rocprofv3: a device copy of known size (the
    reference for scaling the HBM byte counters), the read stream, A x, A^H x,
    the upper-triangle and complex64 products, the 64-column products on
    FP64 and FP32 matrix cores, one BiCGSTAB and one CGNR solve, and one
    batched launch of 1024 n = 256 BiCGSTAB solves."""
    import torch

    from paper_1208_4869_amd import ccg, inputs
    n = A.shape[0]
    src = torch.empty(A.numel() * 2, dtype=torch.float64, device="cuda")
    src.fill_(1.0)
    dst = torch.empty_like(src)
    x = torch.ones(n, dtype=torch.complex128, device="cuda")
    A32 = ccg.ccg_round_c64(A)
    x32 = x.to(torch.complex64)
    P = torch.ones((n, BLOCK_RHS), dtype=torch.complex128, device="cuda")
    Z = torch.empty_like(P)
    wmm = torch.empty(ccg.ccg_workspace_bytes(ccg.WS_MATMAT, n, BLOCK_RHS),
                      dtype=torch.uint8, device="cuda")
    wmm32 = torch.empty(ccg.ccg_workspace_bytes(ccg.WS_MATMAT_C64, n, BLOCK_RHS),
                        dtype=torch.uint8, device="cuda")
    rs_out = ccg.ccg_read_stream(src)
    for _ in range(5):
        dst.copy_(src)
        ccg.ccg_read_stream(src, rs_out)
        ccg.ccg_matvec(ccg.OP_N, A, x)
        ccg.ccg_matvec(ccg.OP_C, A, x)
        ccg.ccg_matvec(ccg.OP_S, A, x)
        ccg.ccg_matvec_c64(A32, x32)
        ccg.ccg_matmat(A, P, Z, work=wmm)
        ccg.ccg_matmat_c64(A32, P, Z, work=wmm32)
    ccg.ccg_bicgstab_ex(A, y, torch.empty_like(x), TOL, MAXIT, flags=1)
    ccg.ccg_cgnr_ex(A, y, torch.empty_like(x), TOL, MAXIT, flags=1)
    del src, dst, A32
    sys_ = [inputs.dense_system(CONFIG0_N, s) for s in range(CONFIG0_BATCH)]
    Ab = torch.from_numpy(np.stack([a for a, _, _ in sys_])).cuda()
    Yb = torch.from_numpy(np.stack([yy for _, _, yy in sys_])).cuda()
    Xb = torch.empty_like(Yb)
    ccg.ccg_solve_small_batched(ccg.WS_BICGSTAB, Ab, Yb, Xb, TOL, MAXIT, ccg.X0_ZERO)
    del Ab, Yb, Xb
    # structured products at m = 100 (lattice kernel: folded transform; a
    # general kernel: the full one) and m = 20 (three-launch path)
    for m, table in ((100, inputs.lattice_table(100)),
                     (100, inputs.cn01(np.random.default_rng(200), 199 ** 3)),
                     (20, inputs.lattice_table(20))):
        op = ccg.T3Operator(m, table)
        xs = torch.from_numpy(inputs.cn01(np.random.default_rng(m), m ** 3)).cuda()
        ys = torch.empty_like(xs)
        wk = op.workspace(ccg.WS_T3_MATVEC)
        for _ in range(5):
            op.matvec(xs, ys, wk)
        del op, wk
    torch.cuda.synchronize()
    log("profile mix done: copy %d bytes x5, read stream x5, matvec N/C/S/c64 x5, A P "
        "FP64 and complex64 (k=%d) x5, 1 BiCGSTAB, 1 CGNR, 1 batch of %d n=%d BiCGSTAB, "
        "structured products x5 (m = 100 lattice and general kernels, m = 20)"
        % (A.numel() * 16, BLOCK_RHS, CONFIG0_BATCH, CONFIG0_N))


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only (--gpus 1, one MI355X); a "
              "system larger than one GPU would be row-sharded across GPUs, "
              "which is not measured here.", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_1208_4869_amd import ccg
    torch.cuda.set_device(0)
    ccg.load()

    A_h, x_true, y_h = make_inputs()
    n = A_h.shape[0]
    A = torch.from_numpy(A_h).cuda()
    y = torch.from_numpy(y_h).cuda()
    torch.cuda.synchronize()

    if args.profile_kernels:
        profile_kernels(A, y)
        return

    # --- headline: BiCGSTAB solves/s.  The v = A p products inside the timed
    # solves (k_gemv_n_role, role v: the dominant kernel, all of its launches
    # full products) are sampled live with HIP events: every 7th of them
    # (six per solve, so the sample rotates through the iterations), one
    # event pair per solve on average.
    x = torch.empty(n, dtype=torch.complex128, device="cuda")
    work = ccg.workspace(ccg.WS_BICGSTAB, n)
    elog = ccg.EventLog(args.steps + 8, stride=PRODUCT_SAMPLE_STRIDE, roles=ccg.PROD_V)
    log("timing %d BiCGSTAB solves (+%d warm-up)" % (args.steps, args.warmup))
    total, lat, res = time_solves(ccg.ccg_bicgstab_ex, A, y, x, work, args.steps,
                                  args.warmup, event_log=elog)
    prod_us = np.array(elog.durations()) * 1e6
    xg = x.cpu().numpy()
    relres = float(np.linalg.norm(y_h - A_h @ xg) / np.linalg.norm(y_h))
    fwd = float(np.linalg.norm(xg - x_true) / np.linalg.norm(x_true))
    if res.info != 0 or not relres <= 1.01 * TOL:
        raise SystemExit("BiCGSTAB did not reach the tolerance: info %d relres %.3e"
                         % (res.info, relres))
    bytes_mv = 16.0 * n * n + 32.0 * n
    t_in = float(np.mean(prod_us)) * 1e-6
    gbs_in = bytes_mv / t_in / 1e9
    log("A x inside the solves: %d samples, mean %.1f us, median %.1f us (%.0f GB/s)"
        % (len(prod_us), prod_us.mean(), np.median(prod_us), gbs_in))
    read_gbs = read_stream_peak()
    trec = measured_traffic()
    trole = measured_traffic("role")
    roofline = {"bound": "hbm",
                "kernel": "k_gemv_n_role, role v (v = A p and the confirming residual) "
                          "inside the timed BiCGSTAB solves",
                "achieved": gbs_in, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": gbs_in / HBM_PEAK_GBS,
                "traffic": trole["k_gemv_n_role_traffic_bytes"] if trole else None,
                "launch_us": t_in * 1e6, "launch_us_median": float(np.median(prod_us)),
                "samples": int(len(prod_us)),
                "sampling": "HIP events around every %dth role-v product launch of the timed "
                            "solves, on their stream" % PRODUCT_SAMPLE_STRIDE,
                "bytes_per_launch": bytes_mv,
                "measured_read_stream_gbs": read_gbs,
                "frac_of_measured_read_stream": gbs_in / read_gbs}
    if args.headline_only:
        out = headline_record(args, total, lat, res, n, relres, fwd)
        out["roofline"] = roofline
        print(json.dumps(out), flush=True)
        return

    # --- CGNR on the same system
    wc = ccg.workspace(ccg.WS_CGNR, n)
    xc = torch.empty_like(x)
    csteps = max(args.steps // 2, 1)
    log("timing %d CGNR solves" % csteps)
    ctot, clat, cres = time_solves(ccg.ccg_cgnr_ex, A, y, xc, wc, csteps, 1)
    xcg = xc.cpu().numpy()
    crel = float(np.linalg.norm(y_h - A_h @ xcg) / np.linalg.norm(y_h))

    # --- COCG / COCR: the lattice matrix is complex symmetric (section 3.4)
    cs = {}
    for name, fn, wsid in (("cocg", ccg.ccg_cocg_ex, ccg.WS_COCG),
                           ("cocr", ccg.ccg_cocr_ex, ccg.WS_COCR)):
        wk = ccg.workspace(wsid, n)
        xs = torch.empty_like(x)
        log("timing %d %s solves" % (csteps, name.upper()))
        stot, slat, sres = time_solves(fn, A, y, xs, wk, csteps, 1)
        xsg = xs.cpu().numpy()
        cs[name] = {"solves_per_s": csteps / stot,
                    "p50_ms": float(np.percentile(slat, 50) * 1e3),
                    "iters": sres.iters, "matvecs": sres.matvecs, "info": sres.info,
                    "relres_true": float(np.linalg.norm(y_h - A_h @ xsg)
                                         / np.linalg.norm(y_h))}

    # --- the plain A x (ccg_matvec: the same inner loop and launch shape
    # without the solver's prologue and epilogue) and A^H x, timed with HIP
    # events over back-to-back launches: secondary figures
    xin = torch.from_numpy(x_true).cuda()
    yout = torch.empty_like(xin)
    wmv = torch.empty(ccg.ccg_workspace_bytes(ccg.WS_MATVEC_C, n), dtype=torch.uint8,
                      device="cuda")
    reps = 50
    tn = time_kernel(lambda: ccg.ccg_matvec(ccg.OP_N, A, xin, yout), reps)
    tc = time_kernel(lambda: ccg.ccg_matvec_ex(ccg.OP_C, A, xin, yout, wmv), reps)
    gbs_n = bytes_mv / tn / 1e9
    gbs_c = bytes_mv / tc / 1e9
    log("plain A x: %.1f us (%.0f GB/s); A^H x: %.1f us (%.0f GB/s)"
        % (tn * 1e6, gbs_n, tc * 1e6, gbs_c))
    roofline["plain_kernel"] = {
        "kernel": "k_gemv_n_plain (ccg_matvec)", "launch_us": tn * 1e6,
        "achieved": gbs_n, "frac": gbs_n / HBM_PEAK_GBS,
        "frac_of_measured_read_stream": gbs_n / read_gbs,
        "traffic": trec.get("k_gemv_n_traffic_bytes") if trec else None,
        "timing": "HIP events over %d back-to-back launches" % reps}

    out = headline_record(args, total, lat, res, n, relres, fwd)
    out.update({
        "roofline": roofline,
        "matvec_h": {"kernel": "k_gemv_c_band + gather (A^H x)",
                     "achieved_gbs": gbs_c, "frac": gbs_c / HBM_PEAK_GBS,
                     "frac_of_measured_read_stream": gbs_c / read_gbs,
                     "launch_us": tc * 1e6},
        "cgnr": {"solves_per_s": csteps / ctot,
                 "p50_ms": float(np.percentile(clat, 50) * 1e3),
                 "iters": cres.iters, "matvecs": cres.matvecs, "info": cres.info,
                 "relres_true": crel},
        "cocg": cs["cocg"],
        "cocr": cs["cocr"],
    })
    if not args.no_config0:
        out["config0"] = config0_leg(max(args.steps * 3, 30))
    if not args.no_sym:
        out["symmetric"] = sym_leg(A, A_h, y, y_h, csteps)
    if not args.no_mixed:
        out["mixed"] = mixed_leg(max(args.steps // 3, 3))
    if not args.no_block:
        out["block"] = block_leg(A, A_h, max(args.steps // 3, 2))
    if not args.no_structured:
        out["structured"] = structured_leg(max(args.steps // 3, 3))
    if not args.no_serve:
        out["serve"] = serve_leg(args.serve_requests, args.serve_rate)
    if not args.no_cpu_baseline:
        log("timing the CPU oracle (bounded sample, ~%.0f s)" % args.cpu_seconds)
        out["cpu_baseline"], out["cpu_baseline_all_cores"] = cpu_baseline(
            A_h, y_h, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
