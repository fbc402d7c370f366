// ccg_small.hip -- many small dense systems at once: BiCGSTAB and CGNR on a
// batch of independent complex128 systems A_b x_b = y_b (n <= 1024), one
// workgroup per system and the whole solve of every system in one launch.
//
// The methods, stop rule, confirmation, restart and info codes are those of
// ccg_bicgstab / ccg_cgnr (section 2.1's bicgstab and cgnr; Usage:
// epsilon_err, maxit): the workgroup walks the same sequence of steps the
// multi-kernel solvers launch -- BiCGSTAB: v = A p | s = r - alpha v |
// t = A s | x, r, next p; CGNR: w = A p | x, r | z = A^H r | p -- and after
// each step's fused reductions thread 0 applies the same scalar step
// (apply_step: alpha, omega, beta, gamma, the stop, budget and breakdown
// tests, the phase change) to the system's record in LDS.  Only the order of
// the floating-point sums differs (a block reduction instead of per-block
// partials), so results agree with the multi-kernel solvers to rounding.
//
// Why one workgroup per system: at n = 256 A is 1 MiB and a product is a
// few microseconds of work, less than a kernel launch costs, so the
// multi-kernel solvers are launch-bound there.  Here the Krylov vectors live
// in LDS (6 n complex128 for BiCGSTAB, 4 n for CGNR), x and y stay in global
// memory (L2-resident), and A streams from memory once per product; a batch
// of independent systems fills the chip with one launch and is bound by the
// HBM stream of all the systems' matrices.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "../../include/ccg.h"
#include "ccg_device.h"
#include "ccg_krylov.h"

namespace ccg {

constexpr int kSmallMaxN = CCG_SMALL_MAX_N;
constexpr int kSmallThreads = 256;
constexpr int kSmallWaves = kSmallThreads / kWave;

struct SmallArgs {
    const d2* A;
    int64_t lda, strideA;
    const d2* Y;
    int64_t strideY;
    d2* X;
    int64_t strideX;
    ccg_result* res;
    int n, maxit, x0zero;
    double tol2;
};

// Block totals of K per-thread values (64-lane butterfly, then the
// wavefronts in index order: fixed order, every run the same bits); every
// thread receives the totals.  lds holds K * kSmallWaves entries.
template <int K>
__device__ __forceinline__ void small_sums(d2 (&v)[K], d2* lds)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    d2 s[K];
#pragma unroll
    for (int k = 0; k < K; ++k) s[k] = wave_sum(v[k]);
    __syncthreads();  // lds may still be read after the previous call
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) lds[k * kSmallWaves + wave] = s[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
        d2 t = lds[k * kSmallWaves];
#pragma unroll
        for (int w = 1; w < kSmallWaves; ++w) t += lds[k * kSmallWaves + w];
        v[k] = t;
    }
}

// The scalar step of reduction `kind` on the totals, by thread 0, then a
// barrier so that every thread reads the new record.  Every thread has
// passed the barriers of small_sums (and so finished reading the record)
// before thread 0 writes it.
__device__ __forceinline__ void small_step(SolverState& L, int kind, d2 t0, d2 t1,
                                           d2 t2 = d2{0.0, 0.0})
{
    if (threadIdx.x == 0) {
        L.pending = kind;
        apply_step(L, t0, t1, nullptr, t2);
    }
    __syncthreads();
}

// y = A in for one system: lane l multiplies the columns l + 64 c (held in
// registers), RG rows at a time per wavefront (wavefront w takes the row
// groups w, w + 4, ...); the RG row sums cross the lanes in the transposing
// butterfly and fin(i, value) runs in the lane that holds row i's total.
// NB = 64-column chunks per row (n <= 64 NB).
template <int NB, class Fin>
__device__ __forceinline__ void small_gemv(const d2* __restrict__ A, int64_t lda, int n,
                                           const d2* in, Fin&& fin)
{
    // rows per group: 32 loads in flight per lane (n = 256, 1024 systems:
    // BiCGSTAB 3.08 against 3.31 ms with 8, 3.20 with 16; CGNR 7.32 against
    // 7.67 and 7.46), two wavefronts per SIMD
    constexpr int RG = NB >= 32 ? 1 : 32 / NB;
    constexpr int LPR = kWave / RG;             // lanes sharing a row total
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    d2 pr[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) {
        const int j = lane + kWave * c;
        pr[c] = j < n ? in[j] : d2{0.0, 0.0};
    }
    for (int r0 = wave * RG; r0 < n; r0 += kSmallWaves * RG) {
        d2 a[RG][NB];
#pragma unroll
        for (int k = 0; k < RG; ++k)
#pragma unroll
            for (int c = 0; c < NB; ++c) {
                const int row = r0 + k, j = lane + kWave * c;
                a[k][c] = (row < n && j < n) ? A[(int64_t)row * lda + j] : d2{0.0, 0.0};
            }
        d2 acc[RG];
#pragma unroll
        for (int k = 0; k < RG; ++k) {
            acc[k] = d2{0.0, 0.0};
#pragma unroll
            for (int c = 0; c < NB; ++c) acc[k] = cfma(a[k][c], pr[c], acc[k]);
        }
        wave_transpose_sum<RG>(acc, lane);
        const int row = r0 + lane / LPR;
        if (lane % LPR == 0 && row < n) fin(row, acc[0]);
    }
}

// z = A^H r for one system: lane l accumulates conj(A_ij) r_i for its
// columns j = l + 64 c over the rows of its wavefront (row groups w, w + 4,
// ... of U rows), and the four wavefronts' sums are added into z in
// wavefront order.
template <int NB>
__device__ __forceinline__ void small_gemv_h(const d2* __restrict__ A, int64_t lda, int n,
                                             const d2* r, d2* z)
{
    constexpr int U = NB >= 8 ? 1 : 8 / NB;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    d2 acc[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) acc[c] = d2{0.0, 0.0};
    for (int r0 = wave * U; r0 < n; r0 += kSmallWaves * U) {
        d2 a[U][NB], ri[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int row = r0 + k;
            ri[k] = row < n ? r[row] : d2{0.0, 0.0};
#pragma unroll
            for (int c = 0; c < NB; ++c) {
                const int j = lane + kWave * c;
                a[k][c] = (row < n && j < n) ? A[(int64_t)row * lda + j] : d2{0.0, 0.0};
            }
        }
#pragma unroll
        for (int k = 0; k < U; ++k)
#pragma unroll
            for (int c = 0; c < NB; ++c) acc[c] = cfma_conj(a[k][c], ri[k], acc[c]);
    }
    for (int w = 0; w < kSmallWaves; ++w) {
        if (wave == w) {
#pragma unroll
            for (int c = 0; c < NB; ++c) {
                const int j = lane + kWave * c;
                if (j < n) z[j] = w == 0 ? acc[c] : z[j] + acc[c];
            }
        }
        __syncthreads();
    }
}

__device__ __forceinline__ void small_result(const SolverState& L, ccg_result* res)
{
    ccg_result o;
    o.info = L.phase == PH_DONE ? L.info : 1;  // slot budget spent (defensive)
    o.iters = L.iters;
    o.matvecs = L.matvecs;
    o.confirms = L.confirms;
    o.relres_rec = L.relres_rec;
    o.relres_true = L.relres_true;
    *res = o;
}

// ||y||^2, then either the x0 = 0 set-up (x = 0, r = y, and for BiCGSTAB
// r^ = p = y) with its combined step, or the norm step followed by the
// set-up residual r = y - A x (x = 0 when y == 0).
template <int NB, bool BICG>
__device__ __forceinline__ void small_setup(const SmallArgs& a, SolverState& L, const d2* A,
                                            const d2* y, d2* x, d2* r, d2* rh, d2* p,
                                            d2* red)
{
    const int n = a.n, tid = threadIdx.x;
    const d2 z = d2{0.0, 0.0};
    if (a.x0zero) {
        d2 t[1] = {z};
        for (int i = tid; i < n; i += kSmallThreads) {
            const d2 yi = y[i];
            x[i] = z;
            r[i] = yi;
            if (BICG) {
                rh[i] = yi;
                p[i] = yi;
            }
            t[0].x += cabs2(yi);
        }
        small_sums<1>(t, red);
        small_step(L, BICG ? PK_NY_SETUP_B0 : PK_NY_SETUP_C0, t[0], z);
        return;
    }
    d2 t[1] = {z};
    for (int i = tid; i < n; i += kSmallThreads) t[0].x += cabs2(y[i]);
    small_sums<1>(t, red);
    small_step(L, PK_NORMY, t[0], z);
    const int ph = L.phase;
    if (ph == PH_ZERO) {
        for (int i = tid; i < n; i += kSmallThreads) x[i] = z;
        __syncthreads();
        small_step(L, PK_ZERO, z, z);
    } else if (ph == PH_RUN) {
        d2 u[1] = {z};
        small_gemv<NB>(A, a.lda, n, x, [&](int i, d2 val) {
            const d2 ri = y[i] - val;
            r[i] = ri;
            if (BICG) {
                rh[i] = ri;
                p[i] = ri;
            }
            u[0].x += cabs2(ri);
        });
        small_sums<1>(u, red);
        small_step(L, BICG ? PK_SETUP_B1 : PK_SETUP_C1, u[0], z);
    }
}

template <int NB>
__global__ __launch_bounds__(kSmallThreads) void k_small_bicgstab(SmallArgs a)
{
    extern __shared__ d2 vecs[];
    __shared__ SolverState L;
    __shared__ d2 red[3 * kSmallWaves];
    constexpr int np = NB * kWave;
    d2 *r = vecs, *rh = r + np, *p = rh + np, *v = p + np, *s = v + np, *t = s + np;
    const int64_t sys = blockIdx.x;
    const d2* A = a.A + sys * a.strideA;
    const d2* y = a.Y + sys * a.strideY;
    d2* x = a.X + sys * a.strideX;
    const int n = a.n, tid = threadIdx.x;
    const d2 z = d2{0.0, 0.0};
    if (tid == 0) init_state(L, a.maxit, a.tol2, 0);
    __syncthreads();
    small_setup<NB, true>(a, L, A, y, x, r, rh, p, red);

    const int64_t max_slots = 2 * (int64_t)a.maxit + 4;
    for (int64_t slot = 0; slot < max_slots && L.phase != PH_DONE; ++slot) {
        // v = A p (iterating, or a new direction), or the confirming
        // residual r = y - A x (with r^ = p = r for a restart)
        int ph = L.phase;
        if (ph == PH_RUN || ph == PH_RESTART) {
            d2 u[2] = {z, z};
            small_gemv<NB>(A, a.lda, n, p, [&](int i, d2 val) {
                v[i] = val;
                u[0] = cfma_conj(rh[i], val, u[0]);
                u[1].x += cabs2(val);
            });
            small_sums<2>(u, red);
            small_step(L, PK_V, u[0], u[1]);
        } else if (ph == PH_CONFIRM) {
            d2 u[1] = {z};
            small_gemv<NB>(A, a.lda, n, x, [&](int i, d2 val) {
                const d2 ri = y[i] - val;
                r[i] = ri;
                rh[i] = ri;
                p[i] = ri;
                u[0].x += cabs2(ri);
            });
            small_sums<1>(u, red);
            small_step(L, PK_CONFIRM_B, u[0], z);
        }
        // s = r - alpha v, ||s||^2, r^H s
        if (L.phase == PH_RUN) {
            const d2 nal = d2{-L.alpha.x, -L.alpha.y};
            d2 u[2] = {z, z};
            for (int i = tid; i < n; i += kSmallThreads) {
                const d2 si = cfma(nal, v[i], r[i]);
                s[i] = si;
                u[0].x += cabs2(si);
                u[1] = cfma_conj(rh[i], si, u[1]);
            }
            small_sums<2>(u, red);
            small_step(L, PK_S2, u[0], u[1]);
        }
        // t = A s, t^H s, ||t||^2, r^H t
        if (L.phase == PH_RUN) {
            d2 u[3] = {z, z, z};
            small_gemv<NB>(A, a.lda, n, s, [&](int i, d2 val) {
                t[i] = val;
                u[0] = cfma_conj(val, s[i], u[0]);
                u[1].x += cabs2(val);
                u[2] = cfma_conj(rh[i], val, u[2]);
            });
            small_sums<3>(u, red);
            small_step(L, PK_T3, u[0], u[1], u[2]);
        }
        // x += alpha p + omega s, r = s - omega t, next p; or, after a
        // half-step exit, x += alpha p
        ph = L.phase;
        if (ph == PH_RUN || ph == PH_HALF) {
            const d2 alpha = L.alpha, omega = L.omega, beta = L.beta;
            const d2 nom = d2{-omega.x, -omega.y};
            d2 u[1] = {z};
            for (int i = tid; i < n; i += kSmallThreads) {
                const d2 pi = p[i];
                d2 xi = cfma(alpha, pi, x[i]);
                if (ph == PH_RUN) {
                    const d2 si = s[i];
                    xi = cfma(omega, si, xi);
                    const d2 ri = cfma(nom, t[i], si);
                    r[i] = ri;
                    u[0].x += cabs2(ri);
                    p[i] = cfma(beta, cfma(nom, v[i], pi), ri);
                }
                x[i] = xi;
            }
            if (ph == PH_RUN) {
                small_sums<1>(u, red);
                small_step(L, PK_XRP, u[0], z);
            } else {
                __syncthreads();
                small_step(L, PK_HALF, z, z);
            }
        }
    }
    if (tid == 0) small_result(L, a.res + sys);
}

template <int NB>
__global__ __launch_bounds__(kSmallThreads) void k_small_cgnr(SmallArgs a)
{
    extern __shared__ d2 vecs[];
    __shared__ SolverState L;
    __shared__ d2 red[kSmallWaves];
    constexpr int np = NB * kWave;
    d2 *r = vecs, *zv = r + np, *p = zv + np, *w = p + np;
    const int64_t sys = blockIdx.x;
    const d2* A = a.A + sys * a.strideA;
    const d2* y = a.Y + sys * a.strideY;
    d2* x = a.X + sys * a.strideX;
    const int n = a.n, tid = threadIdx.x;
    const d2 z = d2{0.0, 0.0};
    if (tid == 0) init_state(L, a.maxit, a.tol2, 0);
    __syncthreads();
    small_setup<NB, false>(a, L, A, y, x, r, nullptr, nullptr, red);

    const int64_t max_slots = 2 * (int64_t)a.maxit + 4;
    for (int64_t slot = 0; slot < max_slots && L.phase != PH_DONE; ++slot) {
        // w = A p, ||w||^2; or the confirming residual r = y - A x
        int ph = L.phase;
        if (ph == PH_RUN) {
            d2 u[1] = {z};
            small_gemv<NB>(A, a.lda, n, p, [&](int i, d2 val) {
                w[i] = val;
                u[0].x += cabs2(val);
            });
            small_sums<1>(u, red);
            small_step(L, PK_W, u[0], z);
        } else if (ph == PH_CONFIRM) {
            d2 u[1] = {z};
            small_gemv<NB>(A, a.lda, n, x, [&](int i, d2 val) {
                const d2 ri = y[i] - val;
                r[i] = ri;
                u[0].x += cabs2(ri);
            });
            small_sums<1>(u, red);
            small_step(L, PK_CONFIRM_C, u[0], z);
        }
        // x += alpha p, r -= alpha w, ||r||^2
        if (L.phase == PH_RUN) {
            const double al = L.alpha.x;
            d2 u[1] = {z};
            for (int i = tid; i < n; i += kSmallThreads) {
                const d2 pi = p[i], wi = w[i];
                d2 xi = x[i], ri = r[i];
                xi.x = __builtin_fma(al, pi.x, xi.x);
                xi.y = __builtin_fma(al, pi.y, xi.y);
                ri.x = __builtin_fma(-al, wi.x, ri.x);
                ri.y = __builtin_fma(-al, wi.y, ri.y);
                x[i] = xi;
                r[i] = ri;
                u[0].x += cabs2(ri);
            }
            small_sums<1>(u, red);
            small_step(L, PK_XR2, u[0], z);
        }
        // z = A^H r, ||z||^2 (continuing, or the first direction after a
        // (re)start)
        ph = L.phase;
        if (ph == PH_RUN || ph == PH_RESTART) {
            small_gemv_h<NB>(A, a.lda, n, r, zv);
            d2 u[1] = {z};
            for (int i = tid; i < n; i += kSmallThreads) u[0].x += cabs2(zv[i]);
            small_sums<1>(u, red);
            small_step(L, ph == PH_RESTART ? PK_Z_RESTART : PK_Z_RUN, u[0], z);
        }
        // p = z (new direction) or p = z + beta p
        if (L.phase == PH_RUN) {
            const bool fresh = L.restart != 0;
            const double beta = L.beta.x;
            for (int i = tid; i < n; i += kSmallThreads) {
                const d2 zi = zv[i];
                if (fresh) {
                    p[i] = zi;
                } else {
                    d2 pi = p[i];
                    pi.x = __builtin_fma(beta, pi.x, zi.x);
                    pi.y = __builtin_fma(beta, pi.y, zi.y);
                    p[i] = pi;
                }
            }
            __syncthreads();
        }
    }
    if (tid == 0) small_result(L, a.res + sys);
}

// ------------------------------------------------------------------ host

template <int NB>
static hipError_t launch_small(int method, const SmallArgs& a, int64_t batch, hipStream_t s)
{
    const size_t lds = (size_t)(method == CCG_WS_BICGSTAB ? 6 : 4) * NB * kWave * sizeof(d2);
    const void* fn = method == CCG_WS_BICGSTAB ? (const void*)k_small_bicgstab<NB>
                                               : (const void*)k_small_cgnr<NB>;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    if (method == CCG_WS_BICGSTAB)
        k_small_bicgstab<NB><<<(unsigned)batch, kSmallThreads, lds, s>>>(a);
    else
        k_small_cgnr<NB><<<(unsigned)batch, kSmallThreads, lds, s>>>(a);
    return hipGetLastError();
}

static int small_impl(int method, int64_t n, int64_t batch, const ccg_z* A, int64_t lda,
                      int64_t strideA, const ccg_z* Y, int64_t strideY, ccg_z* X,
                      int64_t strideX, double tol, int32_t maxit, uint32_t flags,
                      ccg_result* res, void* stream)
{
    if (method != CCG_WS_BICGSTAB && method != CCG_WS_CGNR) return -1;
    if (n < 0 || n > kSmallMaxN) return -2;
    if (batch < 0 || batch > INT32_MAX) return -3;
    const bool work = n > 0 && batch > 0;
    if (work && !A) return -4;
    if (lda < (n > 1 ? n : 1)) return -5;
    if (batch > 1 && n > 0 && strideA < (n - 1) * lda + n) return -6;
    if (work && !Y) return -7;
    if (batch > 1 && strideY < n) return -8;
    if (work && !X) return -9;
    if (batch > 1 && strideX < n) return -10;
    if (!(tol > 0.0) || !std::isfinite(tol)) return -11;
    if (maxit < 0) return -12;
    if (flags & ~CCG_X0_ZERO) return -13;
    if (batch > 0 && !res) return -14;
    if (batch == 0) return 0;
    hipStream_t s = (hipStream_t)stream;
    if (n == 0) {  // a no-op per system with info 0
        ccg_result zero{};
        for (int64_t b = 0; b < batch; ++b) {
            const hipError_t e =
                hipMemcpyAsync(res + b, &zero, sizeof zero, hipMemcpyHostToDevice, s);
            if (e != hipSuccess) return (int)e;
        }
        const hipError_t e = hipStreamSynchronize(s);  // zero lives on this stack
        return e == hipSuccess ? 0 : (int)e;
    }
    SmallArgs a;
    a.A = (const d2*)A;
    a.lda = lda;
    a.strideA = strideA;
    a.Y = (const d2*)Y;
    a.strideY = strideY;
    a.X = (d2*)X;
    a.strideX = strideX;
    a.res = res;
    a.n = (int)n;
    a.maxit = maxit;
    a.x0zero = (flags & CCG_X0_ZERO) ? 1 : 0;
    a.tol2 = tol * tol;
    hipError_t e;
    if (n <= kWave)
        e = launch_small<1>(method, a, batch, s);
    else if (n <= 2 * kWave)
        e = launch_small<2>(method, a, batch, s);
    else if (n <= 4 * kWave)
        e = launch_small<4>(method, a, batch, s);
    else if (n <= 8 * kWave)
        e = launch_small<8>(method, a, batch, s);
    else
        e = launch_small<16>(method, a, batch, s);
    return e == hipSuccess ? 0 : (int)e;
}

}  // namespace ccg

extern "C" {

int ccg_solve_small_batched(int method, int64_t n, int64_t batch, const ccg_z* A, int64_t lda,
                            int64_t strideA, const ccg_z* Y, int64_t strideY, ccg_z* X,
                            int64_t strideX, double tol, int32_t maxit, uint32_t flags,
                            ccg_result* res, void* stream)
{
    return ccg::small_impl(method, n, batch, A, lda, strideA, Y, strideY, X, strideX, tol, maxit,
                           flags, res, stream);
}

}  // extern "C"
