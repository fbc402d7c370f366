// ccg_block.hip -- many right-hand sides at once: the complex product
// Z = A P on FP64 matrix cores, and block BiCGSTAB, where every column keeps
// its own scalars and stop test (the method of the PIM90 set, Codes section
// 2.1, applied to k systems that share A, as a DDA code does for several
// incident fields).
//
// The product.  Z (n x k) = A (n x n) P (n x k), complex128, 8 n^2 k flops on
// about 16 n^2 bytes of A: at k = 64 that is 32 flop/B, above the FP64 ridge
// (78.6 TFLOP/s / 8 TB/s), so the product is bound by the matrix cores.  One
// v_mfma_f64_16x16x4f64 multiplies a 16 x 4 by a 4 x 16 real tile; a complex
// tile step takes four of them (re*re, -im*im into the real part, re*im,
// im*re into the imaginary part).  A block of 4 wavefronts owns 64 rows; each
// wavefront keeps 16 rows x 64 columns of Z in registers (4 column tiles x
// real/imaginary x 4 FP64 per lane), fed from LDS tiles.  The K dimension is
// split into 8 slices,
// slice = blockIdx % 8: blocks are dispatched round robin over the 8 XCDs, so
// every block on an XCD works on the same slice and the XCD's L2 holds that
// slice of P (1 MB at n = 8000, k = 64) while A streams through once.  A
// fixed-order pass adds the 8 slice results, fused with whatever the solver
// needs from the product (the column reductions of the next scalar step).
//
// The solver.  Per slot: direction update | A P | product sum (+ column
// reductions) | column step | s-update | A S | product sum | column step |
// x, r update | column step.  Column steps run in one small block that reads
// the per-block column partials in a fixed order and applies the same scalar
// step as the single right-hand-side solver to each column's own record.
// Columns that have finished are frozen (their x is never written again);
// the product still covers them, since A is read once for all columns anyway.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "../../include/ccg.h"
#include "ccg_device.h"
#include "ccg_host.h"
#include "ccg_krylov.h"

namespace ccg {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kSlices = 8;         // K split, one slice per XCD
constexpr int kRowsPerBlock = 64;  // 4 wavefronts x 16 rows
constexpr int kMaxCols = 64;       // columns per product pass
constexpr int kColBlocks = 1024;   // blocks of the column-wise vector kernels
constexpr int kStepThreads = 512;  // threads of the column step: 8 per column

static inline int kslice_of(int64_t n)
{
    const int64_t per = (n + kSlices - 1) / kSlices;
    return (int)(((per + 7) / 8) * 8);  // a multiple of the LDS stage depth
}

// ------------------------------------------------------------------ GEMM

// Slice s of Z = A B: Zp[s][i][c] = sum over k in slice s of A[i][k] B[k][c],
// for i < n, c < ncols (ncols <= 16 NT).
//
// The block stages tiles of A (64 rows x kKS) and B (kKS x 16 NT) through LDS,
// double buffered, with coalesced loads (each thread fetches two consecutive
// elements of an A row; a wavefront covers 16 rows x 128 bytes), one barrier
// per stage; the global loads of the next stage are in flight while the
// matrix cores work on the current one.  Wavefront w multiplies rows
// 16w..16w+15 of the tile by all 16 NT columns.
constexpr int kKS = 8;  // k per LDS stage (a multiple of the 4-deep MFMA step)

template <int NT>
__global__ __launch_bounds__(kBlock) void k_zgemm(const d2* __restrict__ A, int64_t lda, int n,
                                                  const d2* __restrict__ B, int64_t ldb,
                                                  int ncols, d2* __restrict__ Zp, int kslice)
{
    constexpr int AP = kKS + 1;                       // padded A-tile row (LDS banks)
    constexpr int AE = kRowsPerBlock * kKS / kBlock;  // A elements per thread
    constexpr int BW = 16 * NT;                       // B-tile width
    constexpr int BN = kKS * BW;                      // B-tile elements
    constexpr int BPT = (BN + kBlock - 1) / kBlock;   // B elements per thread
    __shared__ d2 As[2][kRowsPerBlock * AP];
    __shared__ d2 Bs[2][BN];
    const int s = blockIdx.x % kSlices;
    const int rb = blockIdx.x / kSlices;
    const int t = threadIdx.x;
    const int lane = t & (kWave - 1);
    const int w = t / kWave;
    const int li = lane & 15;  // A row / B column within the 16-wide MFMA tile
    const int lk = lane >> 4;  // k within the 4-deep MFMA step
    const int k0 = s * kslice;
    const int k1 = k0 + kslice < n ? k0 + kslice : n;
    d4 cre[NT], cim[NT];
#pragma unroll
    for (int q = 0; q < NT; ++q) {
        cre[q] = d4{0.0, 0.0, 0.0, 0.0};
        cim[q] = d4{0.0, 0.0, 0.0, 0.0};
    }
    // this thread's share of the global tiles
    const int arow = t / (kKS / AE);
    const int aseg = (t % (kKS / AE)) * AE;
    const int grow = rb * kRowsPerBlock + arow < n ? rb * kRowsPerBlock + arow : n - 1;
    const d2* Ar = A + (int64_t)grow * lda;
    d2 ra[AE], rbv[BPT];
    auto gload = [&](int kk) {
#pragma unroll
        for (int e = 0; e < AE; ++e) {
            const int kc = kk + aseg + e;
            ra[e] = Ar[kc < n ? kc : n - 1];
            if (kc >= k1) ra[e] = d2{0.0, 0.0};
        }
#pragma unroll
        for (int m = 0; m < BPT; ++m) {
            const int idx = t + m * kBlock;
            const int kc = kk + idx / BW;
            const int c = idx % BW;
            const bool ok = idx < BN && kc < k1 && c < ncols;
            rbv[m] = B[(int64_t)(ok ? kc : k0) * ldb + (ok ? c : 0)];
            if (!ok) rbv[m] = d2{0.0, 0.0};
        }
    };
    auto lstore = [&](int buf) {
#pragma unroll
        for (int e = 0; e < AE; ++e) As[buf][arow * AP + aseg + e] = ra[e];
#pragma unroll
        for (int m = 0; m < BPT; ++m) {
            const int idx = t + m * kBlock;
            if (idx < BN) Bs[buf][idx] = rbv[m];
        }
    };
    const int nst = k1 > k0 ? (k1 - k0 + kKS - 1) / kKS : 0;
    if (nst > 0) {
        gload(k0);
        lstore(0);
    }
    __syncthreads();
    for (int st = 0; st < nst; ++st) {
        const int cur = st & 1;
        if (st + 1 < nst) gload(k0 + (st + 1) * kKS);
#pragma unroll
        for (int ks = 0; ks < kKS; ks += 4) {
            const d2 a = As[cur][(w * 16 + li) * AP + ks + lk];
            d2 b[NT];
#pragma unroll
            for (int q = 0; q < NT; ++q) b[q] = Bs[cur][(ks + lk) * BW + 16 * q + li];
#pragma unroll
            for (int q = 0; q < NT; ++q) {
                cre[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b[q].x, cre[q], 0, 0, 0);
                cim[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b[q].y, cim[q], 0, 0, 0);
            }
#pragma unroll
            for (int q = 0; q < NT; ++q) {
                cre[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.y, b[q].y, cre[q], 0, 0, 0);
                cim[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b[q].x, cim[q], 0, 0, 0);
            }
        }
        if (st + 1 < nst) lstore(cur ^ 1);
        __syncthreads();
    }
    // result register v of a lane holds row lk + 4 v of the wavefront's 16-row
    // tile, column li (the v_mfma_f64_16x16x4f64 result layout; the
    // integer-input product tests pin it)
#pragma unroll
    for (int q = 0; q < NT; ++q) {
        const int col = 16 * q + li;
        if (col >= ncols) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = rb * kRowsPerBlock + w * 16 + lk + 4 * v;
            if (r < n) Zp[((int64_t)s * n + r) * ncols + col] = d2{cre[q][v], cim[q][v]};
        }
    }
}

// Z[i][c] = sum over slices s (in order) of Zp[s][i][c]
__device__ __forceinline__ d2 slice_sum(const d2* __restrict__ Zp, int64_t n, int ncols,
                                        int64_t i, int c)
{
    d2 z = Zp[i * ncols + c];
#pragma unroll
    for (int s = 1; s < kSlices; ++s) z += Zp[((int64_t)s * n + i) * ncols + c];
    return z;
}

__global__ __launch_bounds__(kBlock) void k_zgemm_sum(const d2* __restrict__ Zp, int n, int ncols,
                                                      d2* __restrict__ Z, int64_t ldz)
{
    const int64_t total = (int64_t)n * ncols;
    for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * kBlock) {
        const int64_t i = e / ncols;
        const int c = (int)(e - i * ncols);
        Z[i * ldz + c] = slice_sum(Zp, n, ncols, i, c);
    }
}

template <int NT>
static void launch_gemm(const d2* A, int64_t lda, int n, const d2* B, int64_t ldb, int ncols,
                        d2* Zp, hipStream_t s)
{
    const int rblocks = (n + kRowsPerBlock - 1) / kRowsPerBlock;
    k_zgemm<NT><<<rblocks * kSlices, kBlock, 0, s>>>(A, lda, n, B, ldb, ncols, Zp, kslice_of(n));
}

static void gemm(const d2* A, int64_t lda, int n, const d2* B, int64_t ldb, int ncols, d2* Zp,
                 hipStream_t s)
{
    switch ((ncols + 15) / 16) {
    case 1: launch_gemm<1>(A, lda, n, B, ldb, ncols, Zp, s); break;
    case 2: launch_gemm<2>(A, lda, n, B, ldb, ncols, Zp, s); break;
    case 3: launch_gemm<3>(A, lda, n, B, ldb, ncols, Zp, s); break;
    default: launch_gemm<4>(A, lda, n, B, ldb, ncols, Zp, s); break;
    }
}

static size_t zpart_bytes(int64_t n, int ncols)
{
    return align256((size_t)kSlices * (size_t)n * (size_t)ncols * sizeof(d2));
}

// ---------------------------------------------------------- block solver

// Stages of the column step, i.e. which reduction the small kernel finishes.
enum ColStage : int {
    CS_NORMY = 0, CS_SETUP0, CS_SETUP1, CS_P1, CS_S, CS_T, CS_XR
};

struct BArgs {
    const d2* A;
    int64_t lda;
    int n, k, kp;            // systems, padded column count (power of two)
    const d2* Y;
    int64_t ldy;
    d2* X;
    int64_t ldx;
    d2 *R, *RH, *P, *V, *S, *T, *B;  // n x kp, row-major
    d2* Zp;                          // slice results
    d2* cpart;                       // [blocks][kp][2] column partials
    SolverState* cst;                // kp records
};

constexpr size_t kStateStride = 256;
static_assert(sizeof(SolverState) <= kStateStride, "column record");

__device__ __forceinline__ SolverState& col_state(const BArgs& a, int j)
{
    return *(SolverState*)((char*)a.cst + (size_t)j * kStateStride);
}

// Element loop of the column-wise kernels: every thread keeps one column
// (kp divides the block size), rows advance by gridDim.x * kBlock / kp.
#define COL_LOOP(a)                                                              \
    const int j = threadIdx.x & ((a).kp - 1);                                    \
    const int64_t total = (int64_t)(a).n * (a).kp;                               \
    for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < total;      \
         e += (int64_t)gridDim.x * kBlock)

// Per-block column partials: threads of the same column add in thread order.
__device__ __forceinline__ void col_partials(const BArgs& a, d2 v0, d2 v1)
{
    __shared__ d2 l0[kBlock], l1[kBlock];
    l0[threadIdx.x] = v0;
    l1[threadIdx.x] = v1;
    __syncthreads();
    const int t = threadIdx.x;
    if (t < a.kp) {
        d2 s0 = l0[t], s1 = l1[t];
        for (int m = t + a.kp; m < kBlock; m += a.kp) {
            s0 += l0[m];
            s1 += l1[m];
        }
        a.cpart[((size_t)blockIdx.x * a.kp + t) * 2] = s0;
        a.cpart[((size_t)blockIdx.x * a.kp + t) * 2 + 1] = s1;
    }
}

__global__ void kb_init(BArgs a, int maxit, double tol2)
{
    const int j = threadIdx.x;
    if (j >= a.kp) return;
    SolverState o;
    const bool real_col = j < a.k;
    o.phase = real_col ? PH_RUN : PH_DONE;
    o.restart = 1;
    o.info = real_col ? -1 : 0;
    o.iters = o.matvecs = o.confirms = 0;
    o.maxit = maxit;
    o.pending = PK_NONE;
    o.pending_blocks = 0;
    o.no_confirm = 0;
    o.pad1 = o.pad2 = 0;
    o.ny2 = o.thr2 = o.rh2 = o.rr = o.gamma = 0.0;
    o.tol2 = tol2;
    o.relres_rec = o.relres_true = __builtin_nan("");
    o.rho = o.rho_old = o.alpha = o.omega = o.beta = d2{0.0, 0.0};
    col_state(a, j) = o;
}

// Column step: finish the column reductions of the previous kernel (nparts
// blocks) and apply the scalar step of `stage` to every column that has one.
// With ring_slot, also report whether every column has finished.
__global__ __launch_bounds__(kStepThreads) void kb_step(BArgs a, int stage, int nparts,
                                                       int* ring_slot)
{
    constexpr int G = kStepThreads / kMaxCols;  // threads per column
    __shared__ d2 g0[G][kMaxCols], g1[G][kMaxCols];
    __shared__ int done[kMaxCols];
    const int j = threadIdx.x & (kMaxCols - 1);
    const int grp = threadIdx.x / kMaxCols;
    // thread (j, grp) adds blocks grp, grp + G, ... in order, eight loads in
    // flight; the G group sums are then added in group order
    d2 s0 = d2{0.0, 0.0}, s1 = d2{0.0, 0.0};
    if (j < a.kp) {
        int b = grp;
        for (; b + 7 * G < nparts; b += 8 * G) {
            d2 u0[8], u1[8];
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                u0[m] = a.cpart[((size_t)(b + m * G) * a.kp + j) * 2];
                u1[m] = a.cpart[((size_t)(b + m * G) * a.kp + j) * 2 + 1];
            }
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                s0 += u0[m];
                s1 += u1[m];
            }
        }
        for (; b < nparts; b += G) {
            s0 += a.cpart[((size_t)b * a.kp + j) * 2];
            s1 += a.cpart[((size_t)b * a.kp + j) * 2 + 1];
        }
    }
    g0[grp][j] = s0;
    g1[grp][j] = s1;
    __syncthreads();
    if (threadIdx.x < a.kp) {
        d2 t0 = g0[0][j], t1 = g1[0][j];
        for (int g = 1; g < G; ++g) {
            t0 += g0[g][j];
            t1 += g1[g][j];
        }
        SolverState L = col_state(a, j);
        const int ph = L.phase;
        int kind = PK_NONE;
        switch (stage) {
        case CS_NORMY: kind = ph == PH_DONE ? PK_NONE : PK_NORMY; break;
        case CS_SETUP0: kind = ph == PH_ZERO ? PK_ZERO : ph == PH_RUN ? PK_SETUP_B0 : PK_NONE; break;
        case CS_SETUP1: kind = ph == PH_ZERO ? PK_ZERO : ph == PH_RUN ? PK_SETUP_B1 : PK_NONE; break;
        case CS_P1:
            kind = (ph == PH_RUN || ph == PH_RESTART) ? PK_V : ph == PH_CONFIRM ? PK_CONFIRM_B
                                                                                : PK_NONE;
            break;
        case CS_S: kind = ph == PH_RUN ? PK_S : PK_NONE; break;
        case CS_T: kind = ph == PH_RUN ? PK_T : PK_NONE; break;
        case CS_XR: kind = ph == PH_RUN ? PK_XR : ph == PH_HALF ? PK_HALF : PK_NONE; break;
        }
        if (kind != PK_NONE) {
            L.pending = kind;
            apply_step(L, t0, t1, nullptr);
            col_state(a, j) = L;
        }
        done[j] = L.phase == PH_DONE;
    }
    if (ring_slot) {
        __syncthreads();
        if (threadIdx.x == 0) {
            int all = 1;
            for (int c = 0; c < a.kp; ++c) all &= done[c];
            __hip_atomic_store(ring_slot, all ? (int)PH_DONE : (int)PH_RUN, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_SYSTEM);
        }
    }
}

__global__ __launch_bounds__(kBlock) void kb_normy(BArgs a)
{
    d2 v0 = d2{0.0, 0.0};
    COL_LOOP(a)
    {
        if (j < a.k) {
            const int64_t i = e / a.kp;
            v0.x += cabs2(a.Y[i * a.ldy + j]);
        }
    }
    col_partials(a, v0, d2{0.0, 0.0});
}

// x0 = 0: x = 0, r = r^ = y
__global__ __launch_bounds__(kBlock) void kb_setup0(BArgs a)
{
    d2 v0 = d2{0.0, 0.0};
    COL_LOOP(a)
    {
        const int ph = col_state(a, j).phase;
        if (j < a.k && (ph == PH_RUN || ph == PH_ZERO)) {
            const int64_t i = e / a.kp;
            a.X[i * a.ldx + j] = d2{0.0, 0.0};
            if (ph == PH_RUN) {
                const d2 yi = a.Y[i * a.ldy + j];
                a.R[e] = yi;
                a.RH[e] = yi;
                v0.x += cabs2(yi);
            }
        }
    }
    col_partials(a, v0, d2{0.0, 0.0});
}

// general x0: B = x (x = 0 for y = 0 columns)
__global__ __launch_bounds__(kBlock) void kb_setx(BArgs a)
{
    COL_LOOP(a)
    {
        const int ph = col_state(a, j).phase;
        const int64_t i = e / a.kp;
        d2 b = d2{0.0, 0.0};
        if (j < a.k && ph == PH_ZERO) a.X[i * a.ldx + j] = d2{0.0, 0.0};
        if (j < a.k && ph == PH_RUN) b = a.X[i * a.ldx + j];
        a.B[e] = b;
    }
}

// r = r^ = y - (A x), ||r||^2
__global__ __launch_bounds__(kBlock) void kb_red_setup(BArgs a)
{
    d2 v0 = d2{0.0, 0.0};
    COL_LOOP(a)
    {
        if (j < a.k && col_state(a, j).phase == PH_RUN) {
            const int64_t i = e / a.kp;
            const d2 ri = a.Y[i * a.ldy + j] - slice_sum(a.Zp, a.n, a.kp, i, j);
            a.R[e] = ri;
            a.RH[e] = ri;
            v0.x += cabs2(ri);
        }
    }
    col_partials(a, v0, d2{0.0, 0.0});
}

// p = r or r + beta (p - omega v); the product input B is p, or x for a
// column that confirms, or 0.
__global__ __launch_bounds__(kBlock) void kb_p(BArgs a)
{
    COL_LOOP(a)
    {
        const SolverState& L = col_state(a, j);
        const int ph = L.phase;
        d2 b = d2{0.0, 0.0};
        if (ph == PH_RUN || ph == PH_RESTART) {
            const d2 ri = a.R[e];
            d2 pe;
            if (L.restart) {
                pe = ri;
            } else {
                const d2 nom = d2{-L.omega.x, -L.omega.y};
                const d2 d = cfma(nom, a.V[e], a.P[e]);
                pe = cfma(L.beta, d, ri);
            }
            a.P[e] = pe;
            b = pe;
        } else if (ph == PH_CONFIRM && j < a.k) {
            const int64_t i = e / a.kp;
            b = a.X[i * a.ldx + j];
        }
        a.B[e] = b;
    }
}

// after the first product: v = A p (+ r^H v, ||v||^2), or the confirming
// residual r = r^ = y - A x (+ ||r||^2)
__global__ __launch_bounds__(kBlock) void kb_red1(BArgs a)
{
    d2 v0 = d2{0.0, 0.0}, v1 = d2{0.0, 0.0};
    COL_LOOP(a)
    {
        const int ph = col_state(a, j).phase;
        if (ph == PH_RUN || ph == PH_RESTART || ph == PH_CONFIRM) {
            const int64_t i = e / a.kp;
            const d2 z = slice_sum(a.Zp, a.n, a.kp, i, j);
            if (ph == PH_CONFIRM) {
                const d2 ri = a.Y[i * a.ldy + j] - z;
                a.R[e] = ri;
                a.RH[e] = ri;
                v0.x += cabs2(ri);
            } else {
                a.V[e] = z;
                v0 = cfma_conj(a.RH[e], z, v0);
                v1.x += cabs2(z);
            }
        }
    }
    col_partials(a, v0, v1);
}

// s = r - alpha v, ||s||^2
__global__ __launch_bounds__(kBlock) void kb_s(BArgs a)
{
    d2 v0 = d2{0.0, 0.0};
    COL_LOOP(a)
    {
        const SolverState& L = col_state(a, j);
        d2 si = d2{0.0, 0.0};
        if (L.phase == PH_RUN) {
            const d2 nal = d2{-L.alpha.x, -L.alpha.y};
            si = cfma(nal, a.V[e], a.R[e]);
            v0.x += cabs2(si);
        }
        a.S[e] = si;
    }
    col_partials(a, v0, d2{0.0, 0.0});
}

// after the second product: t = A s (+ t^H s, ||t||^2)
__global__ __launch_bounds__(kBlock) void kb_red2(BArgs a)
{
    d2 v0 = d2{0.0, 0.0}, v1 = d2{0.0, 0.0};
    COL_LOOP(a)
    {
        if (col_state(a, j).phase == PH_RUN) {
            const int64_t i = e / a.kp;
            const d2 z = slice_sum(a.Zp, a.n, a.kp, i, j);
            a.T[e] = z;
            v0 = cfma_conj(z, a.S[e], v0);
            v1.x += cabs2(z);
        }
    }
    col_partials(a, v0, v1);
}

// x += alpha p + omega s, r = s - omega t (+ ||r||^2, r^H r); after a
// half-step exit x += alpha p.  Finished columns are not touched.
__global__ __launch_bounds__(kBlock) void kb_xr(BArgs a)
{
    d2 v0 = d2{0.0, 0.0}, v1 = d2{0.0, 0.0};
    COL_LOOP(a)
    {
        const SolverState& L = col_state(a, j);
        const int ph = L.phase;
        if ((ph == PH_RUN || ph == PH_HALF) && j < a.k) {
            const int64_t i = e / a.kp;
            d2* xp = a.X + i * a.ldx + j;
            d2 xi = cfma(L.alpha, a.P[e], *xp);
            if (ph == PH_RUN) {
                const d2 si = a.S[e];
                xi = cfma(L.omega, si, xi);
                const d2 nom = d2{-L.omega.x, -L.omega.y};
                const d2 ri = cfma(nom, a.T[e], si);
                a.R[e] = ri;
                v0.x += cabs2(ri);
                v1 = cfma_conj(a.RH[e], ri, v1);
            }
            *xp = xi;
        }
    }
    col_partials(a, v0, v1);
}

// ----------------------------------------------------------------- host

static int pow2_at_least(int k)
{
    int p = 1;
    while (p < k) p <<= 1;
    return p;
}

static int col_blocks(int64_t n, int kp)
{
    int64_t b = ((int64_t)n * kp + kBlock - 1) / kBlock;
    if (b > kColBlocks) b = kColBlocks;
    return (int)(b < 1 ? 1 : b);
}

struct BLayout {
    size_t cst, cpart, mats, zp, total;
    size_t mat_bytes;
};

static BLayout block_layout(int64_t n, int k)
{
    const int kp = pow2_at_least(k);
    BLayout L{};
    size_t off = 0;
    L.cst = off;
    off += align256(kStateStride * kMaxCols);
    L.cpart = off;
    off += align256((size_t)kColBlocks * kp * 2 * sizeof(d2));
    L.mat_bytes = align256((size_t)(n > 0 ? n : 1) * kp * sizeof(d2));
    L.mats = off;
    off += 7 * L.mat_bytes;
    L.zp = off;
    off += zpart_bytes(n > 0 ? n : 1, kp);
    L.total = off;
    return L;
}

static int run_block(const BArgs& a, uint32_t flags, int32_t maxit, double tol2,
                     ccg_result* res, hipStream_t s)
{
    SyncCtx* sc = nullptr;
    hipError_t e = get_sync(&sc);
    if (e != hipSuccess) return (int)e;
    const int gC = col_blocks(a.n, a.kp);

    kb_init<<<1, kMaxCols, 0, s>>>(a, maxit, tol2);
    kb_normy<<<gC, kBlock, 0, s>>>(a);
    kb_step<<<1, kStepThreads, 0, s>>>(a, CS_NORMY, gC, nullptr);
    if (flags & CCG_X0_ZERO) {
        kb_setup0<<<gC, kBlock, 0, s>>>(a);
        kb_step<<<1, kStepThreads, 0, s>>>(a, CS_SETUP0, gC, nullptr);
    } else {
        kb_setx<<<gC, kBlock, 0, s>>>(a);
        gemm(a.A, a.lda, a.n, a.B, a.kp, a.kp, a.Zp, s);
        kb_red_setup<<<gC, kBlock, 0, s>>>(a);
        kb_step<<<1, kStepThreads, 0, s>>>(a, CS_SETUP1, gC, nullptr);
    }
    if ((e = hipGetLastError()) != hipSuccess) return (int)e;

    const int64_t max_slots = 2 * (int64_t)maxit + 4;
    const int ahead = 1;  // a slot holds two matrix products: far longer than enqueueing
    for (int64_t slot = 0; slot < max_slots + ahead; ++slot) {
        if (slot < max_slots) {
            kb_p<<<gC, kBlock, 0, s>>>(a);
            gemm(a.A, a.lda, a.n, a.B, a.kp, a.kp, a.Zp, s);
            kb_red1<<<gC, kBlock, 0, s>>>(a);
            kb_step<<<1, kStepThreads, 0, s>>>(a, CS_P1, gC, nullptr);
            kb_s<<<gC, kBlock, 0, s>>>(a);
            kb_step<<<1, kStepThreads, 0, s>>>(a, CS_S, gC, nullptr);
            gemm(a.A, a.lda, a.n, a.S, a.kp, a.kp, a.Zp, s);
            kb_red2<<<gC, kBlock, 0, s>>>(a);
            kb_step<<<1, kStepThreads, 0, s>>>(a, CS_T, gC, nullptr);
            kb_xr<<<gC, kBlock, 0, s>>>(a);
            kb_step<<<1, kStepThreads, 0, s>>>(a, CS_XR, gC, sc->ring_d + slot % kRing);
            if ((e = hipGetLastError()) != hipSuccess) return (int)e;
            if ((e = hipEventRecord(sc->ev[slot % kRing], s)) != hipSuccess) return (int)e;
        }
        const int64_t seen = slot - ahead;
        if (seen >= 0) {
            if ((e = hipEventSynchronize(sc->ev[seen % kRing])) != hipSuccess) return (int)e;
            if (__atomic_load_n(&sc->ring_h[seen % kRing], __ATOMIC_ACQUIRE) == PH_DONE) break;
        }
    }
    std::vector<char> hs(kStateStride * a.k);
    if ((e = hipMemcpyAsync(hs.data(), a.cst, hs.size(), hipMemcpyDeviceToHost, s)) !=
        hipSuccess)
        return (int)e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return (int)e;
    for (int j = 0; j < a.k; ++j) {
        const SolverState& st = *(const SolverState*)(hs.data() + (size_t)j * kStateStride);
        res[j].info = st.phase == PH_DONE ? st.info : 1;
        res[j].iters = st.iters;
        res[j].matvecs = st.matvecs;
        res[j].confirms = st.confirms;
        res[j].relres_rec = st.relres_rec;
        res[j].relres_true = st.relres_true;
    }
    return 0;
}

static constexpr int64_t kMaxNB = (int64_t)1 << 30;

static int block_ex(int64_t n, int64_t k, const ccg_z* A, int64_t lda, const ccg_z* Y,
                    int64_t ldy, ccg_z* X, int64_t ldx, double tol, int32_t maxit,
                    uint32_t flags, void* work, size_t work_bytes, ccg_result* res, void* stream)
{
    if (n < 0 || n > kMaxNB) return -1;
    if (k < 1 || k > kMaxCols) return -2;
    if (n > 0 && !A) return -3;
    if (lda < (n > 1 ? n : 1)) return -4;
    if (n > 0 && !Y) return -5;
    if (ldy < k) return -6;
    if (n > 0 && !X) return -7;
    if (ldx < k) return -8;
    if (!(tol > 0.0) || !std::isfinite(tol)) return -9;
    if (maxit < 0) return -10;
    if (flags & ~CCG_X0_ZERO) return -11;
    if (n > 0 && (!work || ((uintptr_t)work & 255))) return -12;
    const BLayout L = block_layout(n, (int)k);
    if (n > 0 && work_bytes < L.total) return -13;
    if (!res) return -14;
    if (n == 0) {
        for (int64_t j = 0; j < k; ++j) {
            std::memset(&res[j], 0, sizeof res[j]);
            res[j].relres_rec = res[j].relres_true = 0.0;
        }
        return 0;
    }
    BArgs a{};
    char* base = (char*)work;
    a.A = (const d2*)A;
    a.lda = lda;
    a.n = (int)n;
    a.k = (int)k;
    a.kp = pow2_at_least((int)k);
    a.Y = (const d2*)Y;
    a.ldy = ldy;
    a.X = (d2*)X;
    a.ldx = ldx;
    d2* m[7];
    for (int q = 0; q < 7; ++q) m[q] = (d2*)(base + L.mats + q * L.mat_bytes);
    a.R = m[0]; a.RH = m[1]; a.P = m[2]; a.V = m[3]; a.S = m[4]; a.T = m[5]; a.B = m[6];
    a.Zp = (d2*)(base + L.zp);
    a.cpart = (d2*)(base + L.cpart);
    a.cst = (SolverState*)(base + L.cst);
    return run_block(a, flags, maxit, tol * tol, res, (hipStream_t)stream);
}

}  // namespace ccg

// ============================================================== C ABI

namespace ccg {

// Workspace of the block entry points (ccg_workspace_bytes delegates here).
size_t block_workspace_bytes(int method, int64_t n, int64_t k)
{
    if (n < 0 || k < 1) return 0;
    if (method == CCG_WS_MATMAT) {
        const int kc = (int)(k < kMaxCols ? k : kMaxCols);
        return zpart_bytes(n > 0 ? n : 1, kc);
    }
    if (method == CCG_WS_BICGSTAB_BLOCK && k <= kMaxCols) return block_layout(n, (int)k).total;
    return 0;
}

}  // namespace ccg

extern "C" {

static int matmat_impl(int64_t n, int64_t k, const ccg_z* A, int64_t lda, const ccg_z* B,
                       int64_t ldb, ccg_z* Z, int64_t ldz, void* work, size_t work_bytes,
                       void* stream, bool own)
{
    using namespace ccg;
    if (n < 0 || n > kMaxNB) return -1;
    if (k < 0) return -2;
    if (n > 0 && k > 0 && !A) return -3;
    if (lda < (n > 1 ? n : 1)) return -4;
    if (n > 0 && k > 0 && !B) return -5;
    if (ldb < (k > 1 ? k : 1)) return -6;
    if (n > 0 && k > 0 && !Z) return -7;
    if (ldz < (k > 1 ? k : 1)) return -8;
    if (n == 0 || k == 0) return 0;
    hipStream_t s = (hipStream_t)stream;
    const int kc = (int)(k < kMaxCols ? k : kMaxCols);
    const size_t need = zpart_bytes(n, kc);
    void* zp = work;
    hipError_t e;
    if (own) {
        if ((e = hipMallocAsync(&zp, need, s)) != hipSuccess) return (int)e;
    } else {
        if (!work || ((uintptr_t)work & 255)) return -9;
        if (work_bytes < need) return -10;
    }
    for (int64_t c0 = 0; c0 < k; c0 += kMaxCols) {
        const int nc = (int)(k - c0 < kMaxCols ? k - c0 : kMaxCols);
        gemm((const d2*)A, lda, (int)n, (const d2*)B + c0, ldb, nc, (d2*)zp, s);
        int64_t blocks = ((int64_t)n * nc + kBlock - 1) / kBlock;
        if (blocks > 2048) blocks = 2048;
        k_zgemm_sum<<<(int)blocks, kBlock, 0, s>>>((const d2*)zp, (int)n, nc, (d2*)Z + c0, ldz);
    }
    e = hipGetLastError();
    if (own) {
        hipError_t e2 = hipFreeAsync(zp, s);
        if (e == hipSuccess) e = e2;
    }
    return e == hipSuccess ? 0 : (int)e;
}

int ccg_matmat(int64_t n, int64_t k, const ccg_z* A, int64_t lda, const ccg_z* B, int64_t ldb,
               ccg_z* Z, int64_t ldz, void* stream)
{
    return matmat_impl(n, k, A, lda, B, ldb, Z, ldz, nullptr, 0, stream, true);
}

int ccg_matmat_ex(int64_t n, int64_t k, const ccg_z* A, int64_t lda, const ccg_z* B,
                  int64_t ldb, ccg_z* Z, int64_t ldz, void* work, size_t work_bytes,
                  void* stream)
{
    return matmat_impl(n, k, A, lda, B, ldb, Z, ldz, work, work_bytes, stream, false);
}

int ccg_bicgstab_block_ex(int64_t n, int64_t k, const ccg_z* A, int64_t lda, const ccg_z* Y,
                          int64_t ldy, ccg_z* X, int64_t ldx, double tol, int32_t maxit,
                          uint32_t flags, void* work, size_t work_bytes, ccg_result* res,
                          void* stream)
{
    return ccg::block_ex(n, k, A, lda, Y, ldy, X, ldx, tol, maxit, flags, work, work_bytes,
                         res, stream);
}

int ccg_bicgstab_block(int64_t n, int64_t k, const ccg_z* A, int64_t lda, const ccg_z* Y,
                       int64_t ldy, ccg_z* X, int64_t ldx, double tol, int32_t maxit,
                       int32_t* info, void* stream)
{
    if (!info) return -11;
    if (k < 1 || k > ccg::kMaxCols) return -2;
    std::vector<ccg_result> res((size_t)k);
    if (n == 0) {
        for (int64_t j = 0; j < k; ++j) info[j] = 0;
        return 0;
    }
    if (n < 0) return -1;
    hipStream_t s = (hipStream_t)stream;
    const size_t bytes = ccg::block_layout(n, (int)k).total;
    void* work = nullptr;
    hipError_t e = hipMallocAsync(&work, bytes, s);
    if (e != hipSuccess) return (int)e;
    int rc = ccg::block_ex(n, k, A, lda, Y, ldy, X, ldx, tol, maxit, 0u, work, bytes, res.data(),
                           stream);
    e = hipFreeAsync(work, s);
    if (rc == 0 && e == hipSuccess) e = hipStreamSynchronize(s);
    if (rc != 0) return rc;
    if (e != hipSuccess) return (int)e;
    for (int64_t j = 0; j < k; ++j) info[j] = res[(size_t)j].info;
    return 0;
}

}  // extern "C"
