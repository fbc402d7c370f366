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
#include <algorithm>
#include <deque>
#include <map>
#include <unordered_map>
#include <utility>
#include <vector>

#include "../../include/ccg.h"
#include "ccg_device.h"
#include "ccg_host.h"
#include "ccg_krylov.h"

namespace ccg {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kSlices = 8;         // K split, one slice per XCD
constexpr int kRowsPerBlock = 64;  // 4 wavefronts x 16 rows
constexpr int kMaxCols = 64;       // columns per product pass
// Blocks of the column-wise vector kernels (at most): one per compute unit.
// The column step that follows each of them reads their kp x 2 partials in a
// single block, at about 100 GB/s; with 1024 blocks (2 MB of partials at
// kp = 64) it took 22 us, and 256 made the 64-column block solve 3.6% and the
// mixed one 6.5% faster (128: 1.8% and 3.3%).
constexpr int kColBlocks = 256;
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
// The block stages tiles of A (16 WV rows x kKS) and B (kKS x 16 NT) through
// LDS, double buffered, with coalesced loads (each thread fetches two
// consecutive elements of an A row; a wavefront covers 16 rows x 128 bytes),
// one barrier per stage; the global loads of the next PF stages are in flight
// while the matrix cores work on the current one (PF = 1 except for the
// products that launch_gemm gives a ring, below).  Wavefront w multiplies
// rows 16w..16w+15 of the tile by all 16 NT columns.
//
// Each complex product takes three real matrix-core products rather than
// four (the 3M method): with P1 = Re A Re B, P2 = Im A Im B and
// P3 = (Re A + Im A)(Re B + Im B) accumulated over the slice, Re Z = P1 - P2
// and Im Z = (P3 - P1) - P2.  It does a quarter less matrix-core work; its
// error is bounded normwise like the four-product form's (Higham, SIAM J.
// Matrix Anal. Appl. 13, 1992), about three times the unit roundoff times
// |A| |B| for the imaginary part instead of two, and it is exact on Gaussian
// integers of moderate size.  At n = 8000, k = 64 (20 back-to-back launches
// through ccg_matmat, HIP events, A/B on one box): 543 - 553 us against
// 609 - 612 us; splitting the 64 columns over two wavefronts per 16 rows
// (half the accumulators, two blocks per compute unit) or 16-deep stages
// measured the same.
//
// kHalf (NT = 1, ncols <= 8): the 16 columns of the matrix-core tile hold the
// real parts (columns 0-7) and the imaginary parts (8-15) of the 8 complex
// columns of B, so each 4-deep step takes two real products (Re A and Im A
// times that tile) instead of four on a half-empty tile; lane c and lane
// c + 8 then combine Re Z = Re A Re B - Im A Im B and Im Z = Re A Im B +
// Im A Re B.  The serving products of 5 to 8 columns are HBM bound with it
// rather than bound by the padded matrix-core work.
constexpr int kKS = 8;  // k per LDS stage (a multiple of the 4-deep MFMA step)
constexpr int kHalfCols = 8;  // widest product of the packed form
// Stages whose global loads are in flight at once in the packed form: its
// products are HBM bound (8 to 16 flops per byte of A), and one stage ahead
// (two A elements per thread per barrier) leaves HBM mostly idle.  The ring
// holds the loaded values in registers; each stage stores one slot to LDS,
// waits at the barrier, issues the loads of the stage kHalfRing ahead into
// that slot and multiplies.  Measured through ccg_matmat with 4-wavefront
// blocks (6 / 8 columns, HIP events): n = 4096 50.4 / 49.4 us against 61.6 /
// 59.3 for one stage ahead with 8-wavefront blocks, n = 2048 19.0 / 19.4
// against 24.8 / 25.2; an 8-deep ring was slower than 4 (53.1 / 51.2 at
// n = 4096: more registers, fewer blocks per compute unit).  Above
// kHalfRingMaxN the stand-alone product keeps the one-stage form, which was
// faster there (n = 8000: 180.7 against 189.0 us).  The serving grids keep
// the one-stage form: they batch many requests, so many blocks per compute
// unit are in flight anyway, and their capacity did not change with a ring of
// 4 or 8 (within the 3% spread between boxes).  The matrix-core steps are the
// same in every form, so are the bits.
constexpr int kHalfRing = 4;
constexpr int kHalfRingMaxN = 4096;

// LDS of one zgemm_body shape: two A tiles and two B tiles (the caller
// declares it, so that a kernel with several shapes holds the largest once).
template <int NT, int KS = kKS, int WV = kWavesPerBlock, bool kHalf = false>
struct ZgemmLds {
    static constexpr int ROWS = 16 * WV;                    // rows per block
    static constexpr int AP = KS + 1;                       // padded A-tile row (LDS banks)
    static constexpr int BW = kHalf ? kHalfCols : 16 * NT;  // B-tile width
    static constexpr int BN = KS * BW;                      // B-tile elements
    static constexpr int size = 2 * ROWS * AP + 2 * BN;     // d2 elements
};

template <int NT, int KS = kKS, int WV = kWavesPerBlock, bool kHalf = false, int PF = 1>
__device__ __forceinline__ void zgemm_body(const d2* __restrict__ A, int64_t lda, int n,
                                           const d2* __restrict__ B, int64_t ldb, int ncols,
                                           d2* __restrict__ Zp, int kslice, int bid, d2* lds)
{
    static_assert(!kHalf || NT == 1, "the packed form has one tile");
    using LD = ZgemmLds<NT, KS, WV, kHalf>;
    constexpr int TH = WV * kWave;                    // threads per block
    constexpr int ROWS = LD::ROWS;
    constexpr int AP = LD::AP;
    constexpr int AE = ROWS * KS / TH;                // A elements per thread
    constexpr int BW = LD::BW;
    constexpr int BN = LD::BN;
    constexpr int BPT = (BN + TH - 1) / TH;           // B elements per thread
    d2(*As)[ROWS * AP] = reinterpret_cast<d2(*)[ROWS * AP]>(lds);
    d2(*Bs)[BN] = reinterpret_cast<d2(*)[BN]>(lds + 2 * ROWS * AP);
    const int s = bid % kSlices;
    const int rb = bid / kSlices;
    const int t = threadIdx.x;
    const int lane = t & (kWave - 1);
    const int w = t / kWave;
    const int li = lane & 15;  // A row / B column within the 16-wide MFMA tile
    const int lk = lane >> 4;  // k within the 4-deep MFMA step
    const int k0 = s * kslice;
    const int k1 = k0 + kslice < n ? k0 + kslice : n;
    // kHalf: cre = Re A x [Re B | Im B], cim = Im A x [Re B | Im B].  Else the
    // three real products of each complex one: cre = Re A Re B, cim =
    // Im A Im B, c3 = (Re A + Im A)(Re B + Im B).
    d4 cre[NT], cim[NT], c3[NT];
#pragma unroll
    for (int q = 0; q < NT; ++q) {
        cre[q] = d4{0.0, 0.0, 0.0, 0.0};
        cim[q] = d4{0.0, 0.0, 0.0, 0.0};
        c3[q] = d4{0.0, 0.0, 0.0, 0.0};
    }
    // this thread's share of the global tiles
    const int arow = t / (KS / AE);
    const int aseg = (t % (KS / AE)) * AE;
    const int grow = rb * ROWS + arow < n ? rb * ROWS + arow : n - 1;
    const d2* Ar = A + (int64_t)grow * lda;
    // The loads of a stage only issue here; what falls outside the slice is
    // zeroed when the values go to LDS (after other stages' matrix products),
    // so nothing waits for the loads before the products.  Slot j of the ring
    // holds the loads of stages j, j + PF, j + 2 PF, ...
    d2 ra[PF][AE], rbv[PF][BPT];
    bool aok[PF][AE], bok[PF][BPT];
    auto gload = [&](int j, int kk) {
#pragma unroll
        for (int e = 0; e < AE; ++e) {
            const int kc = kk + aseg + e;
            aok[j][e] = kc < k1;
            ra[j][e] = Ar[kc < k1 ? kc : k0];
        }
#pragma unroll
        for (int m = 0; m < BPT; ++m) {
            const int idx = t + m * TH;
            const int kc = kk + idx / BW;
            const int c = idx % BW;
            bok[j][m] = idx < BN && kc < k1 && c < ncols;
            rbv[j][m] = B[(int64_t)(bok[j][m] ? kc : k0) * ldb + (bok[j][m] ? c : 0)];
        }
    };
    auto lstore = [&](int j, int buf) {
        const d2 z = d2{0.0, 0.0};
#pragma unroll
        for (int e = 0; e < AE; ++e) As[buf][arow * AP + aseg + e] = aok[j][e] ? ra[j][e] : z;
#pragma unroll
        for (int m = 0; m < BPT; ++m) {
            const int idx = t + m * TH;
            if (idx < BN) Bs[buf][idx] = bok[j][m] ? rbv[j][m] : z;
        }
    };
    auto mstage = [&](int cur) {
#pragma unroll
        for (int ks = 0; ks < KS; ks += 4) {
            const d2 a = As[cur][(w * 16 + li) * AP + ks + lk];
            if constexpr (kHalf) {
                // cre: Re A x [Re B | Im B], cim: Im A x [Re B | Im B]
                const d2 bb = Bs[cur][(ks + lk) * BW + (li & (kHalfCols - 1))];
                const double bp = li < kHalfCols ? bb.x : bb.y;
                cre[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, bp, cre[0], 0, 0, 0);
                cim[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, bp, cim[0], 0, 0, 0);
            } else {
                d2 b[NT];
#pragma unroll
                for (int q = 0; q < NT; ++q) b[q] = Bs[cur][(ks + lk) * BW + 16 * q + li];
                const double as = a.x + a.y;
#pragma unroll
                for (int q = 0; q < NT; ++q) {
                    cre[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b[q].x, cre[q], 0, 0, 0);
                    cim[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b[q].y, cim[q], 0, 0, 0);
                    c3[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(as, b[q].x + b[q].y, c3[q], 0, 0,
                                                                 0);
                }
            }
        }
    };
    const int nst = k1 > k0 ? (k1 - k0 + KS - 1) / KS : 0;
    if constexpr (PF == 1) {
        // next stage's loads in flight during this stage's products; one
        // barrier per stage
        if (nst > 0) {
            gload(0, k0);
            lstore(0, 0);
        }
        __syncthreads();
        for (int st = 0; st < nst; ++st) {
            const int cur = st & 1;
            if (st + 1 < nst) gload(0, k0 + (st + 1) * KS);
            mstage(cur);
            if (st + 1 < nst) lstore(0, cur ^ 1);
            __syncthreads();
        }
    } else {
        // PF stages in flight.  Stage st stores slot st mod PF into LDS
        // buffer st mod 2 (whose previous contents, stage st - 2, every
        // wavefront has multiplied before the barrier of stage st - 1),
        // waits at the barrier, refills the slot with stage st + PF and
        // multiplies.  Every slot is loaded and stored in each group of PF
        // stages, also past the slice (those loads re-read its first
        // columns, k0 < k1 <= n, and are zeroed), so the compiler's count of
        // the loads in flight stays exact and a store waits only for its own
        // slot; only the products stop at the last stage.  An empty slice
        // (k0 >= n: small n) loads nothing and stores its zero sums.  nst is
        // the same in the whole block.
        if (nst > 0) {
#pragma unroll
            for (int j = 0; j < PF; ++j) gload(j, k0 + j * KS);
            for (int st0 = 0; st0 < nst; st0 += PF) {
#pragma unroll
                for (int j = 0; j < PF; ++j) {
                    const int st = st0 + j;
                    lstore(j, st & 1);
                    __syncthreads();
                    gload(j, k0 + (st + PF) * KS);
                    if (st < nst) mstage(st & 1);
                }
            }
        }
    }
    // result register v of a lane holds row lk + 4 v of the wavefront's 16-row
    // tile, column li (the v_mfma_f64_16x16x4f64 result layout; the
    // integer-input product tests pin it)
    if constexpr (kHalf) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const double d1 = cre[0][v], d2v = cim[0][v];
            const double o1 = __shfl_xor(d1, kHalfCols, kWave), o2 = __shfl_xor(d2v, kHalfCols, kWave);
            const int r = rb * ROWS + w * 16 + lk + 4 * v;
            if (li < ncols && r < n) Zp[((int64_t)s * n + r) * ncols + li] = d2{d1 - o2, o1 + d2v};
        }
        return;
    }
    // Re = Re A Re B - Im A Im B, Im = (c3 - Re A Re B) - Im A Im B
#pragma unroll
    for (int q = 0; q < NT; ++q) {
        const int col = 16 * q + li;
        if (col >= ncols) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = rb * ROWS + w * 16 + lk + 4 * v;
            if (r < n)
                Zp[((int64_t)s * n + r) * ncols + col] =
                    d2{cre[q][v] - cim[q][v], (c3[q][v] - cre[q][v]) - cim[q][v]};
        }
    }
}

// The stand-alone product (ccg_matmat, the block solvers' products) runs 8
// wavefronts per block: 128 rows share each B tile in LDS, half the B
// traffic per product of the 4-wavefront blocks the serving grids keep.
// Measured at n = 8000, k = 64 (kernel time, HIP events): 517 against 566 us
// for 4 wavefronts, 0.81 of the FP64 matrix peak; a 16-deep stage (579 us,
// LDS-bound to 2 blocks per compute unit), 2-wavefront blocks (586 us) and
// 12- or 32-deep stages were slower.  Every element sums its products in the
// same order whatever the block shape, so all shapes give the same bits.
constexpr int kGemmWaves = 8;

template <int NT, int KS = kKS, int WV = kGemmWaves, bool kHalf = false, int PF = 1>
__global__ __launch_bounds__(WV * kWave) void k_zgemm(const d2* __restrict__ A, int64_t lda,
                                                      int n, const d2* __restrict__ B,
                                                      int64_t ldb, int ncols,
                                                      d2* __restrict__ Zp, int kslice,
                                                      const int* __restrict__ skip)
{
    __shared__ d2 lds[ZgemmLds<NT, KS, WV, kHalf>::size];
    if (skip && *skip) return;
    zgemm_body<NT, KS, WV, kHalf, PF>(A, lda, n, B, ldb, ncols, Zp, kslice, blockIdx.x, lds);
}

// Slice s of Z = A B for at most kVCols columns, on the vector units.  With
// four or fewer right-hand sides the product is HBM bound and a 16-wide
// matrix-core tile would spend most of its work and of its B traffic on
// padding; here wavefront w takes kVRows rows, lane l the columns
// k0 + 64 c + l of the slice, and each lane accumulates kVRows x KP complex
// sums in FP64 (one load of A feeds KP complex FMAs; the lane's B row segment
// serves kVRows rows).  The sums cross the 64 lanes in the transposing
// butterfly.  Same slice split and output layout as zgemm_body: block b takes
// slice b mod 8 (the XCD it runs on) and rows (b / 8) * kVRowsPerBlock ...
constexpr int kVCols = 4;                   // most columns of this product
constexpr int kVRows = 4;                   // rows per wavefront
constexpr int kVRowsPerBlock = kWavesPerBlock * kVRows;

template <int KP>
__device__ __forceinline__ void vgemm_body(const d2* __restrict__ A, int64_t lda, int n,
                                           const d2* __restrict__ B, int64_t ldb, int ncols,
                                           d2* __restrict__ Zp, int kslice, int bid)
{
    const int s = bid % kSlices;
    const int rb = bid / kSlices;
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    const int r0 = rb * kVRowsPerBlock + w * kVRows;
    const int k0 = s * kslice;
    const int k1 = k0 + kslice < n ? k0 + kslice : n;
    constexpr int NV = kVRows * KP;
    d2 acc[NV];
#pragma unroll
    for (int e = 0; e < NV; ++e) acc[e] = d2{0.0, 0.0};
    const d2* Ar[kVRows];
#pragma unroll
    for (int r = 0; r < kVRows; ++r) Ar[r] = A + (int64_t)(r0 + r < n ? r0 + r : n - 1) * lda;
    for (int j = k0 + lane; j < k1; j += kWave) {
        d2 b[KP], a[kVRows];
#pragma unroll
        for (int c = 0; c < KP; ++c) b[c] = c < ncols ? B[(int64_t)j * ldb + c] : d2{0.0, 0.0};
#pragma unroll
        for (int r = 0; r < kVRows; ++r) a[r] = ldnt(Ar[r] + j);
#pragma unroll
        for (int r = 0; r < kVRows; ++r)
#pragma unroll
            for (int c = 0; c < KP; ++c) acc[r * KP + c] = cfma(a[r], b[c], acc[r * KP + c]);
    }
    wave_transpose_sum<NV>(acc, lane);
    constexpr int kShare = kWave / NV;  // lanes holding the same total
    if ((lane & (kShare - 1)) == 0) {
        const int e = lane / kShare;
        const int r = e / KP, c = e % KP;
        if (r0 + r < n && c < ncols) Zp[((int64_t)s * n + r0 + r) * ncols + c] = acc[0];
    }
}

// skip (device word, or null): when set, a solver has no column left that
// needs this product and the launch does nothing.
template <int KP>
__global__ __launch_bounds__(kBlock) void k_vgemm(const d2* __restrict__ A, int64_t lda, int n,
                                                  const d2* __restrict__ B, int64_t ldb,
                                                  int ncols, d2* __restrict__ Zp, int kslice,
                                                  const int* __restrict__ skip)
{
    if (skip && *skip) return;
    vgemm_body<KP>(A, lda, n, B, ldb, ncols, Zp, kslice, blockIdx.x);
}

static inline int vgemm_blocks(int64_t n)
{
    return (int)((n + kVRowsPerBlock - 1) / kVRowsPerBlock) * kSlices;
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

template <int NT, bool kHalf = false>
static void launch_gemm(const d2* A, int64_t lda, int n, const d2* B, int64_t ldb, int ncols,
                        d2* Zp, hipStream_t s, const int* skip)
{
    if constexpr (kHalf) {
        if (n <= kHalfRingMaxN) {  // the packed form's ring
            constexpr int rows = 16 * kWavesPerBlock;
            const int rblocks = (n + rows - 1) / rows;
            k_zgemm<NT, kKS, kWavesPerBlock, kHalf, kHalfRing>
                <<<rblocks * kSlices, kWavesPerBlock * kWave, 0, s>>>(A, lda, n, B, ldb, ncols,
                                                                      Zp, kslice_of(n), skip);
            return;
        }
    }
    // 49 - 64 columns: the 3M accumulators leave one 8-wavefront block per
    // compute unit, whose waves waited on their loads 27% of their cycles
    // with one stage ahead; two stages ahead (the ring of the packed form,
    // same occupancy) took n = 8000 from 544 - 548 to 533 - 535 us (four: no
    // better).  Narrower products keep two blocks per compute unit and one
    // stage.
    constexpr int PF = (!kHalf && NT == 4) ? 2 : 1;
    constexpr int rows = 16 * kGemmWaves;
    const int rblocks = (n + rows - 1) / rows;
    k_zgemm<NT, kKS, kGemmWaves, kHalf, PF><<<rblocks * kSlices, kGemmWaves * kWave, 0, s>>>(
        A, lda, n, B, ldb, ncols, Zp, kslice_of(n), skip);
}

// Z slices = A B: vector units for up to kVCols columns, FP64 matrix cores
// beyond (the packed form up to kHalfCols columns).
static void gemm(const d2* A, int64_t lda, int n, const d2* B, int64_t ldb, int ncols, d2* Zp,
                 hipStream_t s, const int* skip = nullptr)
{
    if (ncols <= kVCols) {
        const int g = vgemm_blocks(n), ks = kslice_of(n);
        if (ncols == 1)
            k_vgemm<1><<<g, kBlock, 0, s>>>(A, lda, n, B, ldb, ncols, Zp, ks, skip);
        else if (ncols == 2)
            k_vgemm<2><<<g, kBlock, 0, s>>>(A, lda, n, B, ldb, ncols, Zp, ks, skip);
        else
            k_vgemm<4><<<g, kBlock, 0, s>>>(A, lda, n, B, ldb, ncols, Zp, ks, skip);
        return;
    }
    if (ncols <= kHalfCols) {
        launch_gemm<1, true>(A, lda, n, B, ldb, ncols, Zp, s, skip);
        return;
    }
    switch ((ncols + 15) / 16) {
    case 1: launch_gemm<1>(A, lda, n, B, ldb, ncols, Zp, s, skip); break;
    case 2: launch_gemm<2>(A, lda, n, B, ldb, ncols, Zp, s, skip); break;
    case 3: launch_gemm<3>(A, lda, n, B, ldb, ncols, Zp, s, skip); break;
    default: launch_gemm<4>(A, lda, n, B, ldb, ncols, Zp, s, skip); break;
    }
}

// ----------------------------------------------------- complex64 product

// Slice s of Z = A32 B for the mixed-precision block solver: A32 complex64,
// B complex128 rounded to complex64 as it is staged, products accumulated in
// FP32 on the matrix cores (v_mfma_f32_16x16x4f32, three real products per
// complex step, the 3M form of zgemm_body: 325 - 337 against 369 - 376 us at
// n = 8000, k = 64, A/B on one box), each slice result widened to FP64 on store
// into the same slice buffer, so the FP64 slice sum and column kernels are
// shared.  Tiles: 64 rows x 16 k per LDS stage (8 KB of A, as the FP64
// kernel's 64 x 8).  Result register v of a lane holds row 4 lk + v, column
// li (the v_mfma_f32_16x16x4f32 layout, unlike the FP64 instruction's
// lk + 4 v; the integer-input product tests pin it).
typedef float f4v __attribute__((ext_vector_type(4)));
constexpr int kKS32 = 16;

static inline int kslice32_of(int64_t n)
{
    const int64_t per = (n + kSlices - 1) / kSlices;
    return (int)(((per + kKS32 - 1) / kKS32) * kKS32);
}

template <int NT, int KS = kKS32, int WV = kWavesPerBlock, int PF = 1>
__device__ __forceinline__ void cgemm_body(const f2* __restrict__ A, int64_t lda, int n,
                                           const d2* __restrict__ B, int64_t ldb, int ncols,
                                           d2* __restrict__ Zp, int kslice, int bid)
{
    constexpr int TH = WV * kWave;
    constexpr int ROWS = 16 * WV;
    constexpr int AP = KS + 1;
    constexpr int AE = ROWS * KS / TH;
    constexpr int BW = 16 * NT;
    constexpr int BN = KS * BW;
    constexpr int BPT = (BN + TH - 1) / TH;
    __shared__ f2 As[2][ROWS * AP];
    __shared__ f2 Bs[2][BN];
    const int s = bid % kSlices;
    const int rb = bid / kSlices;
    const int t = threadIdx.x;
    const int lane = t & (kWave - 1);
    const int w = t / kWave;
    const int li = lane & 15;
    const int lk = lane >> 4;
    const int k0 = s * kslice;
    const int k1 = k0 + kslice < n ? k0 + kslice : n;
    f4v cre[NT], cim[NT], c3[NT];
#pragma unroll
    for (int q = 0; q < NT; ++q) {
        cre[q] = f4v{0.f, 0.f, 0.f, 0.f};
        cim[q] = f4v{0.f, 0.f, 0.f, 0.f};
        c3[q] = f4v{0.f, 0.f, 0.f, 0.f};
    }
    const int arow = t / (KS / AE);
    const int aseg = (t % (KS / AE)) * AE;
    const int grow = rb * ROWS + arow < n ? rb * ROWS + arow : n - 1;
    const f2* Ar = A + (int64_t)grow * lda;
    // as in zgemm_body: the loads only issue here; zeroing outside the slice
    // and the rounding of B to complex64 happen on the way to LDS
    f2 ra[PF][AE];
    d2 rbv[PF][BPT];
    bool aok[PF][AE], bok[PF][BPT];
    auto gload = [&](int j, int kk) {
#pragma unroll
        for (int e = 0; e < AE; ++e) {
            const int kc = kk + aseg + e;
            aok[j][e] = kc < k1;
            ra[j][e] = Ar[kc < k1 ? kc : k0];
        }
#pragma unroll
        for (int m = 0; m < BPT; ++m) {
            const int idx = t + m * TH;
            const int kc = kk + idx / BW;
            const int c = idx % BW;
            bok[j][m] = idx < BN && kc < k1 && c < ncols;
            rbv[j][m] = B[(int64_t)(bok[j][m] ? kc : k0) * ldb + (bok[j][m] ? c : 0)];
        }
    };
    auto lstore = [&](int j, int buf) {
        const f2 z = f2{0.f, 0.f};
#pragma unroll
        for (int e = 0; e < AE; ++e) As[buf][arow * AP + aseg + e] = aok[j][e] ? ra[j][e] : z;
#pragma unroll
        for (int m = 0; m < BPT; ++m) {
            const int idx = t + m * TH;
            if (idx < BN)
                Bs[buf][idx] = bok[j][m] ? f2{(float)rbv[j][m].x, (float)rbv[j][m].y} : z;
        }
    };
    auto mstage = [&](int cur) {
#pragma unroll
        for (int ks = 0; ks < KS; ks += 4) {
            const f2 a = As[cur][(w * 16 + li) * AP + ks + lk];
            f2 b[NT];
#pragma unroll
            for (int q = 0; q < NT; ++q) b[q] = Bs[cur][(ks + lk) * BW + 16 * q + li];
            const float as = a.x + a.y;
#pragma unroll
            for (int q = 0; q < NT; ++q) {
                cre[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b[q].x, cre[q], 0, 0, 0);
                cim[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b[q].y, cim[q], 0, 0, 0);
                c3[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(as, b[q].x + b[q].y, c3[q], 0, 0, 0);
            }
        }
    };
    const int nst = k1 > k0 ? (k1 - k0 + KS - 1) / KS : 0;
    if constexpr (PF == 1) {
        if (nst > 0) {
            gload(0, k0);
            lstore(0, 0);
        }
        __syncthreads();
        for (int st = 0; st < nst; ++st) {
            const int cur = st & 1;
            if (st + 1 < nst) gload(0, k0 + (st + 1) * KS);
            mstage(cur);
            if (st + 1 < nst) lstore(0, cur ^ 1);
            __syncthreads();
        }
    } else if (nst > 0) {
#pragma unroll
        for (int j = 0; j < PF; ++j) gload(j, k0 + j * KS);
        for (int st0 = 0; st0 < nst; st0 += PF) {
#pragma unroll
            for (int j = 0; j < PF; ++j) {
                const int st = st0 + j;
                lstore(j, st & 1);
                __syncthreads();
                gload(j, k0 + (st + PF) * KS);
                if (st < nst) mstage(st & 1);
            }
        }
    }
#pragma unroll
    for (int q = 0; q < NT; ++q) {
        const int col = 16 * q + li;
        if (col >= ncols) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = rb * ROWS + w * 16 + 4 * lk + v;
            if (r < n)
                Zp[((int64_t)s * n + r) * ncols + col] =
                    d2{(double)(cre[q][v] - cim[q][v]),
                       (double)((c3[q][v] - cre[q][v]) - cim[q][v])};
        }
    }
}

// 49 - 64 columns keep two stages of loads in flight (the ring of
// zgemm_body): with three real products per complex one the FP32 matrix-core
// work per stage is short, and n = 8000, k = 64 took 309 - 312 against
// 316 - 318 us (A/B on one box).  Same steps, same bits.
template <int NT, int KS = kKS32, int WV = kGemmWaves, int PF = (NT == 4 ? 2 : 1)>
__global__ __launch_bounds__(WV * kWave) void k_cgemm(const f2* __restrict__ A, int64_t lda,
                                                      int n, const d2* __restrict__ B,
                                                      int64_t ldb, int ncols,
                                                      d2* __restrict__ Zp, int kslice,
                                                      const int* __restrict__ skip)
{
    if (skip && *skip) return;
    cgemm_body<NT, KS, WV, PF>(A, lda, n, B, ldb, ncols, Zp, kslice, blockIdx.x);
}

template <int NT>
static void launch_cgemm(const f2* A, int64_t lda, int n, const d2* B, int64_t ldb, int ncols,
                         d2* Zp, hipStream_t s, const int* skip)
{
    constexpr int rows = 16 * kGemmWaves;
    const int rblocks = (n + rows - 1) / rows;
    k_cgemm<NT><<<rblocks * kSlices, kGemmWaves * kWave, 0, s>>>(A, lda, n, B, ldb, ncols, Zp,
                                                                 kslice32_of(n), skip);
}

static void cgemm(const f2* A, int64_t lda, int n, const d2* B, int64_t ldb, int ncols, d2* Zp,
                  hipStream_t s, const int* skip = nullptr)
{
    switch ((ncols + 15) / 16) {
    case 1: launch_cgemm<1>(A, lda, n, B, ldb, ncols, Zp, s, skip); break;
    case 2: launch_cgemm<2>(A, lda, n, B, ldb, ncols, Zp, s, skip); break;
    case 3: launch_cgemm<3>(A, lda, n, B, ldb, ncols, Zp, s, skip); break;
    default: launch_cgemm<4>(A, lda, n, B, ldb, ncols, Zp, s, skip); break;
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
    const f2* A32;                   // complex64 A: products on FP32 matrix cores
    int64_t lda32;
    int* done;                       // solve alone: set once every column has finished
};

constexpr size_t kStateStride = 256;
static_assert(sizeof(SolverState) <= kStateStride, "column record");

__device__ __forceinline__ SolverState& col_state(const BArgs& a, int j)
{
    return *(SolverState*)((char*)a.cst + (size_t)j * kStateStride);
}

// Element loop of the column-wise kernels: every thread keeps one column
// (kp divides the block size), rows advance by nblk * kBlock / kp.  bid and
// nblk are the block's index and the block count of the system it works on
// (the grid itself, or the system's share of a batched grid).
#define COL_LOOP(a)                                                              \
    const int j = threadIdx.x & ((a).kp - 1);                                    \
    const int64_t total = (int64_t)(a).n * (a).kp;                               \
    for (int64_t e = (int64_t)bid * kBlock + threadIdx.x; e < total;             \
         e += (int64_t)nblk * kBlock)

// Per-block column partials: threads of the same column add in thread order.
__device__ __forceinline__ void col_partials(const BArgs& a, int bid, d2 v0, d2 v1)
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
        a.cpart[((size_t)bid * a.kp + t) * 2] = s0;
        a.cpart[((size_t)bid * a.kp + t) * 2 + 1] = s1;
    }
}

// Column records of a new solve: thread j (of at least kp) writes record j.
__device__ __forceinline__ void kb_init_body(const BArgs& a, int maxit, double tol2,
                                             int no_confirm)
{
    const int j = threadIdx.x;
    if (j == 0 && a.done) *a.done = 0;
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
    o.no_confirm = no_confirm;
    o.pad1 = o.pad2 = 0;
    o.ny2 = o.thr2 = o.rh2 = o.rr = o.gamma = 0.0;
    o.tol2 = tol2;
    o.relres_rec = o.relres_true = __builtin_nan("");
    o.rho = o.rho_old = o.alpha = o.omega = o.beta = d2{0.0, 0.0};
    col_state(a, j) = o;
}

__global__ void kb_init(BArgs a, int maxit, double tol2, int no_confirm)
{
    kb_init_body(a, maxit, tol2, no_confirm);
}

// Column step: finish the column reductions of the previous kernel (nparts
// blocks) and apply the scalar step of `stage` to every column that has one.
// With ring_slot (pinned host word) and/or dev_flag (device word), also
// report whether every column has finished.
__device__ __forceinline__ void kb_step_body(const BArgs& a, int stage, int nparts,
                                             int* ring_slot, int* dev_flag = nullptr)
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
    if (ring_slot || dev_flag) {
        __syncthreads();
        if (threadIdx.x == 0) {
            int all = 1;
            for (int c = 0; c < a.kp; ++c) all &= done[c];
            if (ring_slot)
                __hip_atomic_store(ring_slot, all ? (int)PH_DONE : (int)PH_RUN, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_SYSTEM);
            if (dev_flag) *dev_flag = all;
        }
    }
}

__device__ __forceinline__ void kb_normy_body(const BArgs& a, int bid, int nblk)
{
    d2 v0 = d2{0.0, 0.0};
    COL_LOOP(a)
    {
        if (j < a.k) {
            const int64_t i = e / a.kp;
            v0.x += cabs2(a.Y[i * a.ldy + j]);
        }
    }
    col_partials(a, bid, v0, d2{0.0, 0.0});
}

// x0 = 0: x = 0, r = r^ = y
__device__ __forceinline__ void kb_setup0_body(const BArgs& a, int bid, int nblk)
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
    col_partials(a, bid, v0, d2{0.0, 0.0});
}

// general x0: B = x (x = 0 for y = 0 columns)
__device__ __forceinline__ void kb_setx_body(const BArgs& a, int bid, int nblk)
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
__device__ __forceinline__ void kb_red_setup_body(const BArgs& a, int bid, int nblk)
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
    col_partials(a, bid, v0, d2{0.0, 0.0});
}

// p = r or r + beta (p - omega v); the product input B is p, or x for a
// column that confirms, or 0.
__device__ __forceinline__ void kb_p_body(const BArgs& a, int bid, int nblk)
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
__device__ __forceinline__ void kb_red1_body(const BArgs& a, int bid, int nblk)
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
    col_partials(a, bid, v0, v1);
}

// s = r - alpha v, ||s||^2
__device__ __forceinline__ void kb_s_body(const BArgs& a, int bid, int nblk)
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
    col_partials(a, bid, v0, d2{0.0, 0.0});
}

// after the second product: t = A s (+ t^H s, ||t||^2)
__device__ __forceinline__ void kb_red2_body(const BArgs& a, int bid, int nblk)
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
    col_partials(a, bid, v0, v1);
}

// x += alpha p + omega s, r = s - omega t (+ ||r||^2, r^H r); after a
// half-step exit x += alpha p.  Finished columns are not touched.
__device__ __forceinline__ void kb_xr_body(const BArgs& a, int bid, int nblk)
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
    col_partials(a, bid, v0, v1);
}

// One system per grid.
__global__ __launch_bounds__(kStepThreads) void kb_step(BArgs a, int stage, int nparts,
                                                       int* ring_slot)
{
    kb_step_body(a, stage, nparts, ring_slot, a.done);
}
__global__ __launch_bounds__(kBlock) void kb_normy(BArgs a) { kb_normy_body(a, blockIdx.x, gridDim.x); }
__global__ __launch_bounds__(kBlock) void kb_setup0(BArgs a) { kb_setup0_body(a, blockIdx.x, gridDim.x); }
__global__ __launch_bounds__(kBlock) void kb_setx(BArgs a) { kb_setx_body(a, blockIdx.x, gridDim.x); }
__global__ __launch_bounds__(kBlock) void kb_red_setup(BArgs a) { kb_red_setup_body(a, blockIdx.x, gridDim.x); }
__global__ __launch_bounds__(kBlock) void kb_p(BArgs a) { kb_p_body(a, blockIdx.x, gridDim.x); }
__global__ __launch_bounds__(kBlock) void kb_red1(BArgs a) { kb_red1_body(a, blockIdx.x, gridDim.x); }
__global__ __launch_bounds__(kBlock) void kb_s(BArgs a) { kb_s_body(a, blockIdx.x, gridDim.x); }
__global__ __launch_bounds__(kBlock) void kb_red2(BArgs a) { kb_red2_body(a, blockIdx.x, gridDim.x); }
__global__ __launch_bounds__(kBlock) void kb_xr(BArgs a) { kb_xr_body(a, blockIdx.x, gridDim.x); }

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
    size_t cst, done, cpart, mats, zp, total;
    size_t mat_bytes;
};

static BLayout block_layout(int64_t n, int k)
{
    const int kp = pow2_at_least(k);
    BLayout L{};
    size_t off = 0;
    L.cst = off;
    off += align256(kStateStride * kMaxCols);
    L.done = off;
    off += 256;
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

// Z slices = A B for the block solver: FP64 matrix cores, or the complex64
// copy of A on FP32 matrix cores when the arguments carry one.
static void block_product(const BArgs& a, const d2* B, hipStream_t s)
{
    if (a.A32)
        cgemm(a.A32, a.lda32, a.n, B, a.kp, a.kp, a.Zp, s, a.done);
    else
        gemm(a.A, a.lda, a.n, B, a.kp, a.kp, a.Zp, s, a.done);
}

static int run_block(const BArgs& a, uint32_t flags, int32_t maxit, double tol2,
                     ccg_result* res, hipStream_t s, int no_confirm = 0)
{
    SyncCtx* sc = nullptr;
    hipError_t e = get_sync(&sc);
    if (e != hipSuccess) return (int)e;
    const int gC = col_blocks(a.n, a.kp);

    kb_init<<<1, kMaxCols, 0, s>>>(a, maxit, tol2, no_confirm);
    kb_normy<<<gC, kBlock, 0, s>>>(a);
    kb_step<<<1, kStepThreads, 0, s>>>(a, CS_NORMY, gC, nullptr);
    if (flags & CCG_X0_ZERO) {
        kb_setup0<<<gC, kBlock, 0, s>>>(a);
        kb_step<<<1, kStepThreads, 0, s>>>(a, CS_SETUP0, gC, nullptr);
    } else {
        kb_setx<<<gC, kBlock, 0, s>>>(a);
        block_product(a, a.B, s);
        kb_red_setup<<<gC, kBlock, 0, s>>>(a);
        kb_step<<<1, kStepThreads, 0, s>>>(a, CS_SETUP1, gC, nullptr);
    }
    if ((e = hipGetLastError()) != hipSuccess) return (int)e;

    const int64_t max_slots = 2 * (int64_t)maxit + 4;
    const int ahead = 1;  // a slot holds two matrix products: far longer than enqueueing
    for (int64_t slot = 0; slot < max_slots + ahead; ++slot) {
        if (slot < max_slots) {
            kb_p<<<gC, kBlock, 0, s>>>(a);
            block_product(a, a.B, s);
            kb_red1<<<gC, kBlock, 0, s>>>(a);
            kb_step<<<1, kStepThreads, 0, s>>>(a, CS_P1, gC, nullptr);
            kb_s<<<gC, kBlock, 0, s>>>(a);
            kb_step<<<1, kStepThreads, 0, s>>>(a, CS_S, gC, nullptr);
            block_product(a, a.S, s);
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
    a.done = (int*)(base + L.done);
    return run_block(a, flags, maxit, tol * tol, res, (hipStream_t)stream);
}

}  // namespace ccg


namespace ccg {

// --------------------------------------------------- mixed block solver
//
// FP64 iterative refinement around the block solver run on the complex64
// copy of A (products on FP32 matrix cores, see cgemm_body): per outer step
// R = Y - A X in FP64 (FP64 matrix cores), every column not yet converged
// solves A32 D = R / ||R|| to tol_inner (recursive residual, no
// confirmation) and takes X += ||R|| D in FP64.  The inner Krylov vectors
// stay FP64: they are O(n k) bytes against the O(n^2) of A, whose bytes the
// complex64 copy halves.

struct ColScale {
    double v[kMaxCols];
};

// out[c] = sum over i (in order of blocks of threads) of |M[i][c]|^2
__global__ __launch_bounds__(kBlock) void km_colnorm(const d2* __restrict__ M, int64_t ld,
                                                     int n, double* __restrict__ out)
{
    __shared__ d2 lds[kMaxWaves];
    const int c = blockIdx.x;
    d2 acc = d2{0.0, 0.0};
    for (int i = threadIdx.x; i < n; i += kBlock) acc.x += cabs2(M[(int64_t)i * ld + c]);
    const d2 tot = block_sum(acc, lds);
    if (threadIdx.x == 0) out[c] = tot.x;
}

// R = Y - (sum of the slices of Zp) in columns c < k (Zp null: R = Y); the
// padding columns of R are zero.  R is n x kp, Zp n x k per slice.
__global__ __launch_bounds__(kBlock) void km_resid(const d2* __restrict__ Y, int64_t ldy,
                                                   const d2* __restrict__ Zp, int n, int k,
                                                   int kp, d2* __restrict__ R)
{
    const int64_t total = (int64_t)n * kp;
    for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * kBlock) {
        const int64_t i = e / kp;
        const int c = (int)(e - i * kp);
        d2 r = d2{0.0, 0.0};
        if (c < k) {
            r = Y[i * ldy + c];
            if (Zp) r = r - slice_sum(Zp, n, k, i, c);
        }
        R[e] = r;
    }
}

// Ys = R scaled by column (scale 0 for the columns that sit out)
__global__ __launch_bounds__(kBlock) void km_scale(const d2* __restrict__ R, int n, int kp,
                                                   ColScale sc, d2* __restrict__ Ys)
{
    const int64_t total = (int64_t)n * kp;
    for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * kBlock) {
        const double f = sc.v[e % kp];
        const d2 r = R[e];
        Ys[e] = d2{r.x * f, r.y * f};
    }
}

// An inner solve that met a non-finite value, or broke down before its
// first update (its correction is zero, and the next outer step would repeat
// it), ends the column's refinement: its correction is not applied.
__host__ __device__ __forceinline__ bool inner_ends_refinement(int info, int iters)
{
    return info == 4 || ((info == 2 || info == 3) && iters == 0);
}

// X[:, c] += nr[c] D[:, c] for the columns with nr[c] != 0 (and, when inner
// is not null, whose inner record does not end the refinement); zero:
// X[:, c] = 0 first where zero.v[c] != 0
__global__ __launch_bounds__(kBlock) void km_update(d2* __restrict__ X, int64_t ldx, int n, int k,
                                                    int kp, const d2* __restrict__ D, ColScale nr,
                                                    ColScale zero,
                                                    const char* __restrict__ inner = nullptr)
{
    const int64_t total = (int64_t)n * k;
    for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * kBlock) {
        const int64_t i = e / k;
        const int c = (int)(e - i * k);
        d2* xp = X + i * ldx + c;
        if (zero.v[c] != 0.0) *xp = d2{0.0, 0.0};
        double f = nr.v[c];
        if (inner && f != 0.0) {
            const SolverState* st = (const SolverState*)(inner + (size_t)c * kStateStride);
            if (inner_ends_refinement(st->info, st->iters)) f = 0.0;
        }
        if (f != 0.0) {
            const d2 d = D[i * kp + c];
            *xp = *xp + d2{d.x * f, d.y * f};
        }
    }
}

// Refinement record of a mixed request in the server (device memory): what
// block_mixed_impl keeps on the host, kept here so that the outer steps run
// on the device between batched iterations.
enum MixState { MX_INIT = 0, MX_INNER, MX_FIN };

struct MixRec {
    double ny2[kMaxCols];   // ||y||^2
    double nrm[kMaxCols];   // ||r||^2 of the latest FP64 residual
    double nr[kMaxCols];    // ||r|| of the inner solve now running (0: column sits out)
    double sc[kMaxCols];    // 1 / ||r|| (0: column sits out)
    double relres[kMaxCols];
    int info[kMaxCols], outers[kMaxCols], inner_iters[kMaxCols], mv32[kMaxCols],
        mv64[kMaxCols], live[kMaxCols], zero[kMaxCols];
    int state;              // MixState
    int setup;              // an inner solve starts in this step
    int zeroing;            // x = 0 in the columns zero[] in this step
    int outer;              // FP64 residuals after the first
    int maxit, maxit_inner;
    double tol, tol_inner2;
};

struct BMixLayout {
    BLayout inner;
    size_t R, Ys, D, norms, mix, total;
};

static BMixLayout bmix_layout(int64_t n, int k)
{
    BMixLayout L{};
    L.inner = block_layout(n, k);
    const int kp = pow2_at_least(k);
    const size_t mb = align256((size_t)(n > 0 ? n : 1) * kp * sizeof(d2));
    size_t off = L.inner.total;
    L.R = off;
    off += mb;
    L.Ys = off;
    off += mb;
    L.D = off;
    off += mb;
    L.norms = off;
    off += align256(kMaxCols * sizeof(double));
    L.mix = off;
    off += align256(sizeof(MixRec));
    L.total = off;
    return L;
}

static int elem_blocks(int64_t total)
{
    int64_t b = (total + kBlock - 1) / kBlock;
    if (b > 2048) b = 2048;
    return (int)(b < 1 ? 1 : b);
}

static int block_mixed_impl(int64_t n, int64_t k, const ccg_z* A, int64_t lda, const ccg_c* A32,
                            int64_t lda32, const ccg_z* Y, int64_t ldy, ccg_z* X, int64_t ldx,
                            double tol, int32_t maxit, double tol_inner, int32_t maxit_inner,
                            uint32_t flags, void* work, size_t work_bytes, ccg_mixed_result* res,
                            double* outer_res, void* stream)
{
    if (n < 0 || n > kMaxNB) return -1;
    if (k < 1 || k > kMaxCols) return -2;
    if (n > 0 && !A) return -3;
    if (lda < (n > 1 ? n : 1)) return -4;
    if (n > 0 && !A32) return -5;
    if (lda32 < (n > 1 ? n : 1)) return -6;
    if (n > 0 && !Y) return -7;
    if (ldy < k) return -8;
    if (n > 0 && !X) return -9;
    if (ldx < k) return -10;
    if (!(tol > 0.0) || !std::isfinite(tol)) return -11;
    if (maxit < 0) return -12;
    if (!(tol_inner > 0.0) || !(tol_inner < 1.0)) return -13;
    if (maxit_inner < 1) return -14;
    if (flags & ~CCG_X0_ZERO) return -15;
    if (n > 0 && (!work || ((uintptr_t)work & 255))) return -16;
    const BMixLayout L = bmix_layout(n, (int)k);
    if (n > 0 && work_bytes < L.total) return -17;
    if (!res) return -18;
    for (int64_t j = 0; j < k; ++j) {
        std::memset(&res[j], 0, sizeof res[j]);
        res[j].relres_true = 0.0;
    }
    if (outer_res)
        for (int64_t j = 0; j < k * ((int64_t)maxit + 1); ++j) outer_res[j] = __builtin_nan("");
    if (n == 0) return 0;
    hipStream_t s = (hipStream_t)stream;
    const int kk = (int)k;
    const int kp = pow2_at_least(kk);
    char* base = (char*)work;
    d2* R = (d2*)(base + L.R);
    d2* Ys = (d2*)(base + L.Ys);
    d2* D = (d2*)(base + L.D);
    double* nrm_d = (double*)(base + L.norms);
    // inner solver: A32 D = Ys
    BArgs ai{};
    ai.A = nullptr;
    ai.lda = lda;
    ai.A32 = (const f2*)A32;
    ai.lda32 = lda32;
    ai.n = (int)n;
    ai.k = kk;
    ai.kp = kp;
    ai.Y = Ys;
    ai.ldy = kp;
    ai.X = D;
    ai.ldx = kp;
    d2* m[7];
    for (int q = 0; q < 7; ++q) m[q] = (d2*)(base + L.inner.mats + q * L.inner.mat_bytes);
    ai.R = m[0]; ai.RH = m[1]; ai.P = m[2]; ai.V = m[3]; ai.S = m[4]; ai.T = m[5]; ai.B = m[6];
    ai.Zp = (d2*)(base + L.inner.zp);
    ai.cpart = (d2*)(base + L.inner.cpart);
    ai.cst = (SolverState*)(base + L.inner.cst);
    ai.done = (int*)(base + L.inner.done);

    hipError_t e;
    std::vector<double> nrm(kk), ny2(kk);
    auto colnorms = [&](const d2* M, int64_t ld, double* host) -> int {
        km_colnorm<<<kk, kBlock, 0, s>>>(M, ld, (int)n, nrm_d);
        hipError_t e2 = hipGetLastError();
        if (e2 == hipSuccess)
            e2 = hipMemcpyAsync(host, nrm_d, kk * sizeof(double), hipMemcpyDeviceToHost, s);
        if (e2 == hipSuccess) e2 = hipStreamSynchronize(s);
        return (int)e2;
    };
    int rc = colnorms((const d2*)Y, ldy, ny2.data());
    if (rc) return rc;
    // columns still iterating
    std::vector<char> live(kk, 1);
    ColScale zero{}, none{};
    for (int c = 0; c < kk; ++c) {
        if (!std::isfinite(ny2[c])) {  // x left as given
            res[c].info = 4;
            live[c] = 0;
        } else if (ny2[c] == 0.0) {  // x = 0
            zero.v[c] = 1.0;
            live[c] = 0;
        }
    }
    const bool x0zero = (flags & CCG_X0_ZERO) != 0;
    if (x0zero)
        for (int c = 0; c < kk; ++c)
            if (live[c]) zero.v[c] = 1.0;
    // apply the zeroing now so that the residual below sees it
    km_update<<<elem_blocks(n * k), kBlock, 0, s>>>((d2*)X, ldx, (int)n, kk, kp, D, none, zero);
    std::vector<ccg_result> inner(kk);
    for (int outer = 0;; ++outer) {
        if (outer == 0 && x0zero) {
            km_resid<<<elem_blocks(n * kp), kBlock, 0, s>>>((const d2*)Y, ldy, nullptr, (int)n,
                                                            kk, kp, R);
        } else {
            gemm((const d2*)A, lda, (int)n, (const d2*)X, ldx, kk, ai.Zp, s);
            km_resid<<<elem_blocks(n * kp), kBlock, 0, s>>>((const d2*)Y, ldy, ai.Zp, (int)n, kk,
                                                            kp, R);
            for (int c = 0; c < kk; ++c)
                if (live[c]) res[c].matvecs64++;
        }
        if ((e = hipGetLastError()) != hipSuccess) return (int)e;
        if ((rc = colnorms(R, kp, nrm.data()))) return rc;
        ColScale sc{}, nr{};
        int active = 0;
        for (int c = 0; c < kk; ++c) {
            if (!live[c]) continue;
            const double rel = std::sqrt(nrm[c] / ny2[c]);
            res[c].relres_true = rel;
            if (outer_res) outer_res[(int64_t)c * ((int64_t)maxit + 1) + outer] = rel;
            if (!std::isfinite(nrm[c])) {
                res[c].info = 4;
                live[c] = 0;
            } else if (rel <= tol) {
                res[c].info = 0;
                live[c] = 0;
            } else if (outer >= maxit) {
                res[c].info = 1;
                live[c] = 0;
            } else {
                const double r = std::sqrt(nrm[c]);
                sc.v[c] = 1.0 / r;
                nr.v[c] = r;
                ++active;
            }
        }
        if (!active) break;
        km_scale<<<elem_blocks(n * kp), kBlock, 0, s>>>(R, (int)n, kp, sc, Ys);
        if ((e = hipGetLastError()) != hipSuccess) return (int)e;
        rc = run_block(ai, CCG_X0_ZERO, maxit_inner, tol_inner * tol_inner, inner.data(), s, 1);
        if (rc) return rc;
        for (int c = 0; c < kk; ++c) {
            if (nr.v[c] == 0.0) continue;
            res[c].outer++;
            res[c].inner_iters += inner[c].iters;
            res[c].matvecs32 += inner[c].matvecs;
            if (inner_ends_refinement(inner[c].info, inner[c].iters)) {
                res[c].info = inner[c].info;  // x keeps its value
                live[c] = 0;
                nr.v[c] = 0.0;
            }
        }
        km_update<<<elem_blocks(n * k), kBlock, 0, s>>>((d2*)X, ldx, (int)n, kk, kp, D, nr,
                                                          none);
        if ((e = hipGetLastError()) != hipSuccess) return (int)e;
    }
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return (int)e;
    return 0;
}

// --------------------------------------------------------------- serving
//
// Continuous batching of independent block systems.  Every admitted request
// has a record in a device table; each kernel of a batched iteration runs one
// grid over all records: block b finds its record by a binary search over the
// records' first block indices and runs the block solver's body with its
// index within the record's share.  The block partition, reduction order and
// product slices of a request are those of the same request solved alone,
// whatever else is in the batch.  Product shares start at multiples of 8, so
// the slice of a product block is still the XCD it runs on.

constexpr int kServeCols = 16;  // one 16-wide matrix-core tile (or the vector-unit
                                // product for kp <= kVCols) per request
constexpr int kMaxActive = 128;

struct SlotRec {
    BArgs a;
    int c0, gC;  // column-kernel blocks [c0, c0 + gC) of the batched grid
    int g0, gG;  // matrix-core product blocks [g0, g0 + gG) (0 blocks if none)
    int v0, vG;  // vector-unit product blocks [v0, v0 + vG) (FP64, kp <= kVCols)
    int kslice;
    int slot;    // index of the request's done word
    // set-up of the request's current solve (read by the batched set-up only)
    int maxit, no_confirm;
    double tol2;
    // device sources of Y and X still to be copied into the pool by the
    // batched set-up (null when admission copied them)
    const d2 *ysrc, *xsrc;
    int64_t ldys, ldxs;
    // mixed requests (null mix for FP64 ones): the refinement record, Y and
    // X (n x k) and R (n x kp) of the outer loop, the blocks of its FP64
    // residual product [o0, o0 + oG) (slice length kslice64) and of its
    // column norms [q0, q0 + k)
    MixRec* mix;
    const d2* yo;
    d2 *xo, *ro;
    int o0, oG, q0, kslice64;
};

enum RecGrid { RG_COL, RG_MFMA, RG_VALU, RG_OUT, RG_NORM };

// The record whose blocks of grid `which` contain block b: the last record
// starting at or before b (records with no blocks in that grid are skipped).
__device__ __forceinline__ int find_rec(const SlotRec* __restrict__ tab, int m, int b, int which)
{
    int lo = 0, hi = m - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        const int start = which == RG_MFMA ? tab[mid].g0 : which == RG_VALU ? tab[mid].v0
                        : which == RG_OUT ? tab[mid].o0 : which == RG_NORM ? tab[mid].q0
                        : tab[mid].c0;
        if (start <= b)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// A request whose columns have all finished (done word set by the last
// column step) is skipped by every later batched kernel.
#define SERVE_COL_KERNEL(name)                                                        \
    __global__ __launch_bounds__(kBlock) void kv_##name(                              \
        const SlotRec* __restrict__ tab, int m, const int* __restrict__ sdone)        \
    {                                                                                 \
        const SlotRec& r = tab[find_rec(tab, m, blockIdx.x, RG_COL)];                 \
        if (sdone[r.slot]) return;                                                    \
        const BArgs a = r.a;                                                          \
        kb_##name##_body(a, blockIdx.x - r.c0, r.gC);                                 \
    }
SERVE_COL_KERNEL(normy)
SERVE_COL_KERNEL(setup0)
SERVE_COL_KERNEL(p)
SERVE_COL_KERNEL(red1)
SERVE_COL_KERNEL(s)
SERVE_COL_KERNEL(red2)
SERVE_COL_KERNEL(xr)
#undef SERVE_COL_KERNEL

// The product of every record: FP64 records here, the inner solves of mixed
// requests (records with a complex64 A) in kv_cgemm; each kernel's grid
// covers all records and skips the other kind.
__global__ __launch_bounds__(kBlock) void kv_gemm(const SlotRec* __restrict__ tab, int m,
                                                  const int* __restrict__ sdone, int use_s)
{
    __shared__ d2 zl[ZgemmLds<1>::size];  // the larger of the two forms
    const SlotRec& r = tab[find_rec(tab, m, blockIdx.x, RG_MFMA)];
    if (sdone[r.slot] || r.a.A32 || r.gG == 0) return;
    const BArgs a = r.a;
    if (a.kp <= kHalfCols)
        zgemm_body<1, kKS, kWavesPerBlock, true>(a.A, a.lda, a.n, use_s ? a.S : a.B, a.kp, a.kp,
                                                 a.Zp, r.kslice, blockIdx.x - r.g0, zl);
    else
        zgemm_body<1>(a.A, a.lda, a.n, use_s ? a.S : a.B, a.kp, a.kp, a.Zp, r.kslice,
                      blockIdx.x - r.g0, zl);
}

// The FP64 requests of at most kVCols columns: the vector-unit product, as
// gemm() gives it to ccg_bicgstab_block_ex.
__global__ __launch_bounds__(kBlock) void kv_vgemm(const SlotRec* __restrict__ tab, int m,
                                                   const int* __restrict__ sdone, int use_s)
{
    const SlotRec& r = tab[find_rec(tab, m, blockIdx.x, RG_VALU)];
    if (sdone[r.slot] || r.vG == 0) return;
    const BArgs a = r.a;
    const d2* Bm = use_s ? a.S : a.B;
    const int bid = blockIdx.x - r.v0;
    if (a.kp == 1)
        vgemm_body<1>(a.A, a.lda, a.n, Bm, a.kp, a.kp, a.Zp, r.kslice, bid);
    else if (a.kp == 2)
        vgemm_body<2>(a.A, a.lda, a.n, Bm, a.kp, a.kp, a.Zp, r.kslice, bid);
    else
        vgemm_body<4>(a.A, a.lda, a.n, Bm, a.kp, a.kp, a.Zp, r.kslice, bid);
}

__global__ __launch_bounds__(kBlock) void kv_cgemm(const SlotRec* __restrict__ tab, int m,
                                                   const int* __restrict__ sdone, int use_s)
{
    const SlotRec& r = tab[find_rec(tab, m, blockIdx.x, RG_MFMA)];
    if (sdone[r.slot] || !r.a.A32) return;
    const BArgs a = r.a;
    cgemm_body<1>(a.A32, a.lda32, a.n, use_s ? a.S : a.B, a.kp, a.kp, a.Zp, r.kslice,
                  blockIdx.x - r.g0);
}

// The FP64 products of a batched iteration in one grid: blocks [0, tot_g)
// are the matrix-core shares (kv_gemm's), blocks [tot_g, tot_g + tot_v) the
// vector-unit shares (kv_vgemm's).  The complex64 products of mixed requests
// stay in kv_cgemm (its LDS tiles would lower the occupancy of this grid).
// One launch instead of two, but at the larger register count of the two
// bodies (4 wavefronts per SIMD, where kv_gemm has 7).  Measured on the
// 512-request mix: with every grid merged the median latency at 70% load fell
// by a fifth and the capacity (batches of about 30 000 product blocks) by 3%;
// merging grids of up to kMergedProdBlocks blocks keeps the first and loses
// nothing of the second.
constexpr int kMergedProdBlocks = 16384;
__global__ __launch_bounds__(kBlock) void kv_prod(const SlotRec* __restrict__ tab, int m,
                                                  const int* __restrict__ sdone, int use_s,
                                                  int tot_g)
{
    __shared__ d2 zl[ZgemmLds<1>::size];
    const int b = blockIdx.x;
    if (b < tot_g) {
        const SlotRec& r = tab[find_rec(tab, m, b, RG_MFMA)];
        if (sdone[r.slot] || r.a.A32 || r.gG == 0) return;
        const BArgs a = r.a;
        if (a.kp <= kHalfCols)
            zgemm_body<1, kKS, kWavesPerBlock, true>(a.A, a.lda, a.n, use_s ? a.S : a.B, a.kp,
                                                     a.kp, a.Zp, r.kslice, b - r.g0, zl);
        else
            zgemm_body<1>(a.A, a.lda, a.n, use_s ? a.S : a.B, a.kp, a.kp, a.Zp, r.kslice,
                          b - r.g0, zl);
        return;
    }
    const int bv = b - tot_g;
    const SlotRec& r = tab[find_rec(tab, m, bv, RG_VALU)];
    if (sdone[r.slot] || r.vG == 0) return;
    const BArgs a = r.a;
    const d2* Bm = use_s ? a.S : a.B;
    const int bid = bv - r.v0;
    if (a.kp == 1)
        vgemm_body<1>(a.A, a.lda, a.n, Bm, a.kp, a.kp, a.Zp, r.kslice, bid);
    else if (a.kp == 2)
        vgemm_body<2>(a.A, a.lda, a.n, Bm, a.kp, a.kp, a.Zp, r.kslice, bid);
    else
        vgemm_body<4>(a.A, a.lda, a.n, Bm, a.kp, a.kp, a.Zp, r.kslice, bid);
}

// A32 = complex64(A), n x n, A32 dense (lda32 = n); round to nearest
__global__ __launch_bounds__(kBlock) void km_round(const d2* __restrict__ A, int64_t lda, int n,
                                                   f2* __restrict__ A32)
{
    const int64_t total = (int64_t)n * n;
    for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * kBlock) {
        const int64_t i = e / n;
        const d2 v = A[i * lda + (e - i * n)];
        A32[e] = f2{(float)v.x, (float)v.y};
    }
}

// One block per record.  With ring (pinned, one word per slot), the step also
// reports the request's all-done state to the host and to the done word.
__global__ __launch_bounds__(kStepThreads) void kv_step(const SlotRec* __restrict__ tab,
                                                        int* sdone, int stage, int* ring)
{
    const SlotRec& r = tab[blockIdx.x];
    if (sdone[r.slot]) return;
    const BArgs a = r.a;
    // a mixed request's word tells the host when its refinement is over
    // (ko_decide), not when an inner solve ends
    kb_step_body(a, stage, r.gC, ring && !r.mix ? ring + r.slot : nullptr,
                 ring ? sdone + r.slot : nullptr);
}

// Copy of Y and X (n x k, device sources) into a request's pool matrices
// (leading dimension k), for the records of the batched set-up that have
// them; the column-kernel shares of the set-up table split the elements.
__global__ __launch_bounds__(kBlock) void kv_copy_in(const SlotRec* __restrict__ tab, int m)
{
    const SlotRec& r = tab[find_rec(tab, m, blockIdx.x, RG_COL)];
    if (!r.ysrc) return;
    const int bid = blockIdx.x - r.c0;
    const int k = r.a.k;
    const int64_t total = (int64_t)r.a.n * k;
    for (int64_t e = (int64_t)bid * kBlock + threadIdx.x; e < total;
         e += (int64_t)r.gC * kBlock) {
        const int64_t i = e / k;
        const int64_t j = e - i * k;
        r.a.X[e] = r.xsrc[i * r.ldxs + j];
        const_cast<d2*>(r.a.Y)[e] = r.ysrc[i * r.ldys + j];
    }
}

// First kernel of the batched set-up of the solves that start in a step (a
// table of their records, one block each): the request's done word is
// cleared and its column records written, as kb_init does for a solve alone.
// The set-up continues with kv_normy, kv_step (CS_NORMY), kv_setup0 and
// kv_step (CS_SETUP0) over the same table.
__global__ __launch_bounds__(kMaxCols) void kv_setup_init(const SlotRec* __restrict__ tab,
                                                          int* sdone)
{
    const SlotRec& r = tab[blockIdx.x];
    if (threadIdx.x == 0) sdone[r.slot] = 0;
    const BArgs a = r.a;
    kb_init_body(a, r.maxit, r.tol2, r.no_confirm);
}

// ---------------------------------- mixed requests: the outer loop on the device
//
// A mixed request runs block_mixed_impl's refinement with x0 = 0, each step
// of it as a batched kernel over the table, so that no outer step waits for
// the host.  In every batched iteration, before the inner iteration kernels:
//   ko_update  x += ||r|| D for the records whose inner solve has ended
//              (their done word is set), skipping columns whose inner record
//              ends the refinement
//   ko_gemm    their FP64 residual product A X (the product gemm() picks)
//   ko_resid   R = Y - A X (R = Y for a record just admitted)
//   ko_colnorm ||R[:, c]||^2, one block per column as km_colnorm
//   ko_decide  one block per record: the inner solve's counts, then per
//              column converged / outer budget spent / non-finite, the
//              scales, and the column records of the next inner solve
//   ko_scale   Ys = R / ||R|| (and x = 0 for a record just admitted)
//   ko_normy, ko_step (CS_NORMY), ko_setup0, ko_step (CS_SETUP0): the set-up
//              of the next inner solve, as the batched set-up runs it
// The arithmetic of each step is block_mixed_impl's, element for element, so
// a request's x equals the solver run alone bit for bit.

// Which part of the refinement record r takes in this iteration: 1 its first
// residual (just admitted), 2 an outer step (its inner solve has ended), 0
// none (inner solve running, or finished).
__device__ __forceinline__ int mix_turn(const SlotRec& r, const int* sdone)
{
    if (!r.mix) return 0;
    const int st = r.mix->state;
    return st == MX_INIT ? 1 : (st == MX_INNER && sdone[r.slot]) ? 2 : 0;
}

// A mixed request's record on admission (one block of kMaxCols threads); the
// done word stays set until the first inner solve starts.
__global__ __launch_bounds__(kMaxCols) void ko_init(MixRec* x, int k, int maxit, int maxit_inner,
                                                    double tol, double tol_inner2, int* sdone)
{
    const int c = threadIdx.x;
    x->ny2[c] = x->nrm[c] = x->nr[c] = x->sc[c] = x->relres[c] = 0.0;
    x->info[c] = x->outers[c] = x->inner_iters[c] = x->mv32[c] = x->mv64[c] = 0;
    x->live[c] = c < k ? 1 : 0;
    x->zero[c] = 0;
    if (c == 0) {
        x->state = MX_INIT;
        x->setup = x->zeroing = 0;
        x->outer = 0;
        x->maxit = maxit;
        x->maxit_inner = maxit_inner;
        x->tol = tol;
        x->tol_inner2 = tol_inner2;
        *sdone = 1;
    }
}

__global__ __launch_bounds__(kBlock) void ko_update(const SlotRec* __restrict__ tab, int m,
                                                    const int* __restrict__ sdone)
{
    const SlotRec& r = tab[find_rec(tab, m, blockIdx.x, RG_COL)];
    if (mix_turn(r, sdone) != 2) return;
    const BArgs a = r.a;
    const MixRec* x = r.mix;
    const int k = a.k, kp = a.kp;
    const int64_t total = (int64_t)a.n * k;
    for (int64_t e = (int64_t)(blockIdx.x - r.c0) * kBlock + threadIdx.x; e < total;
         e += (int64_t)r.gC * kBlock) {
        const int64_t i = e / k;
        const int c = (int)(e - i * k);
        double f = x->nr[c];
        if (f != 0.0) {
            const SolverState& st = col_state(a, c);
            if (inner_ends_refinement(st.info, st.iters)) f = 0.0;
        }
        if (f != 0.0) {
            d2* xp = r.xo + i * k + c;
            const d2 d = a.X[i * kp + c];
            *xp = *xp + d2{d.x * f, d.y * f};
        }
    }
}

__global__ __launch_bounds__(kBlock) void ko_gemm(const SlotRec* __restrict__ tab, int m,
                                                  const int* __restrict__ sdone)
{
    __shared__ d2 zl[ZgemmLds<1>::size];
    const SlotRec& r = tab[find_rec(tab, m, blockIdx.x, RG_OUT)];
    if (r.oG == 0 || mix_turn(r, sdone) != 2) return;
    const BArgs a = r.a;
    const int bid = blockIdx.x - r.o0;
    if (a.k == 1)
        vgemm_body<1>(a.A, a.lda, a.n, r.xo, 1, 1, a.Zp, r.kslice64, bid);
    else if (a.k == 2)
        vgemm_body<2>(a.A, a.lda, a.n, r.xo, 2, 2, a.Zp, r.kslice64, bid);
    else if (a.k <= kVCols)
        vgemm_body<4>(a.A, a.lda, a.n, r.xo, a.k, a.k, a.Zp, r.kslice64, bid);
    else if (a.k <= kHalfCols)
        zgemm_body<1, kKS, kWavesPerBlock, true>(a.A, a.lda, a.n, r.xo, a.k, a.k, a.Zp,
                                                 r.kslice64, bid, zl);
    else
        zgemm_body<1>(a.A, a.lda, a.n, r.xo, a.k, a.k, a.Zp, r.kslice64, bid, zl);
}

__global__ __launch_bounds__(kBlock) void ko_resid(const SlotRec* __restrict__ tab, int m,
                                                   const int* __restrict__ sdone)
{
    const SlotRec& r = tab[find_rec(tab, m, blockIdx.x, RG_COL)];
    const int turn = mix_turn(r, sdone);
    if (!turn) return;
    const BArgs a = r.a;
    const int n = a.n, k = a.k, kp = a.kp;
    const int64_t total = (int64_t)n * kp;
    for (int64_t e = (int64_t)(blockIdx.x - r.c0) * kBlock + threadIdx.x; e < total;
         e += (int64_t)r.gC * kBlock) {
        const int64_t i = e / kp;
        const int c = (int)(e - i * kp);
        d2 v = d2{0.0, 0.0};
        if (c < k) {
            v = r.yo[i * k + c];
            if (turn == 2) v = v - slice_sum(a.Zp, n, k, i, c);
        }
        r.ro[e] = v;
    }
}

__global__ __launch_bounds__(kBlock) void ko_colnorm(const SlotRec* __restrict__ tab, int m,
                                                     const int* __restrict__ sdone)
{
    __shared__ d2 lds[kMaxWaves];
    const SlotRec& r = tab[find_rec(tab, m, blockIdx.x, RG_NORM)];
    if (!mix_turn(r, sdone)) return;
    const int c = blockIdx.x - r.q0;
    const int n = r.a.n, kp = r.a.kp;
    d2 acc = d2{0.0, 0.0};
    for (int i = threadIdx.x; i < n; i += kBlock) acc.x += cabs2(r.ro[(int64_t)i * kp + c]);
    const d2 tot = block_sum(acc, lds);
    if (threadIdx.x == 0) r.mix->nrm[c] = tot.x;
}

// One block of kMaxCols threads per record (thread c: column c).  ring: this
// iteration's row of host-visible done words.
__global__ __launch_bounds__(kMaxCols) void ko_decide(const SlotRec* __restrict__ tab, int* sdone,
                                                      int* ring)
{
    __shared__ int act;
    const SlotRec& r = tab[blockIdx.x];
    if (!r.mix) return;
    MixRec* x = r.mix;
    const int turn = mix_turn(r, sdone);
    const int c = threadIdx.x;
    const BArgs a = r.a;
    if (c == 0) act = 0;
    __syncthreads();  // every thread has read the state and the done word
    if (c == 0) x->setup = x->zeroing = 0;
    if (turn && c < a.k) {
        if (turn == 1) {  // y's norms (R = y, x0 = 0); x = 0 where y is finite
            const double v = x->nrm[c];
            x->ny2[c] = v;
            if (!__builtin_isfinite(v)) {  // x left as given
                x->info[c] = 4;
                x->live[c] = 0;
            } else {  // y = 0: x = 0, info 0, done
                x->zero[c] = 1;
                if (v == 0.0) x->live[c] = 0;
            }
        } else if (x->nr[c] != 0.0) {  // the inner solve this column took part in
            const SolverState& st = col_state(a, c);
            x->outers[c]++;
            x->inner_iters[c] += st.iters;
            x->mv32[c] += st.matvecs;
            if (inner_ends_refinement(st.info, st.iters)) {
                x->info[c] = st.info;  // its correction was not applied
                x->live[c] = 0;
            } else {
                x->mv64[c]++;
            }
        }
        const int outer = turn == 1 ? 0 : x->outer + 1;
        double sc = 0.0, nr = 0.0;
        if (x->live[c]) {
            const double nrm = x->nrm[c];
            const double rel = __builtin_sqrt(nrm / x->ny2[c]);
            x->relres[c] = rel;
            if (!__builtin_isfinite(nrm)) {
                x->info[c] = 4;
                x->live[c] = 0;
            } else if (rel <= x->tol) {
                x->info[c] = 0;
                x->live[c] = 0;
            } else if (outer >= x->maxit) {
                x->info[c] = 1;
                x->live[c] = 0;
            } else {
                nr = __builtin_sqrt(nrm);
                sc = 1.0 / nr;
                atomicOr(&act, 1);
            }
        }
        x->sc[c] = sc;
        x->nr[c] = nr;
    }
    __syncthreads();
    if (turn) {
        if (act) {  // the next inner solve: column records, done word cleared
            kb_init_body(a, x->maxit_inner, x->tol_inner2, 1);
            if (c == 0) {
                x->setup = 1;
                x->state = MX_INNER;
                sdone[r.slot] = 0;
            }
        } else if (c == 0) {
            x->state = MX_FIN;
        }
        if (c == 0) {
            if (turn == 2) x->outer++;
            x->zeroing = turn == 1;
        }
    }
    __syncthreads();
    if (c == 0)
        __hip_atomic_store(ring + r.slot, x->state == MX_FIN ? (int)PH_DONE : (int)PH_RUN,
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

__global__ __launch_bounds__(kBlock) void ko_scale(const SlotRec* __restrict__ tab, int m)
{
    const SlotRec& r = tab[find_rec(tab, m, blockIdx.x, RG_COL)];
    if (!r.mix) return;
    const MixRec* x = r.mix;
    const BArgs a = r.a;
    const int k = a.k, kp = a.kp;
    if (x->setup) {
        const int64_t total = (int64_t)a.n * kp;
        for (int64_t e = (int64_t)(blockIdx.x - r.c0) * kBlock + threadIdx.x; e < total;
             e += (int64_t)r.gC * kBlock) {
            const double f = x->sc[e % kp];
            const d2 v = r.ro[e];
            const_cast<d2*>(a.Y)[e] = d2{v.x * f, v.y * f};
        }
    }
    if (x->zeroing) {
        const int64_t total = (int64_t)a.n * k;
        for (int64_t e = (int64_t)(blockIdx.x - r.c0) * kBlock + threadIdx.x; e < total;
             e += (int64_t)r.gC * kBlock)
            if (x->zero[e % k]) r.xo[e] = d2{0.0, 0.0};
    }
}

// The set-up kernels of the batched set-up, for the records whose next inner
// solve starts in this iteration.
__global__ __launch_bounds__(kBlock) void ko_normy(const SlotRec* __restrict__ tab, int m)
{
    const SlotRec& r = tab[find_rec(tab, m, blockIdx.x, RG_COL)];
    if (!r.mix || !r.mix->setup) return;
    const BArgs a = r.a;
    kb_normy_body(a, blockIdx.x - r.c0, r.gC);
}
__global__ __launch_bounds__(kBlock) void ko_setup0(const SlotRec* __restrict__ tab, int m)
{
    const SlotRec& r = tab[find_rec(tab, m, blockIdx.x, RG_COL)];
    if (!r.mix || !r.mix->setup) return;
    const BArgs a = r.a;
    kb_setup0_body(a, blockIdx.x - r.c0, r.gC);
}
__global__ __launch_bounds__(kStepThreads) void ko_step(const SlotRec* __restrict__ tab, int stage)
{
    const SlotRec& r = tab[blockIdx.x];
    if (!r.mix || !r.mix->setup) return;
    const BArgs a = r.a;
    kb_step_body(a, stage, r.gC, nullptr);
}

// First-fit allocator over the pool (offsets and sizes are multiples of 256).
class PoolAlloc {
    std::map<size_t, size_t> free_;  // offset -> bytes
public:
    void init(size_t off, size_t bytes)
    {
        free_.clear();
        if (bytes) free_[off] = bytes;
    }
    bool alloc(size_t bytes, size_t* off)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            const size_t o = it->first, rest = it->second - bytes;
            free_.erase(it);
            if (rest) free_[o + bytes] = rest;
            *off = o;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && off + bytes == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

struct ServeReq {
    int64_t ticket = 0;
    int64_t n = 0;
    int k = 0;
    const d2* A = nullptr;
    int64_t lda = 0;
    const d2* Y = nullptr;
    int64_t ldy = 0;
    d2* X = nullptr;
    int64_t ldx = 0;
    double tol = 0.0;
    int32_t maxit = 0;
    size_t bytes = 0, off = 0;
    int slot = -1;
    int state = CCG_REQ_QUEUED;
    bool retiring = false;      // copy-out enqueued
    bool setup_pending = false; // a solve starts: set-up not yet enqueued
    int64_t ticks = 0, max_ticks = 0, last_tick = -1;
    SlotRec rec{};
    std::vector<ccg_result> res;
    // mixed precision (FP64 refinement around inner solves on complex64 A,
    // its outer loop run by the ko_* kernels of every batched iteration)
    bool mixed = false;
    double tol_inner = 0.0;
    int32_t maxit_inner = 0;
    int64_t solve_id = 0;       // id of the block solve now iterating
    d2* Xd = nullptr;           // pool copy of X
};

// Pool bytes of one request: A, Y, X and the block-solver workspace; a mixed
// request also holds complex64 A and the refinement vectors.
static size_t serve_bytes(int64_t n, int k)
{
    return align256((size_t)n * n * sizeof(d2)) + 2 * align256((size_t)n * k * sizeof(d2)) +
           block_layout(n, k).total;
}

static size_t serve_bytes_mixed(int64_t n, int k)
{
    return align256((size_t)n * n * sizeof(d2)) + align256((size_t)n * n * sizeof(f2)) +
           2 * align256((size_t)n * k * sizeof(d2)) + bmix_layout(n, k).total;
}

}  // namespace ccg

struct ccg_server {
    int device = 0;
    hipStream_t s = nullptr;
    char* pool = nullptr;
    size_t pool_bytes = 0, head = 0;
    int max_active = 0;
    int* sdone_d = nullptr;
    ccg::SlotRec* tab_d = nullptr;
    ccg::PoolAlloc alloc;
    std::deque<ccg::ServeReq*> queue;
    std::deque<int64_t> finished;  // done tickets not yet handed out by next_done
    std::unordered_map<int64_t, ccg::ServeReq*> reqs;
    ccg::ServeReq* slots[ccg::kMaxActive] = {};
    int64_t next_ticket = 1;
    int64_t next_solve = 1;
    // batched iterations: pinned done words [kRing][kMaxActive], one event each
    int* ring_h = nullptr;
    int* ring_d = nullptr;
    hipEvent_t tick_ev[ccg::kRing] = {};
    std::vector<std::pair<int, int64_t>> members[ccg::kRing];  // (slot, solve id)
    int64_t tick = 0, seen = 0;
    // table uploads: pinned staging [kRing][kMaxActive]
    ccg::SlotRec* stage_h = nullptr;
    hipEvent_t stage_ev[ccg::kRing] = {};
    bool stage_pending[ccg::kRing] = {};
    int stage_next = 0;
    std::vector<std::pair<int, int64_t>> table;  // (slot, solve id) of the device table
    // batched set-up: device table of the solves starting in a step, its
    // pinned staging [kRing][kMaxActive] and events
    ccg::SlotRec* stab_d = nullptr;
    ccg::SlotRec* sstage_h = nullptr;
    hipEvent_t sstage_ev[ccg::kRing] = {};
    bool sstage_pending[ccg::kRing] = {};
    int sstage_next = 0;
    int tot_c = 0, tot_g = 0, tot_v = 0;
    // copy-out: pinned column records [kMaxActive][kServeCols]
    char* res_h = nullptr;
    ccg::MixRec* mix_h = nullptr;  // pinned refinement records of retiring mixed requests
    int tot_o = 0, tot_q = 0;      // blocks of the mixed requests' residual products, norms
    hipEvent_t slot_ev[ccg::kMaxActive] = {};
    ccg_server_stats st{};
};

namespace ccg {

// Start a block solve of request r (inner solve of a mixed request, or the
// whole solve of an FP64 one): its set-up joins the batched set-up of the
// next step (serve_setup_batch), after which it iterates.
static int serve_start_solve(ccg_server* S, ServeReq* r, int32_t maxit, double tol2,
                             int no_confirm)
{
    r->rec.maxit = maxit;
    r->rec.tol2 = tol2;
    r->rec.no_confirm = no_confirm;
    r->setup_pending = true;
    r->solve_id = S->next_solve++;
    r->ticks = 0;
    r->max_ticks = 2 * (int64_t)maxit + 4;
    return 0;
}

// True when p is device memory of `device` (then kernels on the server's
// stream may read it in place).
static bool on_device(const void* p, int device)
{
    hipPointerAttribute_t at{};
    if (hipPointerGetAttributes(&at, p) != hipSuccess) {
        (void)hipGetLastError();  // pageable host memory: not an error here
        return false;
    }
    return at.type == hipMemoryTypeDevice && at.device == device;
}

static int serve_admit(ccg_server* S, ServeReq* r, int slot)
{
    const int64_t n = r->n;
    const int k = r->k;
    hipStream_t s = S->s;
    char* base = S->pool + r->off;
    size_t o = 0;
    d2* A = (d2*)(base + o);
    o += align256((size_t)n * n * sizeof(d2));
    f2* A32 = nullptr;
    if (r->mixed) {
        A32 = (f2*)(base + o);
        o += align256((size_t)n * n * sizeof(f2));
    }
    d2* Y = (d2*)(base + o);
    o += align256((size_t)n * k * sizeof(d2));
    d2* X = (d2*)(base + o);
    o += align256((size_t)n * k * sizeof(d2));
    char* w = base + o;
    const BLayout L = block_layout(n, k);
    const int kp = pow2_at_least(k);
    // A in device memory of this GPU is read where it is (the caller keeps it
    // valid and unchanged until the request is done); only host memory is
    // copied into the pool, whose A region stays reserved either way.
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return (int)e;
    const bool borrow = on_device(r->A, S->device);
    const d2* Asrc = borrow ? r->A : A;
    const int64_t lda = borrow ? r->lda : n;
    BArgs a{};
    a.A = Asrc;
    a.lda = lda;
    a.n = (int)n;
    a.k = k;
    a.kp = kp;
    a.Y = Y;
    a.ldy = k;
    a.X = X;
    a.ldx = k;
    d2* m[7];
    for (int q = 0; q < 7; ++q) m[q] = (d2*)(w + L.mats + q * L.mat_bytes);
    a.R = m[0]; a.RH = m[1]; a.P = m[2]; a.V = m[3]; a.S = m[4]; a.T = m[5]; a.B = m[6];
    a.Zp = (d2*)(w + L.zp);
    a.cpart = (d2*)(w + L.cpart);
    a.cst = (SolverState*)(w + L.cst);
    r->Xd = X;
    r->rec.mix = nullptr;
    if (r->mixed) {
        // the block solver runs the inner solves A32 D = Ys; the outer loop
        // keeps Y, X and R
        const BMixLayout M = bmix_layout(n, k);
        a.A32 = A32;
        a.lda32 = n;
        a.Y = (d2*)(w + M.Ys);
        a.ldy = kp;
        a.X = (d2*)(w + M.D);
        a.ldx = kp;
        r->rec.mix = (MixRec*)(w + M.mix);
        r->rec.yo = Y;
        r->rec.xo = X;
        r->rec.ro = (d2*)(w + M.R);
        r->rec.kslice64 = kslice_of(n);
        r->rec.oG = k <= kVCols ? vgemm_blocks(n)
                                : (int)((n + kRowsPerBlock - 1) / kRowsPerBlock) * kSlices;
    }
    const size_t row = (size_t)k * sizeof(d2);
    if (!borrow &&
        (e = hipMemcpy2DAsync(A, n * sizeof(d2), r->A, r->lda * sizeof(d2), n * sizeof(d2), n,
                              hipMemcpyDefault, s)) != hipSuccess)
        return (int)e;
    // x keeps the caller's values in columns the solver never writes.  Y and X
    // in device memory of this GPU (FP64 requests) are copied by the batched
    // set-up, in one kernel for all requests starting in the step; mixed
    // requests need Y at once (its column norms).
    const bool yx_dev = !r->mixed && on_device(r->Y, S->device) && on_device(r->X, S->device);
    if (!yx_dev) {
        if ((e = hipMemcpy2DAsync(Y, row, r->Y, r->ldy * sizeof(d2), row, n, hipMemcpyDefault,
                                  s)) != hipSuccess)
            return (int)e;
        if ((e = hipMemcpy2DAsync(X, row, r->X, r->ldx * sizeof(d2), row, n, hipMemcpyDefault,
                                  s)) != hipSuccess)
            return (int)e;
    }
    r->rec.a = a;
    r->rec.ysrc = yx_dev ? r->Y : nullptr;
    r->rec.xsrc = yx_dev ? r->X : nullptr;
    r->rec.ldys = r->ldy;
    r->rec.ldxs = r->ldx;
    r->rec.gC = col_blocks(n, kp);
    const bool valu = !r->mixed && kp <= kVCols;
    r->rec.gG = valu ? 0 : (int)((n + kRowsPerBlock - 1) / kRowsPerBlock) * kSlices;
    r->rec.vG = valu ? vgemm_blocks(n) : 0;
    r->rec.kslice = r->mixed ? kslice32_of(n) : kslice_of(n);
    r->rec.slot = slot;
    r->slot = slot;
    r->state = CCG_REQ_RUNNING;
    S->slots[slot] = r;
    S->st.admitted++;
    S->st.pool_used += r->bytes;
    if (S->st.pool_used > S->st.pool_peak) S->st.pool_peak = S->st.pool_used;
    int rc;
    if (r->mixed) {
        km_round<<<elem_blocks(n * n), kBlock, 0, s>>>(Asrc, lda, (int)n, A32);
        ko_init<<<1, kMaxCols, 0, s>>>(r->rec.mix, k, r->maxit, r->maxit_inner, r->tol,
                                       r->tol_inner * r->tol_inner, S->sdone_d + slot);
        if ((e = hipGetLastError()) != hipSuccess) return (int)e;
        // the device ends every inner solve within maxit_inner iterations and
        // the refinement within maxit outer steps; this bound only guards
        // against a done word that never arrives
        r->solve_id = S->next_solve++;
        r->ticks = 0;
        r->max_ticks = ((int64_t)r->maxit + 1) * (2 * (int64_t)r->maxit_inner + 6) + 8;
    } else if ((rc = serve_start_solve(S, r, r->maxit, r->tol * r->tol, 0))) {
        return rc;
    }
    return 0;
}

// Enqueue the copy-out of a request whose columns have finished.
static int serve_retire(ccg_server* S, ServeReq* r)
{
    hipStream_t s = S->s;
    const size_t row = (size_t)r->k * sizeof(d2);
    hipError_t e;
    if ((e = hipMemcpy2DAsync(r->X, r->ldx * sizeof(d2), r->Xd, row, row, r->n,
                              hipMemcpyDefault, s)) != hipSuccess)
        return (int)e;
    if (r->mixed) {
        if ((e = hipMemcpyAsync(S->mix_h + r->slot, r->rec.mix, sizeof(MixRec),
                                hipMemcpyDeviceToHost, s)) != hipSuccess)
            return (int)e;
    } else {
        char* dst = S->res_h + (size_t)r->slot * kServeCols * kStateStride;
        if ((e = hipMemcpyAsync(dst, r->rec.a.cst, (size_t)r->k * kStateStride,
                                hipMemcpyDeviceToHost, s)) != hipSuccess)
            return (int)e;
    }
    if ((e = hipEventRecord(S->slot_ev[r->slot], s)) != hipSuccess) return (int)e;
    r->retiring = true;
    return 0;
}

// Requests with an outstanding copy-out: finished ones free their slots and
// pool blocks.  wait: block on them.
static int serve_collect(ccg_server* S, bool wait)
{
    for (int q = 0; q < S->max_active; ++q) {
        ServeReq* r = S->slots[q];
        if (!r || !r->retiring) continue;
        hipError_t e = wait ? hipEventSynchronize(S->slot_ev[q]) : hipEventQuery(S->slot_ev[q]);
        if (e == hipErrorNotReady) continue;
        if (e != hipSuccess) return (int)e;
        r->res.resize(r->k);
        if (r->mixed) {
            const MixRec& x = S->mix_h[q];
            for (int j = 0; j < r->k; ++j) {
                ccg_result& o = r->res[j];
                // a column still live here was cut off by the tick guard
                o.info = x.live[j] && x.state != MX_FIN ? 1 : x.info[j];
                o.iters = x.inner_iters[j];
                o.matvecs = x.mv32[j];
                o.confirms = x.mv64[j];
                o.relres_rec = x.relres[j];
                o.relres_true = x.relres[j];
            }
        } else {
            const char* src = S->res_h + (size_t)q * kServeCols * kStateStride;
            for (int j = 0; j < r->k; ++j) {
                const SolverState& c = *(const SolverState*)(src + (size_t)j * kStateStride);
                ccg_result& o = r->res[j];
                o.info = c.phase == PH_DONE ? c.info : 1;
                o.iters = c.iters;
                o.matvecs = c.matvecs;
                o.confirms = c.confirms;
                o.relres_rec = c.relres_rec;
                o.relres_true = c.relres_true;
            }
        }
        r->state = CCG_REQ_DONE;
        r->retiring = false;
        S->finished.push_back(r->ticket);
        S->alloc.release(r->off, r->bytes);
        S->st.pool_used -= r->bytes;
        S->st.completed++;
        S->slots[q] = nullptr;
    }
    return 0;
}

// Read the done words of tick `seen` (waiting for it): requests that ended
// (a mixed one: its whole refinement) retire.
static int serve_read_tick(ccg_server* S)
{
    const int u = (int)(S->seen % kRing);
    hipError_t e = hipEventSynchronize(S->tick_ev[u]);
    if (e != hipSuccess) return (int)e;
    for (const auto& mt : S->members[u]) {
        ServeReq* r = S->slots[mt.first];
        // the entry must belong to the request's current solve
        if (!r || r->solve_id != mt.second || r->retiring || r->state != CCG_REQ_RUNNING)
            continue;
        const int w = __atomic_load_n(&S->ring_h[u * kMaxActive + mt.first], __ATOMIC_ACQUIRE);
        const bool out_of_budget = r->ticks >= r->max_ticks && r->last_tick == S->seen;
        if (w == PH_DONE || out_of_budget) {
            int rc = serve_retire(S, r);
            if (rc) return rc;
        }
    }
    S->members[u].clear();
    S->seen++;
    return 0;
}

static int serve_upload_table(ccg_server* S, const std::vector<std::pair<int, int64_t>>& want)
{
    const int u = S->stage_next;
    S->stage_next = (S->stage_next + 1) % kRing;
    if (S->stage_pending[u]) {
        hipError_t e = hipEventSynchronize(S->stage_ev[u]);
        if (e != hipSuccess) return (int)e;
        S->stage_pending[u] = false;
    }
    SlotRec* h = S->stage_h + (size_t)u * kMaxActive;
    // the device table lists the largest systems first: every batched grid
    // then ends with the smallest blocks, and its tail is short
    std::vector<int> order(want.size());
    for (size_t i = 0; i < want.size(); ++i) order[i] = (int)i;
    std::stable_sort(order.begin(), order.end(), [&](int p, int q) {
        return S->slots[want[p].first]->n > S->slots[want[q].first]->n;
    });
    int c = 0, g = 0, v = 0, o = 0, nq = 0;
    for (size_t i = 0; i < want.size(); ++i) {
        SlotRec rec = S->slots[want[order[i]].first]->rec;
        rec.c0 = c;
        rec.g0 = g;
        rec.v0 = v;
        rec.o0 = o;
        rec.q0 = nq;
        c += rec.gC;
        g += rec.gG;
        v += rec.vG;
        if (rec.mix) {
            o += rec.oG;
            nq += rec.a.k;
        }
        h[i] = rec;
    }
    S->tot_c = c;
    S->tot_g = g;
    S->tot_v = v;
    S->tot_o = o;
    S->tot_q = nq;
    S->table = want;
    if (want.empty()) return 0;
    hipError_t e = hipMemcpyAsync(S->tab_d, h, want.size() * sizeof(SlotRec),
                                  hipMemcpyHostToDevice, S->s);
    if (e != hipSuccess) return (int)e;
    if ((e = hipEventRecord(S->stage_ev[u], S->s)) != hipSuccess) return (int)e;
    S->stage_pending[u] = true;
    return 0;
}

static bool serve_iterating(const ServeReq* r)
{
    return r && r->state == CCG_REQ_RUNNING && !r->retiring && !r->setup_pending &&
           r->ticks < r->max_ticks;
}

// Enqueue the set-up of every solve that starts now, as one batch: a table of
// their records (column-kernel shares laid out as in the iteration table) and
// five kernels over it, each request's set-up being the one a solve alone runs
// (same block partition, same reduction order).
static int serve_setup_batch(ccg_server* S)
{
    const int u = S->sstage_next;
    SlotRec* h = S->sstage_h + (size_t)u * kMaxActive;
    int m = 0, c = 0;
    bool copy_in = false;
    for (int q = 0; q < S->max_active; ++q) {
        ServeReq* r = S->slots[q];
        if (!r || !r->setup_pending) continue;
        if (m == 0 && S->sstage_pending[u]) {  // staging u is free once its copy ran
            hipError_t e = hipEventSynchronize(S->sstage_ev[u]);
            if (e != hipSuccess) return (int)e;
            S->sstage_pending[u] = false;
        }
        SlotRec rec = r->rec;
        rec.c0 = c;
        c += rec.gC;
        h[m++] = rec;
        copy_in = copy_in || rec.ysrc;
        r->rec.ysrc = r->rec.xsrc = nullptr;  // copied once
        r->setup_pending = false;
    }
    if (m == 0) return 0;
    S->sstage_next = (S->sstage_next + 1) % kRing;
    hipStream_t s = S->s;
    hipError_t e = hipMemcpyAsync(S->stab_d, h, (size_t)m * sizeof(SlotRec),
                                  hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return (int)e;
    if ((e = hipEventRecord(S->sstage_ev[u], s)) != hipSuccess) return (int)e;
    S->sstage_pending[u] = true;
    const SlotRec* tab = S->stab_d;
    if (copy_in) kv_copy_in<<<c, kBlock, 0, s>>>(tab, m);
    kv_setup_init<<<m, kMaxCols, 0, s>>>(tab, S->sdone_d);
    kv_normy<<<c, kBlock, 0, s>>>(tab, m, S->sdone_d);
    kv_step<<<m, kStepThreads, 0, s>>>(tab, S->sdone_d, CS_NORMY, nullptr);
    kv_setup0<<<c, kBlock, 0, s>>>(tab, m, S->sdone_d);
    kv_step<<<m, kStepThreads, 0, s>>>(tab, S->sdone_d, CS_SETUP0, nullptr);
    if ((e = hipGetLastError()) != hipSuccess) return (int)e;
    return 0;
}

// Admission in arrival order while a slot is free and the head fits the pool.
static int serve_admit_queue(ccg_server* S)
{
    while (!S->queue.empty()) {
        int slot = -1;
        for (int q = 0; q < S->max_active && slot < 0; ++q)
            if (!S->slots[q]) slot = q;
        if (slot < 0) break;
        ServeReq* r = S->queue.front();
        size_t off = 0;
        if (!S->alloc.alloc(r->bytes, &off)) {
            // the head waits until retirements free enough of the pool
            S->st.admission_waits++;
            break;
        }
        r->off = off;
        S->queue.pop_front();
        int rc = serve_admit(S, r, slot);
        if (rc) return rc;
    }
    return 0;
}

static int serve_step(ccg_server* S)
{
    int rc;
    hipError_t e;
    // 1. finished copy-outs free their slots and pool blocks; admit
    if ((rc = serve_collect(S, false))) return rc;
    if ((rc = serve_admit_queue(S))) return rc;
    if ((rc = serve_setup_batch(S))) return rc;
    // 2. the table of this iteration: admitted requests still iterating (a
    //    slot may hold another request than in the last table: compare tickets)
    std::vector<std::pair<int, int64_t>> want;
    bool any64 = false, any32 = false, anyv = false;
    for (int q = 0; q < S->max_active; ++q)
        if (serve_iterating(S->slots[q])) {
            want.emplace_back(q, S->slots[q]->solve_id);
            const SlotRec& rec = S->slots[q]->rec;
            (S->slots[q]->mixed ? any32 : rec.vG > 0 ? anyv : any64) = true;
        }
    if (want != S->table && (rc = serve_upload_table(S, want))) return rc;
    // 3. one batched iteration
    if (!want.empty()) {
        while (S->seen + kRing <= S->tick)
            if ((rc = serve_read_tick(S))) return rc;
        const int u = (int)(S->tick % kRing);
        const int m = (int)want.size();
        hipStream_t s = S->s;
        const SlotRec* tab = S->tab_d;
        int* ring = S->ring_d + (size_t)u * kMaxActive;
        if (any32) {  // the outer steps of the mixed requests, then their inner set-ups
            ko_update<<<S->tot_c, kBlock, 0, s>>>(tab, m, S->sdone_d);
            if (S->tot_o > 0) ko_gemm<<<S->tot_o, kBlock, 0, s>>>(tab, m, S->sdone_d);
            ko_resid<<<S->tot_c, kBlock, 0, s>>>(tab, m, S->sdone_d);
            ko_colnorm<<<S->tot_q, kBlock, 0, s>>>(tab, m, S->sdone_d);
            ko_decide<<<m, kMaxCols, 0, s>>>(tab, S->sdone_d, ring);
            ko_scale<<<S->tot_c, kBlock, 0, s>>>(tab, m);
            ko_normy<<<S->tot_c, kBlock, 0, s>>>(tab, m);
            ko_step<<<m, kStepThreads, 0, s>>>(tab, CS_NORMY);
            ko_setup0<<<S->tot_c, kBlock, 0, s>>>(tab, m);
            ko_step<<<m, kStepThreads, 0, s>>>(tab, CS_SETUP0);
        }
        kv_p<<<S->tot_c, kBlock, 0, s>>>(tab, m, S->sdone_d);
        const int tg = any64 ? S->tot_g : 0;
        const int tv = anyv ? S->tot_v : 0;
        const bool merged = tg + tv <= kMergedProdBlocks;
        auto products = [&](int use_s) {
            if (merged) {
                if (tg + tv > 0) kv_prod<<<tg + tv, kBlock, 0, s>>>(tab, m, S->sdone_d, use_s, tg);
            } else {
                if (tg > 0) kv_gemm<<<tg, kBlock, 0, s>>>(tab, m, S->sdone_d, use_s);
                if (tv > 0) kv_vgemm<<<tv, kBlock, 0, s>>>(tab, m, S->sdone_d, use_s);
            }
            if (any32) kv_cgemm<<<S->tot_g, kBlock, 0, s>>>(tab, m, S->sdone_d, use_s);
        };
        products(0);
        kv_red1<<<S->tot_c, kBlock, 0, s>>>(tab, m, S->sdone_d);
        kv_step<<<m, kStepThreads, 0, s>>>(tab, S->sdone_d, CS_P1, nullptr);
        kv_s<<<S->tot_c, kBlock, 0, s>>>(tab, m, S->sdone_d);
        kv_step<<<m, kStepThreads, 0, s>>>(tab, S->sdone_d, CS_S, nullptr);
        products(1);
        kv_red2<<<S->tot_c, kBlock, 0, s>>>(tab, m, S->sdone_d);
        kv_step<<<m, kStepThreads, 0, s>>>(tab, S->sdone_d, CS_T, nullptr);
        kv_xr<<<S->tot_c, kBlock, 0, s>>>(tab, m, S->sdone_d);
        kv_step<<<m, kStepThreads, 0, s>>>(tab, S->sdone_d, CS_XR, ring);
        if ((e = hipGetLastError()) != hipSuccess) return (int)e;
        if ((e = hipEventRecord(S->tick_ev[u], s)) != hipSuccess) return (int)e;
        S->members[u] = want;
        for (const auto& w : want) {
            ServeReq* r = S->slots[w.first];
            r->ticks++;
            r->last_tick = S->tick;
        }
        S->tick++;
        S->st.ticks++;
    }
    // 4. read the stop flags one iteration behind (all of them when idle) and
    //    enqueue the copy-out of what has finished
    const int64_t behind = want.empty() ? 0 : 1;
    while (S->seen + behind < S->tick)
        if ((rc = serve_read_tick(S))) return rc;
    // 5. with nothing left iterating, wait for the copy-outs
    bool iterating = false;
    for (int q = 0; q < S->max_active; ++q)
        iterating = iterating || serve_iterating(S->slots[q]) ||
                    (S->slots[q] && S->slots[q]->setup_pending);
    if (!iterating && (rc = serve_collect(S, true))) return rc;
    int act = 0;
    for (int q = 0; q < S->max_active; ++q)
        if (S->slots[q]) act++;
    S->st.active = act;
    S->st.queued = (int32_t)S->queue.size();
    if (act > S->st.peak_active) S->st.peak_active = act;
    return 0;
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
    if (method == CCG_WS_MATMAT_C64) {
        const int kc = (int)(k < kMaxCols ? k : kMaxCols);
        return zpart_bytes(n > 0 ? n : 1, kc);
    }
    if (method == CCG_WS_BICGSTAB_BLOCK_MIXED && k <= kMaxCols)
        return bmix_layout(n, (int)k).total;
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



int ccg_matmat_c64(int64_t n, int64_t k, const ccg_c* A32, int64_t lda32, const ccg_z* B,
                   int64_t ldb, ccg_z* Z, int64_t ldz, void* work, size_t work_bytes,
                   void* stream)
{
    using namespace ccg;
    if (n < 0 || n > kMaxNB) return -1;
    if (k < 0) return -2;
    if (n > 0 && k > 0 && !A32) return -3;
    if (lda32 < (n > 1 ? n : 1)) return -4;
    if (n > 0 && k > 0 && !B) return -5;
    if (ldb < (k > 1 ? k : 1)) return -6;
    if (n > 0 && k > 0 && !Z) return -7;
    if (ldz < (k > 1 ? k : 1)) return -8;
    if (n == 0 || k == 0) return 0;
    const int kc = (int)(k < kMaxCols ? k : kMaxCols);
    if (!work || ((uintptr_t)work & 255)) return -9;
    if (work_bytes < zpart_bytes(n, kc)) return -10;
    hipStream_t s = (hipStream_t)stream;
    for (int64_t c0 = 0; c0 < k; c0 += kMaxCols) {
        const int nc = (int)(k - c0 < kMaxCols ? k - c0 : kMaxCols);
        cgemm((const f2*)A32, lda32, (int)n, (const d2*)B + c0, ldb, nc, (d2*)work, s);
        int64_t blocks = ((int64_t)n * nc + kBlock - 1) / kBlock;
        if (blocks > 2048) blocks = 2048;
        k_zgemm_sum<<<(int)blocks, kBlock, 0, s>>>((const d2*)work, (int)n, nc, (d2*)Z + c0, ldz);
    }
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? 0 : (int)e;
}

int ccg_bicgstab_block_mixed_ex(int64_t n, int64_t k, const ccg_z* A, int64_t lda,
                                const ccg_c* A32, int64_t lda32, const ccg_z* Y, int64_t ldy,
                                ccg_z* X, int64_t ldx, double tol, int32_t maxit,
                                double tol_inner, int32_t maxit_inner, uint32_t flags, void* work,
                                size_t work_bytes, ccg_mixed_result* res, double* outer_res,
                                void* stream)
{
    return ccg::block_mixed_impl(n, k, A, lda, A32, lda32, Y, ldy, X, ldx, tol, maxit, tol_inner,
                                 maxit_inner, flags, work, work_bytes, res, outer_res, stream);
}

// ------------------------------------------------------------- serving ABI

size_t ccg_server_request_bytes(int64_t n, int64_t k)
{
    if (n < 0 || n > ccg::kMaxNB || k < 1 || k > ccg::kServeCols) return 0;
    return n == 0 ? 0 : ccg::serve_bytes(n, (int)k);
}

size_t ccg_server_request_bytes_mixed(int64_t n, int64_t k)
{
    if (n < 0 || n > ccg::kMaxNB || k < 1 || k > ccg::kServeCols) return 0;
    return n == 0 ? 0 : ccg::serve_bytes_mixed(n, (int)k);
}

int ccg_server_create(void* pool, size_t pool_bytes, int32_t max_active, void* stream,
                      ccg_server** out)
{
    using namespace ccg;
    if (!pool || ((uintptr_t)pool & 255)) return -1;
    const size_t head =
        align256(kMaxActive * sizeof(int)) + 2 * align256(kMaxActive * sizeof(SlotRec));
    if (pool_bytes < head) return -2;
    if (max_active < 1 || max_active > kMaxActive) return -3;
    if (!out) return -5;
    *out = nullptr;
    ccg_server* S = new ccg_server;
    hipError_t e = hipGetDevice(&S->device);
    S->s = (hipStream_t)stream;
    S->pool = (char*)pool;
    S->pool_bytes = pool_bytes;
    S->head = head;
    S->max_active = max_active;
    S->sdone_d = (int*)pool;
    S->tab_d = (SlotRec*)((char*)pool + align256(kMaxActive * sizeof(int)));
    S->stab_d = (SlotRec*)((char*)S->tab_d + align256(kMaxActive * sizeof(SlotRec)));
    S->alloc.init(head, (pool_bytes - head) & ~(size_t)255);
    if (e == hipSuccess)
        e = hipHostMalloc((void**)&S->ring_h, (size_t)kRing * kMaxActive * sizeof(int),
                          hipHostMallocMapped | hipHostMallocCoherent);
    if (e == hipSuccess) e = hipHostGetDevicePointer((void**)&S->ring_d, S->ring_h, 0);
    if (e == hipSuccess)
        e = hipHostMalloc((void**)&S->stage_h, (size_t)kRing * kMaxActive * sizeof(SlotRec),
                          hipHostMallocDefault);
    if (e == hipSuccess)
        e = hipHostMalloc((void**)&S->sstage_h, (size_t)kRing * kMaxActive * sizeof(SlotRec),
                          hipHostMallocDefault);
    if (e == hipSuccess)
        e = hipHostMalloc((void**)&S->res_h, (size_t)kMaxActive * kServeCols * kStateStride,
                          hipHostMallocDefault);
    if (e == hipSuccess)
        e = hipHostMalloc((void**)&S->mix_h, (size_t)kMaxActive * sizeof(MixRec),
                          hipHostMallocDefault);
    for (int q = 0; q < kRing && e == hipSuccess; ++q) {
        e = hipEventCreateWithFlags(&S->tick_ev[q], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&S->stage_ev[q], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&S->sstage_ev[q], hipEventDisableTiming);
    }
    for (int q = 0; q < kMaxActive && e == hipSuccess; ++q)
        e = hipEventCreateWithFlags(&S->slot_ev[q], hipEventDisableTiming);
    if (e != hipSuccess) {
        ccg_server_destroy(S);
        return (int)e;
    }
    *out = S;
    return 0;
}

int ccg_server_destroy(ccg_server* S)
{
    if (!S) return -1;
    hipError_t e = hipStreamSynchronize(S->s);
    for (auto& kv : S->reqs) delete kv.second;
    auto keep = [&e](hipError_t e2) {
        if (e == hipSuccess) e = e2;
    };
    for (int q = 0; q < ccg::kRing; ++q) {
        if (S->tick_ev[q]) keep(hipEventDestroy(S->tick_ev[q]));
        if (S->stage_ev[q]) keep(hipEventDestroy(S->stage_ev[q]));
        if (S->sstage_ev[q]) keep(hipEventDestroy(S->sstage_ev[q]));
    }
    for (int q = 0; q < ccg::kMaxActive; ++q)
        if (S->slot_ev[q]) keep(hipEventDestroy(S->slot_ev[q]));
    if (S->ring_h) keep(hipHostFree(S->ring_h));
    if (S->stage_h) keep(hipHostFree(S->stage_h));
    if (S->sstage_h) keep(hipHostFree(S->sstage_h));
    if (S->res_h) keep(hipHostFree(S->res_h));
    if (S->mix_h) keep(hipHostFree(S->mix_h));
    delete S;
    return e == hipSuccess ? 0 : (int)e;
}

static int server_submit(ccg_server* S, int64_t n, int64_t k, const ccg_z* A, int64_t lda,
                         const ccg_z* Y, int64_t ldy, ccg_z* X, int64_t ldx, double tol,
                         int32_t maxit, bool mixed, double tol_inner, int32_t maxit_inner,
                         int64_t* ticket)
{
    using namespace ccg;
    if (!S) return -1;
    if (n < 0 || n > kMaxNB) return -2;
    if (k < 1 || k > kServeCols) return -3;
    if (n > 0 && !A) return -4;
    if (lda < (n > 1 ? n : 1)) return -5;
    if (n > 0 && !Y) return -6;
    if (ldy < k) return -7;
    if (n > 0 && !X) return -8;
    if (ldx < k) return -9;
    if (!(tol > 0.0) || !std::isfinite(tol)) return -10;
    if (maxit < 0) return -11;
    if (mixed) {
        if (!(tol_inner > 0.0) || !(tol_inner < 1.0)) return -12;
        if (maxit_inner < 1) return -13;
        if (!ticket) return -14;
    } else if (!ticket) {
        return -12;
    }
    const size_t bytes = n == 0 ? 0 : mixed ? serve_bytes_mixed(n, (int)k) : serve_bytes(n, (int)k);
    if (bytes > S->pool_bytes - S->head) {
        S->st.rejected++;
        return CCG_SERVER_REJECTED;
    }
    ServeReq* r = new ServeReq;
    r->ticket = S->next_ticket++;
    r->n = n;
    r->k = (int)k;
    r->A = (const d2*)A;
    r->lda = lda;
    r->Y = (const d2*)Y;
    r->ldy = ldy;
    r->X = (d2*)X;
    r->ldx = ldx;
    r->tol = tol;
    r->maxit = maxit;
    r->mixed = mixed;
    r->tol_inner = tol_inner;
    r->maxit_inner = maxit_inner;
    r->bytes = bytes;
    S->reqs[r->ticket] = r;
    S->st.submitted++;
    if (n == 0) {
        r->state = CCG_REQ_DONE;
        r->res.assign((size_t)k, ccg_result{});
        for (auto& o : r->res) o.relres_rec = o.relres_true = 0.0;
        S->finished.push_back(r->ticket);
        S->st.completed++;
    } else {
        S->queue.push_back(r);
        S->st.queued = (int32_t)S->queue.size();
    }
    *ticket = r->ticket;
    return 0;
}

int ccg_server_submit(ccg_server* S, int64_t n, int64_t k, const ccg_z* A, int64_t lda,
                      const ccg_z* Y, int64_t ldy, ccg_z* X, int64_t ldx, double tol,
                      int32_t maxit, int64_t* ticket)
{
    return server_submit(S, n, k, A, lda, Y, ldy, X, ldx, tol, maxit, false, 0.0, 0, ticket);
}

int ccg_server_submit_mixed(ccg_server* S, int64_t n, int64_t k, const ccg_z* A, int64_t lda,
                            const ccg_z* Y, int64_t ldy, ccg_z* X, int64_t ldx, double tol,
                            int32_t maxit, double tol_inner, int32_t maxit_inner,
                            int64_t* ticket)
{
    return server_submit(S, n, k, A, lda, Y, ldy, X, ldx, tol, maxit, true, tol_inner,
                         maxit_inner, ticket);
}

int ccg_server_step(ccg_server* S, int32_t* active, int32_t* queued)
{
    if (!S) return -1;
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return (int)e;
    if (dev != S->device) return -1;
    int rc = ccg::serve_step(S);
    if (active) *active = S->st.active;
    if (queued) *queued = S->st.queued;
    return rc;
}

int ccg_server_poll(ccg_server* S, int64_t ticket, int32_t* state, ccg_result* res)
{
    if (!S) return -1;
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return -2;
    if (!state) return -3;
    ccg::ServeReq* r = it->second;
    if (r->state == CCG_REQ_DONE && !res) return -4;
    *state = r->state;
    if (r->state == CCG_REQ_DONE) {
        for (int j = 0; j < r->k; ++j) res[j] = r->res[(size_t)j];
        S->reqs.erase(it);
        delete r;
    }
    return 0;
}

int ccg_server_next_done(ccg_server* S, int64_t* ticket)
{
    if (!S) return -1;
    if (!ticket) return -2;
    *ticket = 0;
    while (!S->finished.empty()) {
        const int64_t t = S->finished.front();
        S->finished.pop_front();
        if (S->reqs.count(t)) {  // not released by an earlier poll
            *ticket = t;
            break;
        }
    }
    return 0;
}

int ccg_server_get_stats(const ccg_server* S, ccg_server_stats* out)
{
    if (!S) return -1;
    if (!out) return -2;
    *out = S->st;
    return 0;
}

}  // extern "C"
