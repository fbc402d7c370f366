// ccg_gemv.h -- dense complex128 matrix-vector products on gfx950.
//
// y = A x (row-major A): a block of W wavefronts owns R consecutive rows and
// streams them left to right, the wavefronts interleaved over 64-element
// column chunks, one 16-byte element per lane per load.  A is read with
// nontemporal loads so that it streams through the caches without evicting
// x, which is re-read from L2 once per block (R rows).  Each lane accumulates
// a strided partial sum in FP64 with fused multiply-adds; a 64-lane butterfly
// and a fixed-order sum over the block's wavefronts give the row totals.
//
// y = A^H x on the same row-major A: a block owns a tile of 64 columns and a
// band of rows; lane j of each wavefront walks down column j (coalesced 1 KB
// row segments per wavefront), accumulating conj(A_ij) x_i.  The four
// wavefronts of a block split the band into four sub-bands and add their
// sums in a fixed order; a second pass adds the band partials in band order.
// Both products use only fixed summation orders: results are reproducible
// bit for bit from run to run.
#pragma once

#include "ccg_device.h"

namespace ccg {

// Row sums of R rows starting at row0, computed by a block of W wavefronts:
// wavefront w takes the 64-column chunks w, w + W, w + 2W, ... of all R rows,
// U chunks per step (R*U loads of A in flight per lane), so the W wavefronts
// of a block read W adjacent 1 KB segments of the same rows at a time and
// each x chunk is fetched once per block for R rows.  Rows past n - 1 are
// clamped to n - 1 (their sums are discarded by the caller).  On return
// red[w][r] holds wavefront w's sum for row row0 + r; the row total is
// red[0][r] + red[1][r] + ... in wavefront order (gemv_n_row_total).
//
// pre (optional, with U = 1): this wavefront's first chunk of the R rows,
// already in LDS (R x 64 elements, see gemv_n_prefetch); it is used in place
// of loading that chunk, in the same order, so the sums keep their bits.
template <int R, int U, int W>
__device__ __forceinline__ void gemv_n_block(const d2* __restrict__ A, int64_t lda, int n,
                                             const d2* __restrict__ x, int row0,
                                             d2 (*red)[R], const d2* pre = nullptr)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const d2* Ar[R];
    d2 acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int row = row0 + r < n ? row0 + r : n - 1;
        Ar[r] = A + (int64_t)row * lda + lane;
        acc[r] = d2{0.0, 0.0};
    }
    const d2* xl = x + lane;
    const int nfull = n / kWave;  // chunks with 64 valid columns
    int c = wave;
    if (U == 1 && pre && c < nfull) {
        const d2 xv = xl[c * kWave];
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] = cfma(pre[r * kWave + lane], xv, acc[r]);
        c += W;
    }
    for (; c + (U - 1) * W < nfull; c += U * W) {
        d2 a[R][U];
        d2 xv[U];
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int u = 0; u < U; ++u) a[r][u] = ldnt(Ar[r] + (c + u * W) * kWave);
#pragma unroll
        for (int u = 0; u < U; ++u) xv[u] = xl[(c + u * W) * kWave];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int r = 0; r < R; ++r) acc[r] = cfma(a[r][u], xv[u], acc[r]);
    }
    for (; c * kWave < n; c += W) {
        if (c * kWave + lane < n) {
            const d2 xv = xl[c * kWave];
#pragma unroll
            for (int r = 0; r < R; ++r) acc[r] = cfma(ldnt(Ar[r] + c * kWave), xv, acc[r]);
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const d2 s = wave_sum(acc[r]);
        if (lane == 0) red[wave][r] = s;
    }
    __syncthreads();
}

// Start the loads of this wavefront's first 64-column chunk of rows row0 ..
// row0 + R - 1 (chunk `wave`, when it is a full chunk) straight into LDS
// (global_load_lds: no registers held), pre[r * 64 + lane] for row r, so
// they are in flight while the kernel does other work before its product
// (gemv_n_block with pre).  The caller waits for them (s_waitcnt vmcnt(0))
// before the wavefront reads pre or ends.
template <int R>
__device__ __forceinline__ void gemv_n_prefetch(const d2* __restrict__ A, int64_t lda, int n,
                                                int row0, d2* pre)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    if (wave >= n / kWave) return;  // not a full chunk: loaded the plain way
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int row = row0 + r < n ? row0 + r : n - 1;
        const d2* src = A + (int64_t)row * lda + wave * kWave + lane;
        __builtin_amdgcn_global_load_lds((const void*)src,
                                         (__attribute__((address_space(3))) void*)(pre + r * kWave),
                                         16, 0, 0);
    }
}

// Total of row row0 + r from the per-wavefront sums, in wavefront order.
template <int R, int W>
__device__ __forceinline__ d2 gemv_n_row_total(const d2 (*red)[R], int r)
{
    d2 s = red[0][r];
#pragma unroll
    for (int w = 1; w < W; ++w) s += red[w][r];
    return s;
}

// The same block layout for complex64 A and x (the mixed-precision inner
// products): each lane accumulates its strided partial sums in FP32 with
// fused multiply-adds; the cross-lane and cross-wavefront sums are in FP64.
// With vec16 (A 16-byte aligned, lda even, x 16-byte aligned) a lane loads
// two adjacent complex64 per 16-byte load and a wavefront chunk is 128
// columns; otherwise 8-byte loads and 64-column chunks.  Columns past the
// last full chunk are taken one per lane.
__device__ __forceinline__ void cfmaf(f2& acc, f2 a, f2 x)
{
    acc.x = __builtin_fmaf(a.x, x.x, acc.x);
    acc.x = __builtin_fmaf(-a.y, x.y, acc.x);
    acc.y = __builtin_fmaf(a.x, x.y, acc.y);
    acc.y = __builtin_fmaf(a.y, x.x, acc.y);
}

typedef float f4 __attribute__((ext_vector_type(4)));

template <int R, int W>
__device__ __forceinline__ void gemv_n_block_f(const f2* __restrict__ A, int64_t lda, int n,
                                               const f2* __restrict__ x, int row0,
                                               d2 (*red)[R], bool vec16)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const f2* Ar[R];
    f2 acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int row = row0 + r < n ? row0 + r : n - 1;
        Ar[r] = A + (int64_t)row * lda;
        acc[r] = f2{0.0f, 0.0f};
    }
    int jt;  // first column of the per-lane tail
    if (vec16) {
        const int nfull = n / (2 * kWave);
        for (int c = wave; c < nfull; c += W) {
            const int j = c * 2 * kWave + 2 * lane;
            const f4 xv = *(const f4*)(x + j);
            f4 a[R];
#pragma unroll
            for (int r = 0; r < R; ++r) a[r] = __builtin_nontemporal_load((const f4*)(Ar[r] + j));
#pragma unroll
            for (int r = 0; r < R; ++r) {
                cfmaf(acc[r], f2{a[r].x, a[r].y}, f2{xv.x, xv.y});
                cfmaf(acc[r], f2{a[r].z, a[r].w}, f2{xv.z, xv.w});
            }
        }
        jt = nfull * 2 * kWave;
    } else {
        const int nfull = n / kWave;
        for (int c = wave; c < nfull; c += W) {
            const int j = c * kWave + lane;
            const f2 xv = x[j];
            f2 a[R];
#pragma unroll
            for (int r = 0; r < R; ++r) a[r] = ldnt(Ar[r] + j);
#pragma unroll
            for (int r = 0; r < R; ++r) cfmaf(acc[r], a[r], xv);
        }
        jt = nfull * kWave;
    }
    for (int j = jt + wave * kWave + lane; j < n; j += W * kWave) {
        const f2 xv = x[j];
#pragma unroll
        for (int r = 0; r < R; ++r) cfmaf(acc[r], ldnt(Ar[r] + j), xv);
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const d2 s = wave_sum(d2{(double)acc[r].x, (double)acc[r].y});
        if (lane == 0) red[wave][r] = s;
    }
    __syncthreads();
}

// Launch shape of the A x kernels for a given n.
struct GemvNShape {
    int rows_per_wave;
    int blocks;
};

// Launch shape of the A^H x kernels.
struct GemvCShape {
    int ntiles;     // column tiles of 64
    int nbands;     // row bands
    int band_rows;  // rows per band (the last band may be shorter)
    int blocks() const { return ntiles * nbands; }
};

inline GemvCShape gemv_c_shape(int64_t n)
{
    GemvCShape s;
    s.ntiles = (int)((n + kWave - 1) / kWave);
    // about 1000 blocks: enough to fill 256 CUs, few enough that each block
    // walks a long band (fewer partials, longer streams)
    int64_t want = (1024 + s.ntiles - 1) / s.ntiles;
    int64_t cap = (n + 63) / 64;
    int64_t nb = want < cap ? want : cap;
    if (nb < 1) nb = 1;
    s.band_rows = (int)((n + nb - 1) / nb);
    if (s.band_rows < 1) s.band_rows = 1;
    s.nbands = (int)((n + s.band_rows - 1) / s.band_rows);
    if (s.nbands < 1) s.nbands = 1;
    return s;
}

// Partial sums of conj(A_ij) x_i over one band of rows for one 64-column
// tile, written to part[band * n + j].  Block = 4 wavefronts; wavefront w
// takes the w-th quarter of the band.
template <int U>
__device__ __forceinline__ void gemv_c_band(const d2* __restrict__ A, int64_t lda, int n,
                                            const d2* __restrict__ x, d2* __restrict__ part,
                                            GemvCShape sh)
{
    __shared__ d2 red[kWavesPerBlock][kWave];
    const int tile = blockIdx.x % sh.ntiles;
    const int band = blockIdx.x / sh.ntiles;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int col = tile * kWave + lane;
    const int colc = col < n ? col : n - 1;
    const int rb0 = band * sh.band_rows;
    const int rb1 = rb0 + sh.band_rows < n ? rb0 + sh.band_rows : n;
    const int q = (sh.band_rows + kWavesPerBlock - 1) / kWavesPerBlock;
    const int i0 = rb0 + wave * q < rb1 ? rb0 + wave * q : rb1;
    const int i1 = i0 + q < rb1 ? i0 + q : rb1;
    const d2* Ac = A + colc;
    d2 acc = d2{0.0, 0.0};
    int i = i0;
    for (; i + U <= i1; i += U) {
        d2 a[U];
        d2 xv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) a[u] = ldnt(Ac + (int64_t)(i + u) * lda);
#pragma unroll
        for (int u = 0; u < U; ++u) xv[u] = x[i + u];
#pragma unroll
        for (int u = 0; u < U; ++u) acc = cfma_conj(a[u], xv[u], acc);
    }
    for (; i < i1; ++i) acc = cfma_conj(ldnt(Ac + (int64_t)i * lda), x[i], acc);
    red[wave][lane] = acc;
    __syncthreads();
    if (wave == 0 && col < n) {
        d2 s = red[0][lane];
#pragma unroll
        for (int w = 1; w < kWavesPerBlock; ++w) s += red[w][lane];
        part[(int64_t)band * n + col] = s;
    }
}

// z_j = sum over bands b (in order) of part[b * n + j].
__device__ __forceinline__ d2 gemv_c_gather(const d2* __restrict__ part, int n, int nbands, int j)
{
    d2 s = part[j];
    for (int b = 1; b < nbands; ++b) s += part[(int64_t)b * n + j];
    return s;
}

}  // namespace ccg
