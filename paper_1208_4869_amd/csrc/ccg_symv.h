// ccg_symv.h -- y = A x for a complex symmetric A (A^T = A, the matrices of
// COCG and COCR, section 3.4) read from its upper triangle only (elements
// A_ij with j >= i).  Each stored element is loaded once and used twice,
// A_ij x_j for y_i and A_ij x_i for y_j, so a product moves half the bytes
// of the dense one; below the diagonal nothing is read.
//
// Tiling.  The matrix is cut into S x S tiles, S = 64 CW; a block of four
// wavefronts takes one tile (I, J) with J >= I.  Wavefront w streams the
// RW = S / 4 rows I S + w RW, ... of the tile; lane l takes the columns
// J S + l + 64 c (c < CW), so a wavefront reads coalesced 1 KB row segments
// as in the dense product.  Per lane:
//   row part:    v[r] += A_ij x_j   (one accumulator per row of a group)
//   column part: u[c] += A_ij x_i   (one accumulator per column of the lane)
// The rows are taken 8 at a time; the 8 row accumulators are summed over the
// 64 lanes by a transposing butterfly: at each exchange a lane keeps half of
// its rows and sends the other half to its partner, so three exchanges leave
// every lane with a single row, and a plain butterfly over the 8 lanes that
// share it finishes the total.  The column sums of the four wavefronts are
// added in LDS in wavefront order.  In a diagonal tile the lower elements are not
// loaded and the diagonal enters the row part only.
//
// Partials.  Element e of tile K receives one partial from each tile index
// t = 0 .. T-1: the row part of tile (K, t) for t > K, the column part of
// tile (t, K) for t < K, and for t = K the diagonal tile's row part plus its
// column part.  They are stored at P[t n + e]; the product is the sum over t
// in a fixed order, so results are reproducible bit for bit.
//
// Block order: the off-diagonal tiles first, the diagonal tiles (half the
// elements each) last, so that the smallest pieces of work end the launch.
#pragma once

#include "ccg_device.h"

namespace ccg {

constexpr int kSymWaves = 4;  // wavefronts per tile block (kBlock threads)

__host__ __device__ inline int64_t sym_ntiles(int64_t n, int S) { return (n + S - 1) / S; }
__host__ __device__ inline int64_t sym_nblocks(int64_t T) { return T * (T + 1) / 2; }

// Tile edge for an n x n matrix: the largest of 256 and 128 that still
// gives at least 512 tile blocks (two per compute unit), else 64.  Larger
// tiles write fewer partials (n^2 / S of them; the partial stores cost more
// per byte than the streamed reads of A), smaller ones balance the load
// across the compute units.
__host__ __device__ inline int sym_edge(int64_t n)
{
    for (int S = 256; S >= 128; S /= 2)
        if (sym_nblocks(sym_ntiles(n, S)) >= 512) return S;
    return 64;
}

struct SymGeom {
    int S;     // tile edge, 64, 128 or 256
    int T;     // tiles per edge
    d2* part;  // T x n partials
};

// Tile (I, J) of block b: the strictly upper tiles row by row, then the
// diagonal ones.
__device__ __forceinline__ void sym_tile_of(int64_t b, int64_t T, int& I, int& J)
{
    const int64_t noff = T * (T - 1) / 2;
    if (b >= noff) {
        I = J = (int)(b - noff);
        return;
    }
    // strictly upper row r starts at block r (2T - 1 - r) / 2
    auto start = [T](int64_t r) { return r * (2 * T - 1 - r) / 2; };
    const double tt = 2.0 * (double)T - 1.0;
    int64_t r = (int64_t)((tt - sqrt(tt * tt - 8.0 * (double)b)) * 0.5);
    if (r < 0) r = 0;
    if (r > T - 2) r = T - 2;
    while (r > 0 && start(r) > b) --r;
    while (r < T - 2 && start(r + 1) <= b) ++r;
    I = (int)r;
    J = (int)(r + 1 + (b - start(r)));
}

// Value of lane src of a wavefront, in every lane.
__device__ __forceinline__ double bcast_lane(double v, int src)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, src);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), src);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// LDS of one tile block of NW wavefronts.
template <int CW, int NW = kSymWaves>
struct SymTileLds {
    d2 col[NW][kWave * CW];  // column sums per wavefront
    d2 row[kWave * CW];      // row totals of the tile
};

constexpr int kSymGroup = 8;  // rows per step of a wavefront

// Partials of tile (I, J), I <= J, of y = A x (CONJ: y = conj(A) x, which is
// A^H x for a complex symmetric A), into P (layout above).  FULL:
// an off-diagonal tile with every row and column inside the matrix (no
// masks).  Rows and columns past n - 1 are neither loaded nor stored.  A
// wavefront takes its rows G at a time (G * CW loads in flight
// per lane, G = kSymGroup); each group's row sums go through the transposing
// butterfly and land in LDS.
template <int CW, bool FULL, bool CONJ = false, int G = kSymGroup, int NW = kSymWaves>
__device__ __forceinline__ void symv_tile(const d2* __restrict__ A, int64_t lda, int n,
                                          const d2* __restrict__ x, d2* __restrict__ P,
                                          int I, int J, SymTileLds<CW, NW>& lds)
{
    constexpr int S = kWave * CW;
    constexpr int RW = S / NW;
    static_assert(RW % G == 0, "whole row groups");
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int r0 = I * S + wave * RW;  // first row of this wavefront
    const int c0 = J * S;              // first column of the tile
    const d2 zero = d2{0.0, 0.0};

    d2 xj[CW], u[CW];
#pragma unroll
    for (int c = 0; c < CW; ++c) {
        const int j = c0 + kWave * c + lane;
        xj[c] = (FULL || j < n) ? x[j] : zero;
        u[c] = zero;
    }
    const d2 xown = (lane < RW && (FULL || r0 + lane < n)) ? x[r0 + lane] : zero;
    constexpr int kShare = kWave / G;  // lanes holding the same row total
    const int rsel = lane / kShare;

#pragma unroll 1
    for (int g = 0; g < RW; g += G) {
        d2 a[G][CW];
#pragma unroll
        for (int r = 0; r < G; ++r) {
            const int i = r0 + g + r;
            const d2* Ai = A + (int64_t)i * lda + c0 + lane;
#pragma unroll
            for (int c = 0; c < CW; ++c) {
                const int j = c0 + kWave * c + lane;
                a[r][c] = zero;
                if (FULL || (i < n && j < n && j >= i)) a[r][c] = ldnt(Ai + kWave * c);
            }
        }
        d2 v[G];
#pragma unroll
        for (int r = 0; r < G; ++r) {
            const int i = r0 + g + r;
            const d2 xi = d2{bcast_lane(xown.x, g + r), bcast_lane(xown.y, g + r)};
            d2 acc = zero;
#pragma unroll
            for (int c = 0; c < CW; ++c) {
                const int j = c0 + kWave * c + lane;
                const d2 au = (FULL || j != i) ? a[r][c] : zero;
                if (CONJ) {
                    acc = cfma_conj(a[r][c], xj[c], acc);
                    u[c] = cfma_conj(au, xi, u[c]);
                } else {
                    acc = cfma(a[r][c], xj[c], acc);
                    u[c] = cfma(au, xi, u[c]);
                }
            }
            v[r] = acc;
        }
        wave_transpose_sum<G>(v, lane);
        if ((lane & (kShare - 1)) == 0) lds.row[wave * RW + g + rsel] = v[0];
    }
#pragma unroll
    for (int c = 0; c < CW; ++c) lds.col[wave][kWave * c + lane] = u[c];
    __syncthreads();

    for (int t = threadIdx.x; t < S; t += NW * kWave) {
        d2 s = lds.col[0][t];
#pragma unroll
        for (int w = 1; w < NW; ++w) s += lds.col[w][t];
        if (I != J) {
            if (FULL || c0 + t < n) P[(int64_t)I * n + c0 + t] = s;
            if (FULL || I * S + t < n) P[(int64_t)J * n + I * S + t] = lds.row[t];
        } else if (c0 + t < n) {
            P[(int64_t)I * n + c0 + t] = lds.row[t] + s;
        }
    }
}

// The tile of block b (either form).
template <int CW, bool CONJ = false, int G = kSymGroup, int NW = kSymWaves>
__device__ __forceinline__ void symv_block(const d2* __restrict__ A, int64_t lda, int n,
                                           const d2* __restrict__ x, const SymGeom& g,
                                           int64_t b, SymTileLds<CW, NW>& lds)
{
    int I, J;
    sym_tile_of(b, g.T, I, J);
    if (I != J && (int64_t)(J + 1) * (kWave * CW) <= n)
        symv_tile<CW, true, CONJ, G, NW>(A, lda, n, x, g.part, I, J, lds);
    else
        symv_tile<CW, false, CONJ, G, NW>(A, lda, n, x, g.part, I, J, lds);
}

// Sum over t (in order) of the partials P[t n + e] of element
// e = e0 + lane, e0 = the block's first element; every wavefront returns it.
// The four wavefronts take consecutive quarters of t and are added in
// wavefront order.  red: LDS of kSymWaves x 64 entries.
__device__ __forceinline__ d2 symv_gather(const d2* __restrict__ P, int n, int T, int e,
                                          d2 (*red)[kWave])
{
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int qt = (T + kSymWaves - 1) / kSymWaves;
    const int t0 = wave * qt < T ? wave * qt : T;
    const int t1 = t0 + qt < T ? t0 + qt : T;
    d2 s = d2{0.0, 0.0};
    if (e < n)
        for (int t = t0; t < t1; ++t) s += P[(int64_t)t * n + e];
    red[wave][lane] = s;
    __syncthreads();
    d2 tot = red[0][lane];
#pragma unroll
    for (int w = 1; w < kSymWaves; ++w) tot += red[w][lane];
    return tot;
}

}  // namespace ccg
