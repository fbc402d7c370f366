// ccg_t3.h -- the product with a three-level Toeplitz matrix as a zero-padded
// 3-D FFT convolution, for operators the user defines through their own
// matvec (Usage section: the user's own sparse or structured matrix scheme).
//
// The matrix.  Points of an m x m x m lattice, index i = ix + m iy + m^2 iz;
// A_ij = T(p_i - p_j) for a kernel T given on the displacement box
// [-(m-1), m-1]^3 (the dipole lattice of the benchmark: T(d) = e^{i k |d| -
// |d| / L} / |d| off the diagonal, T(0) the diagonal value).  Then
// (A x)(p) = sum_q T(p - q) x(q), a linear convolution, which equals the
// circular convolution on an M^3 grid with M >= 2m - 1 when x is zero-padded
// and T is wrapped (T(d) stored at d mod M).  Here M is the smallest power of
// two >= max(2m - 1, 16) (at most 256).
//
// The transforms.  A line of M points is held by M/8 threads, 8 points each,
// and transformed by mixed-radix decimation in frequency: phases of radix 8
// (the last one of radix 2, 4 or 8 as log2 M dictates).  A phase of radix R
// on sub-blocks of L points takes, for each offset p1 < L/R of a sub-block,
// the R points p1 + (L/R) p2, forms their R-point DFT in registers (three,
// two or one radix-2 stages with constant twiddles), multiplies output k2 by
// W_L^{p1 k2} (W_L = e^{-2 pi i / L}) and leaves it at p1 + (L/R) k2; the
// next phase works on the sub-blocks of L/R points so formed.  Between
// phases the points move through LDS.  The forward transform so ends in a
// digit-reversed order; every operand of a pointwise product (the kernel's
// transform is made by the same passes) is in that order, and the inverse
// transform undoes the phases in reverse order (conjugate twiddles before
// each inverse R-point DFT), returning natural order, times M.  The factor
// M^3 of the three inverse transforms is folded into the kernel's transform
// at set-up (a power of two: exact).
//
// Tiles.  A workgroup of 256 threads transforms T = 2048 / M whole lines
// (a line never straddles two wavefronts).  The lines of a tile are
// consecutive in the pass's line numbering, which is chosen so that the
// strided side of the pass (the axis being transformed is not the fastest
// of its array) is consecutive lines at a fixed point: those accesses go
// through the LDS tile, T neighbouring values per point, while the
// contiguous side loads or stores each line's run directly.
//
// Passes of one product (x -> y); line numberings:
//   X1: line iy + mp iz,  forward along x; x zero-padded          -> G1[iz][kx][iy]
//   X2: line iz + mp kx,  forward along y                          -> G2[kx][ky][iz]
//   X3: line kx M + ky,   forward along z, times K, inverse along z -> G2 (in place)
//   X4: line iz + mp kx,  inverse along y, keep iy < m              -> G1[iz][kx][iy]
//   X5: line iy + mp iz,  inverse along x, keep ix < m              -> y
// (G1 holds M m mp points, G2 M^2 mp, mp = m rounded up to 8 (the lines
// iy or iz >= m of the numberings are padding and do nothing): only the m
// planes that the zero padding and the final crop leave nonzero are ever
// transformed.)  K is stored per
// line in the order the threads hold it after the forward transform (point
// s of thread u at s M/8 + u), so that X3 reads it with unit stride.
#pragma once

#include "ccg_device.h"

namespace ccg {

constexpr int kT3MinM = 16;   // smallest padded edge (every phase shape has a swizzle)
constexpr int kT3MaxM = 256;  // largest padded edge
constexpr int kT3Pts = 8;     // points per thread

// Padded edge for an m-point lattice edge: the smallest power of two
// >= max(2m - 1, kT3MinM); any such edge gives the same linear convolution.
__host__ __device__ inline int t3_padded(int m)
{
    int M = kT3MinM;
    while (M < 2 * m - 1) M <<= 1;
    return M;
}

template <int M>
struct T3Shape {
    static_assert(M >= kT3MinM && M <= kT3MaxM && (M & (M - 1)) == 0, "padded edge");
    static constexpr int TPL = M / kT3Pts;   // threads per line
    static constexpr int T = kBlock / TPL;    // lines per tile
    static constexpr int LG = M == 16 ? 4 : M == 32 ? 5 : M == 64 ? 6 : M == 128 ? 7 : 8;
    static constexpr int NPH = LG / 3 + (LG % 3 ? 1 : 0);  // phases
    static constexpr int radix(int j) { return j < LG / 3 ? 8 : 1 << (LG % 3); }
    // sub-block length of phase j (every earlier phase has radix 8)
    static constexpr int sublen(int j) { return M >> (3 * j); }
};

// Lines of a pass over `lines` lines.
template <int M>
constexpr int64_t t3_tiles(int64_t lines)
{
    return (lines + T3Shape<M>::T - 1) / T3Shape<M>::T;
}

__host__ __device__ constexpr int t3_bitrev(int j, int R)
{
    return R == 8 ? ((j & 1) << 2) | (j & 2) | ((j >> 2) & 1) : R == 4 ? ((j & 1) << 1) | (j >> 1)
                                                                        : j;
}

// Point (position in the line) of slot s of thread u before phase J
// (natural digit order within the R-point group) and after it (the R-point
// DFT leaves its outputs in bit-reversed slot order).
template <int M, int J>
__device__ __forceinline__ int t3_pos_in(int u, int s)
{
    using S = T3Shape<M>;
    constexpr int R = S::radix(J), L = S::sublen(J), Q = L / R;
    const int g = u + S::TPL * (s / R);
    return (g / Q) * L + (g % Q) + Q * (s % R);
}
template <int M, int J>
__device__ __forceinline__ int t3_pos_out(int u, int s)
{
    using S = T3Shape<M>;
    constexpr int R = S::radix(J);
    return t3_pos_in<M, J>(u, (s / R) * R + t3_bitrev(s % R, R));
}

// LDS index of point p of line il of a tile; a line's row holds M + M/16
// points in both layouts, so that a wavefront's rows are its own in either.
// kPad (the exchanges between phases): one point of padding after every 16,
// which keeps them within two-way bank conflicts and makes every slot's
// index the thread's base plus a constant (an immediate offset of the LDS
// instruction).  Otherwise (the tile's strided loads and stores, consecutive
// threads on consecutive lines): p with its low four bits permuted by higher
// bits of p and by il, which spreads the lines over the banks.
template <int M, bool kPad = false>
__device__ __forceinline__ int t3_lds(int il, int p)
{
    if constexpr (kPad) return il * (M + M / 16) + p + (p >> 4);
    const int f = (((p >> 4) & 3) ^ (((p >> 5) & 3) << 2) ^ (il << 1)) & 15;
    return il * (M + M / 16) + (p ^ f);
}

// Points of the LDS tile of T lines.
template <int M>
constexpr int t3_tile_pts()
{
    return T3Shape<M>::T * (M + M / 16);
}

__device__ __forceinline__ d2 cmul_conj(d2 a, d2 w)  // a * conj(w)
{
    return d2{a.x * w.x + a.y * w.y, a.y * w.x - a.x * w.y};
}

// a * W_N^t (conj: a * conj(W_N^t)) for the small roots of the in-register
// DFTs: N in {2, 4, 8}, t < N/2, both constants after unrolling.
__device__ __forceinline__ d2 t3_wsmall(d2 a, int N, int t, bool conj)
{
    constexpr double c = 0.70710678118654752440;  // sqrt(1/2)
    const int e = t * (8 / N);  // eighths of a turn
    if (e == 0) return a;
    if (e == 2) return conj ? d2{-a.y, a.x} : d2{a.y, -a.x};  // -i (conj: +i)
    if (e == 1)                                               // (1 - i)/sqrt2 (conj: 1 + i)
        return conj ? d2{c * (a.x - a.y), c * (a.x + a.y)} : d2{c * (a.x + a.y), c * (a.y - a.x)};
    // e == 3: (-1 - i)/sqrt2 (conj: -1 + i)
    return conj ? d2{-c * (a.x + a.y), c * (a.x - a.y)} : d2{c * (a.y - a.x), -c * (a.x + a.y)};
}

// R-point DFT of slots [b, b + R): radix-2 decimation in frequency, natural
// order in, bit-reversed order out.
template <int R>
__device__ __forceinline__ void t3_dft(d2 (&v)[kT3Pts], int b)
{
#pragma unroll
    for (int h = R / 2; h >= 1; h >>= 1)
#pragma unroll
        for (int k = 0; k < R; ++k) {
            if (k & h) continue;
            const d2 a = v[b + k], c = v[b + k + h];
            v[b + k] = a + c;
            v[b + k + h] = t3_wsmall(a - c, 2 * h, k & (h - 1), false);
        }
}

// Inverse of t3_dft up to the factor R: bit-reversed in, natural out.
template <int R>
__device__ __forceinline__ void t3_idft(d2 (&v)[kT3Pts], int b)
{
#pragma unroll
    for (int h = 1; h <= R / 2; h <<= 1)
#pragma unroll
        for (int k = 0; k < R; ++k) {
            if (k & h) continue;
            const d2 a = v[b + k], c = t3_wsmall(v[b + k + h], 2 * h, k & (h - 1), true);
            v[b + k] = a + c;
            v[b + k + h] = a - c;
        }
}

// W_M^t for t < M from the table of W_M^t, t < M/2 (W^{t + M/2} = -W^t).
template <int M>
__device__ __forceinline__ d2 t3_tw(const d2* __restrict__ tw, int t)
{
    const d2 w = tw[t & (M / 2 - 1)];
    return (t & (M / 2)) ? d2{-w.x, -w.y} : w;
}

// Twiddle seeds of a thread: for each phase J with twiddles (every phase but
// the last, all of radix 8, one group per thread: p1 = u mod L/8), W_L^{p1}
// and W_L^{4 p1} from the table.  The passes with one transform load them
// at their start, so that their latency overlaps the data loads; the z pass
// (two transforms, more live registers) loads them where each phase needs
// them.
template <int M>
__device__ __forceinline__ void t3_seed(int j, int u, const d2* __restrict__ tw, d2& w1, d2& w4)
{
    const int L = T3Shape<M>::sublen(j);
    const int p1 = u % (L / 8);
    w1 = t3_tw<M>(tw, (M / L) * p1);
    w4 = t3_tw<M>(tw, (M / L) * p1 * 4);
}

template <int M, bool kEager = true>
struct T3Tw {
    static constexpr int NJ = T3Shape<M>::NPH - 1;
    d2 w1[kEager ? NJ : 1], w4[kEager ? NJ : 1];
    const d2* tw;
    int u;
    __device__ __forceinline__ T3Tw(int u_, const d2* __restrict__ tw_) : tw(tw_), u(u_)
    {
        if constexpr (kEager) {
#pragma unroll
            for (int j = 0; j < NJ; ++j) t3_seed<M>(j, u, tw, w1[j], w4[j]);
        }
    }
};

// v[bitrev(k)] times W_L^{p1 k} (kConj: its conjugate), k = 1..7, for phase
// J: W_L^{p1} and W_L^{4 p1} from the seeds, the others as their products
// (each product adds at most a few units of rounding), each applied as soon
// as it is formed so that few stay live.
template <bool kConj>
__device__ __forceinline__ void t3_tmul(d2& x, d2 w)
{
    x = kConj ? cmul_conj(x, w) : cmul(x, w);
}

template <int M, int J, bool kConj, bool kEager>
__device__ __forceinline__ void t3_twiddle(d2 (&v)[kT3Pts], const T3Tw<M, kEager>& sd)
{
    d2 w1, w4;
    if constexpr (kEager) {
        w1 = sd.w1[J];
        w4 = sd.w4[J];
    } else {
        t3_seed<M>(J, sd.u, sd.tw, w1, w4);
    }
    t3_tmul<kConj>(v[t3_bitrev(1, 8)], w1);
    const d2 w2 = cmul(w1, w1);
    t3_tmul<kConj>(v[t3_bitrev(2, 8)], w2);
    const d2 w3 = cmul(w1, w2);
    t3_tmul<kConj>(v[t3_bitrev(3, 8)], w3);
    t3_tmul<kConj>(v[t3_bitrev(4, 8)], w4);
    t3_tmul<kConj>(v[t3_bitrev(5, 8)], cmul(w4, w1));
    t3_tmul<kConj>(v[t3_bitrev(6, 8)], cmul(w4, w2));
    t3_tmul<kConj>(v[t3_bitrev(7, 8)], cmul(w4, w3));
}

// Phase J of the forward transform on the registers of thread u.  kHalf:
// the points >= M/2 are zero (the zero padding: m <= M/2), so in phase 0
// the first radix-2 stage only copies and twiddles.
template <int M, int J, bool kHalf, bool kE>
__device__ __forceinline__ void t3_fphase(d2 (&v)[kT3Pts], const T3Tw<M, kE>& tw)
{
    using S = T3Shape<M>;
    constexpr int R = S::radix(J), L = S::sublen(J);
#pragma unroll
    for (int i = 0; i < kT3Pts / R; ++i) {
        if constexpr (kHalf && J == 0) {
            static_assert(R == 8, "phase 0 has radix 8");
#pragma unroll
            for (int k = 0; k < 4; ++k) v[k + 4] = t3_wsmall(v[k], 8, k, false);
#pragma unroll
            for (int h = 2; h >= 1; h >>= 1)
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    if (k & h) continue;
                    const d2 a = v[k], c = v[k + h];
                    v[k] = a + c;
                    v[k + h] = t3_wsmall(a - c, 2 * h, k & (h - 1), false);
                }
        } else {
            t3_dft<R>(v, i * R);
        }
        if constexpr (L > R) {  // offsets p1 > 0 exist: twiddles W_L^{p1 k2}
            static_assert(R == 8 && kT3Pts / R == 1, "one radix-8 group per thread");
            t3_twiddle<M, J, false>(v, tw);
        }
    }
}

// Inverse of t3_fphase (up to the factor R).  kHalf: only the points < M/2
// of phase 0's output are wanted (the crop to m <= M/2).
template <int M, int J, bool kHalf, bool kE>
__device__ __forceinline__ void t3_iphase(d2 (&v)[kT3Pts], const T3Tw<M, kE>& tw)
{
    using S = T3Shape<M>;
    constexpr int R = S::radix(J), L = S::sublen(J);
#pragma unroll
    for (int i = 0; i < kT3Pts / R; ++i) {
        if constexpr (L > R) t3_twiddle<M, J, true>(v, tw);
        if constexpr (kHalf && J == 0) {
#pragma unroll
            for (int h = 1; h <= 2; h <<= 1)
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    if (k & h) continue;
                    const d2 a = v[k], c = t3_wsmall(v[k + h], 2 * h, k & (h - 1), true);
                    v[k] = a + c;
                    v[k + h] = a - c;
                }
#pragma unroll
            for (int k = 0; k < 4; ++k) v[k] = v[k] + t3_wsmall(v[k + 4], 8, k, true);
        } else {
            t3_idft<R>(v, i * R);
        }
    }
}

// Store the registers at the points they hold after phase J (output side)
// or before it (input side), and read them back for another layout.
template <int M, int J, bool kOut, bool kPad = false>
__device__ __forceinline__ void t3_put(const d2 (&v)[kT3Pts], int u, int il, d2* tile)
{
#pragma unroll
    for (int s = 0; s < kT3Pts; ++s)
        tile[t3_lds<M, kPad>(il, kOut ? t3_pos_out<M, J>(u, s) : t3_pos_in<M, J>(u, s))] = v[s];
}
template <int M, int J, bool kOut, bool kPad = false>
__device__ __forceinline__ void t3_get(d2 (&v)[kT3Pts], int u, int il, const d2* tile)
{
#pragma unroll
    for (int s = 0; s < kT3Pts; ++s)
        v[s] = tile[t3_lds<M, kPad>(il, kOut ? t3_pos_out<M, J>(u, s) : t3_pos_in<M, J>(u, s))];
}

// Between the phases of a transform the points of a line move between
// threads of one wavefront only: ordering the LDS accesses within the
// wavefront suffices (its LDS operations execute in order).
__device__ __forceinline__ void t3_wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Forward transform: natural order in (slot s of thread u = point u + s M/8),
// the last phase's output layout out.
template <int M, bool kHalf, int J = 0, bool kE, bool kPad = true>
__device__ __forceinline__ void t3_forward(d2 (&v)[kT3Pts], int u, int il, d2* tile,
                                           const T3Tw<M, kE>& tw)
{
    t3_fphase<M, J, kHalf>(v, tw);
    if constexpr (J + 1 < T3Shape<M>::NPH) {
        t3_put<M, J, true, kPad>(v, u, il, tile);
        t3_wave_sync();
        t3_get<M, J + 1, false, kPad>(v, u, il, tile);
        t3_wave_sync();
        t3_forward<M, kHalf, J + 1, kE, kPad>(v, u, il, tile, tw);
    }
}

// Inverse transform (times M): the last forward phase's layout in, natural
// order out.
template <int M, bool kHalf, int J = T3Shape<M>::NPH - 1, bool kE, bool kPad = true>
__device__ __forceinline__ void t3_inverse(d2 (&v)[kT3Pts], int u, int il, d2* tile,
                                           const T3Tw<M, kE>& tw)
{
    t3_iphase<M, J, kHalf>(v, tw);
    if constexpr (J > 0) {
        t3_put<M, J, false, kPad>(v, u, il, tile);
        t3_wave_sync();
        t3_get<M, J - 1, true, kPad>(v, u, il, tile);
        t3_wave_sync();
        t3_inverse<M, kHalf, J - 1, kE, kPad>(v, u, il, tile, tw);
    }
}

// Geometry of one structured operator.
struct T3Geom {
    int m, M;
    int mp;          // row length of G1 (iy) and G2 (iz): m rounded up to 8
    const d2* tw;    // M/2 twiddles
    const int* even; // 1: the kernel is even in x and in y (K holds the folded rows)
    const d2* K;     // kernel transform, a row of M per line (register order, scaled by M^-3)
    d2* g1;          // G1[iz][kx][iy]: m M mp points
    d2* g2;          // G2[kx][ky][iz]: M^2 mp points
};

// Frequency held at position q of the forward transform's output: the
// digits of q in the phases' block sizes M/R_0, M/(R_0 R_1), ..., read in
// reverse order (mixed-radix digit reversal).
template <int M>
__device__ __forceinline__ int t3_freq(int q)
{
    using S = T3Shape<M>;
    int k = 0, mul = 1;
#pragma unroll
    for (int j = 0; j < S::NPH; ++j) {
        const int R = S::radix(j), B = S::sublen(j) / R;
        k += ((q / B) % R) * mul;
        mul *= R;
    }
    return k;
}

// Position holding frequency k (the inverse of t3_freq).
template <int M>
__device__ __forceinline__ int t3_pos(int k)
{
    using S = T3Shape<M>;
    int q = 0;
#pragma unroll
    for (int j = 0; j < S::NPH; ++j) {
        const int R = S::radix(j);
        q += (k % R) * (S::sublen(j) / R);
        k /= R;
    }
    return q;
}

// Frequencies in mirror-pair order: 0, M/2, 1, M - 1, 2, M - 2, ...
template <int M>
__device__ __forceinline__ int t3_mirror_seq(int a)
{
    return a == 0 ? 0 : a == 1 ? M / 2 : (a & 1) ? M - (a >> 1) : (a >> 1);
}

// Row of K for the z line at positions (qx, qy).  A kernel with
// T(-dx, dy, dz) = T(dx, dy, dz) = T(dx, -dy, dz) (the lattice kernel, which
// depends on |d| only) has K(-kx, ky, kz) = K(kx, ky, kz) = K(kx, -ky, kz),
// so only the rows of frequencies kx, ky in [0, M/2] are kept: (M/2 + 1)^2
// rows instead of M^2, a quarter of the bytes the z pass streams for K.
template <int M>
__device__ __forceinline__ int t3_krow(int qx, int qy, bool even)
{
    if (!even) return qx * M + qy;
    int fx = t3_freq<M>(qx), fy = t3_freq<M>(qy);
    fx = fx <= M / 2 ? fx : M - fx;
    fy = fy <= M / 2 ? fy : M - fy;
    return fx * (M / 2 + 1) + fy;
}

// Rows of G1 and G2 padded to whole 128-byte lines, so that the T
// neighbouring values a tile moves per point (T a multiple of 8) never
// straddle a cache line.
__host__ __device__ inline int t3_row(int m) { return (m + 7) & ~7; }

// Thread of a tile pass: line il of the tile, index u within the line.
// Indices fit in 32 bits: the largest array, K, has 2^24 points.
template <int M>
struct T3Thread {
    int u, il, line;
    __device__ __forceinline__ T3Thread()
    {
        u = (int)threadIdx.x % T3Shape<M>::TPL;
        il = (int)threadIdx.x / T3Shape<M>::TPL;
        line = (int)blockIdx.x * T3Shape<M>::T + il;
    }
    // natural point of slot s
    __device__ __forceinline__ int point(int s) const { return u + T3Shape<M>::TPL * s; }
};

// The strided side of a tile: thread t moves the points t / T + (256 / T) r
// of the tile's line t % T (consecutive threads on consecutive lines).
template <int M>
struct T3Strided {
    int line, p0;
    __device__ __forceinline__ T3Strided()
    {
        line = (int)blockIdx.x * T3Shape<M>::T + (int)threadIdx.x % T3Shape<M>::T;
        p0 = (int)threadIdx.x / T3Shape<M>::T;
    }
    __device__ __forceinline__ int il() const { return (int)threadIdx.x % T3Shape<M>::T; }
    static constexpr int kStep = kBlock / T3Shape<M>::T;
};

// The registers of every line of the tile through LDS to the strided side:
// point p < np of this thread's strided line goes to out[p * stride]
// (nothing for a padding line: live false).  kNat: the registers hold the
// natural order (an inverse transform's output), else the forward output.
template <int M, bool kNat = false>
__device__ __forceinline__ void t3_tile_store(const T3Thread<M>& th, const d2 (&v)[kT3Pts],
                                              d2* tile, d2* out, int stride, bool live,
                                              int np = M)
{
    using S = T3Shape<M>;
    if constexpr (kNat)
        t3_put<M, 0, false>(v, th.u, th.il, tile);
    else
        t3_put<M, S::NPH - 1, true>(v, th.u, th.il, tile);
    __syncthreads();
    const T3Strided<M> sd;
#pragma unroll
    for (int r = 0; r < kT3Pts; ++r) {
        const int p = sd.p0 + T3Strided<M>::kStep * r;
        const d2 val = tile[t3_lds<M>(sd.il(), p)];
        if (live && p < np) out[p * stride] = val;
    }
}

// The registers of every line of the tile from the strided side (in[p *
// stride] for p < np, zeros beyond and for a padding line) through LDS.
// kNat: natural order (a forward transform's input), else the forward
// output layout (an inverse transform's input).
template <int M, bool kNat = false>
__device__ __forceinline__ void t3_tile_load(const T3Thread<M>& th, d2 (&v)[kT3Pts], d2* tile,
                                             const d2* in, int stride, bool live, int np = M)
{
    using S = T3Shape<M>;
    const T3Strided<M> sd;
    d2 w[kT3Pts];
#pragma unroll
    for (int r = 0; r < kT3Pts; ++r) {
        const int p = sd.p0 + T3Strided<M>::kStep * r;
        w[r] = live && p < np ? in[p * stride] : d2{0.0, 0.0};
    }
#pragma unroll
    for (int r = 0; r < kT3Pts; ++r)
        tile[t3_lds<M>(sd.il(), sd.p0 + T3Strided<M>::kStep * r)] = w[r];
    __syncthreads();
    if constexpr (kNat)
        t3_get<M, 0, false>(v, th.u, th.il, tile);
    else
        t3_get<M, S::NPH - 1, true>(v, th.u, th.il, tile);
    t3_wave_sync();
}

// A line's forward output to a contiguous run out[0, M) (natural position
// order, consecutive threads on consecutive points), through the wavefront's
// own rows of the tile.
template <int M>
__device__ __forceinline__ void t3_row_store(const d2 (&v)[kT3Pts], int u, int il, d2* tile,
                                             d2* out, bool live)
{
    t3_put<M, T3Shape<M>::NPH - 1, true>(v, u, il, tile);
    t3_wave_sync();
#pragma unroll
    for (int s = 0; s < kT3Pts; ++s) {
        const int p = u + T3Shape<M>::TPL * s;
        const d2 val = tile[t3_lds<M>(il, p)];
        if (live) out[p] = val;
    }
    t3_wave_sync();
}

// An inverse transform's input from a contiguous run in[0, M) of forward
// output, through the wavefront's own rows of the tile.
template <int M>
__device__ __forceinline__ void t3_row_load(d2 (&v)[kT3Pts], int u, int il, d2* tile,
                                            const d2* in, bool live)
{
    d2 w[kT3Pts];
#pragma unroll
    for (int s = 0; s < kT3Pts; ++s)
        w[s] = live ? in[u + T3Shape<M>::TPL * s] : d2{0.0, 0.0};
#pragma unroll
    for (int s = 0; s < kT3Pts; ++s) tile[t3_lds<M>(il, u + T3Shape<M>::TPL * s)] = w[s];
    t3_wave_sync();
    t3_get<M, T3Shape<M>::NPH - 1, true>(v, u, il, tile);
    t3_wave_sync();
}

// X1: x (n = m^3) -> G1[(iz M + kx) mp + iy]; line iy + mp iz (iy < m live).
template <int M>
__device__ __forceinline__ void t3_pass_x(const T3Geom g, const d2* __restrict__ in, d2* tile)
{
    const int m = g.m, mp = g.mp;
    const T3Thread<M> th;
    const T3Tw<M> tw(th.u, g.tw);
    const int iy = th.line % mp, iz = th.line / mp;
    const d2* src = in + m * (iy + m * iz);
    d2 v[kT3Pts] = {};
#pragma unroll
    for (int s = 0; s < kT3Pts / 2; ++s) {  // points >= M/2 >= m are padding
        const int ix = th.point(s);
        if (iz < m && iy < m && ix < m) v[s] = src[ix];
    }
    t3_forward<M, true>(v, th.u, th.il, tile, tw);
    const T3Strided<M> sd;
    const int oy = sd.line % mp, oz = sd.line / mp;
    d2* out = g.g1 + oz * M * mp + oy;
    const bool live = oz < m && oy < m;
    t3_tile_store<M>(th, v, tile, out, mp, live);
}

// X2: G1 -> G2[(kx M + ky) mp + iz]; line iz + mp kx (iz < m live).
template <int M>
__device__ __forceinline__ void t3_pass_y(const T3Geom g, d2* tile)
{
    const int m = g.m, mp = g.mp;
    const T3Thread<M> th;
    const T3Tw<M> tw(th.u, g.tw);
    const int iz = th.line % mp, kx = th.line / mp;
    const d2* in = g.g1 + (iz * M + kx) * mp;
    d2 v[kT3Pts] = {};
#pragma unroll
    for (int s = 0; s < kT3Pts / 2; ++s) {
        const int iy = th.point(s);
        if (kx < M && iz < m && iy < m) v[s] = in[iy];
    }
    t3_forward<M, true>(v, th.u, th.il, tile, tw);
    const T3Strided<M> sd;
    const int oz = sd.line % mp, ox = sd.line / mp;
    d2* out = g.g2 + ox * M * mp + oz;
    const bool live = ox < M && oz < m;
    t3_tile_store<M>(th, v, tile, out, mp, live);
}

// X3: along z: forward, times K, inverse; G2 in place; line kx M + ky.  For
// a kernel even in x and y the lines are taken in frequency order with each
// frequency beside its mirror (t3_mirror_seq), so that the up to four lines
// sharing a folded K row run in one workgroup (the mirror in y: the next
// line) or M lines later (the mirror in x: a workgroup M / T later, on the
// same XCD), and the row is read from HBM about once.
template <int M>
__device__ __forceinline__ void t3_pass_z(const T3Geom g, d2* tile)
{
    const int m = g.m;
    const T3Thread<M> th;  // M^2 is a multiple of T: every line exists
    const T3Tw<M, false> tw(th.u, g.tw);
    const bool even = *g.even != 0;
    int qx = th.line / M, qy = th.line % M;
    if (even) {
        qx = t3_pos<M>(t3_mirror_seq<M>(qx));
        qy = t3_pos<M>(t3_mirror_seq<M>(qy));
    }
    d2* row = g.g2 + (qx * M + qy) * g.mp;
    const d2* krow = g.K + t3_krow<M>(qx, qy, even) * M;
    d2 v[kT3Pts];
#pragma unroll
    for (int s = 0; s < kT3Pts / 2; ++s) {  // a clamped load and a select: no branch
        const int iz = th.point(s);
        const d2 val = row[iz < m ? iz : m - 1];
        v[s] = iz < m ? val : d2{0.0, 0.0};
    }
#pragma unroll
    for (int s = kT3Pts / 2; s < kT3Pts; ++s) v[s] = d2{0.0, 0.0};
    t3_forward<M, true, 0, false, true>(v, th.u, th.il, tile, tw);
#pragma unroll
    for (int s = 0; s < kT3Pts; ++s) v[s] = cmul(v[s], krow[th.point(s)]);
    t3_inverse<M, true, T3Shape<M>::NPH - 1, false, true>(v, th.u, th.il, tile, tw);
#pragma unroll
    for (int s = 0; s < kT3Pts / 2; ++s) {  // points < M/2 are the ones kept
        const int iz = th.point(s);
        if (iz < m) row[iz] = v[s];
    }
}

// X4: G2 -> G1 (inverse along y, keep iy < m); line iz + mp kx (iz < m live).
template <int M>
__device__ __forceinline__ void t3_pass_yi(const T3Geom g, d2* tile)
{
    const int m = g.m, mp = g.mp;
    const T3Thread<M> th;
    const T3Tw<M> tw(th.u, g.tw);
    const T3Strided<M> sd;
    const int sz = sd.line % mp, sx = sd.line / mp;
    const d2* in = g.g2 + sx * M * mp + sz;
    const bool live = sx < M && sz < m;
    d2 v[kT3Pts];
    t3_tile_load<M>(th, v, tile, in, mp, live);
    t3_inverse<M, true>(v, th.u, th.il, tile, tw);
    const int iz = th.line % mp, kx = th.line / mp;
    if (kx >= M || iz >= m) return;
    d2* out = g.g1 + (iz * M + kx) * mp;
#pragma unroll
    for (int s = 0; s < kT3Pts / 2; ++s) {
        const int iy = th.point(s);
        if (iy < m) out[iy] = v[s];
    }
}

// X5: G1 -> the product for the points ix < m of line iy + mp iz.  Returns
// the lattice line iy + m iz (or -1 for a padding line or one past the
// last); v[s], s < 4, is the product at point ix = th.point(s) when ix < m
// (the other slots hold no output).
template <int M>
__device__ __forceinline__ int t3_pass_xi(const T3Geom g, const T3Thread<M>& th,
                                          d2 (&v)[kT3Pts], d2* tile)
{
    const int m = g.m, mp = g.mp;
    const T3Tw<M> tw(th.u, g.tw);
    const T3Strided<M> sd;
    const int sy = sd.line % mp, sz = sd.line / mp;
    const d2* in = g.g1 + sz * M * mp + sy;
    const bool live = sz < m && sy < m;
    t3_tile_load<M>(th, v, tile, in, mp, live);
    t3_inverse<M, true>(v, th.u, th.il, tile, tw);
    const int iy = th.line % mp, iz = th.line / mp;
    return iz < m && iy < m ? iy + m * iz : -1;
}

// ------------------------------------------------ small lattices (M <= 64)
//
// With m <= 32 every pass above is a few microseconds of latency, so the
// product takes three launches instead of five, one workgroup of 512
// threads per z-plane for the x and y transforms (each in one round of
// lines), whose plane stays in LDS:
//   XY: plane iz: forward along x (m lines), the plane (kx, iy) in LDS,
//       forward along y (M lines)                        -> G2s[iz][kx][ky]
//   Z:  lines kx M + ky: forward along z, times K, inverse (the strided
//       side is iz: loads and stores through the tile)   -> G2s (in place)
//   YX: plane iz: inverse along y (M lines, keep iy < m), the plane (iy, kx)
//       in LDS, inverse along x (m lines, keep ix < m)   -> y
// G2s holds m M^2 points (within the G2 region of the general path).

constexpr int kT3SmallM = 64;      // largest padded edge of the three-launch path
constexpr int kT3PlaneThreads = 512;  // XY / YX workgroup: every y line of a plane in one round

template <int M>
struct T3PlaneShape {
    static constexpr int TL = kT3PlaneThreads / T3Shape<M>::TPL;  // lines per round
    static_assert(TL >= M, "one round holds the y lines of a plane");
};
template <int M>
using T3PlaneTile = d2[T3PlaneShape<M>::TL * (M + M / 16)];
template <int M>
using T3Plane = d2[(M / 2) * M];  // m <= M/2 rows of M points

// XY for plane blockIdx.x.
template <int M>
__device__ __forceinline__ void t3s_xy(const T3Geom g, const d2* __restrict__ in, d2* tile,
                                       d2* plane)
{
    using S = T3Shape<M>;
    const int m = g.m, iz = blockIdx.x;
    const int u = (int)threadIdx.x % S::TPL, il = (int)threadIdx.x / S::TPL;
    const T3Tw<M> tw(u, g.tw);
    // x lines iy = il < m
    d2 v[kT3Pts] = {};
    const d2* src = in + m * (il + m * iz);
#pragma unroll
    for (int s = 0; s < kT3Pts / 2; ++s) {
        const int ix = u + S::TPL * s;
        if (il < m && ix < m) v[s] = src[ix];
    }
    t3_forward<M, true>(v, u, il, tile, tw);
    // plane[kx][iy]: row kx of M/2 points
    if (il < m) {
#pragma unroll
        for (int s = 0; s < kT3Pts; ++s)
            plane[t3_pos_out<M, S::NPH - 1>(u, s) * (M / 2) + il] = v[s];
    }
    __syncthreads();
    // y lines kx = il < M
    const int kx = il;
#pragma unroll
    for (int s = 0; s < kT3Pts; ++s) v[s] = d2{0.0, 0.0};
#pragma unroll
    for (int s = 0; s < kT3Pts / 2; ++s) {
        const int iy = u + S::TPL * s;
        if (kx < M && iy < m) v[s] = plane[kx * (M / 2) + iy];
    }
    t3_forward<M, true>(v, u, il, tile, tw);
    t3_row_store<M>(v, u, il, tile, g.g2 + ((int64_t)iz * M + kx) * M, kx < M);
}

// Z over G2s: line kx M + ky, its points iz < m at stride M^2.
template <int M>
__device__ __forceinline__ void t3s_z(const T3Geom g, d2* tile)
{
    const int m = g.m;
    const T3Thread<M> th;  // M^2 is a multiple of T: every line exists
    const T3Tw<M> tw(th.u, g.tw);
    const T3Strided<M> sd;
    d2 v[kT3Pts];
    t3_tile_load<M, true>(th, v, tile, g.g2 + sd.line, M * M, true, m);
    t3_forward<M, true>(v, th.u, th.il, tile, tw);
    const d2* krow = g.K + t3_krow<M>(th.line / M, th.line % M, *g.even != 0) * M;
#pragma unroll
    for (int s = 0; s < kT3Pts; ++s) v[s] = cmul(v[s], krow[th.point(s)]);
    t3_inverse<M, true>(v, th.u, th.il, tile, tw);
    t3_wave_sync();
    t3_tile_store<M, true>(th, v, tile, g.g2 + sd.line, M * M, true, m);
}

// YX for plane blockIdx.x: leaves the products of plane line iy = il < m
// in v[s], s < 4, at points ix = u + (M/8) s < m; returns whether the
// thread holds a line.
template <int M>
__device__ __forceinline__ bool t3s_yx(const T3Geom g, d2 (&v)[kT3Pts], d2* tile, d2* plane)
{
    using S = T3Shape<M>;
    const int m = g.m, iz = blockIdx.x;
    const int u = (int)threadIdx.x % S::TPL, il = (int)threadIdx.x / S::TPL;
    const T3Tw<M> tw(u, g.tw);
    // inverse y lines kx = il < M -> plane[iy][kx], iy < m
    const int kx = il;
    t3_row_load<M>(v, u, il, tile, g.g2 + ((int64_t)iz * M + kx) * M, kx < M);
    t3_inverse<M, true>(v, u, il, tile, tw);
#pragma unroll
    for (int s = 0; s < kT3Pts / 2; ++s) {
        const int iy = u + S::TPL * s;
        if (kx < M && iy < m) plane[iy * M + kx] = v[s];
    }
    __syncthreads();
    // inverse x lines iy = il < m
#pragma unroll
    for (int s = 0; s < kT3Pts; ++s)
        v[s] = il < m ? plane[il * M + t3_pos_out<M, S::NPH - 1>(u, s)] : d2{0.0, 0.0};
    t3_inverse<M, true>(v, u, il, tile, tw);
    return il < m;
}

}  // namespace ccg
