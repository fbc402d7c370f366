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
// two >= 2m - 1 (at most 256).
//
// The transforms.  One wavefront transforms one line of M points (lane l
// holds points l, l + 64, ... for M > 64).  Forward: radix-2 decimation in
// frequency (natural order in, bit-reversed order out) with twiddles
// W^t = e^{-2 pi i t / M}; the kernel's transform is produced by the same
// passes, so the pointwise product is taken in the bit-reversed layout and no
// reordering pass is needed.  Inverse: decimation in time with conjugate
// twiddles (bit-reversed in, natural out), which undoes the forward stages
// exactly up to a factor 2 per stage; the factor M^3 is folded into the
// kernel's transform at set-up (a power of two: exact).  Pairs at span h < 64
// are exchanged between lanes with xor shuffles; spans >= 64 are within a
// lane's registers.
//
// Passes of one product (x -> y), each a grid of lines:
//   X1: lines (iy, iz), forward along x; x zero-padded         -> G1[iz][kx][iy]
//   X2: lines (kx, iz), forward along y                          -> G2[kx][ky][iz]
//   X3: lines (kx, ky), forward along z, times K, inverse along z -> G2 (in place)
//   X4: lines (kx, iz), inverse along y, keep iy < m              -> G1[iz][kx][iy]
//   X5: lines (iy, iz), inverse along x, keep ix < m              -> y
// (G1 holds M m^2 points, G2 M^2 m; only the m planes that the zero padding
// and the final crop leave nonzero are ever transformed.)
#pragma once

#include "ccg_device.h"

namespace ccg {

constexpr int kT3MaxM = 256;     // largest padded grid edge
constexpr int kT3LinesPerBlock = kBlock / kWave;

// Padded edge for an m-point lattice edge: the smallest power of two >= 2m - 1.
__host__ __device__ inline int t3_padded(int m)
{
    int M = 1;
    while (M < 2 * m - 1) M <<= 1;
    return M;
}

__device__ __forceinline__ d2 cmul_conj(d2 a, d2 w)  // a * conj(w)
{
    return d2{a.x * w.x + a.y * w.y, a.y * w.x - a.x * w.y};
}

__device__ __forceinline__ d2 shfl_xor_d2(d2 v, int mask)
{
    return d2{__shfl_xor(v.x, mask, kWave), __shfl_xor(v.y, mask, kWave)};
}

// Lane stages of a transform: spans h = top, top/2, ..., 1 with top =
// min(M/2, 32): at most six.  Their twiddles are loaded for all stages before
// the first butterfly (fixed-length loops, unrolled, guarded by h >= 1), so
// the loads are in flight together instead of one per stage.
constexpr int kLaneStages = 6;

__device__ __forceinline__ int t3_top(int M) { return M < kWave ? M / 2 : kWave / 2; }

// Forward transform of one line held as R registers per lane (R = M / 64 for
// M >= 64, else 1 with lanes >= M idle).  tw[t] = e^{-2 pi i t / M}, t < M/2.
template <int R>
__device__ __forceinline__ void t3_fwd(d2 (&v)[R], int M, const d2* __restrict__ tw)
{
    const int l = threadIdx.x & (kWave - 1);
    const int top = t3_top(M);
    d2 w[kLaneStages];
#pragma unroll
    for (int i = 0; i < kLaneStages; ++i) {
        const int h = top >> i;
        w[i] = h >= 1 ? tw[(l & (h - 1)) * (M / (2 * h))] : d2{1.0, 0.0};
    }
    // spans held in registers (h >= 64)
#pragma unroll
    for (int hr = R / 2; hr >= 1; hr >>= 1) {
        const int h = hr * kWave;
        const int step = M / (2 * h);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (r & hr) continue;
            const int e = l + kWave * (r & (hr - 1));  // index within the pair block
            const d2 a = v[r], b = v[r + hr];
            v[r] = a + b;
            v[r + hr] = cmul(a - b, tw[e * step]);
        }
    }
    // spans across lanes
#pragma unroll
    for (int i = 0; i < kLaneStages; ++i) {
        const int h = top >> i;
        if (h < 1) break;
        const bool bottom = (l & h) != 0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const d2 pv = shfl_xor_d2(v[r], h);
            v[r] = bottom ? cmul(pv - v[r], w[i]) : v[r] + pv;
        }
    }
}

// Inverse of t3_fwd up to the factor M (bit-reversed in, natural order out).
template <int R>
__device__ __forceinline__ void t3_inv(d2 (&v)[R], int M, const d2* __restrict__ tw)
{
    const int l = threadIdx.x & (kWave - 1);
    const int top = t3_top(M);
    const int nls = top >= 1 ? 32 - __builtin_clz(top) : 0;  // lane stages
    d2 w[kLaneStages];
#pragma unroll
    for (int i = 0; i < kLaneStages; ++i) {
        const int h = 1 << i;
        w[i] = i < nls ? tw[(l & (h - 1)) * (M / (2 * h))] : d2{1.0, 0.0};
    }
#pragma unroll
    for (int i = 0; i < kLaneStages; ++i) {
        if (i >= nls) break;
        const int h = 1 << i;
        const bool bottom = (l & h) != 0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const d2 u = bottom ? cmul_conj(v[r], w[i]) : v[r];
            const d2 pu = shfl_xor_d2(u, h);
            v[r] = bottom ? pu - u : u + pu;
        }
    }
#pragma unroll
    for (int hr = 1; hr <= R / 2; hr <<= 1) {
        const int h = hr * kWave;
        const int step = M / (2 * h);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (r & hr) continue;
            const int e = l + kWave * (r & (hr - 1));
            const d2 a = v[r], b = cmul_conj(v[r + hr], tw[e * step]);
            v[r] = a + b;
            v[r + hr] = a - b;
        }
    }
}

// Geometry of one structured operator.
struct T3Geom {
    int m, M;
    const d2* tw;  // M/2 twiddles
    const d2* K;   // M^3 kernel transform (bit-reversed layout, scaled by M^-3)
    d2* g1;        // M m^2
    d2* g2;        // M^2 m
};

// Line of a pass: wavefront w of block b takes line b * 4 + w.
__device__ __forceinline__ int t3_line()
{
    return blockIdx.x * kT3LinesPerBlock + (int)(threadIdx.x / kWave);
}

// Point p of a line held by (lane, register r).
__device__ __forceinline__ int t3_point(int r) { return (int)(threadIdx.x & (kWave - 1)) + kWave * r; }

// X1: x (n = m^3) -> G1[(iz M + kx) m + iy].  in may be complex128 only.
template <int R>
__device__ __forceinline__ void t3_pass_x(const T3Geom& g, const d2* __restrict__ in)
{
    const int m = g.m, M = g.M;
    const int line = t3_line();
    if (line >= m * m) return;
    const int iy = line % m, iz = line / m;
    d2 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int ix = t3_point(r);
        v[r] = ix < m ? in[ix + (int64_t)m * (iy + (int64_t)m * iz)] : d2{0.0, 0.0};
    }
    t3_fwd<R>(v, M, g.tw);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int kx = t3_point(r);
        if (kx < M) g.g1[((int64_t)iz * M + kx) * m + iy] = v[r];
    }
}

// X2: G1 -> G2[(kx M + ky) m + iz]
template <int R>
__device__ __forceinline__ void t3_pass_y(const T3Geom& g)
{
    const int m = g.m, M = g.M;
    const int line = t3_line();
    if (line >= M * m) return;
    const int kx = line % M, iz = line / M;
    d2 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int iy = t3_point(r);
        v[r] = iy < m ? g.g1[((int64_t)iz * M + kx) * m + iy] : d2{0.0, 0.0};
    }
    t3_fwd<R>(v, M, g.tw);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int ky = t3_point(r);
        if (ky < M) g.g2[((int64_t)kx * M + ky) * m + iz] = v[r];
    }
}

// X3: along z: forward, times K, inverse; G2 in place
template <int R>
__device__ __forceinline__ void t3_pass_z(const T3Geom& g)
{
    const int m = g.m, M = g.M;
    const int line = t3_line();
    if (line >= M * M) return;
    d2* row = g.g2 + (int64_t)line * m;
    const d2* krow = g.K + (int64_t)line * M;
    d2 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int iz = t3_point(r);
        v[r] = iz < m ? row[iz] : d2{0.0, 0.0};
    }
    t3_fwd<R>(v, M, g.tw);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int kz = t3_point(r);
        if (kz < M) v[r] = cmul(v[r], krow[kz]);
    }
    t3_inv<R>(v, M, g.tw);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int iz = t3_point(r);
        if (iz < m) row[iz] = v[r];
    }
}

// X4: G2 -> G1 (inverse along y, keep iy < m)
template <int R>
__device__ __forceinline__ void t3_pass_yi(const T3Geom& g)
{
    const int m = g.m, M = g.M;
    const int line = t3_line();
    if (line >= M * m) return;
    const int kx = line % M, iz = line / M;
    d2 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int ky = t3_point(r);
        v[r] = ky < M ? g.g2[((int64_t)kx * M + ky) * m + iz] : d2{0.0, 0.0};
    }
    t3_inv<R>(v, M, g.tw);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int iy = t3_point(r);
        if (iy < m) g.g1[((int64_t)iz * M + kx) * m + iy] = v[r];
    }
}

// X5: G1 -> the product for the points ix < m of line (iy, iz).  Returns the
// line index (or -1 past the last line); val[r] is the product at point
// ix = t3_point(r) when ix < m.
template <int R>
__device__ __forceinline__ int t3_pass_xi(const T3Geom& g, d2 (&v)[R])
{
    const int m = g.m, M = g.M;
    const int line = t3_line();
    const bool live = line < m * m;
    const int iy = live ? line % m : 0, iz = live ? line / m : 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int kx = t3_point(r);
        v[r] = live && kx < M ? g.g1[((int64_t)iz * M + kx) * m + iy] : d2{0.0, 0.0};
    }
    // every lane of the wavefront takes part in the shuffles
    t3_inv<R>(v, M, g.tw);
    return live ? line : -1;
}

}  // namespace ccg
