// ccg_device.h -- device-side building blocks for the gfx950 kernels:
// complex128 arithmetic, 64-lane wavefront reductions, and the fixed-order
// block reduction that hands its totals to the last workgroup of a grid.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ccg {

// complex128 as a 16-byte vector: one global_load_dwordx4 per element.
typedef double d2 __attribute__((ext_vector_type(2)));
// complex64 as an 8-byte vector (the mixed-precision inner solver).
typedef float f2 __attribute__((ext_vector_type(2)));

constexpr int kWave = 64;
constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kMaxWaves = 16;  // largest block used: 1024 threads

__device__ __forceinline__ d2 cz(double re, double im) { return d2{re, im}; }

// c + a * b
__device__ __forceinline__ d2 cfma(d2 a, d2 b, d2 c)
{
    c.x = __builtin_fma(a.x, b.x, c.x);
    c.x = __builtin_fma(-a.y, b.y, c.x);
    c.y = __builtin_fma(a.x, b.y, c.y);
    c.y = __builtin_fma(a.y, b.x, c.y);
    return c;
}

// c + conj(a) * b
__device__ __forceinline__ d2 cfma_conj(d2 a, d2 b, d2 c)
{
    c.x = __builtin_fma(a.x, b.x, c.x);
    c.x = __builtin_fma(a.y, b.y, c.x);
    c.y = __builtin_fma(a.x, b.y, c.y);
    c.y = __builtin_fma(-a.y, b.x, c.y);
    return c;
}

__device__ __forceinline__ d2 cmul(d2 a, d2 b)
{
    return d2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

__device__ __forceinline__ double cabs2(d2 a) { return a.x * a.x + a.y * a.y; }

// a / b as a * conj(b) / |b|^2
__device__ __forceinline__ d2 cdiv(d2 a, d2 b)
{
    double d = b.x * b.x + b.y * b.y;
    d2 q = d2{a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
    return d2{q.x / d, q.y / d};
}

__device__ __forceinline__ bool cfinite(d2 a)
{
    return __builtin_isfinite(a.x) && __builtin_isfinite(a.y);
}

__device__ __forceinline__ d2 ldnt(const d2* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ f2 ldnt(const f2* p) { return __builtin_nontemporal_load(p); }

// Vector element access in either precision; arithmetic is done in FP64 and
// a complex64 store rounds to nearest.
__device__ __forceinline__ d2 ldv(const d2* p, int64_t i) { return p[i]; }
__device__ __forceinline__ d2 ldv(const f2* p, int64_t i)
{
    const f2 v = p[i];
    return d2{(double)v.x, (double)v.y};
}
__device__ __forceinline__ void stv(d2* p, int64_t i, d2 v) { p[i] = v; }
__device__ __forceinline__ void stv(f2* p, int64_t i, d2 v) { p[i] = f2{(float)v.x, (float)v.y}; }

// Sum over the 64 lanes of a wavefront; every lane receives the total.
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, kWave);
    return v;
}

__device__ __forceinline__ d2 wave_sum(d2 v) { return d2{wave_sum(v.x), wave_sum(v.y)}; }

// Transposing butterfly: the wavefront totals of NV per-lane partial sums
// with about one exchange per value instead of six.  On entry v[k] is this
// lane's partial sum of value k; at each step a lane keeps half of its values
// and sends the other half to its partner at lane distance H (M values per
// step), so log2(NV) steps leave one value per lane and a plain butterfly
// over the 64 / NV lanes that share it finishes the total: on return v[0]
// holds the total of value lane / (64 / NV).  Fixed order: every run gives
// the same bits.
template <int M, int H, int NV>
__device__ __forceinline__ void transpose_sum_step(d2 (&v)[NV], int lane)
{
    if constexpr (M >= 1) {
        const bool up = (lane & H) != 0;
#pragma unroll
        for (int k = 0; k < M; ++k) {
            const d2 send = up ? v[k] : v[k + M];
            const d2 keep = up ? v[k + M] : v[k];
            v[k] = keep + d2{__shfl_xor(send.x, H, kWave), __shfl_xor(send.y, H, kWave)};
        }
        transpose_sum_step<M / 2, H / 2, NV>(v, lane);
    } else {
#pragma unroll
        for (int h = H; h >= 1; h >>= 1)
            v[0] += d2{__shfl_xor(v[0].x, h, kWave), __shfl_xor(v[0].y, h, kWave)};
    }
}

template <int NV>
__device__ __forceinline__ void wave_transpose_sum(d2 (&v)[NV], int lane)
{
    static_assert(NV >= 1 && NV <= kWave && (NV & (NV - 1)) == 0, "power of two rows");
    transpose_sum_step<NV / 2, kWave / 2, NV>(v, lane);
}

// Sum of one value per thread over the block, in a fixed order (64-lane
// butterfly, then wavefronts in index order).  Valid in thread 0.  `lds` must
// hold one entry per wavefront.
__device__ __forceinline__ d2 block_sum(d2 v, d2* lds)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int nwaves = blockDim.x / kWave;
    const d2 s = wave_sum(v);
    __syncthreads();  // lds may still be read by a previous call
    if (lane == 0) lds[wave] = s;
    __syncthreads();
    d2 t = lds[0];
    for (int w = 1; w < nwaves; ++w) t += lds[w];
    return t;
}

// Per-block partial sums: block b writes its two block totals to
// part[2b], part[2b + 1] with plain stores.  The kernel that runs next on the
// stream adds them up (reduce_partials); the kernel boundary makes them
// visible.  No atomics and no fences: every block of the consumer adds the
// same values in the same order and gets the same bits.
__device__ __forceinline__ void write_partials(d2 v0, d2 v1, d2* part, d2* lds)
{
    const d2 s0 = block_sum(v0, lds);
    const d2 s1 = block_sum(v1, lds);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = s0;
        part[2 * blockIdx.x + 1] = s1;
    }
}

// Totals of the nblocks partial pairs written by the previous kernel.  Every
// thread of the block takes part in the loads; the totals are valid in
// thread 0.  Thread t adds blocks t, t + blockDim.x, ... in increasing order,
// with the loads of kInFlight of them in flight at a time (the order of the
// additions does not depend on kInFlight).
template <int kInFlight = 8>
__device__ __forceinline__ void reduce_partials(const d2* part, int nblocks, d2* lds,
                                                d2& t0, d2& t1)
{
    const int step = blockDim.x;
    d2 a0 = d2{0.0, 0.0}, a1 = d2{0.0, 0.0};
    for (int b0 = threadIdx.x; b0 < nblocks; b0 += kInFlight * step) {
        d2 u0[kInFlight], u1[kInFlight];
#pragma unroll
        for (int m = 0; m < kInFlight; ++m) {
            const int b = b0 + m * step;
            if (b < nblocks) {
                u0[m] = part[2 * b];
                u1[m] = part[2 * b + 1];
            }
        }
#pragma unroll
        for (int m = 0; m < kInFlight; ++m) {
            if (b0 + m * step < nblocks) {
                a0 += u0[m];
                a1 += u1[m];
            }
        }
    }
    t0 = block_sum(a0, lds);
    t1 = block_sum(a1, lds);
}

// Three-term forms: the third block total goes to part3[b] (a separate
// array, so the two-term layout is unchanged).
__device__ __forceinline__ void write_partials3(d2 v0, d2 v1, d2 v2, d2* part, d2* part3,
                                                d2* lds)
{
    const d2 s0 = block_sum(v0, lds);
    const d2 s1 = block_sum(v1, lds);
    const d2 s2 = block_sum(v2, lds);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = s0;
        part[2 * blockIdx.x + 1] = s1;
        part3[blockIdx.x] = s2;
    }
}

template <int kInFlight = 5>
__device__ __forceinline__ void reduce_partials3(const d2* part, const d2* part3, int nblocks,
                                                 d2* lds, d2& t0, d2& t1, d2& t2)
{
    const int step = blockDim.x;
    d2 a0 = d2{0.0, 0.0}, a1 = d2{0.0, 0.0}, a2 = d2{0.0, 0.0};
    for (int b0 = threadIdx.x; b0 < nblocks; b0 += kInFlight * step) {
        d2 u0[kInFlight], u1[kInFlight], u2[kInFlight];
#pragma unroll
        for (int m = 0; m < kInFlight; ++m) {
            const int b = b0 + m * step;
            if (b < nblocks) {
                u0[m] = part[2 * b];
                u1[m] = part[2 * b + 1];
                u2[m] = part3[b];
            }
        }
#pragma unroll
        for (int m = 0; m < kInFlight; ++m) {
            if (b0 + m * step < nblocks) {
                a0 += u0[m];
                a1 += u1[m];
                a2 += u2[m];
            }
        }
    }
    t0 = block_sum(a0, lds);
    t1 = block_sum(a1, lds);
    t2 = block_sum(a2, lds);
}

}  // namespace ccg
