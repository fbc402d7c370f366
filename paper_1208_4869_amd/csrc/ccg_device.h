// ccg_device.h -- device-side building blocks for the gfx950 kernels:
// complex128 arithmetic, 64-lane wavefront reductions, and the fixed-order
// block reduction that hands its totals to the last workgroup of a grid.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ccg {

// complex128 as a 16-byte vector: one global_load_dwordx4 per element.
typedef double d2 __attribute__((ext_vector_type(2)));

constexpr int kWave = 64;
constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;

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

// Sum over the 64 lanes of a wavefront; every lane receives the total.
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, kWave);
    return v;
}

__device__ __forceinline__ d2 wave_sum(d2 v) { return d2{wave_sum(v.x), wave_sum(v.y)}; }

// Block-wide fixed-order reduction of NV complex values, followed by a
// last-block hand-off: every block writes its NV partial sums to
// partials[blockIdx.x * NV + k], takes a ticket, and the block that takes the
// last ticket sums all partials in index order.  Returns true (in every thread
// of that block) in the last block only; `total` is then valid in thread 0.
// The ticket is reset to zero for the next launch.  No float atomics: the
// result is the same on every run.
template <int NV>
__device__ bool reduce_to_last_block(d2 (&v)[NV], d2* partials, unsigned* ticket,
                                     d2 (&total)[NV])
{
    __shared__ d2 lds[kWavesPerBlock][NV];
    __shared__ bool last;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int nwaves = blockDim.x / kWave;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        d2 s = wave_sum(v[k]);
        if (lane == 0) lds[wave][k] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            d2 s = lds[0][k];
            for (int w = 1; w < nwaves; ++w) s += lds[w][k];
            partials[blockIdx.x * NV + k] = s;
        }
        __threadfence();
        unsigned t = atomicAdd(ticket, 1u);
        last = (t == gridDim.x - 1);
    }
    __syncthreads();
    if (!last) return false;
    __threadfence();
    d2 acc[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] = d2{0.0, 0.0};
    for (unsigned b = threadIdx.x; b < gridDim.x; b += blockDim.x) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            d2 p = __builtin_nontemporal_load(&partials[b * NV + k]);
            acc[k] += p;
        }
    }
    __syncthreads();  // lds reuse
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        d2 s = wave_sum(acc[k]);
        if (lane == 0) lds[wave][k] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            d2 s = lds[0][k];
            for (int w = 1; w < nwaves; ++w) s += lds[w][k];
            total[k] = s;
        }
        *ticket = 0u;
    }
    return true;
}

}  // namespace ccg
