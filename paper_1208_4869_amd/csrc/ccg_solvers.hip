// ccg_solvers.hip -- BiCGSTAB, CGNR, COCG and COCR for complex128 A x = y on
// gfx950 (dense A, or the structured lattice operator of ccg_t3.h), the
// mixed-precision BiCGSTAB, and the matrix-vector entry points of the C ABI
// (include/ccg.h).
//
// Methods: the bicgstab and cgnr codes of the PIM90 set (Codes, section 2.1),
// with the matrix-vector product apart from the iteration (Abstract; Usage:
// matvec / cmatvec) and the stop rule driven by a tolerance and a budget
// (Usage: epsilon_err, maxit).  The paper prints no algorithm; the steps are
// van der Vorst's BiCGSTAB and CG on the normal equations, each written as a
// short fixed sequence of kernels per iteration:
//
//   BiCGSTAB slot: v = A p (+ r^H v, |v|^2) | s = r - alpha v (+ |s|^2,
//                  r^H s) | t = A s (+ t^H s, |t|^2, r^H t) | x, r and next
//                  p update (+ |r|^2; beta from rho' = r^H s - omega r^H t)
//   CGNR slot:     w = A p (+ |w|^2) | x, r update (+ |r|^2) | A^H r band
//                  partials | z = band sum (+ |z|^2) | p-update
//
// Every reduction is fused into the kernel that produces its operand, which
// writes one partial sum per block with plain stores; the next kernel on the
// stream starts by adding those partials in a fixed order (every block does
// it and gets the same bits) and runs the method's scalar step (alpha, omega,
// beta, rho, stop and breakdown tests) in device memory; block 0 publishes the
// new state to the other of two state copies.  No atomic read-modify-write;
// no scalar crosses to the host during a solve.  A device phase word drives
// the control flow: every kernel reads it on entry and does its part only in
// the phases where it has one, so the host enqueues the same slot over and
// over and learns that the solve is over from a one-word status that the
// first kernel of the next slot stores to pinned host memory.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/ccg.h"
#include "ccg_device.h"
#include "ccg_gemv.h"
#include "ccg_host.h"
#include "ccg_krylov.h"
#include "ccg_symv.h"
#include "ccg_t3.h"

namespace ccg {

size_t block_workspace_bytes(int method, int64_t n, int64_t k);  // ccg_block.hip

struct Args {
    const d2* A;
    int64_t lda;
    int n;
    GemvCShape csh;
    const d2* y;
    d2* x;
    d2 *r, *rh, *p, *v, *s, *t;  // BiCGSTAB vectors
    d2 *z, *w, *zpart;           // CGNR vectors and A^H band partials
    d2* part[2];                 // per-block partial sums, alternating
    d2* xpart[2];                // third per-block sums (PK_T3), alternating
    SolverState* st[2];          // state copies, alternating
    ccg_hist* hist;
    bool vec16;                  // complex64 A with 16-byte aligned rows
    T3Geom t3;                   // structured product (A unused)
    SymGeom sym;                 // upper-triangle product (sym.T > 0), else dense
    int* status;                 // pinned word: the phase after the prologue, or null
};

constexpr int kR = 4;   // rows per block in A x
constexpr int kU = 1;   // 64-element column chunks per wavefront step in A x
constexpr int kWN = 8;  // wavefronts per block in A x
constexpr int kBlockN = kWN * kWave;
// The plain complex64 A x (ccg_matvec_c64): 2 rows per block of 16
// wavefronts, 3% faster than the complex128 shape on complex64 rows (measured
// at n = 17576: 364 against 377 us).  The solvers' role kernels keep 4 rows
// and 8 wavefronts in both precisions: with twice the blocks, each paying the
// prologue (state, pending reduction) and the block sums of its terms, the
// complex64 role product took 510 instead of about 400 us.
constexpr int kRf = 2;
constexpr int kWNf = 16;
constexpr int kBlockNf = kWNf * kWave;

// Launch shape of the A x role kernels (both element types).
template <class T> struct GemvShape {
    static constexpr int R = kR, W = kWN, threads = kBlockN;
};
constexpr int kUC = 4;  // rows per step in A^H x

// Status word of a slot: the phase in the low 4 bits and, above them,
// -16 log2 of the recursive relative residual (0 when unknown or >= 1), which
// the host uses to stop enqueueing slots ahead when the next one is likely
// to be the last.
constexpr int kStatusPhaseBits = 4;

__device__ __forceinline__ int status_word(int phase, double relres)
{
    int code = 0;
    if (relres > 0.0 && relres < 1.0) {
        const double c = -16.0 * log2(relres);
        code = c < (double)(1 << 26) ? (int)c : (1 << 26) - 1;
    }
    return (code << kStatusPhaseBits) | phase;
}

// Start of every solver kernel: load state copy q into LDS and finish the
// reduction the previous kernel left (same fixed order in every block).
// kInFlight: partial loads in flight per thread.  Eight (five for three
// terms) after a product (thousands of block partials); the product kernels,
// which follow vector kernels of at most 512 blocks, take 2 so that the
// prologue does not set their register count (the A x loop needs 64 VGPRs,
// occupancy 8 with 512-thread blocks).
//
// Two LDS records: Ls[0] holds the state as loaded, Ls[1] the state after the
// pending step.  Thread 0 writes only Ls[1], so every thread's read of the
// loaded record (the pending kind and block count that steer it through the
// prologue) is free of that write even where no barrier separates them (the
// first-wavefront path below); the barrier that ends the step orders the
// write before any thread reads Ls[1].  Returns the record the kernel uses.
template <int kInFlight = 8>
__device__ __forceinline__ SolverState& prologue(const Args& a, int q, SolverState* Ls, d2* lds)
{
    if (threadIdx.x == 0) Ls[0] = *a.st[q];
    __syncthreads();
    const int pending = Ls[0].pending;
    SolverState* L = Ls;
    if (pending != PK_NONE) {
        const d2 z = d2{0.0, 0.0};
        d2 t0 = z, t1 = z, t2 = z;
        const int nb = Ls[0].pending_blocks;
        if (nb <= kWave) {
            // at most one partial per thread, all in the first wavefront: the
            // totals are its sums plus +0 (the bits of the block-wide sum,
            // which adds the other wavefronts' +0 sums), with no barrier
            if (threadIdx.x < kWave) {
                if (nb > 0) {
                    const int b = threadIdx.x;
                    d2 a0 = z, a1 = z, a2 = z;
                    if (b < nb) {
                        a0 += a.part[q][2 * b];
                        a1 += a.part[q][2 * b + 1];
                        if (pending == PK_T3) a2 += a.xpart[q][b];
                    }
                    t0 = wave_sum(a0) + z;
                    t1 = wave_sum(a1) + z;
                    if (pending == PK_T3) t2 = wave_sum(a2) + z;
                }
            }
        } else {
            if (pending == PK_T3)
                reduce_partials3<kInFlight == 8 ? 5 : kInFlight>(a.part[q], a.xpart[q], nb, lds,
                                                                t0, t1, t2);
            else
                reduce_partials<kInFlight>(a.part[q], nb, lds, t0, t1);
        }
        if (threadIdx.x == 0) {
            Ls[1] = Ls[0];
            apply_step(Ls[1], t0, t1, blockIdx.x == 0 ? a.hist : nullptr, t2);
        }
        __syncthreads();
        L = Ls + 1;
    }
    // the first kernel of a slot reports where the previous slot left the
    // method (a plain store to pinned host memory, system scope)
    if (a.status && blockIdx.x == 0 && threadIdx.x == 0)
        __hip_atomic_store(a.status, status_word(L->phase, L->relres_rec), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_SYSTEM);
    return *L;
}

// End of every solver kernel: block 0 writes the state for the next kernel,
// with the reduction this kernel leaves (kind, number of partial pairs).
__device__ __forceinline__ void publish(const Args& a, int q, const SolverState& L, int kind,
                                        int nblocks)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        SolverState o = L;
        o.pending = kind;
        o.pending_blocks = nblocks;
        *a.st[q ^ 1] = o;
    }
}

#define SOLVER_PROLOGUE()                           \
    __shared__ SolverState Ls_[2];                  \
    __shared__ d2 lds[kMaxWaves];                   \
    SolverState& L = prologue(a, q, Ls_, lds)

// The same for the product kernels (see prologue).
#define PRODUCT_PROLOGUE()                          \
    __shared__ SolverState Ls_[2];                  \
    __shared__ d2 lds[kMaxWaves];                   \
    SolverState& L = prologue<2>(a, q, Ls_, lds)

// --------------------------------------------------------- common kernels

__global__ void k_init(SolverState* st, int maxit, double tol2, int no_confirm)
{
    if (threadIdx.x == 0) {
        SolverState o;
        init_state(o, maxit, tol2, no_confirm);
        *st = o;
    }
}

// End of a slot: finish what the slot left and copy the phase word to pinned
// host memory.
__global__ void k_status(Args a, int q, int* ring_slot)
{
    SOLVER_PROLOGUE();
    if (threadIdx.x == 0)
        __hip_atomic_store(ring_slot, status_word(L.phase, L.relres_rec), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_SYSTEM);
    publish(a, q, L, PK_NONE, 0);
}

// First kernel of a solve: the initial state (every block builds the same
// record; block 0 publishes it) and ||y||^2 (the stop threshold follows in
// the next kernel's step).  T is the vector element type: d2 (complex128) or
// f2 (complex64, inner solves).
template <class T = d2>
__global__ __launch_bounds__(kBlock) void k_norm_y(Args a, int q, int maxit, double tol2,
                                                   int no_confirm)
{
    __shared__ SolverState L;
    __shared__ d2 lds[kMaxWaves];
    if (threadIdx.x == 0) init_state(L, maxit, tol2, no_confirm);
    __syncthreads();
    const T* y = (const T*)a.y;
    d2 v0 = d2{0.0, 0.0};
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < a.n; i += gridDim.x * kBlock)
        v0.x += cabs2(ldv(y, i));
    write_partials(v0, d2{0.0, 0.0}, a.part[q ^ 1], lds);
    publish(a, q, L, PK_NORMY, gridDim.x);
}

// Methods sharing the set-up kernels.
enum Method { M_BICG = 0, M_CGNR = 1, M_COCG = 2, M_COCR = 3 };

// First kernel of a solve when the caller says x0 = 0: the initial state
// (every block builds the same record; block 0 publishes it), x = 0, r = y
// (and r^ = p = y for BiCGSTAB), and the partials of ||y||^2 (= ||r||^2; COCG
// also (r, r)), which the next kernel's step takes as both the norm of y and
// the set-up sums.  x is zeroed whatever y holds: with a non-finite y the
// solve ends with info 4 at the iterate x0 = 0.
template <int M, class T = d2>
__global__ __launch_bounds__(kBlock) void k_setup_x0zero(Args a, int q, int maxit, double tol2,
                                                         int no_confirm)
{
    __shared__ SolverState L;
    __shared__ d2 lds[kMaxWaves];
    if (threadIdx.x == 0) init_state(L, maxit, tol2, no_confirm);
    __syncthreads();
    T* x = (T*)a.x;
    T* r = (T*)a.r;
    T* rh = (T*)a.rh;
    const T* y = (const T*)a.y;
    d2 v0 = d2{0.0, 0.0}, v1 = d2{0.0, 0.0};
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < a.n; i += gridDim.x * kBlock) {
        stv(x, i, d2{0.0, 0.0});
        const d2 yi = ldv(y, i);
        stv(r, i, yi);
        if (M == M_BICG) {
            stv(rh, i, yi);
            stv((T*)a.p, i, yi);  // first direction
        }
        v0.x += cabs2(yi);
        if (M == M_COCG) v1 = cfma(yi, yi, v1);
    }
    write_partials(v0, v1, a.part[q ^ 1], lds);
    publish(a, q, L, M == M_BICG ? PK_NY_SETUP_B0 : M == M_COCG ? PK_NY_SETUP_G0 : PK_NY_SETUP_C0,
            gridDim.x);
}

// ------------------------------------------------- A x kernels with roles

enum Role {
    ROLE_SETUP_B,  // BiCGSTAB set-up residual (also r^)
    ROLE_SETUP_C,  // CGNR / COCR set-up residual
    ROLE_SETUP_G,  // COCG set-up residual (+ (r, r))
    ROLE_V,        // BiCGSTAB v = A p
    ROLE_T,        // BiCGSTAB t = A s
    ROLE_W,        // CGNR w = A p
    ROLE_Q,        // COCG q = A p
    ROLE_U         // COCR u = A r
};

template <Role RO>
__device__ __forceinline__ int role_mode(int ph)
{
    switch (RO) {
    case ROLE_SETUP_B:
    case ROLE_SETUP_C:
    case ROLE_SETUP_G:
        return (ph == PH_RUN || ph == PH_ZERO) ? ph : -1;
    case ROLE_V:
    case ROLE_Q:
    case ROLE_U:
        return (ph == PH_RUN || ph == PH_RESTART || ph == PH_CONFIRM) ? ph : -1;
    case ROLE_T:
        return ph == PH_RUN ? ph : -1;
    case ROLE_W:
        return (ph == PH_RUN || ph == PH_CONFIRM) ? ph : -1;
    }
    return -1;
}

template <Role RO>
__device__ __forceinline__ constexpr bool role_setup()
{
    return RO == ROLE_SETUP_B || RO == ROLE_SETUP_C || RO == ROLE_SETUP_G;
}

// The vector a product of role RO multiplies in mode `mode`: x for the
// residual-type products (set-up, confirmation), else the role's Krylov vector.
template <Role RO>
__device__ __forceinline__ const d2* role_input(const Args& a, int mode)
{
    const bool resid = role_setup<RO>() || mode == PH_CONFIRM;
    return resid ? a.x : RO == ROLE_T ? a.s : RO == ROLE_U ? a.r : a.p;
}

// Element i of a product of role RO is val: store what the role stores and
// return its dot-product terms (in FP64; complex64 vectors are rounded on
// store and the terms use the stored values).
struct Terms {
    d2 t0, t1, t2;  // t2: r^H t (BiCGSTAB's t = A s only)
};

template <Role RO, class T>
__device__ __forceinline__ Terms role_finish(const Args& a, int mode, int i, const d2 val)
{
    const d2 z = d2{0.0, 0.0};
    const bool resid = role_setup<RO>() || mode == PH_CONFIRM;
    if (resid) {
        T* r = (T*)a.r;
        stv(r, i, ldv((const T*)a.y, i) - val);
        const d2 ri = ldv(r, i);
        if (RO == ROLE_SETUP_B || RO == ROLE_V) {
            stv((T*)a.rh, i, ri);
            stv((T*)a.p, i, ri);  // the direction of a (re)start
        }
        const d2 b = (RO == ROLE_SETUP_G || RO == ROLE_Q) ? cfma(ri, ri, z) : z;
        return Terms{d2{cabs2(ri), 0.0}, b, z};
    }
    if (RO == ROLE_Q) {
        a.v[i] = val;  // q
        return Terms{cfma(a.p[i], val, z), z, z};
    }
    if (RO == ROLE_U) {
        a.z[i] = val;  // u
        return Terms{cfma(a.r[i], val, z), z, z};
    }
    if (RO == ROLE_V) {
        T* v = (T*)a.v;
        stv(v, i, val);
        const d2 vs = ldv(v, i);
        return Terms{cfma_conj(ldv((const T*)a.rh, i), vs, z), d2{cabs2(vs), 0.0}, z};
    }
    if (RO == ROLE_T) {
        T* tv = (T*)a.t;
        stv(tv, i, val);
        const d2 ts = ldv(tv, i);
        return Terms{cfma_conj(ts, ldv((const T*)a.s, i), z), d2{cabs2(ts), 0.0},
                     cfma_conj(ldv((const T*)a.rh, i), ts, z)};
    }
    a.w[i] = val;  // ROLE_W
    return Terms{d2{cabs2(val), 0.0}, z, z};
}

// The reduction a product of role RO leaves for the next kernel.
template <Role RO>
__device__ __forceinline__ int role_kind(int mode)
{
    if (RO == ROLE_SETUP_B) return PK_SETUP_B1;
    if (RO == ROLE_SETUP_C) return PK_SETUP_C1;
    if (RO == ROLE_SETUP_G) return PK_SETUP_G1;
    if (mode == PH_CONFIRM)
        return RO == ROLE_V ? PK_CONFIRM_B : RO == ROLE_Q ? PK_CONFIRM_G : PK_CONFIRM_C;
    return RO == ROLE_V ? PK_V : RO == ROLE_T ? PK_T3 : RO == ROLE_W ? PK_W
         : RO == ROLE_Q ? PK_Q : PK_U;
}

// The block sums of a product of role RO (three for t = A s).
template <Role RO>
__device__ __forceinline__ void role_partials(const Args& a, int q, d2 v0, d2 v1, d2 v2,
                                              d2* lds)
{
    if (RO == ROLE_T)
        write_partials3(v0, v1, v2, a.part[q ^ 1], a.xpart[q ^ 1], lds);
    else
        write_partials(v0, v1, a.part[q ^ 1], lds);
}

// role_partials when only the first wavefront holds nonzero terms (the
// dense product's R rows): the block totals are that wavefront's sums, so no
// block-wide reduction is needed.  Adding +0 keeps the bits of block_sum,
// which adds the other wavefronts' +0 sums to it.
template <Role RO>
__device__ __forceinline__ void role_partials_wave0(const Args& a, int q, d2 v0, d2 v1, d2 v2)
{
    if (threadIdx.x >= kWave) return;
    const d2 z = d2{0.0, 0.0};
    const d2 s0 = wave_sum(v0) + z;
    const d2 s1 = wave_sum(v1) + z;
    d2 s2 = z;
    if (RO == ROLE_T) s2 = wave_sum(v2) + z;
    if (threadIdx.x == 0) {
        d2* part = a.part[q ^ 1];
        part[2 * blockIdx.x] = s0;
        part[2 * blockIdx.x + 1] = s1;
        if (RO == ROLE_T) a.xpart[q ^ 1][blockIdx.x] = s2;
    }
}

// The complex128 form first starts the loads of each wavefront's first chunk
// of A into LDS (A is the same whatever the phase decides), so they are in
// flight during the prologue; the prologue's latency (state, pending
// reduction, scalar step) otherwise delays the stream of every block.
template <Role RO, class T = d2>
__global__ __launch_bounds__(GemvShape<T>::threads) __attribute__((amdgpu_waves_per_eu(8, 8)))
void k_gemv_n_role(Args a, int q)
{
    constexpr int R = GemvShape<T>::R, W = GemvShape<T>::W;
    constexpr bool kPre = sizeof(T) == sizeof(d2);
    __shared__ d2 pre[kPre ? W * R * kWave : 1];
    const int row0 = blockIdx.x * R;
    d2* my_pre = pre + (threadIdx.x / kWave) * R * kWave;
    if constexpr (kPre) gemv_n_prefetch<R>(a.A, a.lda, a.n, row0, my_pre);
    PRODUCT_PROLOGUE();
    if constexpr (kPre) __builtin_amdgcn_s_waitcnt(0);  // the prefetch has landed
    const int mode = role_mode<RO>(L.phase);
    if (mode < 0) { publish(a, q, L, PK_NONE, 0); return; }
    const int n = a.n;
    const int t = threadIdx.x;

    if (mode == PH_ZERO) {  // y == 0: zero this block's rows of x
        if (t < R && row0 + t < n) stv((T*)a.x, row0 + t, d2{0.0, 0.0});
        publish(a, q, L, PK_ZERO, 0);
        return;
    }
    const d2* in = role_input<RO>(a, mode);

    __shared__ d2 red[W][R];
    d2 pv0 = d2{0.0, 0.0}, pv1 = d2{0.0, 0.0}, pv2 = d2{0.0, 0.0};
    if constexpr (sizeof(T) == sizeof(f2))
        gemv_n_block_f<R, W>((const f2*)a.A, a.lda, n, (const f2*)in, row0, red, a.vec16);
    else
        gemv_n_block<R, kU, W>(a.A, a.lda, n, in, row0, red, my_pre);
    // thread r of the first wavefront finishes row row0 + r
    const int i = row0 + t;
    if (t < R && i < n) {
        const Terms tm = role_finish<RO, T>(a, mode, i, gemv_n_row_total<R, W>(red, t));
        pv0 = tm.t0;
        pv1 = tm.t1;
        pv2 = tm.t2;
    }
    role_partials_wave0<RO>(a, q, pv0, pv1, pv2);  // the terms sit in the first wavefront
    publish(a, q, L, role_kind<RO>(mode), gridDim.x);
}

// ------------------------------------- structured (three-level Toeplitz) products
//
// The same roles with the product computed by the five FFT passes of
// ccg_t3.h.  The first pass applies the pending scalar step (and so learns
// the phase and the input vector); the passes in between are the plain ones
// (k_t3p_*); the last pass finishes the product and does what k_gemv_n_role
// does with each element.

template <Role RO, int M>
__global__ __launch_bounds__(kBlock) void k_t3_x(Args a, int q)
{
    SOLVER_PROLOGUE();
    __shared__ d2 tile[t3_tile_pts<M>()];
    const int mode = role_mode<RO>(L.phase);
    if (mode >= 0 && mode != PH_ZERO) t3_pass_x<M>(a.t3, role_input<RO>(a, mode), tile);
    publish(a, q, L, PK_NONE, 0);
}

template <Role RO, int M>
__global__ __launch_bounds__(kBlock) void k_t3_role(Args a, int q)
{
    SOLVER_PROLOGUE();
    __shared__ d2 tile[t3_tile_pts<M>()];
    const int mode = role_mode<RO>(L.phase);
    if (mode < 0) { publish(a, q, L, PK_NONE, 0); return; }
    if (mode == PH_ZERO) {  // y == 0: x = 0
        for (int i = blockIdx.x * kBlock + threadIdx.x; i < a.n; i += gridDim.x * kBlock)
            a.x[i] = d2{0.0, 0.0};
        publish(a, q, L, PK_ZERO, 0);
        return;
    }
    const T3Thread<M> th;
    d2 v[kT3Pts];
    const int line = t3_pass_xi<M>(a.t3, th, v, tile);
    d2 pv0 = d2{0.0, 0.0}, pv1 = d2{0.0, 0.0}, pv2 = d2{0.0, 0.0};
    if (line >= 0) {
#pragma unroll
        for (int s = 0; s < kT3Pts / 2; ++s) {  // points < M/2: every ix < m
            const int ix = th.point(s);
            if (ix < a.t3.m) {
                const Terms tm = role_finish<RO, d2>(a, mode, ix + a.t3.m * line, v[s]);
                pv0 += tm.t0;
                pv1 += tm.t1;
                pv2 += tm.t2;
            }
        }
    }
    role_partials<RO>(a, q, pv0, pv1, pv2, lds);
    publish(a, q, L, role_kind<RO>(mode), gridDim.x);
}

// The same roles on small lattices (padded edge <= 64): three launches (the
// per-plane XY and YX kernels of ccg_t3.h around the z pass).
template <Role RO, int M>
__global__ __launch_bounds__(kT3PlaneThreads) void k_t3s_xy_role(Args a, int q)
{
    SOLVER_PROLOGUE();
    __shared__ T3PlaneTile<M> tile;
    __shared__ T3Plane<M> plane;
    const int mode = role_mode<RO>(L.phase);
    if (mode >= 0 && mode != PH_ZERO) t3s_xy<M>(a.t3, role_input<RO>(a, mode), tile, plane);
    publish(a, q, L, PK_NONE, 0);
}

template <Role RO, int M>
__global__ __launch_bounds__(kT3PlaneThreads) void k_t3s_yx_role(Args a, int q)
{
    SOLVER_PROLOGUE();
    __shared__ T3PlaneTile<M> tile;
    __shared__ T3Plane<M> plane;
    const int mode = role_mode<RO>(L.phase);
    if (mode < 0) { publish(a, q, L, PK_NONE, 0); return; }
    if (mode == PH_ZERO) {  // y == 0: x = 0
        for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += gridDim.x * blockDim.x)
            a.x[i] = d2{0.0, 0.0};
        publish(a, q, L, PK_ZERO, 0);
        return;
    }
    d2 v[kT3Pts];
    const bool live = t3s_yx<M>(a.t3, v, tile, plane);
    const int m = a.t3.m;
    const int u = (int)threadIdx.x % T3Shape<M>::TPL, iy = (int)threadIdx.x / T3Shape<M>::TPL;
    d2 pv0 = d2{0.0, 0.0}, pv1 = d2{0.0, 0.0}, pv2 = d2{0.0, 0.0};
    if (live) {
#pragma unroll
        for (int s = 0; s < kT3Pts / 2; ++s) {
            const int ix = u + T3Shape<M>::TPL * s;
            if (ix < m) {
                const Terms tm =
                    role_finish<RO, d2>(a, mode, ix + m * (iy + m * (int)blockIdx.x), v[s]);
                pv0 += tm.t0;
                pv1 += tm.t1;
                pv2 += tm.t2;
            }
        }
    }
    role_partials<RO>(a, q, pv0, pv1, pv2, lds);
    publish(a, q, L, role_kind<RO>(mode), gridDim.x);
}

// ------------------------------ upper-triangle products of complex symmetric A
//
// The same roles with the product read from the upper triangle (ccg_symv.h):
// the tile pass applies the pending scalar step and writes the partials; the
// gather pass sums them and does what k_gemv_n_role does with each element.

template <Role RO, int CW>
__global__ __launch_bounds__(kBlock) void k_sym_tile(Args a, int q)
{
    SOLVER_PROLOGUE();
    __shared__ SymTileLds<CW> tl;
    const int mode = role_mode<RO>(L.phase);
    if (mode >= 0 && mode != PH_ZERO)
        symv_block<CW>(a.A, a.lda, a.n, role_input<RO>(a, mode), a.sym, blockIdx.x, tl);
    publish(a, q, L, PK_NONE, 0);
}

template <Role RO>
__global__ __launch_bounds__(kBlock) void k_sym_role(Args a, int q)
{
    SOLVER_PROLOGUE();
    const int mode = role_mode<RO>(L.phase);
    if (mode < 0) { publish(a, q, L, PK_NONE, 0); return; }
    const int e = blockIdx.x * kWave + (int)(threadIdx.x & (kWave - 1));
    const bool wave0 = threadIdx.x < kWave;
    if (mode == PH_ZERO) {  // y == 0: x = 0
        if (wave0 && e < a.n) a.x[e] = d2{0.0, 0.0};
        publish(a, q, L, PK_ZERO, 0);
        return;
    }
    __shared__ d2 red[kSymWaves][kWave];
    const d2 val = symv_gather(a.sym.part, a.n, a.sym.T, e, red);
    d2 pv0 = d2{0.0, 0.0}, pv1 = d2{0.0, 0.0}, pv2 = d2{0.0, 0.0};
    if (wave0 && e < a.n) {
        const Terms tm = role_finish<RO, d2>(a, mode, e, val);
        pv0 = tm.t0;
        pv1 = tm.t1;
        pv2 = tm.t2;
    }
    role_partials_wave0<RO>(a, q, pv0, pv1, pv2);  // the terms sit in the first wavefront
    publish(a, q, L, role_kind<RO>(mode), gridDim.x);
}

// ------------------------------------------------------- BiCGSTAB vectors

// The vector kernels load the operands of a thread's first element before
// their prologue: they do not depend on the pending step, so their latency
// overlaps the prologue's state and partial loads.
__device__ __forceinline__ d2 first_ld(const d2* v, int i0, int n)
{
    return i0 < n ? v[i0] : d2{0.0, 0.0};
}

// s = r - alpha v, ||s||^2, r^H s
template <class T = d2>
__global__ __launch_bounds__(kBlock) void k_bicg_s(Args a, int q)
{
    T* s = (T*)a.s;
    const T* r = (const T*)a.r;
    const T* v = (const T*)a.v;
    const T* rh = (const T*)a.rh;
    const int i0 = blockIdx.x * kBlock + threadIdx.x;
    const d2 zero = d2{0.0, 0.0};
    const d2 v_0 = i0 < a.n ? ldv(v, i0) : zero;
    const d2 r_0 = i0 < a.n ? ldv(r, i0) : zero;
    const d2 rh_0 = i0 < a.n ? ldv(rh, i0) : zero;
    SOLVER_PROLOGUE();
    if (L.phase != PH_RUN) { publish(a, q, L, PK_NONE, 0); return; }
    const d2 nal = d2{-L.alpha.x, -L.alpha.y};
    d2 v0 = zero, v1 = zero;
    for (int i = i0; i < a.n; i += gridDim.x * kBlock) {
        const bool first = i == i0;
        stv(s, i, cfma(nal, first ? v_0 : ldv(v, i), first ? r_0 : ldv(r, i)));
        const d2 si = ldv(s, i);
        v0.x += cabs2(si);
        v1 = cfma_conj(first ? rh_0 : ldv(rh, i), si, v1);
    }
    write_partials(v0, v1, a.part[q ^ 1], lds);
    publish(a, q, L, PK_S2, gridDim.x);
}

// x += alpha p + omega s, r = s - omega t, ||r||^2, and the next direction
// p = r + beta (p - omega v) with the beta of PK_T3; or, after a half-step
// exit, x += alpha p.
template <class T = d2>
__global__ __launch_bounds__(kBlock) void k_bicg_xrp(Args a, int q)
{
    T* x = (T*)a.x;
    T* r = (T*)a.r;
    T* p = (T*)a.p;
    const T* s = (const T*)a.s;
    const T* tv = (const T*)a.t;
    const T* v = (const T*)a.v;
    const int i0 = blockIdx.x * kBlock + threadIdx.x;
    const d2 zero = d2{0.0, 0.0};
    const bool in0 = i0 < a.n;
    const d2 p_0 = in0 ? ldv(p, i0) : zero;
    const d2 x_0 = in0 ? ldv(x, i0) : zero;
    const d2 s_0 = in0 ? ldv(s, i0) : zero;
    const d2 t_0 = in0 ? ldv(tv, i0) : zero;
    const d2 v_0 = in0 ? ldv(v, i0) : zero;
    SOLVER_PROLOGUE();
    const int ph = L.phase;
    if (ph != PH_RUN && ph != PH_HALF) { publish(a, q, L, PK_NONE, 0); return; }
    const d2 alpha = L.alpha;
    const d2 omega = L.omega;
    const d2 beta = L.beta;
    const d2 nom = d2{-omega.x, -omega.y};
    d2 v0 = zero;
    for (int i = i0; i < a.n; i += gridDim.x * kBlock) {
        const bool first = i == i0;
        const d2 pi = first ? p_0 : ldv(p, i);
        d2 xi = cfma(alpha, pi, first ? x_0 : ldv(x, i));
        if (ph == PH_RUN) {
            const d2 si = first ? s_0 : ldv(s, i);
            xi = cfma(omega, si, xi);
            stv(r, i, cfma(nom, first ? t_0 : ldv(tv, i), si));
            const d2 ri = ldv(r, i);
            v0.x += cabs2(ri);
            const d2 d = cfma(nom, first ? v_0 : ldv(v, i), pi);  // p - omega v
            stv(p, i, cfma(beta, d, ri));
        }
        stv(x, i, xi);
    }
    if (ph == PH_HALF) { publish(a, q, L, PK_HALF, 0); return; }
    write_partials(v0, d2{0.0, 0.0}, a.part[q ^ 1], lds);
    publish(a, q, L, PK_XRP, gridDim.x);
}

// ----------------------------------------------------------- CGNR vectors

// x += alpha p, r -= alpha w, ||r||^2
__global__ __launch_bounds__(kBlock) void k_cgnr_xr(Args a, int q)
{
    const int i0 = blockIdx.x * kBlock + threadIdx.x;
    const d2 p_0 = first_ld(a.p, i0, a.n), w_0 = first_ld(a.w, i0, a.n);
    const d2 x_0 = first_ld(a.x, i0, a.n), r_0 = first_ld(a.r, i0, a.n);
    SOLVER_PROLOGUE();
    if (L.phase != PH_RUN) { publish(a, q, L, PK_NONE, 0); return; }
    const double al = L.alpha.x;
    d2 v0 = d2{0.0, 0.0};
    for (int i = i0; i < a.n; i += gridDim.x * kBlock) {
        const bool first = i == i0;
        const d2 pi = first ? p_0 : a.p[i];
        const d2 wi = first ? w_0 : a.w[i];
        d2 xi = first ? x_0 : a.x[i];
        xi.x = __builtin_fma(al, pi.x, xi.x);
        xi.y = __builtin_fma(al, pi.y, xi.y);
        d2 ri = first ? r_0 : a.r[i];
        ri.x = __builtin_fma(-al, wi.x, ri.x);
        ri.y = __builtin_fma(-al, wi.y, ri.y);
        a.x[i] = xi;
        a.r[i] = ri;
        v0.x += cabs2(ri);
    }
    write_partials(v0, d2{0.0, 0.0}, a.part[q ^ 1], lds);
    publish(a, q, L, PK_XR2, gridDim.x);
}

// A^H r, band partials
__global__ __launch_bounds__(kBlock) void k_cgnr_z1(Args a, int q)
{
    SOLVER_PROLOGUE();
    if (L.phase == PH_RUN || L.phase == PH_RESTART)
        gemv_c_band<kUC>(a.A, a.lda, a.n, a.r, a.zpart, a.csh);
    publish(a, q, L, PK_NONE, 0);
}

// z = sum of band partials, ||z||^2
__global__ __launch_bounds__(kBlock) void k_cgnr_z2(Args a, int q)
{
    SOLVER_PROLOGUE();
    const int ph = L.phase;
    if (ph != PH_RUN && ph != PH_RESTART) { publish(a, q, L, PK_NONE, 0); return; }
    d2 v0 = d2{0.0, 0.0};
    for (int j = blockIdx.x * kBlock + threadIdx.x; j < a.n; j += gridDim.x * kBlock) {
        const d2 zj = gemv_c_gather(a.zpart, a.n, a.csh.nbands, j);
        a.z[j] = zj;
        v0.x += cabs2(zj);
    }
    write_partials(v0, d2{0.0, 0.0}, a.part[q ^ 1], lds);
    publish(a, q, L, ph == PH_RESTART ? PK_Z_RESTART : PK_Z_RUN, gridDim.x);
}

// A^H r = conj(A) r from the upper triangle of a complex symmetric A: tile
// partials (the upper-triangle form of k_cgnr_z1)
template <int CW>
__global__ __launch_bounds__(kBlock) void k_cgnr_z1_sym(Args a, int q)
{
    SOLVER_PROLOGUE();
    __shared__ SymTileLds<CW> tl;
    if (L.phase == PH_RUN || L.phase == PH_RESTART)
        symv_block<CW, true>(a.A, a.lda, a.n, a.r, a.sym, blockIdx.x, tl);
    publish(a, q, L, PK_NONE, 0);
}

// z = sum of the tile partials, ||z||^2 (the upper-triangle form of k_cgnr_z2)
__global__ __launch_bounds__(kBlock) void k_cgnr_z2_sym(Args a, int q)
{
    SOLVER_PROLOGUE();
    const int ph = L.phase;
    if (ph != PH_RUN && ph != PH_RESTART) { publish(a, q, L, PK_NONE, 0); return; }
    __shared__ d2 red[kSymWaves][kWave];
    const int j = blockIdx.x * kWave + (int)(threadIdx.x & (kWave - 1));
    const d2 zj = symv_gather(a.sym.part, a.n, a.sym.T, j, red);
    d2 v0 = d2{0.0, 0.0};
    if (threadIdx.x < kWave && j < a.n) {
        a.z[j] = zj;
        v0.x = cabs2(zj);
    }
    write_partials(v0, d2{0.0, 0.0}, a.part[q ^ 1], lds);
    publish(a, q, L, ph == PH_RESTART ? PK_Z_RESTART : PK_Z_RUN, gridDim.x);
}

// p = z (new direction) or p = z + beta p
__global__ __launch_bounds__(kBlock) void k_cgnr_p(Args a, int q)
{
    const int i0 = blockIdx.x * kBlock + threadIdx.x;
    const d2 z_0 = first_ld(a.z, i0, a.n), p_0 = first_ld(a.p, i0, a.n);
    SOLVER_PROLOGUE();
    if (L.phase == PH_RUN) {
        const bool fresh = L.restart != 0;
        const double beta = L.beta.x;
        for (int i = i0; i < a.n; i += gridDim.x * kBlock) {
            const bool first = i == i0;
            const d2 zi = first ? z_0 : a.z[i];
            if (fresh) {
                a.p[i] = zi;
            } else {
                d2 pi = first ? p_0 : a.p[i];
                pi.x = __builtin_fma(beta, pi.x, zi.x);
                pi.y = __builtin_fma(beta, pi.y, zi.y);
                a.p[i] = pi;
            }
        }
    }
    publish(a, q, L, PK_NONE, 0);
}

// ------------------------------------------------------ COCG / COCR vectors
// (section 3.4: complex symmetric A; the bilinear form (a, b) = sum a_i b_i)

// COCG: p = r (new direction) or p = r + beta p
__global__ __launch_bounds__(kBlock) void k_cocg_p(Args a, int q)
{
    const int i0 = blockIdx.x * kBlock + threadIdx.x;
    const d2 r_0 = first_ld(a.r, i0, a.n), p_0 = first_ld(a.p, i0, a.n);
    SOLVER_PROLOGUE();
    if (L.phase == PH_RUN || L.phase == PH_RESTART) {
        const bool fresh = L.restart != 0;
        const d2 beta = L.beta;
        for (int i = i0; i < a.n; i += gridDim.x * kBlock) {
            const bool first = i == i0;
            const d2 ri = first ? r_0 : a.r[i];
            a.p[i] = fresh ? ri : cfma(beta, first ? p_0 : a.p[i], ri);
        }
    }
    publish(a, q, L, PK_NONE, 0);
}

// COCG: x += alpha p, r -= alpha q, ||r||^2, (r, r)
__global__ __launch_bounds__(kBlock) void k_cocg_xr(Args a, int q)
{
    const int i0 = blockIdx.x * kBlock + threadIdx.x;
    const d2 p_0 = first_ld(a.p, i0, a.n), x_0 = first_ld(a.x, i0, a.n);
    const d2 v_0 = first_ld(a.v, i0, a.n), r_0 = first_ld(a.r, i0, a.n);
    SOLVER_PROLOGUE();
    if (L.phase != PH_RUN) { publish(a, q, L, PK_NONE, 0); return; }
    const d2 alpha = L.alpha;
    const d2 nal = d2{-alpha.x, -alpha.y};
    d2 v0 = d2{0.0, 0.0}, v1 = d2{0.0, 0.0};
    for (int i = i0; i < a.n; i += gridDim.x * kBlock) {
        const bool first = i == i0;
        a.x[i] = cfma(alpha, first ? p_0 : a.p[i], first ? x_0 : a.x[i]);
        const d2 ri = cfma(nal, first ? v_0 : a.v[i], first ? r_0 : a.r[i]);
        a.r[i] = ri;
        v0.x += cabs2(ri);
        v1 = cfma(ri, ri, v1);
    }
    write_partials(v0, v1, a.part[q ^ 1], lds);
    publish(a, q, L, PK_XR_G, gridDim.x);
}

// COCR: p = r + beta p, w = u + beta w (p = r, w = u for a new direction),
// (w, w)
__global__ __launch_bounds__(kBlock) void k_cocr_pw(Args a, int q)
{
    const int i0 = blockIdx.x * kBlock + threadIdx.x;
    const d2 r_0 = first_ld(a.r, i0, a.n), u_0 = first_ld(a.z, i0, a.n);
    const d2 p_0 = first_ld(a.p, i0, a.n), w_0 = first_ld(a.w, i0, a.n);
    SOLVER_PROLOGUE();
    if (L.phase != PH_RUN) { publish(a, q, L, PK_NONE, 0); return; }
    const bool fresh = L.restart != 0;
    const d2 beta = L.beta;
    d2 v0 = d2{0.0, 0.0};
    for (int i = i0; i < a.n; i += gridDim.x * kBlock) {
        const bool first = i == i0;
        const d2 ri = first ? r_0 : a.r[i];
        const d2 ui = first ? u_0 : a.z[i];
        d2 pi, wi;
        if (fresh) {
            pi = ri;
            wi = ui;
        } else {
            pi = cfma(beta, first ? p_0 : a.p[i], ri);
            wi = cfma(beta, first ? w_0 : a.w[i], ui);
        }
        a.p[i] = pi;
        a.w[i] = wi;
        v0 = cfma(wi, wi, v0);
    }
    write_partials(v0, d2{0.0, 0.0}, a.part[q ^ 1], lds);
    publish(a, q, L, PK_WW, gridDim.x);
}

// COCR: x += alpha p, r -= alpha w, ||r||^2
__global__ __launch_bounds__(kBlock) void k_cocr_xr(Args a, int q)
{
    const int i0 = blockIdx.x * kBlock + threadIdx.x;
    const d2 p_0 = first_ld(a.p, i0, a.n), x_0 = first_ld(a.x, i0, a.n);
    const d2 w_0 = first_ld(a.w, i0, a.n), r_0 = first_ld(a.r, i0, a.n);
    SOLVER_PROLOGUE();
    if (L.phase != PH_RUN) { publish(a, q, L, PK_NONE, 0); return; }
    const d2 alpha = L.alpha;
    const d2 nal = d2{-alpha.x, -alpha.y};
    d2 v0 = d2{0.0, 0.0};
    for (int i = i0; i < a.n; i += gridDim.x * kBlock) {
        const bool first = i == i0;
        a.x[i] = cfma(alpha, first ? p_0 : a.p[i], first ? x_0 : a.x[i]);
        const d2 ri = cfma(nal, first ? w_0 : a.w[i], first ? r_0 : a.r[i]);
        a.r[i] = ri;
        v0.x += cabs2(ri);
    }
    write_partials(v0, d2{0.0, 0.0}, a.part[q ^ 1], lds);
    publish(a, q, L, PK_XR_R, gridDim.x);
}

// --------------------------------------------------------- plain products

__global__ __launch_bounds__(kBlockN) void k_gemv_n_plain(const d2* __restrict__ A, int64_t lda,
                                                          int n, const d2* __restrict__ x,
                                                          d2* __restrict__ y)
{
    __shared__ d2 red[kWN][kR];
    const int row0 = blockIdx.x * kR;
    gemv_n_block<kR, kU, kWN>(A, lda, n, x, row0, red);
    const int t = threadIdx.x;
    if (t < kR && row0 + t < n) y[row0 + t] = gemv_n_row_total<kR, kWN>(red, t);
}

// y = A x in complex64 (the inner product of the mixed-precision solver)
__global__ __launch_bounds__(kBlockNf) void k_gemv_n_plain_f(const f2* __restrict__ A, int64_t lda,
                                                            int n, const f2* __restrict__ x,
                                                            f2* __restrict__ y, bool vec16)
{
    __shared__ d2 red[kWNf][kRf];
    const int row0 = blockIdx.x * kRf;
    gemv_n_block_f<kRf, kWNf>(A, lda, n, x, row0, red, vec16);
    const int t = threadIdx.x;
    if (t < kRf && row0 + t < n) stv(y, row0 + t, gemv_n_row_total<kRf, kWNf>(red, t));
}

__global__ __launch_bounds__(kBlock) void k_gemv_c_band_plain(const d2* __restrict__ A,
                                                              int64_t lda, int n,
                                                              const d2* __restrict__ x,
                                                              d2* __restrict__ part,
                                                              GemvCShape sh)
{
    gemv_c_band<kUC>(A, lda, n, x, part, sh);
}

__global__ __launch_bounds__(kBlock) void k_gemv_c_gather_plain(const d2* __restrict__ part,
                                                                int n, int nbands,
                                                                d2* __restrict__ y)
{
    for (int j = blockIdx.x * kBlock + threadIdx.x; j < n; j += gridDim.x * kBlock)
        y[j] = gemv_c_gather(part, n, nbands, j);
}

template <int CW>
__global__ __launch_bounds__(kBlock) void k_symv_plain(const d2* __restrict__ A, int64_t lda,
                                                       int n, const d2* __restrict__ x,
                                                       SymGeom g)
{
    __shared__ SymTileLds<CW> tl;
    symv_block<CW>(A, lda, n, x, g, blockIdx.x, tl);
}

__global__ __launch_bounds__(kBlock) void k_symv_gather_plain(SymGeom g, int n,
                                                              d2* __restrict__ y)
{
    __shared__ d2 red[kSymWaves][kWave];
    const int e = blockIdx.x * kWave + (int)(threadIdx.x & (kWave - 1));
    const d2 val = symv_gather(g.part, n, g.T, e, red);
    if (threadIdx.x < kWave && e < n) y[e] = val;
}


// ------------------------------------------ structured product, plain and set-up

template <int M>
__global__ __launch_bounds__(kBlock) void k_t3p_x(T3Geom g, const d2* __restrict__ x)
{
    __shared__ d2 tile[t3_tile_pts<M>()];
    t3_pass_x<M>(g, x, tile);
}
template <int M>
__global__ __launch_bounds__(kBlock) void k_t3p_y(T3Geom g)
{
    __shared__ d2 tile[t3_tile_pts<M>()];
    t3_pass_y<M>(g, tile);
}
template <int M>
__global__ __launch_bounds__(kBlock) void k_t3p_z(T3Geom g)
{
    __shared__ d2 tile[t3_tile_pts<M>()];
    t3_pass_z<M>(g, tile);
}
template <int M>
__global__ __launch_bounds__(kBlock) void k_t3p_yi(T3Geom g)
{
    __shared__ d2 tile[t3_tile_pts<M>()];
    t3_pass_yi<M>(g, tile);
}
template <int M>
__global__ __launch_bounds__(kBlock) void k_t3p_xi(T3Geom g, d2* __restrict__ y)
{
    __shared__ d2 tile[t3_tile_pts<M>()];
    const T3Thread<M> th;
    d2 v[kT3Pts];
    const int line = t3_pass_xi<M>(g, th, v, tile);
    if (line < 0) return;
#pragma unroll
    for (int s = 0; s < kT3Pts / 2; ++s) {  // points < M/2: every ix < m
        const int ix = th.point(s);
        if (ix < g.m) y[ix + g.m * line] = v[s];
    }
}

template <int M>
__global__ __launch_bounds__(kT3PlaneThreads) void k_t3s_xy(T3Geom g, const d2* __restrict__ x)
{
    __shared__ T3PlaneTile<M> tile;
    __shared__ T3Plane<M> plane;
    t3s_xy<M>(g, x, tile, plane);
}
template <int M>
__global__ __launch_bounds__(kBlock) void k_t3s_z(T3Geom g)
{
    __shared__ d2 tile[t3_tile_pts<M>()];
    t3s_z<M>(g, tile);
}
template <int M>
__global__ __launch_bounds__(kT3PlaneThreads) void k_t3s_yx(T3Geom g, d2* __restrict__ y)
{
    __shared__ T3PlaneTile<M> tile;
    __shared__ T3Plane<M> plane;
    d2 v[kT3Pts];
    if (!t3s_yx<M>(g, v, tile, plane)) return;
    const int m = g.m;
    const int u = (int)threadIdx.x % T3Shape<M>::TPL, iy = (int)threadIdx.x / T3Shape<M>::TPL;
    d2* out = y + m * (iy + m * (int)blockIdx.x);
#pragma unroll
    for (int s = 0; s < kT3Pts / 2; ++s) {
        const int ix = u + T3Shape<M>::TPL * s;
        if (ix < m) out[ix] = v[s];
    }
}

// tw[t] = e^{-2 pi i t / M}
__global__ void k_t3_twiddle(d2* tw, int M)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < M / 2) {
        double sn, cs;
        sincospi(2.0 * t / M, &sn, &cs);
        tw[t] = d2{cs, -sn};
    }
}

// Kernel value at padded grid coordinate c (the displacement c, or c - M for
// the wrapped negative displacements); outside the displacement box: none.
__device__ __forceinline__ bool t3_disp(int c, int m, int M, int& d)
{
    if (c <= m - 1) { d = c; return true; }
    if (c >= M - (m - 1)) { d = c - M; return true; }
    return false;
}

// Whether the kernel table is even in x and in y: T(-dx, dy, dz) and
// T(dx, -dy, dz) equal T(dx, dy, dz) bit for bit.  k_t3_even_init sets the
// flag, k_t3_even clears it at any pair that differs.
__global__ void k_t3_even_init(int* even) { *even = 1; }

__global__ __launch_bounds__(kBlock) void k_t3_even(const d2* __restrict__ table, int m,
                                                    int* even)
{
    const int w = 2 * m - 1;
    const int64_t n = (int64_t)w * w * w;
    bool odd = false;
    for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * kBlock) {
        const int ax = (int)(e % w), ay = (int)((e / w) % w);
        const int64_t row = e - ax - (int64_t)ay * w;  // (az, 0, 0)
        const d2 t = table[e];
        const d2 tx = table[row + (int64_t)ay * w + (w - 1 - ax)];
        const d2 ty = table[row + (int64_t)(w - 1 - ay) * w + ax];
        odd |= __builtin_bit_cast(uint64_t, t.x) != __builtin_bit_cast(uint64_t, tx.x) ||
               __builtin_bit_cast(uint64_t, t.y) != __builtin_bit_cast(uint64_t, tx.y) ||
               __builtin_bit_cast(uint64_t, t.x) != __builtin_bit_cast(uint64_t, ty.x) ||
               __builtin_bit_cast(uint64_t, t.y) != __builtin_bit_cast(uint64_t, ty.y);
    }
    if (odd) *even = 0;  // every writer writes the same value
}

// Set-up pass 1: lines y + M z of the wrapped kernel, forward along x ->
// S1[(z M + kx) M + y].  table: (2m-1)^3 values, displacement (dx, dy, dz) at
// ((dz + m-1)(2m-1) + (dy + m-1))(2m-1) + (dx + m-1).
template <int M>
__global__ __launch_bounds__(kBlock) void k_t3_s1(const d2* __restrict__ table, T3Geom g,
                                                  d2* __restrict__ S1)
{
    __shared__ d2 tile[t3_tile_pts<M>()];
    const int m = g.m, w = 2 * m - 1;
    const T3Thread<M> th;  // every line of the M^2 exists (M^2 is a multiple of T)
    const int y = th.line % M, z = th.line / M;
    int dy = 0, dz = 0;
    const bool yz = t3_disp(y, m, M, dy) && t3_disp(z, m, M, dz);
    d2 v[kT3Pts];
#pragma unroll
    for (int s = 0; s < kT3Pts; ++s) {
        int dx = 0;
        const bool ok = yz && t3_disp(th.point(s), m, M, dx);
        v[s] = ok ? table[((int64_t)(dz + m - 1) * w + (dy + m - 1)) * w + (dx + m - 1)]
                  : d2{0.0, 0.0};
    }
    t3_forward<M, false>(v, th.u, th.il, tile, T3Tw<M>(th.u, g.tw));
    const T3Strided<M> sd;
    d2* out = S1 + (sd.line / M) * M * M + sd.line % M;
    t3_tile_store<M>(th, v, tile, out, M, true);
}

// Set-up pass 2: lines z + M kx, forward along y -> S2[(kx M + ky) M + z]
template <int M>
__global__ __launch_bounds__(kBlock) void k_t3_s2(T3Geom g, const d2* __restrict__ S1,
                                                  d2* __restrict__ S2)
{
    __shared__ d2 tile[t3_tile_pts<M>()];
    const T3Thread<M> th;
    const d2* in = S1 + ((th.line % M) * M + th.line / M) * M;
    d2 v[kT3Pts];
#pragma unroll
    for (int s = 0; s < kT3Pts; ++s) v[s] = in[th.point(s)];
    t3_forward<M, false>(v, th.u, th.il, tile, T3Tw<M>(th.u, g.tw));
    const T3Strided<M> sd;
    d2* out = S2 + (sd.line / M) * M * M + sd.line % M;
    t3_tile_store<M>(th, v, tile, out, M, true);
}

// Set-up pass 3: lines kx M + ky of S2, forward along z, times M^-3 (exact)
// -> K, in register order, at the row t3_krow gives (a kernel even in x and
// y: only the lines whose frequencies are both <= M/2).
template <int M>
__global__ __launch_bounds__(kBlock) void k_t3_s3(T3Geom g, const d2* __restrict__ S2,
                                                  d2* __restrict__ K, double scale)
{
    __shared__ d2 tile[t3_tile_pts<M>()];
    const T3Thread<M> th;
    const d2* in = S2 + th.line * M;
    d2 v[kT3Pts];
#pragma unroll
    for (int s = 0; s < kT3Pts; ++s) v[s] = in[th.point(s)];
    t3_forward<M, false>(v, th.u, th.il, tile, T3Tw<M>(th.u, g.tw));
    const int qx = th.line / M, qy = th.line % M;
    const bool even = *g.even != 0;
    if (even && (t3_freq<M>(qx) > M / 2 || t3_freq<M>(qy) > M / 2)) return;
    d2* row = K + t3_krow<M>(qx, qy, even) * M;
#pragma unroll
    for (int s = 0; s < kT3Pts; ++s) row[th.point(s)] = d2{v[s].x * scale, v[s].y * scale};
}

// ================================================================== host

template <class T = d2>
static inline int blocks_n(int64_t n)
{
    int64_t b = (n + GemvShape<T>::R - 1) / GemvShape<T>::R;
    return (int)(b < 1 ? 1 : b);
}

static inline int blocks_e(int64_t n)
{
    int64_t b = (n + kBlock - 1) / kBlock;
    if (b > 512) b = 512;
    return (int)(b < 1 ? 1 : b);
}

static constexpr int64_t kMaxN = (int64_t)1 << 30;

// complex64 rows start on 16-byte boundaries (16-byte loads of two elements)
static inline bool rows16(const void* A, int64_t lda)
{
    return ((uintptr_t)A & 15) == 0 && (lda & 1) == 0;
}

struct Layout {
    size_t state, partials, part_bytes, xpartials, xpart_bytes, vec, zpart, spart, total;
    int nvec;
};

// Tile geometry of the upper-triangle product of an n x n matrix.
static SymGeom sym_geom(int64_t n, void* part)
{
    SymGeom g;
    g.S = sym_edge(n);
    g.T = (int)sym_ntiles(n, g.S);
    g.part = (d2*)part;
    return g;
}

static size_t sym_part_bytes(int64_t n)
{
    const SymGeom g = sym_geom(n > 0 ? n : 1, nullptr);
    return align256((size_t)g.T * (size_t)(n > 0 ? n : 1) * sizeof(d2));
}

// sym: the products read the upper triangle of a complex symmetric A (room
// for their tile partials).
static Layout layout(int method, int64_t n, int64_t min_partials = 0, bool sym = false)
{
    Layout L{};
    const GemvCShape csh = gemv_c_shape(n > 0 ? n : 1);
    int64_t pb = blocks_n(n);
    if (pb < 512) pb = 512;
    if (pb < min_partials) pb = min_partials;
    if (csh.blocks() > pb) pb = csh.blocks();
    const size_t vbytes = align256((size_t)(n > 0 ? n : 1) * sizeof(d2));
    size_t off = 0;
    L.state = off;  // two SolverState copies of 512 bytes
    off += 1024;
    L.partials = off;  // two buffers of pb partial pairs
    L.part_bytes = align256((size_t)pb * 2 * sizeof(d2));
    off += 2 * L.part_bytes;
    L.xpartials = off;  // two buffers of pb third sums
    L.xpart_bytes = align256((size_t)pb * sizeof(d2));
    off += 2 * L.xpart_bytes;
    L.nvec = method == CCG_WS_BICGSTAB ? 6 : method == CCG_WS_CGNR ? 4
           : method == CCG_WS_COCG ? 3 : method == CCG_WS_COCR ? 4 : 0;
    L.vec = off;
    off += (size_t)L.nvec * vbytes;
    L.zpart = off;
    if (method == CCG_WS_CGNR || method == CCG_WS_MATVEC_C)
        off += align256((size_t)csh.nbands * (size_t)(n > 0 ? n : 1) * sizeof(d2));
    L.spart = off;
    if (sym) off += sym_part_bytes(n);
    L.total = off;
    return L;
}

// Slots the host keeps queued ahead of the one whose status it reads.  A
// slot at n >= 4096 lasts well over 100 us, far longer than the host needs
// to enqueue the next one, so one slot ahead keeps the GPU busy; small
// systems run slots of a few tens of microseconds and keep two queued.
static inline int lookahead(int64_t n) { return n >= 4096 ? 1 : 2; }

static int check_common(int64_t n, const void* A, int64_t lda, const void* y, const void* x,
                        double tol, int32_t maxit)
{
    if (n < 0 || n > kMaxN) return -1;
    if (n > 0 && !A) return -2;
    if (lda < (n > 1 ? n : 1)) return -3;
    if (n > 0 && !y) return -4;
    if (n > 0 && !x) return -5;
    if (!(tol > 0.0) || !std::isfinite(tol)) return -6;
    if (maxit < 0) return -7;
    return 0;
}

static Args make_args(int method, int64_t n, const ccg_z* A, int64_t lda, const ccg_z* y,
                      ccg_z* x, void* work, ccg_hist* hist, bool sym = false)
{
    const Layout L = layout(method, n, 0, sym);
    char* base = (char*)work;
    const size_t vbytes = align256((size_t)n * sizeof(d2));
    Args a{};
    a.A = (const d2*)A;
    a.lda = lda;
    a.n = (int)n;
    a.csh = gemv_c_shape(n);
    a.y = (const d2*)y;
    a.x = (d2*)x;
    d2* vec[6] = {};
    for (int k = 0; k < L.nvec; ++k) vec[k] = (d2*)(base + L.vec + k * vbytes);
    if (method == CCG_WS_BICGSTAB) {
        a.r = vec[0]; a.rh = vec[1]; a.p = vec[2]; a.v = vec[3]; a.s = vec[4]; a.t = vec[5];
    } else if (method == CCG_WS_COCG) {
        a.r = vec[0]; a.p = vec[1]; a.v = vec[2];  // v holds q = A p
    } else {  // CGNR, COCR (z holds u = A r for COCR)
        a.r = vec[0]; a.z = vec[1]; a.p = vec[2]; a.w = vec[3];
        if (method == CCG_WS_CGNR) a.zpart = (d2*)(base + L.zpart);
    }
    a.part[0] = (d2*)(base + L.partials);
    a.part[1] = (d2*)(base + L.partials + L.part_bytes);
    a.xpart[0] = (d2*)(base + L.xpartials);
    a.xpart[1] = (d2*)(base + L.xpartials + L.xpart_bytes);
    a.st[0] = (SolverState*)(base + L.state);
    a.st[1] = (SolverState*)(base + L.state + 512);
    a.hist = hist;
    a.sym = sym ? sym_geom(n, base + L.spart) : SymGeom{0, 0, nullptr};
    return a;
}

static void read_result(const SolverState& s, ccg_result* res)
{
    res->info = s.info;
    res->iters = s.iters;
    res->matvecs = s.matvecs;
    res->confirms = s.confirms;
    res->relres_rec = s.relres_rec;
    res->relres_true = s.relres_true;
}

static int ws_of(int M)
{
    return M == M_BICG ? CCG_WS_BICGSTAB : M == M_CGNR ? CCG_WS_CGNR
         : M == M_COCG ? CCG_WS_COCG : CCG_WS_COCR;
}

// Padded edges of the structured product: one instantiation per power of two.
#define T3_DISPATCH(Mv, call)                      \
    switch (Mv) {                                  \
    case 16: call(16); break;                      \
    case 32: call(32); break;                      \
    case 64: call(64); break;                      \
    case 128: call(128); break;                    \
    default: call(256); break;                     \
    }

// Workgroups of the first and last pass of a product (and so the partial
// count of a structured solver's product): one per z-plane on the
// three-launch path, else tiles over the lines of the x passes.
static int t3_edge_tiles(int64_t m)
{
    const int M = t3_padded((int)m);
    int64_t t = 0;
#define T3_TILES(Mc) t = Mc <= kT3SmallM ? m : t3_tiles<Mc>(t3_row((int)m) * m)
    T3_DISPATCH(M, T3_TILES)
#undef T3_TILES
    return (int)(t > 0 ? t : 1);
}

// The five passes of a structured product of role RO (state copy q in, q
// advanced past them).  Only the first and the last pass take part in the
// state chain; the three middle passes run unconditionally on the grids
// (when the first pass had nothing to transform they work on stale grid
// data that the last pass then ignores), which spares each of them the
// dependent load of the state at its start.
template <Role RO, int M>
static void launch_t3_role(const Args& a, int& q, hipStream_t s)
{
    const int64_t m = a.t3.m, mp = a.t3.mp;
    Args b = a;  // only the first pass reports a status word
    b.status = nullptr;
    if constexpr (M <= kT3SmallM) {
        k_t3s_xy_role<RO, M><<<(int)m, kT3PlaneThreads, 0, s>>>(a, q);
        q ^= 1;
        k_t3s_z<M><<<(int)t3_tiles<M>(M * M), kBlock, 0, s>>>(a.t3);
        k_t3s_yx_role<RO, M><<<(int)m, kT3PlaneThreads, 0, s>>>(b, q);
    } else {
        k_t3_x<RO, M><<<(int)t3_tiles<M>(mp * m), kBlock, 0, s>>>(a, q);
        q ^= 1;
        k_t3p_y<M><<<(int)t3_tiles<M>(mp * M), kBlock, 0, s>>>(a.t3);
        k_t3p_z<M><<<(int)t3_tiles<M>(M * M), kBlock, 0, s>>>(a.t3);
        k_t3p_yi<M><<<(int)t3_tiles<M>(mp * M), kBlock, 0, s>>>(a.t3);
        k_t3_role<RO, M><<<(int)t3_tiles<M>(mp * m), kBlock, 0, s>>>(b, q);
    }
    q ^= 1;
}

// The two passes of an upper-triangle product of role RO.
template <Role RO>
static void launch_sym_role(const Args& a, int& q, hipStream_t s)
{
    Args b = a;  // only the first pass reports a status word
    b.status = nullptr;
    const int64_t nb = sym_nblocks(a.sym.T);
    if (a.sym.S == 4 * kWave)
        k_sym_tile<RO, 4><<<(unsigned)nb, kBlock, 0, s>>>(a, q);
    else if (a.sym.S == 2 * kWave)
        k_sym_tile<RO, 2><<<(unsigned)nb, kBlock, 0, s>>>(a, q);
    else
        k_sym_tile<RO, 1><<<(unsigned)nb, kBlock, 0, s>>>(a, q);
    q ^= 1;
    k_sym_role<RO><<<(unsigned)((a.n + kWave - 1) / kWave), kBlock, 0, s>>>(b, q);
    q ^= 1;
}

// The event log of the calling host thread (ccg_set_event_log), or null.
static thread_local ccg_event_log* t_event_log = nullptr;

// The CCG_PROD_* kind of a product of role RO.
template <Role RO>
static constexpr uint32_t prod_kind()
{
    return (RO == ROLE_SETUP_B || RO == ROLE_SETUP_C || RO == ROLE_SETUP_G) ? CCG_PROD_SETUP
         : RO == ROLE_V ? CCG_PROD_V
         : RO == ROLE_T ? CCG_PROD_T : RO == ROLE_W ? CCG_PROD_W
         : RO == ROLE_Q ? CCG_PROD_Q : CCG_PROD_U;
}

// A dense complex128 A x launch of the solvers, bracketed by a pair of the
// attached event log's events when it is a sampled launch of a kind the log
// counts and the log has pairs left.
template <Role RO>
static void launch_gemv_logged(const Args& a, int q, hipStream_t s)
{
    ccg_event_log* lg = t_event_log;
    bool rec = false;
    if (lg && (lg->roles == 0 || (lg->roles & prod_kind<RO>()))) {
        rec = lg->events && lg->count >= 0 && lg->count < lg->capacity &&
              (lg->stride <= 1 || lg->seen % lg->stride == 0);
        lg->seen++;
    }
    // a failed record only leaves that pair unset; the solve goes on
    if (rec) (void)hipEventRecord((hipEvent_t)lg->events[2 * lg->count], s);
    k_gemv_n_role<RO, d2><<<blocks_n<d2>(a.n), GemvShape<d2>::threads, 0, s>>>(a, q);
    if (rec) {
        (void)hipEventRecord((hipEvent_t)lg->events[2 * lg->count + 1], s);
        lg->count++;
    }
}

// A product of role RO: dense (one k_gemv_n_role launch, or the two passes
// of the upper-triangle product when a.sym is set) or structured.
template <Role RO, class T, bool S3>
static void launch_product(const Args& a, int& q, hipStream_t s)
{
    if constexpr (S3) {
#define T3_ROLE(Mc) launch_t3_role<RO, Mc>(a, q, s)
        T3_DISPATCH(a.t3.M, T3_ROLE)
#undef T3_ROLE
    } else if (sizeof(T) == sizeof(d2) && a.sym.T > 0) {
        launch_sym_role<RO>(a, q, s);
    } else if constexpr (sizeof(T) == sizeof(d2)) {
        launch_gemv_logged<RO>(a, q, s);
        q ^= 1;
    } else {
        k_gemv_n_role<RO, T><<<blocks_n<T>(a.n), GemvShape<T>::threads, 0, s>>>(a, q);
        q ^= 1;
    }
}

// Wait until the pinned status word idx has been written (it holds
// kStatusEmpty until then) and return it.  The wait only reads host memory;
// after about a millisecond without the word it also polls the stream, so
// that a failed launch ends the wait with its error.  (Any stream query or
// event wait makes the runtime open the next dispatch with a cache
// invalidation, a few microseconds per slot, so the fast path makes none.)
constexpr int kStatusEmpty = -1;

static int wait_status(SyncCtx* sc, int idx, hipStream_t s, int* phase, double* relres)
{
    int v = kStatusEmpty;
    for (uint64_t spin = 1;; ++spin) {
        v = __atomic_load_n(&sc->ring_h[idx], __ATOMIC_ACQUIRE);
        if (v != kStatusEmpty) break;
        if (spin >= (1u << 14) && (spin & 1023) == 0) {
            const hipError_t e = hipStreamQuery(s);
            if (e == hipSuccess) {  // drained: the word must be there now
                v = __atomic_load_n(&sc->ring_h[idx], __ATOMIC_ACQUIRE);
                if (v == kStatusEmpty) return (int)hipErrorUnknown;
                break;
            }
            if (e != hipErrorNotReady) return (int)e;
        }
        __builtin_ia32_pause();
    }
    *phase = v & ((1 << kStatusPhaseBits) - 1);
    const int code = v >> kStatusPhaseBits;
    *relres = code > 0 ? std::exp2(-code / 16.0) : -1.0;
    return 0;
}

// Enqueue set-up, then slots until the status word of a slot reads PH_DONE.
// Every solver kernel reads state copy q and writes copy q ^ 1; the host
// tracks q across the launches it makes.  The status of slot j is written by
// the first kernel of slot j + 1 after its prologue (the last slot the host
// may enqueue is followed by a status kernel), into pinned word j mod kRing,
// which the host clears before it enqueues the writer.  S3: products by the
// structured operator.
template <int M, class T = d2, bool S3 = false>
static int run_solver(const Args& a, uint32_t flags, int32_t maxit, double tol2,
                      ccg_result* res, hipStream_t s, int no_confirm = 0)
{
    static_assert(!(S3 && M == M_CGNR), "CGNR needs A^H: dense only");
    SyncCtx* sc = nullptr;
    hipError_t e = get_sync(&sc);
    if (e != hipSuccess) return (int)e;
    const int gE = blocks_e(a.n);
    const int gC = a.csh.blocks();
    int q = 0;
    auto flip = [&q]() { const int cur = q; q ^= 1; return cur; };

    if (flags & CCG_X0_ZERO) {
        k_setup_x0zero<M == M_COCR ? M_CGNR : M, T>
            <<<gE, kBlock, 0, s>>>(a, flip(), maxit, tol2, no_confirm);
    } else {
        k_norm_y<T><<<gE, kBlock, 0, s>>>(a, flip(), maxit, tol2, no_confirm);
        if (M == M_BICG)
            launch_product<ROLE_SETUP_B, T, S3>(a, q, s);
        else if (M == M_COCG)
            launch_product<ROLE_SETUP_G, T, S3>(a, q, s);
        else
            launch_product<ROLE_SETUP_C, T, S3>(a, q, s);
    }
    if ((e = hipGetLastError()) != hipSuccess) return (int)e;

    // Each slot advances the method by at most one iteration or one
    // confirmation; a confirmation is always preceded by an iteration or
    // by the set-up, so 2 * maxit + 4 slots always suffice.
    //
    // Look-ahead: the host keeps `ahead` slots queued beyond the one whose
    // status it reads, except past the slot that is likely to be the last:
    // when a status reads CONFIRM (the next slot confirms) or the residual
    // ratio of the last two statuses predicts convergence within the next
    // slot, nothing is enqueued after the presumed confirmation slot, and a
    // one-block status kernel reports that slot instead of the first kernel
    // of a slot that would have run for nothing.  A wrong guess costs one such
    // status kernel; the slots then continue as before.
    const int64_t max_slots = 2 * (int64_t)maxit + 4;
    const int ahead = S3 ? 2 : lookahead(a.n);  // structured slots are short
    const double tol = std::sqrt(tol2);
    int64_t next = 0;                 // next slot to enqueue
    int64_t seen = 0;                 // next slot whose status the host reads
    int64_t reported = -1;            // last slot followed by a status kernel
    int64_t stop_at = INT64_MAX;      // enqueue nothing past this slot
    double prev_rr = -1.0;
    for (;;) {
        while (next < max_slots && next <= seen + ahead && next <= stop_at) {
            Args f = a;  // the slot's first kernel reports slot - 1
            f.status = nullptr;
            if (next > 0 && reported != next - 1) {
                const int w = (int)((next - 1) % kRing);
                __atomic_store_n(&sc->ring_h[w], kStatusEmpty, __ATOMIC_RELEASE);
                f.status = sc->ring_d + w;
            }
            if (M == M_BICG) {
                launch_product<ROLE_V, T, S3>(f, q, s);
                k_bicg_s<T><<<gE, kBlock, 0, s>>>(a, flip());
                launch_product<ROLE_T, T, S3>(a, q, s);
                k_bicg_xrp<T><<<gE, kBlock, 0, s>>>(a, flip());
            } else if (M == M_CGNR && a.sym.T > 0) {
                launch_sym_role<ROLE_W>(f, q, s);
                k_cgnr_xr<<<gE, kBlock, 0, s>>>(a, flip());
                const unsigned nb = (unsigned)sym_nblocks(a.sym.T);
                if (a.sym.S == 4 * kWave)
                    k_cgnr_z1_sym<4><<<nb, kBlock, 0, s>>>(a, flip());
                else if (a.sym.S == 2 * kWave)
                    k_cgnr_z1_sym<2><<<nb, kBlock, 0, s>>>(a, flip());
                else
                    k_cgnr_z1_sym<1><<<nb, kBlock, 0, s>>>(a, flip());
                k_cgnr_z2_sym<<<(unsigned)((a.n + kWave - 1) / kWave), kBlock, 0, s>>>(a, flip());
                k_cgnr_p<<<gE, kBlock, 0, s>>>(a, flip());
            } else if (M == M_CGNR) {
                launch_gemv_logged<ROLE_W>(f, flip(), s);
                k_cgnr_xr<<<gE, kBlock, 0, s>>>(a, flip());
                k_cgnr_z1<<<gC, kBlock, 0, s>>>(a, flip());
                k_cgnr_z2<<<gE, kBlock, 0, s>>>(a, flip());
                k_cgnr_p<<<gE, kBlock, 0, s>>>(a, flip());
            } else if (M == M_COCG) {
                k_cocg_p<<<gE, kBlock, 0, s>>>(f, flip());
                launch_product<ROLE_Q, T, S3>(a, q, s);
                k_cocg_xr<<<gE, kBlock, 0, s>>>(a, flip());
            } else {
                launch_product<ROLE_U, T, S3>(f, q, s);
                k_cocr_pw<<<gE, kBlock, 0, s>>>(a, flip());
                k_cocr_xr<<<gE, kBlock, 0, s>>>(a, flip());
            }
            ++next;
        }
        // the last enqueued slot has no follower for now: a status kernel
        // reports it
        if (next > seen && reported != next - 1 && (next == max_slots || next > stop_at)) {
            const int w = (int)((next - 1) % kRing);
            __atomic_store_n(&sc->ring_h[w], kStatusEmpty, __ATOMIC_RELEASE);
            k_status<<<1, kBlock, 0, s>>>(a, flip(), sc->ring_d + w);
            reported = next - 1;
        }
        if ((e = hipGetLastError()) != hipSuccess) return (int)e;
        if (seen >= next) break;  // slot budget spent (defensive)
        int phase = 0;
        double rr = -1.0;
        int rc = wait_status(sc, (int)(seen % kRing), s, &phase, &rr);
        if (rc) return rc;
        if (phase == PH_DONE) break;
        if (phase == PH_CONFIRM || phase == PH_HALF) {
            stop_at = seen + 1;
        } else {
            stop_at = INT64_MAX;
            if (phase == PH_RUN && prev_rr > 0.0 && rr > 0.0 && rr < prev_rr &&
                rr * (rr / prev_rr) <= 2.0 * tol)
                stop_at = seen + 2;  // slot seen + 1 is predicted to converge
        }
        prev_rr = rr;
        ++seen;
    }
    SolverState hs;
    if ((e = hipMemcpyAsync(&hs, a.st[q], sizeof hs, hipMemcpyDeviceToHost, s)) != hipSuccess)
        return (int)e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return (int)e;
    read_result(hs, res);
    if (hs.phase != PH_DONE) res->info = 1;  // defensive: slot budget spent
    return 0;
}

template <int M>
static int solve_ex(int64_t n, const ccg_z* A, int64_t lda, const ccg_z* y, ccg_z* x,
                    double tol, int32_t maxit, uint32_t flags, void* work, size_t work_bytes,
                    ccg_result* res, ccg_hist* hist, void* stream)
{
    int bad = check_common(n, A, lda, y, x, tol, maxit);
    if (bad) return bad;
    if (flags & ~(CCG_X0_ZERO | CCG_A_SYM_UPPER)) return -8;
    const bool sym = (flags & CCG_A_SYM_UPPER) != 0;
    const int method = ws_of(M);
    if (n > 0 && !work) return -9;
    if (n > 0 && ((uintptr_t)work & 255)) return -9;
    if (n > 0 && work_bytes < layout(method, n, 0, sym).total) return -10;
    if (!res) return -11;
    if (n == 0) {
        std::memset(res, 0, sizeof *res);
        res->relres_rec = res->relres_true = 0.0;
        return 0;
    }
    const Args a = make_args(method, n, A, lda, y, x, work, hist, sym);
    return run_solver<M>(a, flags, maxit, tol * tol, res, (hipStream_t)stream);
}

template <int M>
static int solve_short(int64_t n, const ccg_z* A, int64_t lda, const ccg_z* y, ccg_z* x,
                       double tol, int32_t maxit, int32_t* info, void* stream)
{
    int bad = check_common(n, A, lda, y, x, tol, maxit);
    if (bad) return bad;
    if (!info) return -8;
    ccg_result res{};
    if (n == 0) {
        *info = 0;
        return 0;
    }
    hipStream_t s = (hipStream_t)stream;
    const size_t bytes = layout(ws_of(M), n).total;
    void* work = nullptr;
    hipError_t e = hipMallocAsync(&work, bytes, s);
    if (e != hipSuccess) return (int)e;
    int rc = solve_ex<M>(n, A, lda, y, x, tol, maxit, 0u, work, bytes, &res, nullptr, stream);
    e = hipFreeAsync(work, s);
    if (rc == 0 && e == hipSuccess) e = hipStreamSynchronize(s);
    if (rc != 0) return rc;
    if (e != hipSuccess) return (int)e;
    *info = res.info;
    return 0;
}

static int matvec_impl(int op, int64_t n, const ccg_z* A, int64_t lda, const ccg_z* x,
                       ccg_z* y, void* work, size_t work_bytes, void* stream, bool own_ws)
{
    if (op != CCG_OP_N && op != CCG_OP_C && op != CCG_OP_S) return -1;
    if (n < 0 || n > kMaxN) return -2;
    if (n > 0 && !A) return -3;
    if (lda < (n > 1 ? n : 1)) return -4;
    if (n > 0 && !x) return -5;
    if (n > 0 && !y) return -6;
    if (n == 0) return 0;
    const char *xb = (const char*)x, *yb = (const char*)y;
    const size_t vb = (size_t)n * sizeof(d2);
    if (xb < yb + vb && yb < xb + vb) return -6;  // x and y overlap
    hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    if (op == CCG_OP_N) {
        k_gemv_n_plain<<<blocks_n(n), kBlockN, 0, s>>>((const d2*)A, lda, (int)n, (const d2*)x,
                                                     (d2*)y);
        e = hipGetLastError();
        return e == hipSuccess ? 0 : (int)e;
    }
    if (op == CCG_OP_S) {
        const size_t need = sym_part_bytes(n);
        void* part = work;
        if (own_ws) {
            if ((e = hipMallocAsync(&part, need, s)) != hipSuccess) return (int)e;
        } else {
            if (!work) return -7;
            if (work_bytes < need) return -8;
        }
        const SymGeom g = sym_geom(n, part);
        const unsigned nb = (unsigned)sym_nblocks(g.T);
        if (g.S == 4 * kWave)
            k_symv_plain<4><<<nb, kBlock, 0, s>>>((const d2*)A, lda, (int)n, (const d2*)x, g);
        else if (g.S == 2 * kWave)
            k_symv_plain<2><<<nb, kBlock, 0, s>>>((const d2*)A, lda, (int)n, (const d2*)x, g);
        else
            k_symv_plain<1><<<nb, kBlock, 0, s>>>((const d2*)A, lda, (int)n, (const d2*)x, g);
        k_symv_gather_plain<<<(unsigned)((n + kWave - 1) / kWave), kBlock, 0, s>>>(g, (int)n,
                                                                                  (d2*)y);
        e = hipGetLastError();
        if (own_ws) {
            hipError_t e2 = hipFreeAsync(part, s);
            if (e == hipSuccess) e = e2;
        }
        return e == hipSuccess ? 0 : (int)e;
    }
    const GemvCShape sh = gemv_c_shape(n);
    const size_t need = (size_t)sh.nbands * (size_t)n * sizeof(d2);
    void* part = work;
    if (own_ws) {
        if ((e = hipMallocAsync(&part, need, s)) != hipSuccess) return (int)e;
    } else {
        if (!work) return -7;
        if (work_bytes < need) return -8;
    }
    k_gemv_c_band_plain<<<sh.blocks(), kBlock, 0, s>>>((const d2*)A, lda, (int)n,
                                                       (const d2*)x, (d2*)part, sh);
    k_gemv_c_gather_plain<<<blocks_e(n), kBlock, 0, s>>>((const d2*)part, (int)n, sh.nbands,
                                                         (d2*)y);
    e = hipGetLastError();
    if (own_ws) {
        hipError_t e2 = hipFreeAsync(part, s);
        if (e == hipSuccess) e = e2;
    }
    return e == hipSuccess ? 0 : (int)e;
}

// ------------------------------------------------------------ read stream
//
// ccg_read_stream: a measurement aid outside the method -- one pass that
// reads a buffer with the products' 16-byte nontemporal loads and nothing
// else, so the HBM read rate the chip delivers to that load pattern can be
// set beside the products' rates.  Block b reads the b-th slab of
// CCG_READ_STREAM_SLAB bytes as consecutive 4 KB rows (256 threads x 16 B),
// kReadUnroll rows in flight per thread -- the contiguous per-block streams
// of the products; a grid-stride walk with loads spread over the whole
// buffer measured 10-20% slower.  Every block writes the sum of what it read,
// so no load can be dropped.
constexpr int kReadUnroll = 16;
constexpr int64_t kReadSlab16 = CCG_READ_STREAM_SLAB / 16;

__global__ __launch_bounds__(kBlock) void k_read_stream(const d2* __restrict__ src, int64_t n16,
                                                        d2* __restrict__ out)
{
    __shared__ d2 lds[kMaxWaves];
    const int64_t b0 = (int64_t)blockIdx.x * kReadSlab16;
    const int64_t e1 = b0 + kReadSlab16 < n16 ? b0 + kReadSlab16 : n16;
    int64_t i = b0 + threadIdx.x;
    d2 acc = d2{0.0, 0.0};
    for (; i + (kReadUnroll - 1) * kBlock < e1; i += kReadUnroll * kBlock) {
        d2 v[kReadUnroll];
#pragma unroll
        for (int u = 0; u < kReadUnroll; ++u) v[u] = ldnt(src + i + u * kBlock);
#pragma unroll
        for (int u = 0; u < kReadUnroll; ++u) acc += v[u];
    }
    for (; i < e1; i += kBlock) acc += ldnt(src + i);
    const d2 tot = block_sum(acc, lds);
    if (threadIdx.x == 0) out[blockIdx.x] = tot;
}

static int read_stream_impl(const void* src, size_t bytes, void* out, size_t out_bytes,
                            void* stream)
{
    if (bytes > 0 && !src) return -1;
    if (bytes % 16 || ((uintptr_t)src & 15)) return -2;
    const int64_t n16 = (int64_t)(bytes / 16);
    const int64_t blocks = (n16 + kReadSlab16 - 1) / kReadSlab16;
    if (blocks > 0 && (!out || ((uintptr_t)out & 15))) return -3;
    if (out_bytes < (size_t)blocks * 16) return -4;
    if (blocks > INT32_MAX) return -2;
    if (blocks == 0) return 0;
    k_read_stream<<<(unsigned)blocks, kBlock, 0, (hipStream_t)stream>>>((const d2*)src, n16,
                                                                         (d2*)out);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? 0 : (int)e;
}

// --------------------------------------------- allocation-free products
//
// ccg_matvec_noalloc: the products of ccg_matvec for callers that cannot
// allocate device memory.  The partial sums of the A^H x band walk and of the
// upper-triangle tiles go to a fixed device array instead of a stream-ordered
// allocation.  Every GPU holds its own copy of a __device__ array (the loader
// places one per device) until the process ends; host code never passes the
// array's name to a kernel (on the host that name is a stand-in, not a device
// address) but the address hipGetSymbolAddress returns for the current
// device, looked up once per device on the first call there.  Both partial
// kinds are written in full before they are read (every band or tile writes
// its partial of every element it covers), so nothing needs clearing between
// calls; calls that overlap on one GPU share the array and race.
constexpr size_t kNoAllocScratchBytes = (size_t)CCG_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices];

// The device address of `scratch` on the current device.
static int noalloc_scratch(void** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return (int)e;
    if (dev < 0 || dev >= kMaxDevices) return (int)hipErrorInvalidDevice;
    std::lock_guard<std::mutex> guard(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return (int)e;
        if (!ptr) return (int)hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return 0;
}

// Bytes of partial sums a product of kind op needs at size n (0 for A x).
static size_t noalloc_need(int op, int64_t n)
{
    if (op == CCG_OP_C) {
        const GemvCShape sh = gemv_c_shape(n);
        return (size_t)sh.nbands * (size_t)n * sizeof(d2);
    }
    if (op == CCG_OP_S) return sym_part_bytes(n);
    return 0;
}

static int matvec_noalloc_impl(int op, int64_t n, const ccg_z* A, int64_t lda, const ccg_z* x,
                               ccg_z* y, void* stream)
{
    if (op != CCG_OP_N && op != CCG_OP_C && op != CCG_OP_S) return -1;
    if (n < 0 || n > kMaxN) return -2;
    if (n == 0 || op == CCG_OP_N)
        return matvec_impl(op, n, A, lda, x, y, nullptr, 0, stream, false);
    if (noalloc_need(op, n) > kNoAllocScratchBytes) return -2;  // beyond the fixed array
    void* ptr = nullptr;
    const int rc = noalloc_scratch(&ptr);
    if (rc) return rc;
    return matvec_impl(op, n, A, lda, x, y, ptr, kNoAllocScratchBytes, stream, false);
}

// ------------------------------------------------------- mixed precision
//
// FP64 iterative refinement around an inner complex64 BiCGSTAB (the single /
// double switch of the ddprecision module, Usage section, used inside one
// solve): the outer residual r = y - A x comes from the complex128 A in FP64,
// the correction d solves A32 d = r / ||r|| in complex64 (FP32 product
// accumulation, FP64 reductions and scalars) to a loose relative tolerance,
// and x += ||r|| d is applied in FP64.  The outer loop stops on the FP64 true
// residual, so info 0 means ||y - A x|| <= tol ||y|| exactly as for
// ccg_bicgstab.

// r = y - A x with FP64 products, block partials of ||r||^2
__global__ __launch_bounds__(kBlockN) void k_mix_resid(const d2* __restrict__ A, int64_t lda,
                                                       int n, const d2* __restrict__ x,
                                                       const d2* __restrict__ y,
                                                       d2* __restrict__ r, d2* part)
{
    __shared__ d2 red[kWN][kR];
    __shared__ d2 lds[kMaxWaves];
    const int row0 = blockIdx.x * kR;
    gemv_n_block<kR, kU, kWN>(A, lda, n, x, row0, red);
    const int t = threadIdx.x;
    d2 v0 = d2{0.0, 0.0};
    if (t < kR && row0 + t < n) {
        const d2 ri = y[row0 + t] - gemv_n_row_total<kR, kWN>(red, t);
        r[row0 + t] = ri;
        v0.x = cabs2(ri);
    }
    write_partials(v0, d2{0.0, 0.0}, part, lds);
}

// r = y (x0 = 0) and x = 0, block partials of ||r||^2
__global__ __launch_bounds__(kBlock) void k_mix_copy(int n, const d2* __restrict__ y,
                                                     d2* __restrict__ x, d2* __restrict__ r,
                                                     d2* part)
{
    __shared__ d2 lds[kMaxWaves];
    d2 v0 = d2{0.0, 0.0};
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        const d2 yi = y[i];
        r[i] = yi;
        x[i] = d2{0.0, 0.0};
        v0.x += cabs2(yi);
    }
    write_partials(v0, d2{0.0, 0.0}, part, lds);
}

// block partials of ||y||^2
__global__ __launch_bounds__(kBlock) void k_mix_norm(int n, const d2* __restrict__ y, d2* part)
{
    __shared__ d2 lds[kMaxWaves];
    d2 v0 = d2{0.0, 0.0};
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock)
        v0.x += cabs2(y[i]);
    write_partials(v0, d2{0.0, 0.0}, part, lds);
}

__global__ __launch_bounds__(kBlock) void k_mix_zero(int n, d2* __restrict__ x)
{
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock)
        x[i] = d2{0.0, 0.0};
}

// total of nblocks partial pairs -> out (one block)
__global__ __launch_bounds__(kBlock) void k_mix_total(const d2* part, int nblocks, d2* out)
{
    __shared__ d2 lds[kMaxWaves];
    d2 t0, t1;
    reduce_partials(part, nblocks, lds, t0, t1);
    if (threadIdx.x == 0) *out = t0;
}

// r32 = complex64(r * scale)
__global__ __launch_bounds__(kBlock) void k_mix_round(int n, const d2* __restrict__ r,
                                                      double scale, f2* __restrict__ r32)
{
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        const d2 v = r[i];
        r32[i] = f2{(float)(v.x * scale), (float)(v.y * scale)};
    }
}

// x += scale * d32 in FP64
__global__ __launch_bounds__(kBlock) void k_mix_update(int n, const f2* __restrict__ d32,
                                                       double scale, d2* __restrict__ x)
{
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        const f2 d = d32[i];
        d2 xi = x[i];
        xi.x = __builtin_fma(scale, (double)d.x, xi.x);
        xi.y = __builtin_fma(scale, (double)d.y, xi.y);
        x[i] = xi;
    }
}

// dst = complex64(src), row by row
__global__ __launch_bounds__(kBlock) void k_round_c64(int64_t rows, int64_t cols,
                                                      const d2* __restrict__ src, int64_t lds_,
                                                      f2* __restrict__ dst, int64_t ldd)
{
    const int64_t total = rows * cols;
    for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * kBlock) {
        const int64_t i = e / cols, j = e - i * cols;
        const d2 v = src[i * lds_ + j];
        dst[i * ldd + j] = f2{(float)v.x, (float)v.y};
    }
}

struct MixLayout {
    size_t inner, r64, r32, d32, part, tot, total;
};

static MixLayout mix_layout(int64_t n)
{
    MixLayout L{};
    const size_t nn = (size_t)(n > 0 ? n : 1);
    size_t off = 0;
    L.inner = off;
    off += layout(CCG_WS_BICGSTAB, n).total;  // complex128-sized: room for complex64
    L.r64 = off;
    off += align256(nn * sizeof(d2));
    L.r32 = off;
    off += align256(nn * sizeof(f2));
    L.d32 = off;
    off += align256(nn * sizeof(f2));
    L.part = off;
    int64_t pb = blocks_n(n) > blocks_e(n) ? blocks_n(n) : blocks_e(n);
    off += align256((size_t)pb * 2 * sizeof(d2));
    L.tot = off;
    off += 256;
    L.total = off;
    return L;
}

static int mixed_impl(int64_t n, const ccg_z* A, int64_t lda, const ccg_c* A32, int64_t lda32,
                      const ccg_z* y, ccg_z* x, double tol, int32_t maxit, double tol_inner,
                      int32_t maxit_inner, uint32_t flags, void* work, size_t work_bytes,
                      ccg_mixed_result* res, double* outer_res, void* stream)
{
    if (n < 0 || n > kMaxN) return -1;
    if (n > 0 && !A) return -2;
    if (lda < (n > 1 ? n : 1)) return -3;
    if (n > 0 && !A32) return -4;
    if (lda32 < (n > 1 ? n : 1)) return -5;
    if (n > 0 && !y) return -6;
    if (n > 0 && !x) return -7;
    if (!(tol > 0.0) || !std::isfinite(tol)) return -8;
    if (maxit < 0) return -9;
    if (!(tol_inner > 0.0) || !(tol_inner < 1.0)) return -10;
    if (maxit_inner < 1) return -11;
    if (flags & ~CCG_X0_ZERO) return -12;
    const MixLayout ML = mix_layout(n);
    if (n > 0 && (!work || ((uintptr_t)work & 255))) return -13;
    if (n > 0 && work_bytes < ML.total) return -14;
    if (!res) return -15;
    std::memset(res, 0, sizeof *res);
    res->relres_true = __builtin_nan("");
    if (outer_res)
        for (int32_t j = 0; j <= maxit; ++j) outer_res[j] = __builtin_nan("");
    if (n == 0) {
        res->relres_true = 0.0;
        return 0;
    }
    hipStream_t s = (hipStream_t)stream;
    char* base = (char*)work;
    d2* r64 = (d2*)(base + ML.r64);
    f2* r32 = (f2*)(base + ML.r32);
    f2* d32 = (f2*)(base + ML.d32);
    d2* part = (d2*)(base + ML.part);
    d2* tot = (d2*)(base + ML.tot);
    const int gN = blocks_n(n), gE = blocks_e(n);
    hipError_t e;

    // the inner solver: BiCGSTAB on complex64 vectors, A32 d = r32
    Args in = make_args(CCG_WS_BICGSTAB, n, nullptr, lda32, nullptr, nullptr, base + ML.inner,
                        nullptr);
    in.A = (const d2*)A32;
    in.y = (const d2*)r32;
    in.x = (d2*)d32;
    in.vec16 = rows16(A32, lda32);  // the inner vectors are 256-byte aligned

    // ||y||^2
    k_mix_norm<<<gE, kBlock, 0, s>>>((int)n, (const d2*)y, part);
    k_mix_total<<<1, kBlock, 0, s>>>(part, gE, tot);
    d2 hy;
    if ((e = hipMemcpyAsync(&hy, tot, sizeof hy, hipMemcpyDeviceToHost, s)) != hipSuccess)
        return (int)e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return (int)e;
    const double ny2 = hy.x;
    if (!std::isfinite(ny2)) {  // x is left as it was
        res->info = 4;
        return 0;
    }
    if (ny2 == 0.0) {  // y = 0: x = 0
        k_mix_zero<<<gE, kBlock, 0, s>>>((int)n, (d2*)x);
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return (int)e;
        res->relres_true = 0.0;
        return 0;
    }
    auto residual_norm2 = [&](bool x_zero, double* rr) -> int {
        if (x_zero) {
            // r = y, x = 0: ||r||^2 is ||y||^2, summed by the same blocks in
            // the same order as k_mix_norm did above (the same bits), so no
            // second round trip to the host
            k_mix_copy<<<gE, kBlock, 0, s>>>((int)n, (const d2*)y, (d2*)x, r64, part);
            *rr = ny2;
            return (int)hipGetLastError();
        }
        k_mix_resid<<<gN, kBlockN, 0, s>>>((const d2*)A, lda, (int)n, (const d2*)x,
                                           (const d2*)y, r64, part);
        k_mix_total<<<1, kBlock, 0, s>>>(part, gN, tot);
        d2 h;
        if ((e = hipMemcpyAsync(&h, tot, sizeof h, hipMemcpyDeviceToHost, s)) != hipSuccess)
            return (int)e;
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return (int)e;
        *rr = h.x;
        return 0;
    };

    const double thr2 = tol * tol * ny2;
    for (int outer = 0;; ++outer) {
        double rr = 0.0;
        int rc = residual_norm2(outer == 0 && (flags & CCG_X0_ZERO), &rr);
        if (rc) return rc;
        if (outer > 0 || !(flags & CCG_X0_ZERO)) res->matvecs64++;
        res->relres_true = std::sqrt(rr / ny2);
        if (outer_res) outer_res[outer] = res->relres_true;
        if (!std::isfinite(rr)) { res->info = 4; break; }
        if (rr <= thr2) { res->info = 0; break; }
        if (outer >= maxit) { res->info = 1; break; }
        const double nr = std::sqrt(rr);
        k_mix_round<<<gE, kBlock, 0, s>>>((int)n, r64, 1.0 / nr, r32);
        ccg_result ir{};
        rc = run_solver<M_BICG, f2>(in, CCG_X0_ZERO, maxit_inner, tol_inner * tol_inner, &ir, s,
                                    /*no_confirm=*/1);
        if (rc) return rc;
        res->outer++;
        res->inner_iters += ir.iters;
        res->matvecs32 += ir.matvecs;
        if (ir.info == 4) { res->info = 4; break; }
        // a breakdown before the first inner update leaves d = 0: the next
        // step would repeat this one exactly
        if ((ir.info == 2 || ir.info == 3) && ir.iters == 0) { res->info = ir.info; break; }
        k_mix_update<<<gE, kBlock, 0, s>>>((int)n, d32, nr, (d2*)x);
        if ((e = hipGetLastError()) != hipSuccess) return (int)e;
    }
    return 0;
}


// ------------------------------------------------------ structured operator

static constexpr int64_t kT3MaxEdge = kT3MaxM / 2;  // lattice edge m <= 128

// The operator buffer: twiddles | evenness flag | K (M^3 points, or the
// (M/2 + 1)^2 M of the folded rows) | set-up scratch (M^3).
struct T3OpLayout {
    int M;
    size_t tw, even, K, S, total;
};

static T3OpLayout t3_op_layout(int64_t m)
{
    T3OpLayout L{};
    L.M = t3_padded((int)m);
    const size_t M3 = (size_t)L.M * L.M * L.M;
    L.tw = 0;
    L.even = align256((size_t)(L.M / 2) * sizeof(d2));
    L.K = L.even + 256;
    L.S = L.K + align256(M3 * sizeof(d2));
    L.total = L.S + align256(M3 * sizeof(d2));
    return L;
}

// Scratch of one product: G1 (M m mp) and G2 (M^2 mp).
static size_t t3_grid_bytes(int64_t m)
{
    const size_t M = (size_t)t3_padded((int)m), mp = (size_t)t3_row((int)m);
    return align256(M * m * mp * sizeof(d2)) + align256(M * M * mp * sizeof(d2));
}

static T3Geom t3_geom(int64_t m, const void* op, void* grids)
{
    const T3OpLayout L = t3_op_layout(m);
    T3Geom g{};
    g.m = (int)m;
    g.M = L.M;
    g.mp = t3_row((int)m);
    g.tw = (const d2*)((const char*)op + L.tw);
    g.even = (const int*)((const char*)op + L.even);
    g.K = (const d2*)((const char*)op + L.K);
    g.g1 = (d2*)grids;
    g.g2 = (d2*)((char*)grids + align256((size_t)L.M * m * g.mp * sizeof(d2)));
    return g;
}

static size_t t3_workspace(int method, int64_t m)
{
    if (method == CCG_WS_T3_MATVEC) return t3_grid_bytes(m);
    const int64_t n = m * m * m;
    return layout(method, n, t3_edge_tiles(m)).total + t3_grid_bytes(m);
}

template <int M>
static void t3_matvec_launch(const T3Geom& g, const d2* x, d2* y, hipStream_t s)
{
    const int64_t m = g.m, mp = g.mp;
    if constexpr (M <= kT3SmallM) {
        k_t3s_xy<M><<<(int)m, kT3PlaneThreads, 0, s>>>(g, x);
        k_t3s_z<M><<<(int)t3_tiles<M>(M * M), kBlock, 0, s>>>(g);
        k_t3s_yx<M><<<(int)m, kT3PlaneThreads, 0, s>>>(g, y);
    } else {
        k_t3p_x<M><<<(int)t3_tiles<M>(mp * m), kBlock, 0, s>>>(g, x);
        k_t3p_y<M><<<(int)t3_tiles<M>(mp * M), kBlock, 0, s>>>(g);
        k_t3p_z<M><<<(int)t3_tiles<M>(M * M), kBlock, 0, s>>>(g);
        k_t3p_yi<M><<<(int)t3_tiles<M>(mp * M), kBlock, 0, s>>>(g);
        k_t3p_xi<M><<<(int)t3_tiles<M>(mp * m), kBlock, 0, s>>>(g, y);
    }
}

template <int M>
static void t3_setup_launch(const T3Geom& g, const d2* table, d2* K, d2* S, hipStream_t s)
{
    k_t3_twiddle<<<(M / 2 + kBlock - 1) / kBlock, kBlock, 0, s>>>((d2*)g.tw, M);
    int* even = (int*)g.even;
    k_t3_even_init<<<1, 1, 0, s>>>(even);
    const int64_t w = 2 * g.m - 1;
    const int64_t eb = (w * w * w + kBlock - 1) / kBlock;
    k_t3_even<<<(int)(eb < 4096 ? eb : 4096), kBlock, 0, s>>>(table, g.m, even);
    const int tiles = (int)t3_tiles<M>(M * M);
    // K's region holds pass 1's output until pass 3 writes the transform
    k_t3_s1<M><<<tiles, kBlock, 0, s>>>(table, g, K);
    k_t3_s2<M><<<tiles, kBlock, 0, s>>>(g, K, S);
    k_t3_s3<M><<<tiles, kBlock, 0, s>>>(g, S, K, std::ldexp(1.0, -3 * T3Shape<M>::LG));
}

static int t3_setup_impl(int64_t m, const ccg_z* table, void* op, size_t op_bytes, void* stream)
{
    if (m < 1 || m > kT3MaxEdge) return -1;
    if (!table) return -2;
    if (!op || ((uintptr_t)op & 255)) return -3;
    const T3OpLayout L = t3_op_layout(m);
    if (op_bytes < L.total) return -4;
    hipStream_t s = (hipStream_t)stream;
    T3Geom g = t3_geom(m, op, nullptr);
    d2* K = (d2*)((char*)op + L.K);
    d2* S = (d2*)((char*)op + L.S);
#define T3_SETUP(Mc) t3_setup_launch<Mc>(g, (const d2*)table, K, S, s)
    T3_DISPATCH(L.M, T3_SETUP)
#undef T3_SETUP
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? 0 : (int)e;
}

static int t3_matvec_impl(int64_t m, const void* op, const ccg_z* x, ccg_z* y, void* work,
                          size_t work_bytes, void* stream)
{
    if (m < 0 || m > kT3MaxEdge) return -1;
    if (m == 0) return 0;
    if (!op || ((uintptr_t)op & 255)) return -2;
    if (!x) return -3;
    if (!y) return -4;
    if (!work || ((uintptr_t)work & 255)) return -5;
    if (work_bytes < t3_grid_bytes(m)) return -6;
    const T3Geom g = t3_geom(m, op, work);
    hipStream_t s = (hipStream_t)stream;
#define T3_MATVEC(Mc) t3_matvec_launch<Mc>(g, (const d2*)x, (d2*)y, s)
    T3_DISPATCH(g.M, T3_MATVEC)
#undef T3_MATVEC
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? 0 : (int)e;
}

template <int M>
static int t3_solve(int64_t m, const void* op, const ccg_z* y, ccg_z* x, double tol,
                    int32_t maxit, uint32_t flags, void* work, size_t work_bytes,
                    ccg_result* res, ccg_hist* hist, void* stream)
{
    if (m < 0 || m > kT3MaxEdge) return -1;
    if (m > 0 && (!op || ((uintptr_t)op & 255))) return -2;
    if (m > 0 && !y) return -3;
    if (m > 0 && !x) return -4;
    if (!(tol > 0.0) || !std::isfinite(tol)) return -5;
    if (maxit < 0) return -6;
    if (flags & ~CCG_X0_ZERO) return -7;
    const int method = ws_of(M);
    if (m > 0 && (!work || ((uintptr_t)work & 255))) return -8;
    if (m > 0 && work_bytes < t3_workspace(method, m)) return -9;
    if (!res) return -10;
    if (m == 0) {
        std::memset(res, 0, sizeof *res);
        res->relres_rec = res->relres_true = 0.0;
        return 0;
    }
    const int64_t n = m * m * m;
    const Layout L = layout(method, n, t3_edge_tiles(m));
    // make_args carves the vectors and partial buffers with the default
    // partial count; rebuild them here with the structured one
    Args a = make_args(method, n, nullptr, 1, y, x, work, hist);
    char* base = (char*)work;
    a.part[0] = (d2*)(base + L.partials);
    a.part[1] = (d2*)(base + L.partials + L.part_bytes);
    a.xpart[0] = (d2*)(base + L.xpartials);
    a.xpart[1] = (d2*)(base + L.xpartials + L.xpart_bytes);
    const size_t vbytes = align256((size_t)n * sizeof(d2));
    d2* vec[6] = {};
    for (int k = 0; k < L.nvec; ++k) vec[k] = (d2*)(base + L.vec + k * vbytes);
    if (method == CCG_WS_BICGSTAB) {
        a.r = vec[0]; a.rh = vec[1]; a.p = vec[2]; a.v = vec[3]; a.s = vec[4]; a.t = vec[5];
    } else if (method == CCG_WS_COCG) {
        a.r = vec[0]; a.p = vec[1]; a.v = vec[2];
    } else {
        a.r = vec[0]; a.z = vec[1]; a.p = vec[2]; a.w = vec[3];
    }
    a.t3 = t3_geom(m, op, base + L.total);
    return run_solver<M, d2, true>(a, flags, maxit, tol * tol, res, (hipStream_t)stream);
}
}  // namespace ccg

// ============================================================== C ABI

extern "C" {

size_t ccg_workspace_bytes(int method, int64_t n, int64_t nrhs)
{
    if (n < 0 || nrhs < 1) return 0;
    if (method == CCG_WS_MATMAT || method == CCG_WS_BICGSTAB_BLOCK ||
        method == CCG_WS_MATMAT_C64 || method == CCG_WS_BICGSTAB_BLOCK_MIXED)
        return ccg::block_workspace_bytes(method, n, nrhs);
    if (method == CCG_WS_MATVEC_C) {
        const ccg::GemvCShape sh = ccg::gemv_c_shape(n > 0 ? n : 1);
        return (size_t)sh.nbands * (size_t)(n > 0 ? n : 1) * sizeof(ccg_z);
    }
    if (method == CCG_WS_BICGSTAB || method == CCG_WS_CGNR || method == CCG_WS_COCG ||
        method == CCG_WS_COCR)
        return ccg::layout(method, n).total;
    if (method == CCG_WS_MATVEC_S) return ccg::sym_part_bytes(n);
    if (method == (CCG_WS_BICGSTAB | CCG_WS_SYM) || method == (CCG_WS_CGNR | CCG_WS_SYM) ||
        method == (CCG_WS_COCG | CCG_WS_SYM) || method == (CCG_WS_COCR | CCG_WS_SYM))
        return ccg::layout(method & ~CCG_WS_SYM, n, 0, true).total;
    if (method == CCG_WS_BICGSTAB_MIXED) return ccg::mix_layout(n).total;
    return 0;
}

int ccg_matvec(int op, int64_t n, const ccg_z* A, int64_t lda, const ccg_z* x, ccg_z* y,
               void* stream)
{
    return ccg::matvec_impl(op, n, A, lda, x, y, nullptr, 0, stream, true);
}

int ccg_matvec_ex(int op, int64_t n, const ccg_z* A, int64_t lda, const ccg_z* x, ccg_z* y,
                  void* work, size_t work_bytes, void* stream)
{
    return ccg::matvec_impl(op, n, A, lda, x, y, work, work_bytes, stream, false);
}

int ccg_read_stream(const void* src, size_t bytes, void* out, size_t out_bytes, void* stream)
{
    return ccg::read_stream_impl(src, bytes, out, out_bytes, stream);
}

int ccg_set_event_log(ccg_event_log* log)
{
    if (log && (log->capacity < 0 || (log->capacity > 0 && !log->events))) return -1;
    ccg::t_event_log = log;
    return 0;
}

int ccg_matvec_noalloc(int op, int64_t n, const ccg_z* A, int64_t lda, const ccg_z* x,
                       ccg_z* y, void* stream)
{
    return ccg::matvec_noalloc_impl(op, n, A, lda, x, y, stream);
}

int ccg_bicgstab(int64_t n, const ccg_z* A, int64_t lda, const ccg_z* y, ccg_z* x, double tol,
                 int32_t maxit, int32_t* info, void* stream)
{
    return ccg::solve_short<ccg::M_BICG>(n, A, lda, y, x, tol, maxit, info, stream);
}

int ccg_cgnr(int64_t n, const ccg_z* A, int64_t lda, const ccg_z* y, ccg_z* x, double tol,
             int32_t maxit, int32_t* info, void* stream)
{
    return ccg::solve_short<ccg::M_CGNR>(n, A, lda, y, x, tol, maxit, info, stream);
}

int ccg_bicgstab_ex(int64_t n, const ccg_z* A, int64_t lda, const ccg_z* y, ccg_z* x,
                    double tol, int32_t maxit, uint32_t flags, void* work, size_t work_bytes,
                    ccg_result* res, ccg_hist* hist, void* stream)
{
    return ccg::solve_ex<ccg::M_BICG>(n, A, lda, y, x, tol, maxit, flags, work, work_bytes, res, hist,
                               stream);
}

int ccg_cgnr_ex(int64_t n, const ccg_z* A, int64_t lda, const ccg_z* y, ccg_z* x, double tol,
                int32_t maxit, uint32_t flags, void* work, size_t work_bytes, ccg_result* res,
                ccg_hist* hist, void* stream)
{
    return ccg::solve_ex<ccg::M_CGNR>(n, A, lda, y, x, tol, maxit, flags, work, work_bytes, res,
                                hist, stream);
}

int ccg_bicgstab_mixed_ex(int64_t n, const ccg_z* A, int64_t lda, const ccg_c* A32,
                          int64_t lda32, const ccg_z* y, ccg_z* x, double tol, int32_t maxit,
                          double tol_inner, int32_t maxit_inner, uint32_t flags, void* work,
                          size_t work_bytes, ccg_mixed_result* res, double* outer_res,
                          void* stream)
{
    return ccg::mixed_impl(n, A, lda, A32, lda32, y, x, tol, maxit, tol_inner, maxit_inner,
                           flags, work, work_bytes, res, outer_res, stream);
}

int ccg_matvec_c64(int64_t n, const ccg_c* A, int64_t lda, const ccg_c* x, ccg_c* y,
                   void* stream)
{
    if (n < 0 || n > ccg::kMaxN) return -1;
    if (n > 0 && !A) return -2;
    if (lda < (n > 1 ? n : 1)) return -3;
    if (n > 0 && !x) return -4;
    if (n > 0 && !y) return -5;
    if (n == 0) return 0;
    const char *xb = (const char*)x, *yb = (const char*)y;
    const size_t vb = (size_t)n * sizeof(ccg_c);
    if (xb < yb + vb && yb < xb + vb) return -5;
    const bool v16 = ccg::rows16(A, lda) && ((uintptr_t)x & 15) == 0;
    const int nblk = (int)((n + ccg::kRf - 1) / ccg::kRf);
    ccg::k_gemv_n_plain_f<<<nblk, ccg::kBlockNf, 0, (hipStream_t)stream>>>(
        (const ccg::f2*)A, lda, (int)n, (const ccg::f2*)x, (ccg::f2*)y, v16);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? 0 : (int)e;
}

int ccg_round_c64(int64_t rows, int64_t cols, const ccg_z* src, int64_t lds, ccg_c* dst,
                  int64_t ldd, void* stream)
{
    if (rows < 0) return -1;
    if (cols < 0) return -2;
    if (rows > 0 && cols > 0 && !src) return -3;
    if (lds < (cols > 1 ? cols : 1)) return -4;
    if (rows > 0 && cols > 0 && !dst) return -5;
    if (ldd < (cols > 1 ? cols : 1)) return -6;
    if (rows == 0 || cols == 0) return 0;
    int64_t blocks = (rows * cols + ccg::kBlock - 1) / ccg::kBlock;
    if (blocks > 4096) blocks = 4096;
    ccg::k_round_c64<<<(int)blocks, ccg::kBlock, 0, (hipStream_t)stream>>>(
        rows, cols, (const ccg::d2*)src, lds, (ccg::f2*)dst, ldd);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? 0 : (int)e;
}

int ccg_cocg(int64_t n, const ccg_z* A, int64_t lda, const ccg_z* y, ccg_z* x, double tol,
             int32_t maxit, int32_t* info, void* stream)
{
    return ccg::solve_short<ccg::M_COCG>(n, A, lda, y, x, tol, maxit, info, stream);
}

int ccg_cocr(int64_t n, const ccg_z* A, int64_t lda, const ccg_z* y, ccg_z* x, double tol,
             int32_t maxit, int32_t* info, void* stream)
{
    return ccg::solve_short<ccg::M_COCR>(n, A, lda, y, x, tol, maxit, info, stream);
}

int ccg_cocg_ex(int64_t n, const ccg_z* A, int64_t lda, const ccg_z* y, ccg_z* x, double tol,
                int32_t maxit, uint32_t flags, void* work, size_t work_bytes, ccg_result* res,
                ccg_hist* hist, void* stream)
{
    return ccg::solve_ex<ccg::M_COCG>(n, A, lda, y, x, tol, maxit, flags, work, work_bytes,
                                      res, hist, stream);
}

int ccg_cocr_ex(int64_t n, const ccg_z* A, int64_t lda, const ccg_z* y, ccg_z* x, double tol,
                int32_t maxit, uint32_t flags, void* work, size_t work_bytes, ccg_result* res,
                ccg_hist* hist, void* stream)
{
    return ccg::solve_ex<ccg::M_COCR>(n, A, lda, y, x, tol, maxit, flags, work, work_bytes,
                                      res, hist, stream);
}

size_t ccg_t3_op_bytes(int64_t m)
{
    if (m < 1 || m > ccg::kT3MaxEdge) return 0;
    return ccg::t3_op_layout(m).total;
}

size_t ccg_t3_workspace_bytes(int method, int64_t m)
{
    if (m < 1 || m > ccg::kT3MaxEdge) return 0;
    if (method != CCG_WS_T3_MATVEC && method != CCG_WS_BICGSTAB && method != CCG_WS_COCG &&
        method != CCG_WS_COCR)
        return 0;
    return ccg::t3_workspace(method, m);
}

int ccg_t3_setup(int64_t m, const ccg_z* table, void* op, size_t op_bytes, void* stream)
{
    return ccg::t3_setup_impl(m, table, op, op_bytes, stream);
}

int ccg_t3_matvec(int64_t m, const void* op, const ccg_z* x, ccg_z* y, void* work,
                  size_t work_bytes, void* stream)
{
    return ccg::t3_matvec_impl(m, op, x, y, work, work_bytes, stream);
}

int ccg_t3_bicgstab_ex(int64_t m, const void* op, const ccg_z* y, ccg_z* x, double tol,
                       int32_t maxit, uint32_t flags, void* work, size_t work_bytes,
                       ccg_result* res, ccg_hist* hist, void* stream)
{
    return ccg::t3_solve<ccg::M_BICG>(m, op, y, x, tol, maxit, flags, work, work_bytes, res,
                                      hist, stream);
}

int ccg_t3_cocg_ex(int64_t m, const void* op, const ccg_z* y, ccg_z* x, double tol,
                   int32_t maxit, uint32_t flags, void* work, size_t work_bytes, ccg_result* res,
                   ccg_hist* hist, void* stream)
{
    return ccg::t3_solve<ccg::M_COCG>(m, op, y, x, tol, maxit, flags, work, work_bytes, res,
                                      hist, stream);
}

int ccg_t3_cocr_ex(int64_t m, const void* op, const ccg_z* y, ccg_z* x, double tol,
                   int32_t maxit, uint32_t flags, void* work, size_t work_bytes, ccg_result* res,
                   ccg_hist* hist, void* stream)
{
    return ccg::t3_solve<ccg::M_COCR>(m, op, y, x, tol, maxit, flags, work, work_bytes, res,
                                      hist, stream);
}

}  // extern "C"
