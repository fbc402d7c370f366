// ccg_solvers.hip -- BiCGSTAB and CGNR for dense complex128 A x = y on
// gfx950, and the matrix-vector entry points of the C ABI (include/ccg.h).
//
// Methods: the bicgstab and cgnr codes of the PIM90 set (Codes, section 2.1),
// with the matrix-vector product apart from the iteration (Abstract; Usage:
// matvec / cmatvec) and the stop rule driven by a tolerance and a budget
// (Usage: epsilon_err, maxit).  The paper prints no algorithm; the steps are
// van der Vorst's BiCGSTAB and CG on the normal equations, each written as a
// short fixed sequence of kernels per iteration:
//
//   BiCGSTAB slot: p-update | v = A p (+ r^H v, |v|^2) | s = r - alpha v
//                  (+ |s|^2) | t = A s (+ t^H s, |t|^2) | x, r update
//                  (+ |r|^2, r^H r)
//   CGNR slot:     w = A p (+ |w|^2) | x, r update (+ |r|^2) | A^H r band
//                  partials | z = band sum (+ |z|^2) | p-update
//
// Every reduction is fused into the kernel that produces its operand; the
// block partials go to the last block of the grid (atomic ticket), which adds
// them in a fixed order and runs the method's scalar step (alpha, omega,
// beta, rho, stop and breakdown tests) in device memory.  No scalar crosses to
// the host during a solve.  A device phase word drives the control flow:
// every kernel reads it on entry and does its part only in the phases where it
// has one, so the host enqueues the same slot over and over and learns that
// the solve is over from a one-word status copied to pinned host memory at
// the end of each slot, a few slots behind the device.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/ccg.h"
#include "ccg_device.h"
#include "ccg_gemv.h"

namespace ccg {

// ------------------------------------------------------------------ state

enum Phase : int {
    PH_RUN = 0,      // iterating
    PH_HALF = 1,     // BiCGSTAB converged at s: finish x, then confirm
    PH_CONFIRM = 2,  // compute the true residual next
    PH_RESTART = 3,  // true residual replaced r: start a new direction
    PH_ZERO = 4,     // y == 0: x = 0 and stop
    PH_DONE = 5,
};

enum Ticket : int {
    T_NORMY = 0, T_SETUP, T_V, T_S, T_T, T_XR, T_W, T_XR2, T_Z2, T_COUNT
};

struct alignas(16) SolverState {
    int phase, restart, info, iters;
    int matvecs, confirms, maxit, pad0;
    double ny2, thr2, rh2, rr;
    double relres_rec, relres_true, gamma, pad1;
    d2 rho, rho_old, alpha, omega, beta;
    unsigned tickets[16];
};
static_assert(sizeof(SolverState) <= 1024, "state block");

struct Args {
    const d2* A;
    int64_t lda;
    int n;
    int nbands_c;
    GemvCShape csh;
    const d2* y;
    d2* x;
    d2 *r, *rh, *p, *v, *s, *t;  // BiCGSTAB vectors
    d2 *z, *w, *zpart;           // CGNR vectors and A^H band partials
    d2* partials;
    SolverState* st;
    ccg_hist* hist;
    double tol2;
};

constexpr int kR = 4;  // rows per wavefront in A x
constexpr int kU = 2;  // 64-element column chunks per step in A x
constexpr int kUC = 8; // rows per step in A^H x

__device__ __forceinline__ int read_phase(const SolverState* st)
{
    return __builtin_amdgcn_readfirstlane(*(volatile const int*)&st->phase);
}

__device__ __forceinline__ void finish(SolverState* st, int info)
{
    st->info = info;
    st->phase = PH_DONE;
}

__device__ __forceinline__ double relres(double sq, double ny2) { return sqrt(sq / ny2); }

// After r = y - A x (or r = y when x0 = 0) at set-up.
__device__ void setup_scalar(SolverState* st, double rr, bool bicg)
{
    if (!__builtin_isfinite(rr)) { finish(st, 4); return; }
    st->rr = rr;
    st->relres_rec = relres(rr, st->ny2);
    if (rr <= st->thr2) { st->phase = PH_CONFIRM; return; }
    st->restart = 1;
    if (bicg) {
        st->rh2 = rr;
        st->rho = d2{rr, 0.0};
        if (st->maxit <= 0) { finish(st, 1); return; }
        st->phase = PH_RUN;
    } else {
        st->phase = PH_RESTART;  // z = A^H r, p = z come next
    }
}

// After the true residual rt = y - A x of a confirmation.
__device__ void confirm_scalar(SolverState* st, double rtt, bool bicg)
{
    st->matvecs++;
    st->confirms++;
    st->relres_true = relres(rtt, st->ny2);
    if (!__builtin_isfinite(rtt)) { finish(st, 4); return; }
    if (rtt <= st->thr2) { finish(st, 0); return; }
    st->rr = rtt;
    st->relres_rec = relres(rtt, st->ny2);
    if (st->iters >= st->maxit) { finish(st, 1); return; }
    if (bicg) {
        st->rh2 = rtt;
        st->rho = d2{rtt, 0.0};
        st->restart = 1;
    }
    st->phase = PH_RESTART;
}

// --------------------------------------------------------- common kernels

__global__ void k_init(SolverState* st, int maxit)
{
    if (threadIdx.x < 16) st->tickets[threadIdx.x] = 0u;
    if (threadIdx.x == 0) {
        st->phase = PH_RUN;
        st->restart = 1;
        st->info = -1;
        st->iters = st->matvecs = st->confirms = 0;
        st->maxit = maxit;
        st->ny2 = st->thr2 = st->rh2 = st->rr = st->gamma = 0.0;
        st->relres_rec = st->relres_true = __builtin_nan("");
        st->rho = st->rho_old = st->alpha = st->omega = st->beta = d2{0.0, 0.0};
    }
}

// Copy the phase word to pinned host memory (end-of-slot status).
__global__ void k_status(const SolverState* st, int* ring_slot)
{
    if (threadIdx.x == 0) {
        int ph = *(volatile const int*)&st->phase;
        __hip_atomic_store(ring_slot, ph, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

// ||y||^2 and the stop threshold.
__global__ __launch_bounds__(kBlock) void k_norm_y(Args a)
{
    d2 pv[1] = {d2{0.0, 0.0}};
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < a.n; i += gridDim.x * kBlock)
        pv[0].x += cabs2(a.y[i]);
    d2 tot[1];
    if (reduce_to_last_block<1>(pv, a.partials, &a.st->tickets[T_NORMY], tot) &&
        threadIdx.x == 0) {
        SolverState* st = a.st;
        double ny2 = tot[0].x;
        st->ny2 = ny2;
        if (!__builtin_isfinite(ny2)) finish(st, 4);
        else if (ny2 == 0.0) st->phase = PH_ZERO;
        else st->thr2 = a.tol2 * ny2;
    }
}

// Set-up when the caller says x0 = 0: x = 0, r = y (and r^ = y).
template <bool BICG>
__global__ __launch_bounds__(kBlock) void k_setup_x0zero(Args a)
{
    const int ph = read_phase(a.st);
    if (ph != PH_RUN && ph != PH_ZERO) return;
    d2 pv[1] = {d2{0.0, 0.0}};
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < a.n; i += gridDim.x * kBlock) {
        a.x[i] = d2{0.0, 0.0};
        if (ph == PH_RUN) {
            const d2 yi = a.y[i];
            a.r[i] = yi;
            if (BICG) a.rh[i] = yi;
            pv[0].x += cabs2(yi);
        }
    }
    d2 tot[1];
    if (reduce_to_last_block<1>(pv, a.partials, &a.st->tickets[T_SETUP], tot) &&
        threadIdx.x == 0) {
        SolverState* st = a.st;
        if (ph == PH_ZERO) {
            st->relres_rec = st->relres_true = 0.0;
            finish(st, 0);
        } else {
            setup_scalar(st, tot[0].x, BICG);
        }
    }
}

// ------------------------------------------------- A x kernels with roles

enum Role { ROLE_SETUP_B, ROLE_SETUP_C, ROLE_V, ROLE_T, ROLE_W };

template <Role RO>
__device__ __forceinline__ int role_mode(int ph)
{
    switch (RO) {
    case ROLE_SETUP_B:
    case ROLE_SETUP_C:
        return (ph == PH_RUN || ph == PH_ZERO) ? ph : -1;
    case ROLE_V:
        return (ph == PH_RUN || ph == PH_RESTART || ph == PH_CONFIRM) ? ph : -1;
    case ROLE_T:
        return ph == PH_RUN ? ph : -1;
    case ROLE_W:
        return (ph == PH_RUN || ph == PH_CONFIRM) ? ph : -1;
    }
    return -1;
}

template <Role RO>
__global__ __launch_bounds__(kBlock) void k_gemv_n_role(Args a)
{
    const int mode = role_mode<RO>(read_phase(a.st));
    if (mode < 0) return;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave_id = blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
    const int row0 = wave_id * kR;
    const int n = a.n;

    // residual-type products read x; the others read a Krylov vector
    const bool resid = (RO == ROLE_SETUP_B || RO == ROLE_SETUP_C || mode == PH_CONFIRM);
    const d2* in = resid ? a.x : (RO == ROLE_T ? a.s : a.p);

    d2 pv[2] = {d2{0.0, 0.0}, d2{0.0, 0.0}};
    if (mode == PH_ZERO) {
        // y == 0: zero this wavefront's rows of x
        if (lane < kR && row0 + lane < n) a.x[row0 + lane] = d2{0.0, 0.0};
    } else if (row0 < n) {
        d2 acc[kR];
        gemv_n_wave<kR, kU>(a.A, a.lda, n, in, row0, acc);
        // lane 0 finishes the wavefront's rows: output and dot-product terms
        if (lane == 0) {
#pragma unroll
            for (int r = 0; r < kR; ++r) {
                const int i = row0 + r;
                if (i >= n) break;
                const d2 val = acc[r];
                if (resid) {
                    const d2 ri = a.y[i] - val;
                    a.r[i] = ri;
                    if (RO == ROLE_SETUP_B || RO == ROLE_V) a.rh[i] = ri;
                    pv[0].x += cabs2(ri);
                } else if (RO == ROLE_V) {
                    a.v[i] = val;
                    pv[0] = cfma_conj(a.rh[i], val, pv[0]);
                    pv[1].x += cabs2(val);
                } else if (RO == ROLE_T) {
                    a.t[i] = val;
                    pv[0] = cfma_conj(val, a.s[i], pv[0]);
                    pv[1].x += cabs2(val);
                } else {  // ROLE_W
                    a.w[i] = val;
                    pv[0].x += cabs2(val);
                }
            }
        }
    }

    unsigned* ticket = &a.st->tickets[RO == ROLE_SETUP_B || RO == ROLE_SETUP_C ? T_SETUP
                                      : RO == ROLE_V ? T_V : RO == ROLE_T ? T_T : T_W];
    d2 tot[2];
    if (!reduce_to_last_block<2>(pv, a.partials, ticket, tot) || threadIdx.x != 0) return;

    SolverState* st = a.st;
    if (mode == PH_ZERO) {
        st->relres_rec = st->relres_true = 0.0;
        finish(st, 0);
        return;
    }
    if (RO == ROLE_SETUP_B || RO == ROLE_SETUP_C) {
        st->matvecs++;
        setup_scalar(st, tot[0].x, RO == ROLE_SETUP_B);
        return;
    }
    if (mode == PH_CONFIRM) {
        confirm_scalar(st, tot[0].x, RO == ROLE_V);
        return;
    }
    st->matvecs++;
    if (RO == ROLE_V) {  // alpha = rho / sigma
        const d2 sigma = tot[0];
        const double vv = tot[1].x;
        st->restart = 0;
        if (!cfinite(sigma) || !__builtin_isfinite(vv)) { finish(st, 4); return; }
        if (cabs2(sigma) <= 1e-28 * st->rh2 * vv) { finish(st, 2); return; }
        const d2 al = cdiv(st->rho, sigma);
        if (!cfinite(al)) { finish(st, 4); return; }
        st->alpha = al;
        if (a.hist) {
            a.hist[st->iters].alpha_re = al.x;
            a.hist[st->iters].alpha_im = al.y;
        }
        st->phase = PH_RUN;
    } else if (RO == ROLE_T) {  // omega = t^H s / t^H t
        const d2 ts = tot[0];
        const double tt = tot[1].x;
        if (!__builtin_isfinite(tt) || !cfinite(ts)) { finish(st, 4); return; }
        if (tt == 0.0) { finish(st, 3); return; }
        const d2 om = d2{ts.x / tt, ts.y / tt};
        if (om.x == 0.0 && om.y == 0.0) { finish(st, 3); return; }
        st->omega = om;
        if (a.hist) {
            a.hist[st->iters].omega_re = om.x;
            a.hist[st->iters].omega_im = om.y;
        }
    } else {  // ROLE_W: alpha = gamma / |w|^2
        const double ww = tot[0].x;
        if (!__builtin_isfinite(ww)) { finish(st, 4); return; }
        if (ww == 0.0) { finish(st, 2); return; }
        const double al = st->gamma / ww;
        st->alpha = d2{al, 0.0};
        if (a.hist) {
            a.hist[st->iters].alpha_re = al;
            a.hist[st->iters].alpha_im = 0.0;
        }
    }
}

// ------------------------------------------------------- BiCGSTAB vectors

// p = r (new direction) or p = r + beta (p - omega v)
__global__ __launch_bounds__(kBlock) void k_bicg_p(Args a)
{
    const int ph = read_phase(a.st);
    if (ph != PH_RUN && ph != PH_RESTART) return;
    const bool fresh = __builtin_amdgcn_readfirstlane(*(volatile const int*)&a.st->restart) != 0;
    const d2 beta = a.st->beta;
    const d2 omega = a.st->omega;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < a.n; i += gridDim.x * kBlock) {
        const d2 ri = a.r[i];
        if (fresh) {
            a.p[i] = ri;
        } else {
            const d2 q = cfma(d2{-omega.x, -omega.y}, a.v[i], a.p[i]);  // p - omega v
            a.p[i] = cfma(beta, q, ri);
        }
    }
}

// s = r - alpha v, |s|^2; half-step stop test
__global__ __launch_bounds__(kBlock) void k_bicg_s(Args a)
{
    if (read_phase(a.st) != PH_RUN) return;
    const d2 alpha = a.st->alpha;
    const d2 nal = d2{-alpha.x, -alpha.y};
    d2 pv[1] = {d2{0.0, 0.0}};
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < a.n; i += gridDim.x * kBlock) {
        const d2 si = cfma(nal, a.v[i], a.r[i]);
        a.s[i] = si;
        pv[0].x += cabs2(si);
    }
    d2 tot[1];
    if (!reduce_to_last_block<1>(pv, a.partials, &a.st->tickets[T_S], tot) ||
        threadIdx.x != 0)
        return;
    SolverState* st = a.st;
    const double ss = tot[0].x;
    if (!__builtin_isfinite(ss)) { finish(st, 4); return; }
    if (a.hist) a.hist[st->iters].res_half = relres(ss, st->ny2);
    if (ss <= st->thr2) {
        st->relres_rec = relres(ss, st->ny2);
        st->phase = PH_HALF;
    }
}

// x += alpha p + omega s, r = s - omega t, |r|^2, r^H r; or, after a
// half-step exit, x += alpha p.
__global__ __launch_bounds__(kBlock) void k_bicg_xr(Args a)
{
    const int ph = read_phase(a.st);
    if (ph != PH_RUN && ph != PH_HALF) return;
    const d2 alpha = a.st->alpha;
    const d2 omega = a.st->omega;
    const d2 nom = d2{-omega.x, -omega.y};
    d2 pv[2] = {d2{0.0, 0.0}, d2{0.0, 0.0}};
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < a.n; i += gridDim.x * kBlock) {
        d2 xi = cfma(alpha, a.p[i], a.x[i]);
        if (ph == PH_RUN) {
            const d2 si = a.s[i];
            xi = cfma(omega, si, xi);
            const d2 ri = cfma(nom, a.t[i], si);
            a.r[i] = ri;
            pv[0].x += cabs2(ri);
            pv[1] = cfma_conj(a.rh[i], ri, pv[1]);
        }
        a.x[i] = xi;
    }
    d2 tot[2];
    if (!reduce_to_last_block<2>(pv, a.partials, &a.st->tickets[T_XR], tot) ||
        threadIdx.x != 0)
        return;
    SolverState* st = a.st;
    st->iters++;
    if (ph == PH_HALF) {
        st->phase = PH_CONFIRM;
        return;
    }
    const double rr = tot[0].x;
    const d2 rho_new = tot[1];
    if (!__builtin_isfinite(rr)) { finish(st, 4); return; }
    if (a.hist) a.hist[st->iters - 1].res_full = relres(rr, st->ny2);
    st->rr = rr;
    st->relres_rec = relres(rr, st->ny2);
    if (rr <= st->thr2) { st->phase = PH_CONFIRM; return; }
    if (st->iters >= st->maxit) { finish(st, 1); return; }
    if (!cfinite(rho_new)) { finish(st, 4); return; }
    if (cabs2(rho_new) <= 1e-28 * st->rh2 * rr) { finish(st, 2); return; }
    const d2 beta = cmul(cdiv(rho_new, st->rho), cdiv(st->alpha, st->omega));
    if (!cfinite(beta)) { finish(st, 4); return; }
    st->rho_old = st->rho;
    st->rho = rho_new;
    st->beta = beta;
    if (a.hist) {
        a.hist[st->iters].beta_re = beta.x;
        a.hist[st->iters].beta_im = beta.y;
    }
}

// ----------------------------------------------------------- CGNR vectors

// x += alpha p, r -= alpha w, |r|^2; stop test
__global__ __launch_bounds__(kBlock) void k_cgnr_xr(Args a)
{
    if (read_phase(a.st) != PH_RUN) return;
    const double al = a.st->alpha.x;
    d2 pv[1] = {d2{0.0, 0.0}};
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < a.n; i += gridDim.x * kBlock) {
        const d2 pi = a.p[i];
        const d2 wi = a.w[i];
        d2 xi = a.x[i];
        xi.x = __builtin_fma(al, pi.x, xi.x);
        xi.y = __builtin_fma(al, pi.y, xi.y);
        d2 ri = a.r[i];
        ri.x = __builtin_fma(-al, wi.x, ri.x);
        ri.y = __builtin_fma(-al, wi.y, ri.y);
        a.x[i] = xi;
        a.r[i] = ri;
        pv[0].x += cabs2(ri);
    }
    d2 tot[1];
    if (!reduce_to_last_block<1>(pv, a.partials, &a.st->tickets[T_XR2], tot) ||
        threadIdx.x != 0)
        return;
    SolverState* st = a.st;
    st->iters++;
    const double rr = tot[0].x;
    if (!__builtin_isfinite(rr)) { finish(st, 4); return; }
    if (a.hist) a.hist[st->iters - 1].res_full = relres(rr, st->ny2);
    st->rr = rr;
    st->relres_rec = relres(rr, st->ny2);
    if (rr <= st->thr2) st->phase = PH_CONFIRM;
}

// A^H r, band partials
__global__ __launch_bounds__(kBlock) void k_cgnr_z1(Args a)
{
    const int ph = read_phase(a.st);
    if (ph != PH_RUN && ph != PH_RESTART) return;
    gemv_c_band<kUC>(a.A, a.lda, a.n, a.r, a.zpart, a.csh);
}

// z = sum of band partials, |z|^2; gamma, beta
__global__ __launch_bounds__(kBlock) void k_cgnr_z2(Args a)
{
    const int ph = read_phase(a.st);
    if (ph != PH_RUN && ph != PH_RESTART) return;
    d2 pv[1] = {d2{0.0, 0.0}};
    for (int j = blockIdx.x * kBlock + threadIdx.x; j < a.n; j += gridDim.x * kBlock) {
        const d2 zj = gemv_c_gather(a.zpart, a.n, a.csh.nbands, j);
        a.z[j] = zj;
        pv[0].x += cabs2(zj);
    }
    d2 tot[1];
    if (!reduce_to_last_block<1>(pv, a.partials, &a.st->tickets[T_Z2], tot) ||
        threadIdx.x != 0)
        return;
    SolverState* st = a.st;
    st->matvecs++;
    const double g = tot[0].x;
    if (!__builtin_isfinite(g)) { finish(st, 4); return; }
    if (g == 0.0) { finish(st, 2); return; }
    if (ph == PH_RESTART) {
        st->gamma = g;
        st->restart = 1;
        st->phase = PH_RUN;
    } else {
        const double beta = g / st->gamma;
        if (a.hist) {
            a.hist[st->iters - 1].beta_re = beta;
            a.hist[st->iters - 1].beta_im = 0.0;
        }
        st->beta = d2{beta, 0.0};
        st->gamma = g;
        st->restart = 0;
    }
    if (st->iters >= st->maxit) finish(st, 1);
}

// p = z (new direction) or p = z + beta p
__global__ __launch_bounds__(kBlock) void k_cgnr_p(Args a)
{
    if (read_phase(a.st) != PH_RUN) return;
    const bool fresh = __builtin_amdgcn_readfirstlane(*(volatile const int*)&a.st->restart) != 0;
    const double beta = a.st->beta.x;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < a.n; i += gridDim.x * kBlock) {
        const d2 zi = a.z[i];
        if (fresh) {
            a.p[i] = zi;
        } else {
            d2 pi = a.p[i];
            pi.x = __builtin_fma(beta, pi.x, zi.x);
            pi.y = __builtin_fma(beta, pi.y, zi.y);
            a.p[i] = pi;
        }
    }
}

// --------------------------------------------------------- plain products

__global__ __launch_bounds__(kBlock) void k_gemv_n_plain(const d2* __restrict__ A, int64_t lda,
                                                         int n, const d2* __restrict__ x,
                                                         d2* __restrict__ y)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int row0 = (blockIdx.x * kWavesPerBlock + threadIdx.x / kWave) * kR;
    if (row0 >= n) return;
    d2 acc[kR];
    gemv_n_wave<kR, kU>(A, lda, n, x, row0, acc);
    if (lane == 0) {
#pragma unroll
        for (int r = 0; r < kR; ++r)
            if (row0 + r < n) y[row0 + r] = acc[r];
    }
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

// ================================================================== host

static inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

static inline int blocks_n(int64_t n)
{
    const int64_t rows_per_block = (int64_t)kR * kWavesPerBlock;
    int64_t b = (n + rows_per_block - 1) / rows_per_block;
    return (int)(b < 1 ? 1 : b);
}

static inline int blocks_e(int64_t n)
{
    int64_t b = (n + kBlock - 1) / kBlock;
    if (b > 512) b = 512;
    return (int)(b < 1 ? 1 : b);
}

static constexpr int64_t kMaxN = (int64_t)1 << 30;

struct Layout {
    size_t state, partials, vec, zpart, total;
    int nvec;
};

static Layout layout(int method, int64_t n)
{
    Layout L{};
    const GemvCShape csh = gemv_c_shape(n > 0 ? n : 1);
    int64_t pb = blocks_n(n);
    if (pb < 512) pb = 512;
    if (csh.blocks() > pb) pb = csh.blocks();
    const size_t vbytes = align256((size_t)(n > 0 ? n : 1) * sizeof(d2));
    size_t off = 0;
    L.state = off;
    off += 1024;
    L.partials = off;
    off += align256((size_t)pb * 2 * sizeof(d2));
    L.nvec = method == CCG_WS_BICGSTAB ? 6 : method == CCG_WS_CGNR ? 4 : 0;
    L.vec = off;
    off += (size_t)L.nvec * vbytes;
    L.zpart = off;
    if (method == CCG_WS_CGNR || method == CCG_WS_MATVEC_C)
        off += align256((size_t)csh.nbands * (size_t)(n > 0 ? n : 1) * sizeof(d2));
    L.total = off;
    return L;
}

// Pinned, device-mapped ring of status words and the events that mark the
// end of each slot; one set per host thread and device, kept for the life of
// the process.
constexpr int kRing = 8;
constexpr int kLookahead = 2;

struct SyncCtx {
    int device = -1;
    int* ring_h = nullptr;
    int* ring_d = nullptr;
    hipEvent_t ev[kRing];
};

static hipError_t get_sync(SyncCtx** out)
{
    thread_local std::vector<SyncCtx*> ctxs;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    for (SyncCtx* c : ctxs)
        if (c->device == dev) { *out = c; return hipSuccess; }
    SyncCtx* c = new SyncCtx;
    c->device = dev;
    e = hipHostMalloc((void**)&c->ring_h, kRing * sizeof(int),
                      hipHostMallocMapped | hipHostMallocCoherent);
    if (e != hipSuccess) { delete c; return e; }
    e = hipHostGetDevicePointer((void**)&c->ring_d, c->ring_h, 0);
    if (e != hipSuccess) return e;
    for (int k = 0; k < kRing; ++k) {
        e = hipEventCreateWithFlags(&c->ev[k], hipEventDisableTiming);
        if (e != hipSuccess) return e;
    }
    ctxs.push_back(c);
    *out = c;
    return hipSuccess;
}

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
                      ccg_z* x, void* work, ccg_hist* hist, double tol)
{
    const Layout L = layout(method, n);
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
    } else {
        a.r = vec[0]; a.z = vec[1]; a.p = vec[2]; a.w = vec[3];
        a.zpart = (d2*)(base + L.zpart);
    }
    a.partials = (d2*)(base + L.partials);
    a.st = (SolverState*)(base + L.state);
    a.hist = hist;
    a.tol2 = tol * tol;
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

// Enqueue set-up, then slots until the status ring reports PH_DONE.
template <bool BICG>
static int run_solver(const Args& a, uint32_t flags, int32_t maxit, ccg_result* res,
                      hipStream_t s)
{
    SyncCtx* sc = nullptr;
    hipError_t e = get_sync(&sc);
    if (e != hipSuccess) return (int)e;
    const int gN = blocks_n(a.n);
    const int gE = blocks_e(a.n);
    const int gC = a.csh.blocks();

    k_init<<<1, 64, 0, s>>>(a.st, maxit);
    k_norm_y<<<gE, kBlock, 0, s>>>(a);
    if (flags & CCG_X0_ZERO)
        k_setup_x0zero<BICG><<<gE, kBlock, 0, s>>>(a);
    else if (BICG)
        k_gemv_n_role<ROLE_SETUP_B><<<gN, kBlock, 0, s>>>(a);
    else
        k_gemv_n_role<ROLE_SETUP_C><<<gN, kBlock, 0, s>>>(a);
    if ((e = hipGetLastError()) != hipSuccess) return (int)e;

    // Each slot advances the method by at most one iteration or one
    // confirmation; a confirmation is always preceded by an iteration or
    // by the set-up, so 2 * maxit + 4 slots always suffice.
    const int64_t max_slots = 2 * (int64_t)maxit + 4;
    for (int64_t slot = 0; slot < max_slots + kLookahead; ++slot) {
        if (slot < max_slots) {
            if (BICG) {
                k_bicg_p<<<gE, kBlock, 0, s>>>(a);
                k_gemv_n_role<ROLE_V><<<gN, kBlock, 0, s>>>(a);
                k_bicg_s<<<gE, kBlock, 0, s>>>(a);
                k_gemv_n_role<ROLE_T><<<gN, kBlock, 0, s>>>(a);
                k_bicg_xr<<<gE, kBlock, 0, s>>>(a);
            } else {
                k_gemv_n_role<ROLE_W><<<gN, kBlock, 0, s>>>(a);
                k_cgnr_xr<<<gE, kBlock, 0, s>>>(a);
                k_cgnr_z1<<<gC, kBlock, 0, s>>>(a);
                k_cgnr_z2<<<gE, kBlock, 0, s>>>(a);
                k_cgnr_p<<<gE, kBlock, 0, s>>>(a);
            }
            k_status<<<1, 64, 0, s>>>(a.st, sc->ring_d + slot % kRing);
            if ((e = hipGetLastError()) != hipSuccess) return (int)e;
            if ((e = hipEventRecord(sc->ev[slot % kRing], s)) != hipSuccess) return (int)e;
        }
        const int64_t seen = slot - kLookahead;
        if (seen >= 0) {
            if ((e = hipEventSynchronize(sc->ev[seen % kRing])) != hipSuccess) return (int)e;
            if (__atomic_load_n(&sc->ring_h[seen % kRing], __ATOMIC_ACQUIRE) == PH_DONE) break;
        }
    }
    SolverState hs;
    if ((e = hipMemcpyAsync(&hs, a.st, sizeof hs, hipMemcpyDeviceToHost, s)) != hipSuccess)
        return (int)e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return (int)e;
    read_result(hs, res);
    if (hs.phase != PH_DONE) res->info = 1;  // defensive: slot budget spent
    return 0;
}

template <bool BICG>
static int solve_ex(int64_t n, const ccg_z* A, int64_t lda, const ccg_z* y, ccg_z* x,
                    double tol, int32_t maxit, uint32_t flags, void* work, size_t work_bytes,
                    ccg_result* res, ccg_hist* hist, void* stream)
{
    int bad = check_common(n, A, lda, y, x, tol, maxit);
    if (bad) return bad;
    if (flags & ~CCG_X0_ZERO) return -8;
    const int method = BICG ? CCG_WS_BICGSTAB : CCG_WS_CGNR;
    if (n > 0 && !work) return -9;
    if (n > 0 && ((uintptr_t)work & 255)) return -9;
    if (n > 0 && work_bytes < layout(method, n).total) return -10;
    if (!res) return -11;
    if (n == 0) {
        std::memset(res, 0, sizeof *res);
        res->relres_rec = res->relres_true = 0.0;
        return 0;
    }
    const Args a = make_args(method, n, A, lda, y, x, work, hist, tol);
    return run_solver<BICG>(a, flags, maxit, res, (hipStream_t)stream);
}

template <bool BICG>
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
    const size_t bytes = layout(BICG ? CCG_WS_BICGSTAB : CCG_WS_CGNR, n).total;
    void* work = nullptr;
    hipError_t e = hipMallocAsync(&work, bytes, s);
    if (e != hipSuccess) return (int)e;
    int rc = solve_ex<BICG>(n, A, lda, y, x, tol, maxit, 0u, work, bytes, &res, nullptr, stream);
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
    if (op != CCG_OP_N && op != CCG_OP_C) return -1;
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
        k_gemv_n_plain<<<blocks_n(n), kBlock, 0, s>>>((const d2*)A, lda, (int)n, (const d2*)x,
                                                     (d2*)y);
        e = hipGetLastError();
        return e == hipSuccess ? 0 : (int)e;
    }
    const GemvCShape sh = gemv_c_shape(n);
    const size_t need = (size_t)sh.nbands * (size_t)n * sizeof(d2);
    void* part = work;
    if (own_ws) {
        if ((e = hipMallocAsync(&part, need, s)) != hipSuccess) return (int)e;
    } else {
        if (!work) return -8;
        if (work_bytes < need) return -9;
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

}  // namespace ccg

// ============================================================== C ABI

extern "C" {

size_t ccg_workspace_bytes(int method, int64_t n, int64_t nrhs)
{
    if (n < 0 || nrhs < 1) return 0;
    if (method == CCG_WS_MATVEC_C) {
        const ccg::GemvCShape sh = ccg::gemv_c_shape(n > 0 ? n : 1);
        return (size_t)sh.nbands * (size_t)(n > 0 ? n : 1) * sizeof(ccg_z);
    }
    if (method == CCG_WS_BICGSTAB || method == CCG_WS_CGNR)
        return ccg::layout(method, n).total;
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

int ccg_bicgstab(int64_t n, const ccg_z* A, int64_t lda, const ccg_z* y, ccg_z* x, double tol,
                 int32_t maxit, int32_t* info, void* stream)
{
    return ccg::solve_short<true>(n, A, lda, y, x, tol, maxit, info, stream);
}

int ccg_cgnr(int64_t n, const ccg_z* A, int64_t lda, const ccg_z* y, ccg_z* x, double tol,
             int32_t maxit, int32_t* info, void* stream)
{
    return ccg::solve_short<false>(n, A, lda, y, x, tol, maxit, info, stream);
}

int ccg_bicgstab_ex(int64_t n, const ccg_z* A, int64_t lda, const ccg_z* y, ccg_z* x,
                    double tol, int32_t maxit, uint32_t flags, void* work, size_t work_bytes,
                    ccg_result* res, ccg_hist* hist, void* stream)
{
    return ccg::solve_ex<true>(n, A, lda, y, x, tol, maxit, flags, work, work_bytes, res, hist,
                               stream);
}

int ccg_cgnr_ex(int64_t n, const ccg_z* A, int64_t lda, const ccg_z* y, ccg_z* x, double tol,
                int32_t maxit, uint32_t flags, void* work, size_t work_bytes, ccg_result* res,
                ccg_hist* hist, void* stream)
{
    return ccg::solve_ex<false>(n, A, lda, y, x, tol, maxit, flags, work, work_bytes, res,
                                hist, stream);
}

}  // extern "C"
