// ccg_krylov.h -- the scalar side of the Krylov solvers: phases, the
// pending-reduction kinds, the per-system state record and the scalar step
// that turns reduction totals into alpha, omega, beta, gamma and the stop,
// budget and breakdown decisions.  Shared by the single right-hand-side
// solvers and the block solver (one record per column).
#pragma once

#include "../../include/ccg.h"
#include "ccg_device.h"

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

// Reduction left for the next kernel to finish, and the scalar step that
// goes with it.
enum Pending : int {
    PK_NONE = 0,
    PK_NORMY,      // ||y||^2
    PK_SETUP_B0,   // block BiCGSTAB set-up, r = y (x0 = 0): ||r||^2
    PK_SETUP_B1,   // BiCGSTAB set-up, r = y - A x: ||r||^2
    PK_SETUP_C1,   // CGNR set-up, r = y - A x
    PK_ZERO,       // y == 0: x has been zeroed
    PK_V,          // r^H v, ||v||^2        -> alpha
    PK_CONFIRM_B,  // ||y - A x||^2 (BiCGSTAB)
    PK_CONFIRM_C,  // ||y - A x||^2 (CGNR)
    PK_S,          // ||s||^2               -> half-step test
    PK_T,          // t^H s, ||t||^2        -> omega
    PK_XR,         // ||r||^2, r^H r        -> stop test, beta
    PK_HALF,       // x += alpha p done after a half-step exit
    PK_W,          // ||w||^2               -> alpha (CGNR)
    PK_XR2,        // ||r||^2               -> stop test (CGNR)
    PK_Z_RUN,      // ||z||^2               -> beta (CGNR)
    PK_Z_RESTART,  // ||z||^2               -> gamma of a new direction (CGNR)
    PK_SETUP_G1,   // COCG set-up, r = y - A x: ||r||^2, (r, r)
    PK_CONFIRM_G,  // ||y - A x||^2, (r, r) of the true residual (COCG)
    PK_Q,          // (p, A p)              -> alpha (COCG)
    PK_XR_G,       // ||r||^2, (r, r)       -> stop test, beta (COCG)
    PK_U,          // (r, A r)              -> beta, budget (COCR)
    PK_WW,         // (A p, A p)            -> alpha (COCR)
    PK_XR_R,       // ||r||^2               -> stop test (COCR)
    // BiCGSTAB with the next direction formed in the x, r update (four
    // launches per iteration): rho' = r^H s - omega r^H t, so beta is known
    // before r is; its breakdown test waits for ||r||.
    PK_S2,         // ||s||^2, r^H s        -> half-step test
    PK_T3,         // t^H s, ||t||^2, r^H t -> omega, rho', beta
    PK_XRP,        // ||r||^2               -> stop test, rho' breakdown, beta
    // x0 = 0: ||y||^2 and the set-up sums come from one kernel (r = y, so
    // ||r||^2 = ||y||^2): the ||y|| step, then the set-up step
    PK_NY_SETUP_B0,  // BiCGSTAB
    PK_NY_SETUP_C0,  // CGNR, COCR
    PK_NY_SETUP_G0,  // COCG (+ (r, r))
};

// The solver's scalars in device memory.  Two copies alternate: a launch
// reads copy q and block 0 writes copy q ^ 1, so no block of a launch ever
// reads what its own launch writes.
struct alignas(16) SolverState {
    int phase, restart, info, iters;
    int matvecs, confirms, maxit, pending;
    int pending_blocks, no_confirm, pad1, pad2;  // no_confirm: inner solves stop on
                                                 // the recursive residual
    double ny2, thr2, rh2, rr;
    double relres_rec, relres_true, gamma, tol2;
    d2 rho, rho_old, alpha, omega, beta;
    d2 rhs, rho_next;  // r^H s of this iteration; rho' for the next one (PK_T3)
};
static_assert(sizeof(SolverState) <= 512, "state block");

// A fresh record: iterating, nothing pending, no scalars yet.
__device__ __forceinline__ void init_state(SolverState& o, int maxit, double tol2,
                                           int no_confirm)
{
    o.phase = PH_RUN;
    o.restart = 1;
    o.info = -1;
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
}

__device__ __forceinline__ void finish(SolverState& L, int info)
{
    L.info = info;
    L.phase = PH_DONE;
}

__device__ __forceinline__ double relres(double sq, double ny2) { return sqrt(sq / ny2); }

// After r = y - A x (or r = y when x0 = 0) at set-up.
__device__ inline void setup_step(SolverState& L, double rr, bool bicg)
{
    if (!__builtin_isfinite(rr)) { finish(L, 4); return; }
    L.rr = rr;
    L.relres_rec = relres(rr, L.ny2);
    if (rr <= L.thr2) {
        if (L.no_confirm) finish(L, 0);
        else L.phase = PH_CONFIRM;
        return;
    }
    L.restart = 1;
    if (bicg) {
        L.rh2 = rr;
        L.rho = d2{rr, 0.0};
        if (L.maxit <= 0) { finish(L, 1); return; }
        L.phase = PH_RUN;
    } else {
        L.phase = PH_RESTART;  // z = A^H r, p = z come next
    }
}

// After the true residual rt = y - A x of a confirmation.
__device__ inline void confirm_step(SolverState& L, double rtt, bool bicg)
{
    L.matvecs++;
    L.confirms++;
    L.relres_true = relres(rtt, L.ny2);
    if (!__builtin_isfinite(rtt)) { finish(L, 4); return; }
    if (rtt <= L.thr2) { finish(L, 0); return; }
    L.rr = rtt;
    L.relres_rec = relres(rtt, L.ny2);
    if (L.iters >= L.maxit) { finish(L, 1); return; }
    if (bicg) {
        L.rh2 = rtt;
        L.rho = d2{rtt, 0.0};
        L.restart = 1;
    }
    L.phase = PH_RESTART;
}

// COCG at a (re)start: rho = (r, r) of the new residual.
__device__ inline void cocg_rho_step(SolverState& L, d2 rho)
{
    if (!cfinite(rho)) { finish(L, 4); return; }
    if (rho.x == 0.0 && rho.y == 0.0) { finish(L, 2); return; }
    L.rho = rho;
    L.restart = 1;
}

// ||y||^2: the stop threshold, or y == 0 (x = 0), or a non-finite y.
__device__ inline void normy_step(SolverState& L, double ny2)
{
    L.ny2 = ny2;
    if (!__builtin_isfinite(ny2)) finish(L, 4);
    else if (ny2 == 0.0) L.phase = PH_ZERO;
    else L.thr2 = L.tol2 * ny2;
}

// COCG set-up on ||r||^2 and (r, r).
__device__ inline void cocg_setup_step(SolverState& L, double rr, d2 rho)
{
    if (!__builtin_isfinite(rr)) { finish(L, 4); return; }
    L.rr = rr;
    L.relres_rec = relres(rr, L.ny2);
    if (rr <= L.thr2) { L.phase = PH_CONFIRM; return; }
    cocg_rho_step(L, rho);
    if (L.phase == PH_DONE) return;
    if (L.maxit <= 0) { finish(L, 1); return; }
    L.phase = PH_RESTART;
}

// The scalar step of the method that finishes the pending reduction with
// totals t0, t1 (and t2 for PK_T3).  Runs in thread 0 of every block of the
// consuming kernel on identical inputs, so every block takes the same
// decision; only block 0 writes the per-iteration record (hist non-null
// there).
__device__ inline void apply_step(SolverState& L, d2 t0, d2 t1, ccg_hist* hist,
                                  d2 t2 = d2{0.0, 0.0})
{
    const int k = L.pending;
    L.pending = PK_NONE;
    L.pending_blocks = 0;
    switch (k) {
    case PK_NORMY:
        normy_step(L, t0.x);
        break;
    case PK_NY_SETUP_B0:
    case PK_NY_SETUP_C0:
    case PK_NY_SETUP_G0:
        normy_step(L, t0.x);
        if (L.phase == PH_ZERO) {  // y == 0: x has been zeroed
            L.relres_rec = L.relres_true = 0.0;
            finish(L, 0);
        } else if (L.phase == PH_RUN) {
            if (k == PK_NY_SETUP_G0)
                cocg_setup_step(L, t0.x, t1);
            else
                setup_step(L, t0.x, k == PK_NY_SETUP_B0);
        }
        break;
    case PK_ZERO:
        L.relres_rec = L.relres_true = 0.0;
        finish(L, 0);
        break;
    case PK_SETUP_B1:
        L.matvecs++;
        setup_step(L, t0.x, true);
        break;
    case PK_SETUP_B0:
        setup_step(L, t0.x, true);
        break;
    case PK_SETUP_C1:
        L.matvecs++;
        setup_step(L, t0.x, false);
        break;
    case PK_CONFIRM_B:
        confirm_step(L, t0.x, true);
        break;
    case PK_CONFIRM_C:
        confirm_step(L, t0.x, false);
        break;
    case PK_V: {  // alpha = rho / sigma
        const d2 sigma = t0;
        const double vv = t1.x;
        L.matvecs++;
        L.restart = 0;
        if (!cfinite(sigma) || !__builtin_isfinite(vv)) { finish(L, 4); break; }
        if (cabs2(sigma) <= 1e-28 * L.rh2 * vv) { finish(L, 2); break; }
        const d2 al = cdiv(L.rho, sigma);
        if (!cfinite(al)) { finish(L, 4); break; }
        L.alpha = al;
        if (hist) {
            hist[L.iters].alpha_re = al.x;
            hist[L.iters].alpha_im = al.y;
        }
        L.phase = PH_RUN;
        break;
    }
    case PK_S: {  // half-step stop test on ||s||
        const double ss = t0.x;
        if (!__builtin_isfinite(ss)) { finish(L, 4); break; }
        if (hist) hist[L.iters].res_half = relres(ss, L.ny2);
        if (ss <= L.thr2) {
            L.relres_rec = relres(ss, L.ny2);
            L.phase = PH_HALF;
        }
        break;
    }
    case PK_T: {  // omega = t^H s / t^H t
        const d2 ts = t0;
        const double tt = t1.x;
        L.matvecs++;
        if (!__builtin_isfinite(tt) || !cfinite(ts)) { finish(L, 4); break; }
        if (tt == 0.0) { finish(L, 3); break; }
        const d2 om = d2{ts.x / tt, ts.y / tt};
        if (om.x == 0.0 && om.y == 0.0) { finish(L, 3); break; }
        L.omega = om;
        if (hist) {
            hist[L.iters].omega_re = om.x;
            hist[L.iters].omega_im = om.y;
        }
        break;
    }
    case PK_XR: {  // stop test on ||r||, then beta for the next direction
        const double rr = t0.x;
        const d2 rho_new = t1;
        L.iters++;
        if (!__builtin_isfinite(rr)) { finish(L, 4); break; }
        if (hist) hist[L.iters - 1].res_full = relres(rr, L.ny2);
        L.rr = rr;
        L.relres_rec = relres(rr, L.ny2);
        if (rr <= L.thr2) {
            if (L.no_confirm) finish(L, 0);
            else L.phase = PH_CONFIRM;
            break;
        }
        if (L.iters >= L.maxit) { finish(L, 1); break; }
        if (!cfinite(rho_new)) { finish(L, 4); break; }
        if (cabs2(rho_new) <= 1e-28 * L.rh2 * rr) { finish(L, 2); break; }
        const d2 beta = cmul(cdiv(rho_new, L.rho), cdiv(L.alpha, L.omega));
        if (!cfinite(beta)) { finish(L, 4); break; }
        L.rho_old = L.rho;
        L.rho = rho_new;
        L.beta = beta;
        if (hist) {
            hist[L.iters].beta_re = beta.x;
            hist[L.iters].beta_im = beta.y;
        }
        break;
    }
    case PK_S2: {  // half-step stop test on ||s||; keep r^H s
        const double ss = t0.x;
        if (!__builtin_isfinite(ss)) { finish(L, 4); break; }
        if (hist) hist[L.iters].res_half = relres(ss, L.ny2);
        L.rhs = t1;
        if (ss <= L.thr2) {
            L.relres_rec = relres(ss, L.ny2);
            L.phase = PH_HALF;
        }
        break;
    }
    case PK_T3: {  // omega = t^H s / t^H t; rho' = r^H s - omega r^H t; beta
        const d2 ts = t0;
        const double tt = t1.x;
        L.matvecs++;
        if (!__builtin_isfinite(tt) || !cfinite(ts)) { finish(L, 4); break; }
        if (tt == 0.0) { finish(L, 3); break; }
        const d2 om = d2{ts.x / tt, ts.y / tt};
        if (om.x == 0.0 && om.y == 0.0) { finish(L, 3); break; }
        L.omega = om;
        if (hist) {
            hist[L.iters].omega_re = om.x;
            hist[L.iters].omega_im = om.y;
        }
        const d2 nom = d2{-om.x, -om.y};
        L.rho_next = cfma(nom, t2, L.rhs);
        // beta is formed now (the x, r update also forms the next p); the
        // tests on rho' and beta wait for ||r|| (PK_XRP)
        L.beta = cmul(cdiv(L.rho_next, L.rho), cdiv(L.alpha, om));
        break;
    }
    case PK_XRP: {  // stop test on ||r||, then the tests on rho' and beta
        const double rr = t0.x;
        const d2 rho_new = L.rho_next;
        L.iters++;
        if (!__builtin_isfinite(rr)) { finish(L, 4); break; }
        if (hist) hist[L.iters - 1].res_full = relres(rr, L.ny2);
        L.rr = rr;
        L.relres_rec = relres(rr, L.ny2);
        if (rr <= L.thr2) {
            if (L.no_confirm) finish(L, 0);
            else L.phase = PH_CONFIRM;
            break;
        }
        if (L.iters >= L.maxit) { finish(L, 1); break; }
        if (!cfinite(rho_new)) { finish(L, 4); break; }
        if (cabs2(rho_new) <= 1e-28 * L.rh2 * rr) { finish(L, 2); break; }
        if (!cfinite(L.beta)) { finish(L, 4); break; }
        L.rho_old = L.rho;
        L.rho = rho_new;
        if (hist) {
            hist[L.iters].beta_re = L.beta.x;
            hist[L.iters].beta_im = L.beta.y;
        }
        break;
    }
    case PK_HALF:
        L.iters++;
        if (L.no_confirm) finish(L, 0);
        else L.phase = PH_CONFIRM;
        break;
    case PK_W: {  // alpha = gamma / ||w||^2
        const double ww = t0.x;
        L.matvecs++;
        if (!__builtin_isfinite(ww)) { finish(L, 4); break; }
        if (ww == 0.0) { finish(L, 2); break; }
        const double al = L.gamma / ww;
        L.alpha = d2{al, 0.0};
        if (hist) {
            hist[L.iters].alpha_re = al;
            hist[L.iters].alpha_im = 0.0;
        }
        break;
    }
    case PK_XR2: {
        const double rr = t0.x;
        L.iters++;
        if (!__builtin_isfinite(rr)) { finish(L, 4); break; }
        if (hist) hist[L.iters - 1].res_full = relres(rr, L.ny2);
        L.rr = rr;
        L.relres_rec = relres(rr, L.ny2);
        if (rr <= L.thr2) L.phase = PH_CONFIRM;
        break;
    }
    case PK_Z_RESTART:
    case PK_Z_RUN: {
        const double g = t0.x;
        L.matvecs++;
        if (!__builtin_isfinite(g)) { finish(L, 4); break; }
        if (g == 0.0) { finish(L, 2); break; }
        if (k == PK_Z_RESTART) {
            L.gamma = g;
            L.restart = 1;
            L.phase = PH_RUN;
        } else {
            const double beta = g / L.gamma;
            if (hist) {
                hist[L.iters - 1].beta_re = beta;
                hist[L.iters - 1].beta_im = 0.0;
            }
            L.beta = d2{beta, 0.0};
            L.gamma = g;
            L.restart = 0;
        }
        if (L.iters >= L.maxit) finish(L, 1);
        break;
    }
    case PK_SETUP_G1:
        L.matvecs++;
        cocg_setup_step(L, t0.x, t1);
        break;
    case PK_CONFIRM_G:
        confirm_step(L, t0.x, false);
        if (L.phase == PH_RESTART) cocg_rho_step(L, t1);
        break;
    case PK_Q: {  // alpha = rho / (p, A p)
        const d2 pq = t0;
        L.matvecs++;
        L.restart = 0;
        if (!cfinite(pq)) { finish(L, 4); break; }
        if (pq.x == 0.0 && pq.y == 0.0) { finish(L, 2); break; }
        const d2 al = cdiv(L.rho, pq);
        L.alpha = al;
        if (hist) {
            hist[L.iters].alpha_re = al.x;
            hist[L.iters].alpha_im = al.y;
        }
        L.phase = PH_RUN;
        break;
    }
    case PK_XR_G: {  // stop test, then beta = (r, r)' / (r, r)
        const double rr = t0.x;
        const d2 rho_new = t1;
        L.iters++;
        if (!__builtin_isfinite(rr)) { finish(L, 4); break; }
        if (hist) hist[L.iters - 1].res_full = relres(rr, L.ny2);
        L.rr = rr;
        L.relres_rec = relres(rr, L.ny2);
        if (rr <= L.thr2) { L.phase = PH_CONFIRM; break; }
        if (!cfinite(rho_new)) { finish(L, 4); break; }
        if (rho_new.x == 0.0 && rho_new.y == 0.0) { finish(L, 2); break; }
        const d2 beta = cdiv(rho_new, L.rho);
        if (hist) {
            hist[L.iters - 1].beta_re = beta.x;
            hist[L.iters - 1].beta_im = beta.y;
        }
        L.beta = beta;
        L.rho = rho_new;
        if (L.iters >= L.maxit) finish(L, 1);
        break;
    }
    case PK_U: {  // rho' = (r, A r); beta = rho'/rho unless a new direction
        const d2 rho_new = t0;
        L.matvecs++;
        if (L.phase == PH_RESTART) L.restart = 1;
        if (!cfinite(rho_new)) { finish(L, 4); break; }
        if (rho_new.x == 0.0 && rho_new.y == 0.0) { finish(L, 2); break; }
        if (!L.restart) {
            const d2 beta = cdiv(rho_new, L.rho);
            if (hist) {
                hist[L.iters - 1].beta_re = beta.x;
                hist[L.iters - 1].beta_im = beta.y;
            }
            L.beta = beta;
        }
        L.rho = rho_new;
        if (L.iters >= L.maxit) { finish(L, 1); break; }
        L.phase = PH_RUN;
        break;
    }
    case PK_WW: {  // alpha = rho / (A p, A p)
        const d2 ww = t0;
        L.restart = 0;
        if (!cfinite(ww)) { finish(L, 4); break; }
        if (ww.x == 0.0 && ww.y == 0.0) { finish(L, 2); break; }
        const d2 al = cdiv(L.rho, ww);
        L.alpha = al;
        if (hist) {
            hist[L.iters].alpha_re = al.x;
            hist[L.iters].alpha_im = al.y;
        }
        break;
    }
    case PK_XR_R: {
        const double rr = t0.x;
        L.iters++;
        if (!__builtin_isfinite(rr)) { finish(L, 4); break; }
        if (hist) hist[L.iters - 1].res_full = relres(rr, L.ny2);
        L.rr = rr;
        L.relres_rec = relres(rr, L.ny2);
        if (rr <= L.thr2) L.phase = PH_CONFIRM;
        break;
    }
    default:
        break;
    }
}

}  // namespace ccg
