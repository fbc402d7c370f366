/*
 * ccg_oracle.c -- CPU oracle of the complex Krylov solvers.
 *
 * TEST INFRASTRUCTURE ONLY.  The test suite, the package smoke check and the
 * benchmark's CPU-baseline leg are the only code that may load this library.
 * The product library never links, calls or falls back to it, and this file
 * shares no code, header or constant table with it.
 *
 * What is computed.  CCGPAK solves A x = y for a complex square matrix A
 * (Introduction, the problem statement "Ax = y"), with the matrix-vector
 * product kept apart from the iteration (Abstract; Usage, the matvec and
 * cmatvec routines).  Of the PIM90 set (Codes, section 2.1) this oracle
 * provides bicgstab and cgnr.  The paper names these methods but prints no
 * algorithm, so the steps follow the published methods it points to:
 *   - BiCGSTAB: van der Vorst (1992), as presented in the Templates book that
 *     the Introduction recommends; complex, unpreconditioned.
 *   - CGNR: conjugate gradients applied to the normal equations
 *     A^H A x = A^H y, which minimises ||y - A x||_2 over a growing Krylov
 *     space (PIM90 set, section 2.1; Templates).
 *   - COCG and COCR for complex symmetric A (A^T = A): the methods of the
 *     "next releases" section 3.4 (COCR of Sogabe and Zhang, 2007, compared
 *     there with COCG).  Both are the CG and CR recurrences with the
 *     unconjugated bilinear form (a, b) = sum a_i b_i in place of the inner
 *     product; one product with A per iteration.
 *   - Mixed precision BiCGSTAB: FP64 iterative refinement around an inner
 *     complex64 BiCGSTAB -- the single/double precision switch of the
 *     ddprecision module (Abstract; Usage section) used inside one solve.
 *     The inner products accumulate in FP32; the inner dot products and
 *     scalars are FP64; the outer residual and update are FP64.  A second
 *     form keeps the inner Krylov vectors in complex128 (the form the solver
 *     for many right-hand sides uses): only the product is complex64, its
 *     input rounded to complex64 and its FP32 sums widened back.
 *   - CG: Hestenes-Stiefel conjugate gradients for Hermitian positive-definite
 *     A.  Not in the paper's list; kept only as a pinned reference that other
 *     tests compare CGNR and BiCGSTAB against.
 *
 * Conventions (readings of what the paper leaves open):
 *   - A is row-major: element (i, j) is A[i*lda + j].
 *   - The inner product conjugates its first argument: <a, b> = sum conj(a_i) b_i
 *     (what Fortran's dot_product does for complex arguments, the intrinsic
 *     the Introduction and section 2.1 say replaced the BLAS calls).
 *   - The iteration stops when ||r||_2 <= tol * ||y||_2 on the recursive
 *     residual; a true residual y - A x then confirms it, and when the
 *     confirmation fails the true residual replaces r and the method restarts
 *     inside the same iteration budget (tolerance epsilon_err and budget maxit
 *     of the cgmodule structure, Usage section).
 *   - info: 0 converged, 1 iteration budget spent, 2 breakdown of rho or sigma
 *     (BiCGSTAB), of ||w|| or ||A^H r|| (CGNR), or of a bilinear form (r, r),
 *     (p, A p), (r, A r) or (A p, A p) (COCG, COCR), 3 breakdown of omega or
 *     t^H t (BiCGSTAB), 4 non-finite value met.
 *
 * Arithmetic: C11 double complex, one thread, every sum a left-to-right loop.
 * Build with -ffp-contract=off so that no multiply-add is fused.  A second
 * build of this same file with OpenMP exists for timing on all host cores
 * only: it splits the rows of the dense product among threads, which leaves
 * every sum, and so every result, bit for bit as in the one-thread build.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex zc;

#define ORACLE_X0_ZERO 1u /* caller says x holds zero on entry: skip y - A x */

typedef struct {
    int32_t info;     /* 0..4, meaning above */
    int32_t iters;    /* completed iterations (a half-step exit counts) */
    int32_t matvecs;  /* applications of A or A^H */
    int32_t confirms; /* true-residual checks made */
    double relres_rec;  /* last recursive ||r|| / ||y|| */
    double relres_true; /* last true ||y - A x|| / ||y|| */
} oracle_stats;

/* One record per iteration; fields a method does not use stay NaN. */
typedef struct {
    double alpha_re, alpha_im;
    double omega_re, omega_im;
    double beta_re, beta_im;
    double res_half; /* BiCGSTAB: ||s|| / ||y|| */
    double res_full; /* ||r|| / ||y|| after the iteration */
} oracle_hist;

/* ---------------------------------------------------------------- helpers */

static double norm2sq(int64_t n, const zc* v)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i)
        s += creal(v[i]) * creal(v[i]) + cimag(v[i]) * cimag(v[i]);
    return s;
}

/* <a, b> = sum_i conj(a_i) * b_i */
static zc dotc(int64_t n, const zc* a, const zc* b)
{
    zc s = 0.0;
    for (int64_t i = 0; i < n; ++i)
        s += conj(a[i]) * b[i];
    return s;
}

/* (a, b) = sum_i a_i * b_i, the bilinear form of COCG / COCR */
static zc dotu(int64_t n, const zc* a, const zc* b)
{
    zc s = 0.0;
    for (int64_t i = 0; i < n; ++i)
        s += a[i] * b[i];
    return s;
}

/* a / b written out as a * conj(b) / |b|^2 */
static zc zdiv(zc a, zc b)
{
    double d = creal(b) * creal(b) + cimag(b) * cimag(b);
    zc q = a * conj(b);
    return CMPLX(creal(q) / d, cimag(q) / d);
}

static double abs2(zc z) { return creal(z) * creal(z) + cimag(z) * cimag(z); }

static int zfinite(zc z) { return isfinite(creal(z)) && isfinite(cimag(z)); }

static void zcopy(int64_t n, const zc* src, zc* dst)
{
    for (int64_t i = 0; i < n; ++i)
        dst[i] = src[i];
}

static void zzero(int64_t n, zc* v)
{
    for (int64_t i = 0; i < n; ++i)
        v[i] = 0.0;
}

/* Threads the OpenMP build uses from now on (want > 0), and how many it
 * will use; 1 in the one-thread build. */
int oracle_threads(int want)
{
#ifdef _OPENMP
    if (want > 0) omp_set_num_threads(want);
    return omp_get_max_threads();
#else
    (void)want;
    return 1;
#endif
}

/* -------------------------------------------------------- matrix products */

/* y = A x : y_i = sum_j A_ij x_j  (the user matvec of the Usage section).
 * In the OpenMP build (timing only) the rows are shared out among threads;
 * every row's sum keeps its left-to-right order, so the bits are the same. */
void oracle_matvec(int64_t n, const zc* A, int64_t lda, const zc* x, zc* y)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        zc s = 0.0;
        for (int64_t j = 0; j < n; ++j)
            s += A[i * lda + j] * x[j];
        y[i] = s;
    }
}

/* y = A^H x : y_j = sum_i conj(A_ij) x_i, summed over i in increasing order
 * (the cmatvec of the Usage section, read as the conjugate transpose that
 * CGNR needs). */
void oracle_matvec_h(int64_t n, const zc* A, int64_t lda, const zc* x, zc* y)
{
    for (int64_t j = 0; j < n; ++j)
        y[j] = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        zc xi = x[i];
        for (int64_t j = 0; j < n; ++j)
            y[j] += conj(A[i * lda + j]) * xi;
    }
}

/* y = A x for a complex symmetric A (A^T = A, the matrices of COCG and COCR,
 * section 3.4) of which only the upper triangle is stored:
 *   y_i = sum_{j < i} A_ji x_j + sum_{j >= i} A_ij x_j,
 * summed over j in increasing order.  Elements below the diagonal are never
 * read.  On a matrix that is symmetric in full this is oracle_matvec's sum
 * term for term, in the same order. */
void oracle_matvec_sym_upper(int64_t n, const zc* A, int64_t lda, const zc* x, zc* y)
{
    for (int64_t i = 0; i < n; ++i) {
        zc s = 0.0;
        for (int64_t j = 0; j < i; ++j)
            s += A[j * lda + i] * x[j];
        for (int64_t j = i; j < n; ++j)
            s += A[i * lda + j] * x[j];
        y[i] = s;
    }
}

/* rt = y - A x */
static void residual(int64_t n, const zc* A, int64_t lda, const zc* y,
                     const zc* x, zc* rt)
{
    oracle_matvec(n, A, lda, x, rt);
    for (int64_t i = 0; i < n; ++i)
        rt[i] = y[i] - rt[i];
}

static int bad_args(int64_t n, int64_t lda, double tol, int32_t maxit)
{
    if (n < 0) return -1;
    if (lda < (n > 1 ? n : 1)) return -3;
    if (!(tol > 0.0) || !isfinite(tol)) return -6;
    if (maxit < 0) return -7;
    return 0;
}

static void stats_init(oracle_stats* st)
{
    memset(st, 0, sizeof *st);
    st->relres_rec = NAN;
    st->relres_true = NAN;
}

static void hist_init(oracle_hist* h, int32_t maxit)
{
    if (!h) return;
    for (int32_t k = 0; k < maxit; ++k) {
        h[k].alpha_re = h[k].alpha_im = NAN;
        h[k].omega_re = h[k].omega_im = NAN;
        h[k].beta_re = h[k].beta_im = NAN;
        h[k].res_half = h[k].res_full = NAN;
    }
}

/* Shared set-up of both solvers: the quick exits and r = y - A x.
 * Returns 1 when the solve is already finished (st->info is set). */
static int setup(int64_t n, const zc* A, int64_t lda, const zc* y, zc* x,
                 uint32_t flags, zc* r, double* ny2_out, double* rr_out,
                 oracle_stats* st)
{
    if (n == 0) {
        st->info = 0;
        return 1;
    }
    double ny2 = norm2sq(n, y);
    if (!isfinite(ny2)) {
        st->info = 4;
        return 1;
    }
    if (ny2 == 0.0) { /* y = 0: the solution is x = 0 */
        zzero(n, x);
        st->info = 0;
        st->relres_rec = st->relres_true = 0.0;
        return 1;
    }
    if (flags & ORACLE_X0_ZERO) {
        zzero(n, x);
        zcopy(n, y, r);
    } else {
        residual(n, A, lda, y, x, r);
        st->matvecs++;
    }
    double rr = norm2sq(n, r);
    if (!isfinite(rr)) {
        st->info = 4;
        return 1;
    }
    st->relres_rec = sqrt(rr / ny2);
    *ny2_out = ny2;
    *rr_out = rr;
    return 0;
}

/* Confirm a converged recursive residual with the true one.  Returns 1 when
 * the solve is finished (info set), 0 when r has been replaced by the true
 * residual and the method must restart. */
static int confirm(int64_t n, const zc* A, int64_t lda, const zc* y,
                   const zc* x, zc* r, zc* work, double ny2, double thr2,
                   int32_t k, int32_t maxit, double* rr, oracle_stats* st)
{
    residual(n, A, lda, y, x, work);
    st->matvecs++;
    st->confirms++;
    double rtt = norm2sq(n, work);
    st->relres_true = sqrt(rtt / ny2);
    if (!isfinite(rtt)) {
        st->info = 4;
        return 1;
    }
    if (rtt <= thr2) {
        st->info = 0;
        return 1;
    }
    zcopy(n, work, r);
    *rr = rtt;
    st->relres_rec = sqrt(rtt / ny2);
    if (k >= maxit) {
        st->info = 1;
        return 1;
    }
    return 0;
}

/* --------------------------------------------------------------- BiCGSTAB */

int oracle_bicgstab(int64_t n, const zc* A, int64_t lda, const zc* y, zc* x,
                    double tol, int32_t maxit, uint32_t flags,
                    oracle_stats* st, oracle_hist* hist)
{
    stats_init(st);
    int bad = bad_args(n, lda, tol, maxit);
    if (bad) return bad;
    hist_init(hist, maxit);

    zc* work = (zc*)malloc(sizeof(zc) * (size_t)(7 * (n > 0 ? n : 1)));
    if (!work) return -100;
    zc *r = work, *rh = r + n, *p = rh + n, *v = p + n, *s = v + n,
       *t = s + n, *tmp = t + n;

    double ny2 = 0.0, rr = 0.0;
    if (setup(n, A, lda, y, x, flags, r, &ny2, &rr, st)) {
        free(work);
        return 0;
    }
    const double thr2 = tol * tol * ny2;
    int32_t k = 0;
    int need_confirm = rr <= thr2;
    int restart = 1, first = 1;
    double rh2 = 0.0;
    zc rho = 0.0, rho_old = 1.0, alpha = 1.0, omega = 1.0;

    for (;;) {
        if (need_confirm) {
            need_confirm = 0;
            if (confirm(n, A, lda, y, x, r, tmp, ny2, thr2, k, maxit, &rr, st))
                break;
            restart = 1;
        }
        if (restart) { /* shadow residual: fixed to the current residual */
            zcopy(n, r, rh);
            rh2 = rr;
            first = 1;
            restart = 0;
        }
        if (k >= maxit) {
            st->info = 1;
            break;
        }
        rho = dotc(n, rh, r);
        if (!zfinite(rho)) {
            st->info = 4;
            break;
        }
        if (abs2(rho) <= 1e-28 * rh2 * rr) {
            st->info = 2;
            break;
        }
        if (first) {
            zcopy(n, r, p);
            first = 0;
        } else {
            zc beta = zdiv(rho, rho_old) * zdiv(alpha, omega);
            if (!zfinite(beta)) {
                st->info = 4;
                break;
            }
            if (hist) {
                hist[k].beta_re = creal(beta);
                hist[k].beta_im = cimag(beta);
            }
            for (int64_t i = 0; i < n; ++i)
                p[i] = r[i] + beta * (p[i] - omega * v[i]);
        }

        oracle_matvec(n, A, lda, p, v);
        st->matvecs++;
        zc sigma = dotc(n, rh, v);
        double vv = norm2sq(n, v);
        if (!zfinite(sigma) || !isfinite(vv)) {
            st->info = 4;
            break;
        }
        if (abs2(sigma) <= 1e-28 * rh2 * vv) {
            st->info = 2;
            break;
        }
        alpha = zdiv(rho, sigma);
        if (!zfinite(alpha)) {
            st->info = 4;
            break;
        }
        if (hist) {
            hist[k].alpha_re = creal(alpha);
            hist[k].alpha_im = cimag(alpha);
        }

        for (int64_t i = 0; i < n; ++i)
            s[i] = r[i] - alpha * v[i];
        double ss = norm2sq(n, s);
        if (!isfinite(ss)) {
            st->info = 4;
            break;
        }
        if (hist) hist[k].res_half = sqrt(ss / ny2);
        if (ss <= thr2) { /* converged half-way through the iteration */
            for (int64_t i = 0; i < n; ++i)
                x[i] = x[i] + alpha * p[i];
            k++;
            st->relres_rec = sqrt(ss / ny2);
            need_confirm = 1;
            continue;
        }

        oracle_matvec(n, A, lda, s, t);
        st->matvecs++;
        double tt = norm2sq(n, t);
        zc ts = dotc(n, t, s);
        if (!isfinite(tt) || !zfinite(ts)) {
            st->info = 4;
            break;
        }
        if (tt == 0.0) {
            st->info = 3;
            break;
        }
        omega = CMPLX(creal(ts) / tt, cimag(ts) / tt);
        if (omega == 0.0) {
            st->info = 3;
            break;
        }
        if (hist) {
            hist[k].omega_re = creal(omega);
            hist[k].omega_im = cimag(omega);
        }
        for (int64_t i = 0; i < n; ++i) {
            x[i] = x[i] + alpha * p[i] + omega * s[i];
            r[i] = s[i] - omega * t[i];
        }
        rr = norm2sq(n, r);
        k++;
        if (!isfinite(rr)) {
            st->info = 4;
            break;
        }
        if (hist) hist[k - 1].res_full = sqrt(rr / ny2);
        st->relres_rec = sqrt(rr / ny2);
        rho_old = rho;
        if (rr <= thr2) need_confirm = 1;
    }
    st->iters = k;
    free(work);
    return 0;
}

/* ------------------------------------------------------------------- CGNR */

int oracle_cgnr(int64_t n, const zc* A, int64_t lda, const zc* y, zc* x,
                double tol, int32_t maxit, uint32_t flags, oracle_stats* st,
                oracle_hist* hist)
{
    stats_init(st);
    int bad = bad_args(n, lda, tol, maxit);
    if (bad) return bad;
    hist_init(hist, maxit);

    zc* work = (zc*)malloc(sizeof(zc) * (size_t)(5 * (n > 0 ? n : 1)));
    if (!work) return -100;
    zc *r = work, *z = r + n, *p = z + n, *w = p + n, *tmp = w + n;

    double ny2 = 0.0, rr = 0.0;
    if (setup(n, A, lda, y, x, flags, r, &ny2, &rr, st)) {
        free(work);
        return 0;
    }
    const double thr2 = tol * tol * ny2;
    int32_t k = 0;
    int need_confirm = rr <= thr2;
    int restart = 1;
    double gamma = 0.0;

    for (;;) {
        if (need_confirm) {
            need_confirm = 0;
            if (confirm(n, A, lda, y, x, r, tmp, ny2, thr2, k, maxit, &rr, st))
                break;
            restart = 1;
        }
        if (restart) { /* z = A^H r, p = z */
            oracle_matvec_h(n, A, lda, r, z);
            st->matvecs++;
            gamma = norm2sq(n, z);
            if (!isfinite(gamma)) {
                st->info = 4;
                break;
            }
            if (gamma == 0.0) {
                st->info = 2;
                break;
            }
            zcopy(n, z, p);
            restart = 0;
        }
        if (k >= maxit) {
            st->info = 1;
            break;
        }

        oracle_matvec(n, A, lda, p, w);
        st->matvecs++;
        double ww = norm2sq(n, w);
        if (!isfinite(ww)) {
            st->info = 4;
            break;
        }
        if (ww == 0.0) {
            st->info = 2;
            break;
        }
        double alpha = gamma / ww;
        for (int64_t i = 0; i < n; ++i) {
            x[i] = x[i] + alpha * p[i];
            r[i] = r[i] - alpha * w[i];
        }
        rr = norm2sq(n, r);
        k++;
        if (!isfinite(rr)) {
            st->info = 4;
            break;
        }
        if (hist) {
            hist[k - 1].alpha_re = alpha;
            hist[k - 1].alpha_im = 0.0;
            hist[k - 1].res_full = sqrt(rr / ny2);
        }
        st->relres_rec = sqrt(rr / ny2);
        if (rr <= thr2) {
            need_confirm = 1;
            continue;
        }

        oracle_matvec_h(n, A, lda, r, z);
        st->matvecs++;
        double gamma_new = norm2sq(n, z);
        if (!isfinite(gamma_new)) {
            st->info = 4;
            break;
        }
        if (gamma_new == 0.0) {
            st->info = 2;
            break;
        }
        double beta = gamma_new / gamma;
        if (hist) {
            hist[k - 1].beta_re = beta;
            hist[k - 1].beta_im = 0.0;
        }
        for (int64_t i = 0; i < n; ++i)
            p[i] = z[i] + beta * p[i];
        gamma = gamma_new;
    }
    st->iters = k;
    free(work);
    return 0;
}

/* ------------------------------------------------------------------- COCG */

/* COCG: CG with the bilinear form, for complex symmetric A.
 *   p = r, rho = (r, r); per iteration: q = A p, alpha = rho / (p, q),
 *   x += alpha p, r -= alpha q, stop test, rho' = (r, r), beta = rho'/rho,
 *   p = r + beta p.  (r, r) = 0 or (p, q) = 0 with r != 0 is a breakdown. */
int oracle_cocg(int64_t n, const zc* A, int64_t lda, const zc* y, zc* x,
                double tol, int32_t maxit, uint32_t flags, oracle_stats* st,
                oracle_hist* hist)
{
    stats_init(st);
    int bad = bad_args(n, lda, tol, maxit);
    if (bad) return bad;
    hist_init(hist, maxit);

    zc* work = (zc*)malloc(sizeof(zc) * (size_t)(4 * (n > 0 ? n : 1)));
    if (!work) return -100;
    zc *r = work, *p = r + n, *q = p + n, *tmp = q + n;

    double ny2 = 0.0, rr = 0.0;
    if (setup(n, A, lda, y, x, flags, r, &ny2, &rr, st)) {
        free(work);
        return 0;
    }
    const double thr2 = tol * tol * ny2;
    int32_t k = 0;
    int need_confirm = rr <= thr2;
    int restart = 1;
    zc rho = 0.0;

    for (;;) {
        if (need_confirm) {
            need_confirm = 0;
            if (confirm(n, A, lda, y, x, r, tmp, ny2, thr2, k, maxit, &rr, st))
                break;
            restart = 1;
        }
        if (restart) { /* p = r, rho = (r, r) */
            rho = dotu(n, r, r);
            if (!zfinite(rho)) {
                st->info = 4;
                break;
            }
            if (rho == 0.0) {
                st->info = 2;
                break;
            }
            zcopy(n, r, p);
            restart = 0;
        }
        if (k >= maxit) {
            st->info = 1;
            break;
        }
        oracle_matvec(n, A, lda, p, q);
        st->matvecs++;
        zc pq = dotu(n, p, q);
        if (!zfinite(pq)) {
            st->info = 4;
            break;
        }
        if (pq == 0.0) {
            st->info = 2;
            break;
        }
        zc alpha = zdiv(rho, pq);
        for (int64_t i = 0; i < n; ++i) {
            x[i] = x[i] + alpha * p[i];
            r[i] = r[i] - alpha * q[i];
        }
        rr = norm2sq(n, r);
        k++;
        if (!isfinite(rr)) {
            st->info = 4;
            break;
        }
        if (hist) {
            hist[k - 1].alpha_re = creal(alpha);
            hist[k - 1].alpha_im = cimag(alpha);
            hist[k - 1].res_full = sqrt(rr / ny2);
        }
        st->relres_rec = sqrt(rr / ny2);
        if (rr <= thr2) {
            need_confirm = 1;
            continue;
        }
        zc rho_new = dotu(n, r, r);
        if (!zfinite(rho_new)) {
            st->info = 4;
            break;
        }
        if (rho_new == 0.0) {
            st->info = 2;
            break;
        }
        zc beta = zdiv(rho_new, rho);
        if (hist) {
            hist[k - 1].beta_re = creal(beta);
            hist[k - 1].beta_im = cimag(beta);
        }
        for (int64_t i = 0; i < n; ++i)
            p[i] = r[i] + beta * p[i];
        rho = rho_new;
    }
    st->iters = k;
    free(work);
    return 0;
}

/* ------------------------------------------------------------------- COCR */

/* COCR (Sogabe and Zhang): CR with the bilinear form, for complex symmetric
 * A.  Keeps u = A r and w = A p; one product (u = A r) per iteration.
 *   u = A r, p = r, w = u, rho = (r, u); per iteration:
 *   alpha = rho / (w, w), x += alpha p, r -= alpha w, stop test, u = A r,
 *   rho' = (r, u), beta = rho'/rho, p = r + beta p, w = u + beta w. */
int oracle_cocr(int64_t n, const zc* A, int64_t lda, const zc* y, zc* x,
                double tol, int32_t maxit, uint32_t flags, oracle_stats* st,
                oracle_hist* hist)
{
    stats_init(st);
    int bad = bad_args(n, lda, tol, maxit);
    if (bad) return bad;
    hist_init(hist, maxit);

    zc* work = (zc*)malloc(sizeof(zc) * (size_t)(5 * (n > 0 ? n : 1)));
    if (!work) return -100;
    zc *r = work, *u = r + n, *p = u + n, *w = p + n, *tmp = w + n;

    double ny2 = 0.0, rr = 0.0;
    if (setup(n, A, lda, y, x, flags, r, &ny2, &rr, st)) {
        free(work);
        return 0;
    }
    const double thr2 = tol * tol * ny2;
    int32_t k = 0;
    int need_confirm = rr <= thr2;
    int restart = 1;
    zc rho = 0.0;

    for (;;) {
        if (need_confirm) {
            need_confirm = 0;
            if (confirm(n, A, lda, y, x, r, tmp, ny2, thr2, k, maxit, &rr, st))
                break;
            restart = 1;
        }
        if (restart) { /* u = A r, p = r, w = u, rho = (r, u) */
            oracle_matvec(n, A, lda, r, u);
            st->matvecs++;
            rho = dotu(n, r, u);
            if (!zfinite(rho)) {
                st->info = 4;
                break;
            }
            if (rho == 0.0) {
                st->info = 2;
                break;
            }
            zcopy(n, r, p);
            zcopy(n, u, w);
            restart = 0;
        }
        if (k >= maxit) {
            st->info = 1;
            break;
        }
        zc ww = dotu(n, w, w);
        if (!zfinite(ww)) {
            st->info = 4;
            break;
        }
        if (ww == 0.0) {
            st->info = 2;
            break;
        }
        zc alpha = zdiv(rho, ww);
        for (int64_t i = 0; i < n; ++i) {
            x[i] = x[i] + alpha * p[i];
            r[i] = r[i] - alpha * w[i];
        }
        rr = norm2sq(n, r);
        k++;
        if (!isfinite(rr)) {
            st->info = 4;
            break;
        }
        if (hist) {
            hist[k - 1].alpha_re = creal(alpha);
            hist[k - 1].alpha_im = cimag(alpha);
            hist[k - 1].res_full = sqrt(rr / ny2);
        }
        st->relres_rec = sqrt(rr / ny2);
        if (rr <= thr2) {
            need_confirm = 1;
            continue;
        }
        oracle_matvec(n, A, lda, r, u);
        st->matvecs++;
        zc rho_new = dotu(n, r, u);
        if (!zfinite(rho_new)) {
            st->info = 4;
            break;
        }
        if (rho_new == 0.0) {
            st->info = 2;
            break;
        }
        zc beta = zdiv(rho_new, rho);
        if (hist) {
            hist[k - 1].beta_re = creal(beta);
            hist[k - 1].beta_im = cimag(beta);
        }
        for (int64_t i = 0; i < n; ++i) {
            p[i] = r[i] + beta * p[i];
            w[i] = u[i] + beta * w[i];
        }
        rho = rho_new;
    }
    st->iters = k;
    free(work);
    return 0;
}

/* -------------------------------------------------------- mixed precision */

typedef float complex fc;

typedef struct {
    int32_t info;        /* 0..4 from the outer loop */
    int32_t outer;       /* refinement steps (inner solves) */
    int32_t inner_iters; /* inner iterations, all steps */
    int32_t matvecs64;   /* FP64 residual products */
    int32_t matvecs32;   /* complex64 products */
    int32_t pad;
    double relres_true;  /* last FP64 ||y - A x|| / ||y|| */
} oracle_mixed_stats;

/* y = A x in complex64, every row summed left to right in FP32 */
void oracle_matvec_c64(int64_t n, const fc* A, int64_t lda, const fc* x, fc* y)
{
    for (int64_t i = 0; i < n; ++i) {
        fc s = 0.0f;
        for (int64_t j = 0; j < n; ++j)
            s += A[i * lda + j] * x[j];
        y[i] = s;
    }
}

static double norm2sq_c64(int64_t n, const fc* v)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double re = crealf(v[i]), im = cimagf(v[i]);
        s += re * re + im * im;
    }
    return s;
}

/* sum conj(a_i) b_i in FP64 over complex64 vectors */
static zc dotc_c64(int64_t n, const fc* a, const fc* b)
{
    zc s = 0.0;
    for (int64_t i = 0; i < n; ++i)
        s += conj((zc)a[i]) * (zc)b[i];
    return s;
}

/* Inner BiCGSTAB on complex64 vectors for A32 x = b from x = 0: the same
 * steps as oracle_bicgstab, each vector update done in FP64 and rounded to
 * complex64 on store, dot products and scalars in FP64, stop on the
 * recursive residual (no confirmation).  Returns info; *iters, *matvecs. */
static int inner_bicgstab_c64(int64_t n, const fc* A, int64_t lda, const fc* b, fc* x,
                              double tol, int32_t maxit, int32_t* iters, int32_t* matvecs,
                              fc* w)
{
    fc *r = w, *rh = r + n, *p = rh + n, *v = p + n, *s = v + n, *t = s + n;
    for (int64_t i = 0; i < n; ++i) {
        x[i] = 0.0f;
        r[i] = b[i];
        rh[i] = b[i];
    }
    const double nb2 = norm2sq_c64(n, b);
    const double thr2 = tol * tol * nb2;
    double rr = nb2, rh2 = nb2;
    zc rho_old = 1.0, alpha = 1.0, omega = 1.0;
    int first = 1;
    int32_t k = 0;
    *iters = 0;
    if (!isfinite(rr)) return 4;
    if (rr <= thr2) return 0;
    while (k < maxit) {
        zc rho = dotc_c64(n, rh, r);
        if (!zfinite(rho)) return 4;
        if (abs2(rho) <= 1e-28 * rh2 * rr) return 2;
        if (first) {
            for (int64_t i = 0; i < n; ++i) p[i] = r[i];
            first = 0;
        } else {
            zc beta = zdiv(rho, rho_old) * zdiv(alpha, omega);
            for (int64_t i = 0; i < n; ++i)
                p[i] = (fc)((zc)r[i] + beta * ((zc)p[i] - omega * (zc)v[i]));
        }
        oracle_matvec_c64(n, A, lda, p, v);
        (*matvecs)++;
        zc sigma = dotc_c64(n, rh, v);
        double vv = norm2sq_c64(n, v);
        if (!zfinite(sigma) || !isfinite(vv)) return 4;
        if (abs2(sigma) <= 1e-28 * rh2 * vv) return 2;
        alpha = zdiv(rho, sigma);
        for (int64_t i = 0; i < n; ++i) s[i] = (fc)((zc)r[i] - alpha * (zc)v[i]);
        double ss = norm2sq_c64(n, s);
        if (!isfinite(ss)) return 4;
        if (ss <= thr2) {
            for (int64_t i = 0; i < n; ++i) x[i] = (fc)((zc)x[i] + alpha * (zc)p[i]);
            *iters = k + 1;
            return 0;
        }
        oracle_matvec_c64(n, A, lda, s, t);
        (*matvecs)++;
        double tt = norm2sq_c64(n, t);
        zc ts = dotc_c64(n, t, s);
        if (!isfinite(tt) || !zfinite(ts)) return 4;
        if (tt == 0.0) return 3;
        omega = CMPLX(creal(ts) / tt, cimag(ts) / tt);
        if (omega == 0.0) return 3;
        for (int64_t i = 0; i < n; ++i) {
            x[i] = (fc)((zc)x[i] + alpha * (zc)p[i] + omega * (zc)s[i]);
            r[i] = (fc)((zc)s[i] - omega * (zc)t[i]);
        }
        rr = norm2sq_c64(n, r);
        k++;
        *iters = k;
        if (!isfinite(rr)) return 4;
        rho_old = rho;
        if (rr <= thr2) return 0;
    }
    return 1;
}

/* FP64 iterative refinement: r = y - A x (FP64, complex128 A); stop when
 * ||r|| <= tol ||y|| (info 0) or after maxit steps (info 1); otherwise solve
 * A32 d = r / ||r|| with the inner complex64 BiCGSTAB to tol_inner and set
 * x += ||r|| d in FP64.  outer_res (maxit + 1 entries or NULL) receives
 * ||r|| / ||y|| at every outer check. */
int oracle_bicgstab_mixed(int64_t n, const zc* A, int64_t lda, const fc* A32, int64_t lda32,
                          const zc* y, zc* x, double tol, int32_t maxit, double tol_inner,
                          int32_t maxit_inner, uint32_t flags, oracle_mixed_stats* st,
                          double* outer_res)
{
    memset(st, 0, sizeof *st);
    st->relres_true = NAN;
    if (n < 0) return -1;
    if (lda < (n > 1 ? n : 1) || lda32 < (n > 1 ? n : 1)) return -3;
    if (!(tol > 0.0) || !isfinite(tol) || maxit < 0) return -6;
    if (!(tol_inner > 0.0) || !(tol_inner < 1.0) || maxit_inner < 1) return -10;
    if (n == 0) {
        st->relres_true = 0.0;
        return 0;
    }
    double ny2 = norm2sq(n, y);
    if (!isfinite(ny2)) {
        st->info = 4;
        return 0;
    }
    if (ny2 == 0.0) {
        zzero(n, x);
        st->relres_true = 0.0;
        return 0;
    }
    zc* r = (zc*)malloc(sizeof(zc) * (size_t)n);
    fc* f = (fc*)malloc(sizeof(fc) * (size_t)(8 * n));
    if (!r || !f) {
        free(r);
        free(f);
        return -100;
    }
    fc *r32 = f, *d32 = f + n, *w = f + 2 * n;
    const double thr2 = tol * tol * ny2;
    for (int32_t outer = 0;; ++outer) {
        if (outer == 0 && (flags & ORACLE_X0_ZERO)) {
            zzero(n, x);
            zcopy(n, y, r);
        } else {
            residual(n, A, lda, y, x, r);
            st->matvecs64++;
        }
        double rr = norm2sq(n, r);
        st->relres_true = sqrt(rr / ny2);
        if (outer_res) outer_res[outer] = st->relres_true;
        if (!isfinite(rr)) {
            st->info = 4;
            break;
        }
        if (rr <= thr2) {
            st->info = 0;
            break;
        }
        if (outer >= maxit) {
            st->info = 1;
            break;
        }
        const double nr = sqrt(rr);
        const double scale = 1.0 / nr;
        for (int64_t i = 0; i < n; ++i)
            r32[i] = (fc)CMPLX(creal(r[i]) * scale, cimag(r[i]) * scale);
        int32_t it = 0;
        int info_in = inner_bicgstab_c64(n, A32, lda32, r32, d32, tol_inner, maxit_inner, &it,
                                         &st->matvecs32, w);
        st->outer++;
        st->inner_iters += it;
        if (info_in == 4) {
            st->info = 4;
            break;
        }
        if ((info_in == 2 || info_in == 3) && it == 0) {
            /* breakdown before the first inner update: d = 0, and the next
             * step would repeat this one exactly */
            st->info = info_in;
            break;
        }
        for (int64_t i = 0; i < n; ++i)
            x[i] = x[i] + nr * (zc)d32[i];
    }
    free(r);
    free(f);
    return 0;
}

/* ----------------------------------- mixed precision, FP64 inner vectors */

/* The complex64 product applied to a complex128 vector: x rounded to
 * complex64, each row summed left to right in FP32, the sum widened to
 * complex128 (the inner product of the mixed solver for many right-hand
 * sides, whose Krylov vectors stay complex128). */
void oracle_matvec_c64_wide(int64_t n, const fc* A, int64_t lda, const zc* x, zc* y)
{
    for (int64_t i = 0; i < n; ++i) {
        fc s = 0.0f;
        for (int64_t j = 0; j < n; ++j)
            s += A[i * lda + j] * (fc)x[j];
        y[i] = (zc)s;
    }
}

/* Inner BiCGSTAB for A32 d = b from d = 0: the steps of oracle_bicgstab on
 * complex128 vectors with FP64 dot products and scalars, every product
 * oracle_matvec_c64_wide, stop on the recursive residual (no confirmation).
 * Returns info; *iters, *matvecs. */
static int inner_bicgstab_wide(int64_t n, const fc* A, int64_t lda, const zc* b, zc* x,
                               double tol, int32_t maxit, int32_t* iters, int32_t* matvecs,
                               zc* w)
{
    zc *r = w, *rh = r + n, *p = rh + n, *v = p + n, *s = v + n, *t = s + n;
    for (int64_t i = 0; i < n; ++i) {
        x[i] = 0.0;
        r[i] = b[i];
        rh[i] = b[i];
    }
    const double nb2 = norm2sq(n, b);
    const double thr2 = tol * tol * nb2;
    double rr = nb2, rh2 = nb2;
    zc rho_old = 1.0, alpha = 1.0, omega = 1.0;
    int first = 1;
    int32_t k = 0;
    *iters = 0;
    if (!isfinite(rr)) return 4;
    if (rr <= thr2) return 0;
    while (k < maxit) {
        zc rho = dotc(n, rh, r);
        if (!zfinite(rho)) return 4;
        if (abs2(rho) <= 1e-28 * rh2 * rr) return 2;
        if (first) {
            zcopy(n, r, p);
            first = 0;
        } else {
            zc beta = zdiv(rho, rho_old) * zdiv(alpha, omega);
            if (!zfinite(beta)) return 4;
            for (int64_t i = 0; i < n; ++i)
                p[i] = r[i] + beta * (p[i] - omega * v[i]);
        }
        oracle_matvec_c64_wide(n, A, lda, p, v);
        (*matvecs)++;
        zc sigma = dotc(n, rh, v);
        double vv = norm2sq(n, v);
        if (!zfinite(sigma) || !isfinite(vv)) return 4;
        if (abs2(sigma) <= 1e-28 * rh2 * vv) return 2;
        alpha = zdiv(rho, sigma);
        if (!zfinite(alpha)) return 4;
        for (int64_t i = 0; i < n; ++i) s[i] = r[i] - alpha * v[i];
        double ss = norm2sq(n, s);
        if (!isfinite(ss)) return 4;
        if (ss <= thr2) {
            for (int64_t i = 0; i < n; ++i) x[i] = x[i] + alpha * p[i];
            *iters = k + 1;
            return 0;
        }
        oracle_matvec_c64_wide(n, A, lda, s, t);
        (*matvecs)++;
        double tt = norm2sq(n, t);
        zc ts = dotc(n, t, s);
        if (!isfinite(tt) || !zfinite(ts)) return 4;
        if (tt == 0.0) return 3;
        omega = CMPLX(creal(ts) / tt, cimag(ts) / tt);
        if (omega == 0.0) return 3;
        for (int64_t i = 0; i < n; ++i) {
            x[i] = x[i] + alpha * p[i] + omega * s[i];
            r[i] = s[i] - omega * t[i];
        }
        rr = norm2sq(n, r);
        k++;
        *iters = k;
        if (!isfinite(rr)) return 4;
        rho_old = rho;
        if (rr <= thr2) return 0;
    }
    return 1;
}

/* FP64 iterative refinement as oracle_bicgstab_mixed, with the inner solve
 * keeping its Krylov vectors in complex128: r = y - A x (FP64, complex128 A);
 * stop when ||r|| <= tol ||y|| (info 0) or after maxit steps (info 1);
 * otherwise solve A32 d = r / ||r|| (the scaling in FP64, no rounding of the
 * right-hand side) with inner_bicgstab_wide to tol_inner, and set
 * x += ||r|| d in FP64.  An inner non-finite value ends the refinement with
 * info 4, an inner breakdown before the first inner update (d = 0) with the
 * inner info 2 or 3; x is then left as it was.  outer_res (maxit + 1 entries
 * or NULL) receives ||r|| / ||y|| at every outer check. */
int oracle_bicgstab_mixed_wide(int64_t n, const zc* A, int64_t lda, const fc* A32,
                               int64_t lda32, const zc* y, zc* x, double tol, int32_t maxit,
                               double tol_inner, int32_t maxit_inner, uint32_t flags,
                               oracle_mixed_stats* st, double* outer_res)
{
    memset(st, 0, sizeof *st);
    st->relres_true = NAN;
    if (n < 0) return -1;
    if (lda < (n > 1 ? n : 1) || lda32 < (n > 1 ? n : 1)) return -3;
    if (!(tol > 0.0) || !isfinite(tol) || maxit < 0) return -6;
    if (!(tol_inner > 0.0) || !(tol_inner < 1.0) || maxit_inner < 1) return -10;
    if (n == 0) {
        st->relres_true = 0.0;
        return 0;
    }
    double ny2 = norm2sq(n, y);
    if (!isfinite(ny2)) {
        st->info = 4;
        return 0;
    }
    if (ny2 == 0.0) {
        zzero(n, x);
        st->relres_true = 0.0;
        return 0;
    }
    zc* w = (zc*)malloc(sizeof(zc) * (size_t)(9 * n));
    if (!w) return -100;
    zc *r = w, *b = w + n, *d = w + 2 * n, *inner = w + 3 * n;
    const double thr2 = tol * tol * ny2;
    for (int32_t outer = 0;; ++outer) {
        if (outer == 0 && (flags & ORACLE_X0_ZERO)) {
            zzero(n, x);
            zcopy(n, y, r);
        } else {
            residual(n, A, lda, y, x, r);
            st->matvecs64++;
        }
        double rr = norm2sq(n, r);
        st->relres_true = sqrt(rr / ny2);
        if (outer_res) outer_res[outer] = st->relres_true;
        if (!isfinite(rr)) {
            st->info = 4;
            break;
        }
        if (rr <= thr2) {
            st->info = 0;
            break;
        }
        if (outer >= maxit) {
            st->info = 1;
            break;
        }
        const double nr = sqrt(rr);
        const double scale = 1.0 / nr;
        for (int64_t i = 0; i < n; ++i)
            b[i] = CMPLX(creal(r[i]) * scale, cimag(r[i]) * scale);
        int32_t it = 0;
        int info_in = inner_bicgstab_wide(n, A32, lda32, b, d, tol_inner, maxit_inner, &it,
                                          &st->matvecs32, inner);
        st->outer++;
        st->inner_iters += it;
        if (info_in == 4) {
            st->info = 4;
            break;
        }
        if ((info_in == 2 || info_in == 3) && it == 0) {
            st->info = info_in;
            break;
        }
        for (int64_t i = 0; i < n; ++i)
            x[i] = x[i] + CMPLX(nr * creal(d[i]), nr * cimag(d[i]));
    }
    free(w);
    return 0;
}

/* --------------------------------------------------------------------- CG */

/* Hestenes-Stiefel CG for Hermitian positive-definite A.  Stops on the
 * recursive residual ||r|| <= tol ||y||; reports the true residual too. */
int oracle_cg(int64_t n, const zc* A, int64_t lda, const zc* y, zc* x,
              double tol, int32_t maxit, uint32_t flags, oracle_stats* st,
              oracle_hist* hist)
{
    stats_init(st);
    int bad = bad_args(n, lda, tol, maxit);
    if (bad) return bad;
    hist_init(hist, maxit);

    zc* work = (zc*)malloc(sizeof(zc) * (size_t)(4 * (n > 0 ? n : 1)));
    if (!work) return -100;
    zc *r = work, *p = r + n, *q = p + n, *tmp = q + n;

    double ny2 = 0.0, rr = 0.0;
    if (setup(n, A, lda, y, x, flags, r, &ny2, &rr, st)) {
        free(work);
        return 0;
    }
    const double thr2 = tol * tol * ny2;
    int32_t k = 0;
    st->info = 1;
    if (rr <= thr2) {
        st->info = 0;
    } else {
        zcopy(n, r, p);
        while (k < maxit) {
            oracle_matvec(n, A, lda, p, q);
            st->matvecs++;
            double pq = creal(dotc(n, p, q));
            if (!isfinite(pq)) {
                st->info = 4;
                break;
            }
            if (pq <= 0.0) { /* not positive definite along p */
                st->info = 2;
                break;
            }
            double alpha = rr / pq;
            for (int64_t i = 0; i < n; ++i) {
                x[i] = x[i] + alpha * p[i];
                r[i] = r[i] - alpha * q[i];
            }
            double rr_new = norm2sq(n, r);
            k++;
            if (hist) {
                hist[k - 1].alpha_re = alpha;
                hist[k - 1].alpha_im = 0.0;
                hist[k - 1].res_full = sqrt(rr_new / ny2);
            }
            st->relres_rec = sqrt(rr_new / ny2);
            if (!isfinite(rr_new)) {
                st->info = 4;
                break;
            }
            if (rr_new <= thr2) {
                st->info = 0;
                break;
            }
            double beta = rr_new / rr;
            if (hist) {
                hist[k - 1].beta_re = beta;
                hist[k - 1].beta_im = 0.0;
            }
            for (int64_t i = 0; i < n; ++i)
                p[i] = r[i] + beta * p[i];
            rr = rr_new;
        }
    }
    residual(n, A, lda, y, x, tmp);
    st->relres_true = sqrt(norm2sq(n, tmp) / ny2);
    st->iters = k;
    free(work);
    return 0;
}
