/*
 * ccg.h -- C ABI of the MI355X (gfx950) complex Krylov solvers.
 *
 * Problem: solve A x = y for a dense complex square matrix A (Introduction,
 * the problem statement "Ax = y").  The matrix-vector product is an entry
 * point of its own, apart from the iterations (Abstract; Usage section: the
 * matvec and cmatvec routines), and the solvers are two of the PIM90 set
 * (Codes, section 2.1): bicgstab (BiCGSTAB) and cgnr (CG on the normal
 * equations).  The tolerance and iteration budget play the part of the
 * cgmodule structure's epsilon_err and maxit (Usage section).
 *
 * Types and layout
 *   ccg_z      one complex128, real part first (16 bytes).  Bit-compatible with
 *              C99 double _Complex, std::complex<double> and torch.complex128.
 *   A          n x n, row-major: element (i, j) at A[i*lda + j], lda >= n.
 *   vectors    contiguous (stride 1), n elements.
 *   stream     a hipStream_t passed as void*; NULL means the null stream.
 *
 * Ownership
 *   A, x, y, work and hist are device pointers owned by the caller.  The
 *   library keeps no pointer after a call returns.  info and res are host
 *   pointers.  A and y are only read; x is read (initial guess) and written
 *   (solution).
 *
 * Return value of every entry point
 *   0 on success; -k when argument k (1-based) is illegal, in which case no
 *   work is enqueued; a positive hipError_t when the HIP runtime fails.
 *
 * Solver status (*info, res->info)
 *   0  converged: ||y - A x||_2 <= tol * ||y||_2, checked on the true residual
 *   1  iteration budget maxit spent
 *   2  breakdown: rho or sigma (BiCGSTAB); ||A p|| or ||A^H r|| zero (CGNR);
 *      a zero bilinear form (r, r), (p, A p), (r, A r) or (A p, A p) (COCG,
 *      COCR)
 *   3  breakdown: t^H t or omega zero (BiCGSTAB)
 *   4  a non-finite value was met (x is left at the last finite iterate:
 *      x0 as given, or x = 0 under CCG_X0_ZERO when y itself is not finite)
 *   n == 0 is a no-op with info 0; y == 0 gives x = 0 with info 0.
 *
 * Concurrency: calls on different streams with different workspaces are
 * independent.  The solvers wait on their stream before they return; the
 * matrix-vector products do not wait.
 */
#ifndef CCG_H
#define CCG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    double re, im;
} ccg_z;

typedef struct {
    float re, im;
} ccg_c; /* complex64, real part first (8 bytes); torch.complex64 */

/* Outcome of a solve (host struct). */
typedef struct {
    int32_t info;       /* status, codes above */
    int32_t iters;      /* completed iterations; a half-step exit counts */
    int32_t matvecs;    /* applications of A or A^H, confirmations included */
    int32_t confirms;   /* true-residual checks made */
    double relres_rec;  /* last recursive ||r|| / ||y|| */
    double relres_true; /* last true ||y - A x|| / ||y|| */
} ccg_result;

/* Per-iteration record (device array of maxit entries, optional).  Fields a
 * method does not produce are left as they were (callers fill with NaN).
 * BiCGSTAB: alpha, omega, beta (the beta used to form this iteration's
 * direction), res_half = ||s||/||y||, res_full = ||r||/||y||.
 * CGNR: alpha (real), beta (real, formed at the end of the iteration),
 * res_full = ||r||/||y||. */
typedef struct {
    double alpha_re, alpha_im;
    double omega_re, omega_im;
    double beta_re, beta_im;
    double res_half, res_full;
} ccg_hist;

enum { CCG_OP_N = 0, CCG_OP_C = 1, CCG_OP_S = 2 };

/* Method ids for ccg_workspace_bytes. */
enum {
    CCG_WS_MATVEC_C = 1, /* scratch of ccg_matvec_ex with op = CCG_OP_C */
    CCG_WS_BICGSTAB = 2,
    CCG_WS_CGNR = 3,
    CCG_WS_MATMAT = 4,         /* scratch of ccg_matmat_ex (nrhs = k) */
    CCG_WS_BICGSTAB_BLOCK = 5, /* ccg_bicgstab_block_ex (nrhs = k <= 64) */
    CCG_WS_COCG = 6,
    CCG_WS_COCR = 7,
    CCG_WS_BICGSTAB_MIXED = 8,
    CCG_WS_T3_MATVEC = 9, /* scratch of ccg_t3_matvec (ccg_t3_workspace_bytes) */
    CCG_WS_MATMAT_C64 = 10,           /* scratch of ccg_matmat_c64 (nrhs = k) */
    CCG_WS_BICGSTAB_BLOCK_MIXED = 11, /* ccg_bicgstab_block_mixed_ex (k <= 64) */
    CCG_WS_MATVEC_S = 12              /* scratch of ccg_matvec_ex, op = CCG_OP_S */
};

/* Added to CCG_WS_BICGSTAB, CCG_WS_CGNR, CCG_WS_COCG or CCG_WS_COCR: the
 * workspace of that solver run with the flag CCG_A_SYM_UPPER (room for the
 * tile partials of the upper-triangle product, n * ceil(n / S) * 16 bytes
 * more, S = 64, 128 or 256 the product's tile edge). */
#define CCG_WS_SYM 0x100

/* Outcome of a mixed-precision solve (host struct). */
typedef struct {
    int32_t info;        /* status, codes above (from the FP64 outer loop) */
    int32_t outer;       /* refinement steps (inner solves) */
    int32_t inner_iters; /* inner BiCGSTAB iterations, all steps */
    int32_t matvecs64;   /* complex128 products (outer residuals) */
    int32_t matvecs32;   /* complex64 products (inner solves) */
    int32_t pad;
    double relres_true;  /* last FP64 ||y - A x|| / ||y|| */
} ccg_mixed_result;

/* Flags of the _ex solvers. */
#define CCG_X0_ZERO 1u /* x holds no guess: start from x = 0, skip y - A x */
/* A is complex symmetric (A^T = A, not checked; the matrices of COCG and
 * COCR, section 3.4): every product reads only the upper triangle (elements
 * (i, j) with j >= i), half the bytes of a dense product; what lies below the
 * diagonal is never read and may hold anything.  CGNR's A^H r is then
 * conj(A) r from the same triangle.  The workspace is
 * ccg_workspace_bytes(method | CCG_WS_SYM, n, 1). */
#define CCG_A_SYM_UPPER 2u

/*
 * y = op(A) x, op(A) = A (op = CCG_OP_N) or A^H (op = CCG_OP_C), or y = A x
 * for a complex symmetric A read from its upper triangle (op = CCG_OP_S:
 * y_i = sum_{j<i} A_ji x_j + sum_{j>=i} A_ij x_j; below the diagonal nothing
 * is read).  The user matvec / cmatvec of the Usage section; cmatvec is read
 * as the conjugate transpose, which CGNR needs.  Sums are in FP64 with a
 * fixed order (results are bitwise reproducible from run to run).  x and y
 * must not overlap.  Enqueued on stream, no wait.  CCG_OP_C and CCG_OP_S
 * take a stream-ordered scratch of ccg_workspace_bytes(CCG_WS_MATVEC_C or
 * CCG_WS_MATVEC_S, n, 1) bytes from the HIP stream-ordered allocator;
 * ccg_matvec_ex takes it from the caller instead.
 * Arguments: 1 op, 2 n >= 0, 3 A, 4 lda >= max(1,n), 5 x, 6 y, 7 stream.
 */
int ccg_matvec(int op, int64_t n, const ccg_z* A, int64_t lda, const ccg_z* x,
               ccg_z* y, void* stream);

/* As ccg_matvec, with caller scratch (7: work, 8: work_bytes; unused for
 * CCG_OP_N, may be NULL/0 there). Argument 9 is the stream. */
int ccg_matvec_ex(int op, int64_t n, const ccg_z* A, int64_t lda,
                  const ccg_z* x, ccg_z* y, void* work, size_t work_bytes,
                  void* stream);

/*
 * As ccg_matvec, allocating nothing: for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation).  The partial sums of CCG_OP_C and CCG_OP_S go to a
 * fixed device array of CCG_NOALLOC_SCRATCH_BYTES, one per GPU, held from the
 * library's loading until the process ends; CCG_OP_N needs none.  Returns -2
 * when n is out of range or its partials exceed that array (CCG_OP_C needs
 * at most 16 n + 1 MiB bytes, so any n below 2^20; CCG_OP_S needs
 * n * ceil(n / S) * 16 bytes for its tile edge S, so n <= 16384), with no
 * work enqueued.  Every call on one GPU shares that
 * GPU's array: calls that overlap on one GPU (other streams, other threads)
 * race.  The results are bitwise those of ccg_matvec.  Enqueued on stream,
 * no wait.  Arguments as ccg_matvec: 1 op, 2 n, 3 A, 4 lda, 5 x, 6 y,
 * 7 stream.
 */
#define CCG_NOALLOC_SCRATCH_BYTES (16u << 20)
int ccg_matvec_noalloc(int op, int64_t n, const ccg_z* A, int64_t lda,
                       const ccg_z* x, ccg_z* y, void* stream);

/*
 * Many small systems at once: BiCGSTAB (method CCG_WS_BICGSTAB) or CGNR
 * (CCG_WS_CGNR) on batch independent dense systems A_b x_b = y_b of one size
 * n <= CCG_SMALL_MAX_N (the problem "Ax = y" of the Introduction, solved by
 * section 2.1's bicgstab and cgnr for many right-hand sides and matrices at
 * once).  Same methods, stop rule, confirmation, restart and info codes as
 * ccg_bicgstab_ex / ccg_cgnr_ex; every system takes its own decisions, and
 * its result does not depend on the rest of the batch (bitwise).  One
 * workgroup per system runs its whole solve inside one kernel launch, with
 * the Krylov vectors in LDS, so a batch is one launch bound by the HBM
 * stream of the matrices.
 * Layout: system b's matrix at A + b * strideA (row-major, lda >= n), its
 * right-hand side at Y + b * strideY and its x at X + b * strideX (n
 * contiguous elements each; strides are in elements and only checked when
 * batch > 1).  X holds the initial guesses (ignored under CCG_X0_ZERO).
 * res: device array of batch ccg_result, written by the kernel.  All
 * pointers are device pointers.  Asynchronous: nothing is waited for, res
 * is valid once the stream has passed the launch.
 * Arguments: 1 method, 2 n (0..CCG_SMALL_MAX_N), 3 batch >= 0, 4 A, 5 lda,
 * 6 strideA >= (n - 1) lda + n, 7 Y, 8 strideY >= n, 9 X, 10 strideX >= n,
 * 11 tol (> 0, finite), 12 maxit >= 0, 13 flags (CCG_X0_ZERO or 0), 14 res,
 * 15 stream.
 */
#define CCG_SMALL_MAX_N 1024
int ccg_solve_small_batched(int method, int64_t n, int64_t batch,
                            const ccg_z* A, int64_t lda, int64_t strideA,
                            const ccg_z* Y, int64_t strideY, ccg_z* X,
                            int64_t strideX, double tol, int32_t maxit,
                            uint32_t flags, ccg_result* res, void* stream);

/*
 * Measurement aid, outside the method: HIP events around the solvers' dense
 * complex128 products, so that a caller can time the product kernel inside
 * its solves (the A x that dominates their bytes) rather than apart from
 * them.  events holds 2 * capacity hipEvent_t (as void*) created by the
 * caller with timing enabled; count is the number of (start, end) pairs
 * recorded so far and seen the number of products counted while attached,
 * both advanced by the library.  While a log is attached, the dense
 * complex128 A x launches of ccg_bicgstab*, ccg_cgnr*, ccg_cocg* and
 * ccg_cocr* that the calling host thread makes, of the kinds in the mask
 * roles (CCG_PROD_*; 0: every kind), are counted, and every stride-th of
 * them (seen % stride == 0; stride <= 1: all) is bracketed by
 * hipEventRecord(events[2 count]) and hipEventRecord(events[2 count + 1]) on
 * the solve's stream, until capacity pairs are used.  (Each record costs a
 * few microseconds of stream time; a stride spreads a few samples over many
 * solves.)  The log is per host thread; the library keeps the pointer until
 * ccg_set_event_log(NULL), so the caller keeps the struct alive until then.
 * Returns -1 for a negative capacity or a null events array with
 * capacity > 0.
 */
typedef struct {
    void** events;    /* 2 * capacity hipEvent_t, caller-created and -owned */
    int32_t capacity; /* event pairs */
    int32_t count;    /* pairs recorded; advanced by the library */
    int32_t stride;   /* record every stride-th counted product (<= 1: each) */
    int32_t seen;     /* products counted while attached; advanced by the library */
    uint32_t roles;   /* CCG_PROD_* mask of the products counted; 0: all */
    int32_t pad;
} ccg_event_log;
/* Kinds of the solvers' dense products (ccg_event_log.roles). */
enum {
    CCG_PROD_SETUP = 1, /* set-up residuals y - A x */
    CCG_PROD_V = 2,     /* BiCGSTAB v = A p, and its confirming residuals */
    CCG_PROD_T = 4,     /* BiCGSTAB t = A s */
    CCG_PROD_W = 8,     /* CGNR w = A p, and its confirming residuals */
    CCG_PROD_Q = 16,    /* COCG q = A p, and its confirming residuals */
    CCG_PROD_U = 32     /* COCR u = A r, and its confirming residuals */
};
int ccg_set_event_log(ccg_event_log* log);

/*
 * Measurement aid, outside the method: one pass that reads bytes bytes at src
 * (device; 16-byte aligned, bytes a multiple of 16) with the 16-byte
 * nontemporal loads the products use, and nothing else -- the HBM read rate
 * the chip delivers to that load pattern, beside which the products' rates
 * are set.  One block per slab of CCG_READ_STREAM_SLAB bytes writes the
 * 16-byte sum of what it read to out (device, 16-byte aligned, out_bytes >=
 * 16 * ceil(bytes / CCG_READ_STREAM_SLAB)), so no load can be dropped.
 * Asynchronous on stream.  Returns -1 null src, -2 misaligned src or bytes,
 * -3 bad out, -4 out too small.
 */
#define CCG_READ_STREAM_SLAB 262144
int ccg_read_stream(const void* src, size_t bytes, void* out, size_t out_bytes,
                    void* stream);

/* Bytes of device workspace the _ex entry points need (256-byte aligned
 * start required).  nrhs is 1 for the single right-hand-side solvers. */
size_t ccg_workspace_bytes(int method, int64_t n, int64_t nrhs);

/*
 * BiCGSTAB (section 2.1, bicgstab; van der Vorst's method, unpreconditioned,
 * shadow residual fixed to the starting residual).  x holds the initial
 * guess.  Stops on ||r|| <= tol ||y|| (at the half step s or at r), confirms
 * with the true residual, and on a failed confirmation restarts from it
 * within the same budget.  Allocates its workspace, waits on stream, writes
 * *info.
 * Arguments: 1 n, 2 A, 3 lda, 4 y, 5 x, 6 tol (> 0, finite), 7 maxit >= 0,
 * 8 info (host, not NULL), 9 stream.
 */
int ccg_bicgstab(int64_t n, const ccg_z* A, int64_t lda, const ccg_z* y,
                 ccg_z* x, double tol, int32_t maxit, int32_t* info,
                 void* stream);

/*
 * CGNR (section 2.1, cgnr): conjugate gradients on A^H A x = A^H y, one
 * product with A and one with A^H per iteration.  Same stop rule,
 * confirmation, arguments and waiting as ccg_bicgstab.
 */
int ccg_cgnr(int64_t n, const ccg_z* A, int64_t lda, const ccg_z* y, ccg_z* x,
             double tol, int32_t maxit, int32_t* info, void* stream);

/*
 * Extended forms: caller workspace, flags, outcome and per-iteration record.
 * Arguments: 1 n, 2 A, 3 lda, 4 y, 5 x, 6 tol, 7 maxit, 8 flags (CCG_X0_ZERO,
 * CCG_A_SYM_UPPER, or 0), 9 work (device, 256-byte aligned), 10 work_bytes
 * (>= the ccg_workspace_bytes figure), 11 res (host, not NULL), 12 hist
 * (device array of maxit ccg_hist, or NULL), 13 stream.  Wait on stream
 * before returning.
 */
int ccg_bicgstab_ex(int64_t n, const ccg_z* A, int64_t lda, const ccg_z* y,
                    ccg_z* x, double tol, int32_t maxit, uint32_t flags,
                    void* work, size_t work_bytes, ccg_result* res,
                    ccg_hist* hist, void* stream);

int ccg_cgnr_ex(int64_t n, const ccg_z* A, int64_t lda, const ccg_z* y,
                ccg_z* x, double tol, int32_t maxit, uint32_t flags,
                void* work, size_t work_bytes, ccg_result* res, ccg_hist* hist,
                void* stream);

/*
 * COCG and COCR for complex symmetric A (A^T = A, not checked): the methods
 * of the "next releases" section 3.4 (COCR of Sogabe and Zhang, compared
 * there with COCG).  CG and CR with the unconjugated bilinear form
 * (a, b) = sum a_i b_i; one product with A per iteration.  Same stop rule,
 * confirmation, restart, arguments, waiting and info codes as
 * ccg_bicgstab / ccg_bicgstab_ex (workspace ids CCG_WS_COCG, CCG_WS_COCR).
 * COCG's record holds alpha and beta (complex) and res_full; COCR's the same.
 */
int ccg_cocg(int64_t n, const ccg_z* A, int64_t lda, const ccg_z* y, ccg_z* x,
             double tol, int32_t maxit, int32_t* info, void* stream);
int ccg_cocr(int64_t n, const ccg_z* A, int64_t lda, const ccg_z* y, ccg_z* x,
             double tol, int32_t maxit, int32_t* info, void* stream);
int ccg_cocg_ex(int64_t n, const ccg_z* A, int64_t lda, const ccg_z* y,
                ccg_z* x, double tol, int32_t maxit, uint32_t flags,
                void* work, size_t work_bytes, ccg_result* res, ccg_hist* hist,
                void* stream);
int ccg_cocr_ex(int64_t n, const ccg_z* A, int64_t lda, const ccg_z* y,
                ccg_z* x, double tol, int32_t maxit, uint32_t flags,
                void* work, size_t work_bytes, ccg_result* res, ccg_hist* hist,
                void* stream);

/*
 * Mixed precision BiCGSTAB (the single/double switch of the ddprecision
 * module, Usage section, used inside one solve): FP64 iterative refinement
 * around an inner complex64 BiCGSTAB.  Each outer step takes the residual
 * r = y - A x with the complex128 A in FP64, solves A32 d = r / ||r|| with
 * complex64 vectors and products (FP32 accumulation; the dot products and the
 * alpha / omega / beta / rho scalars stay FP64) to the relative tolerance
 * tol_inner, stopping on its recursive residual, and applies x += ||r|| d in
 * FP64.  The outer loop stops when the FP64 true residual meets tol (info 0)
 * or after maxit steps (info 1).  An inner budget or a later inner breakdown
 * only ends that inner solve; an inner non-finite value ends the refinement
 * with info 4, and an inner breakdown before the first inner update (d = 0,
 * so the next step would repeat this one) ends it with the inner info 2 or
 * 3; x is then left as it was.  A32 is the complex64 copy of A
 * (ccg_round_c64), lda32 >= n.
 * Arguments: 1 n, 2 A, 3 lda, 4 A32, 5 lda32, 6 y, 7 x, 8 tol, 9 maxit
 * (outer steps), 10 tol_inner (0 < tol_inner < 1), 11 maxit_inner >= 1,
 * 12 flags (CCG_X0_ZERO or 0), 13 work, 14 work_bytes (>=
 * ccg_workspace_bytes(CCG_WS_BICGSTAB_MIXED, n, 1)), 15 res (host),
 * 16 outer_res (host array of maxit + 1 doubles or NULL: ||r|| / ||y|| at
 * every outer check, NaN past the last), 17 stream.  Waits on stream.
 */
int ccg_bicgstab_mixed_ex(int64_t n, const ccg_z* A, int64_t lda,
                          const ccg_c* A32, int64_t lda32, const ccg_z* y,
                          ccg_z* x, double tol, int32_t maxit, double tol_inner,
                          int32_t maxit_inner, uint32_t flags, void* work,
                          size_t work_bytes, ccg_mixed_result* res,
                          double* outer_res, void* stream);

/* y = A x in complex64, the inner product of the mixed-precision solver: each
 * lane accumulates in FP32 with fused multiply-adds, lanes and wavefronts are
 * added in FP64 and the total rounded to complex64.  Same layout and
 * asynchrony as ccg_matvec.  Arguments: 1 n, 2 A (complex64), 3 lda, 4 x,
 * 5 y, 6 stream. */
int ccg_matvec_c64(int64_t n, const ccg_c* A, int64_t lda, const ccg_c* x,
                   ccg_c* y, void* stream);

/* dst = complex64(src) for a rows x cols row-major block (round to nearest).
 * Arguments: 1 rows, 2 cols, 3 src, 4 lds >= cols, 5 dst, 6 ldd >= cols,
 * 7 stream.  Asynchronous. */
int ccg_round_c64(int64_t rows, int64_t cols, const ccg_z* src, int64_t lds,
                  ccg_c* dst, int64_t ldd, void* stream);

/*
 * Z = A B for k right-hand sides at once: B and Z are n x k, row-major
 * (element (i, c) at B[i*ldb + c], ldb >= k; same for Z).  The user matvec of
 * the Usage section applied to k vectors; on FP64 matrix cores
 * (v_mfma_f64_16x16x4f64), FP64 accumulation in a fixed order (reproducible
 * bit for bit).  Beyond 8 columns each complex product is formed from three
 * real ones (Re A Re B, Im A Im B, (Re A + Im A)(Re B + Im B)): every element
 * is within about 3 (n + 2) u |A| |B| of the exact product, u = 2^-53, and
 * exact on Gaussian integers of moderate size.  Columns are processed 64 at a
 * time.  B and Z must not
 * overlap.  Asynchronous; ccg_matmat takes a stream-ordered scratch of
 * ccg_workspace_bytes(CCG_WS_MATMAT, n, k) bytes, ccg_matmat_ex takes it from
 * the caller (256-byte aligned).
 * Arguments: 1 n, 2 k >= 0, 3 A, 4 lda, 5 B, 6 ldb, 7 Z, 8 ldz, [9 work,
 * 10 work_bytes,] stream.
 */
int ccg_matmat(int64_t n, int64_t k, const ccg_z* A, int64_t lda, const ccg_z* B,
               int64_t ldb, ccg_z* Z, int64_t ldz, void* stream);
int ccg_matmat_ex(int64_t n, int64_t k, const ccg_z* A, int64_t lda,
                  const ccg_z* B, int64_t ldb, ccg_z* Z, int64_t ldz, void* work,
                  size_t work_bytes, void* stream);

/*
 * Block BiCGSTAB: the k systems A x_c = y_c (columns of Y, X; n x k,
 * row-major, 1 <= k <= 64) solved together.  Every column has its own rho,
 * alpha, omega, beta, stop test, confirmation and info, exactly as
 * ccg_bicgstab would give it; the two products of an iteration are one
 * matrix-matrix product each for all columns.  A column that has finished is
 * frozen (its x is not written again).  Y is read; X holds the initial
 * guesses and receives the solutions.
 * ccg_bicgstab_block: arguments 1 n, 2 k, 3 A, 4 lda, 5 Y, 6 ldy >= k, 7 X,
 * 8 ldx >= k, 9 tol, 10 maxit, 11 info (host array of k), 12 stream;
 * allocates its workspace, waits on stream.
 * ccg_bicgstab_block_ex: arguments 1-10 as above, 11 flags (CCG_X0_ZERO or 0),
 * 12 work (device, 256-byte aligned), 13 work_bytes (>= the
 * ccg_workspace_bytes(CCG_WS_BICGSTAB_BLOCK, n, k) figure), 14 res (host
 * array of k ccg_result), 15 stream; waits on stream.
 */
int ccg_bicgstab_block(int64_t n, int64_t k, const ccg_z* A, int64_t lda,
                       const ccg_z* Y, int64_t ldy, ccg_z* X, int64_t ldx,
                       double tol, int32_t maxit, int32_t* info, void* stream);
int ccg_bicgstab_block_ex(int64_t n, int64_t k, const ccg_z* A, int64_t lda,
                          const ccg_z* Y, int64_t ldy, ccg_z* X, int64_t ldx,
                          double tol, int32_t maxit, uint32_t flags, void* work,
                          size_t work_bytes, ccg_result* res, void* stream);

/*
 * Z = A32 B with A32 complex64 (the copy made by ccg_round_c64), B and Z
 * complex128 n x k row-major: B is rounded to complex64 as it is read, the
 * products (three real ones per complex one, as in ccg_matmat) accumulate in
 * FP32 on the FP32 matrix cores (v_mfma_f32_16x16x4f32), each of the 8
 * K-slices is widened to FP64 and the slices are added in FP64 in a fixed
 * order.  The product of the mixed block solver below.  Arguments: 1 n, 2 k, 3 A32, 4 lda32, 5 B, 6 ldb, 7 Z, 8 ldz,
 * 9 work (256-byte aligned, >= ccg_workspace_bytes(CCG_WS_MATMAT_C64, n, k)),
 * 10 work_bytes, 11 stream.  Asynchronous.
 */
int ccg_matmat_c64(int64_t n, int64_t k, const ccg_c* A32, int64_t lda32,
                   const ccg_z* B, int64_t ldb, ccg_z* Z, int64_t ldz,
                   void* work, size_t work_bytes, void* stream);

/*
 * Mixed-precision block BiCGSTAB: ccg_bicgstab_mixed_ex for k right-hand
 * sides at once (1 <= k <= 64).  Per outer step the FP64 residual
 * R = Y - A X (FP64 matrix cores); every column not yet within tol solves
 * A32 D = R / ||R|| with the block solver on the complex64 product
 * (ccg_matmat_c64) to tol_inner (recursive residual) and takes
 * X += ||R|| D in FP64.  The inner Krylov vectors stay complex128 (O(n k)
 * bytes; the complex64 copy halves the O(n^2) bytes of A).  Per column: info
 * 0 within tol, 1 after maxit outer steps, 4 non-finite (x left as given),
 * and the inner-breakdown rule of ccg_bicgstab_mixed_ex (info 4, 2 or 3);
 * y = 0 gives x = 0.  Arguments: 1 n, 2 k, 3 A, 4 lda, 5 A32, 6 lda32, 7 Y,
 * 8 ldy >= k, 9 X, 10 ldx >= k, 11 tol, 12 maxit (outer), 13 tol_inner
 * (0 < tol_inner < 1), 14 maxit_inner >= 1, 15 flags (CCG_X0_ZERO or 0),
 * 16 work (>= ccg_workspace_bytes(CCG_WS_BICGSTAB_BLOCK_MIXED, n, k)),
 * 17 work_bytes, 18 res (host array of k ccg_mixed_result), 19 outer_res
 * (host array of k * (maxit + 1) doubles or NULL: column c's ||r|| / ||y||
 * at outer check j in outer_res[c * (maxit + 1) + j], NaN where not
 * reached), 20 stream.  Waits on stream.
 */
int ccg_bicgstab_block_mixed_ex(int64_t n, int64_t k, const ccg_z* A,
                                int64_t lda, const ccg_c* A32, int64_t lda32,
                                const ccg_z* Y, int64_t ldy, ccg_z* X,
                                int64_t ldx, double tol, int32_t maxit,
                                double tol_inner, int32_t maxit_inner,
                                uint32_t flags, void* work, size_t work_bytes,
                                ccg_mixed_result* res, double* outer_res,
                                void* stream);

/*
 * Structured product: A is a three-level Toeplitz matrix on an m x m x m
 * lattice (n = m^3, point index ix + m iy + m^2 iz), A_ij = T(p_i - p_j) for
 * a kernel T on the displacement box [-(m-1), m-1]^3 -- the shape of the
 * discrete-dipole systems of the Introduction, used through the user's own
 * matrix scheme that the Usage section leaves to the caller's matvec.  The
 * product is a zero-padded 3-D FFT convolution on an M^3 grid (M the
 * smallest power of two >= max(2m - 1, 16); 1 <= m <= 128): O(n log n) work
 * and O(n) memory instead of the dense 16 n^2 bytes.  A kernel even in x and
 * in y (T(-dx, dy, dz) = T(dx, dy, dz) = T(dx, -dy, dz) bit for bit, as the
 * lattice kernel, a function of |d|) is detected at set-up; its transform is
 * then kept for the frequencies |kx|, |ky| <= M/2 only, a quarter of the
 * bytes each product streams for it.
 *
 * ccg_t3_setup: 1 m, 2 table (device, (2m-1)^3 complex128; displacement
 * (dx, dy, dz) at ((dz+m-1)(2m-1) + (dy+m-1))(2m-1) + (dx+m-1); the zero
 * displacement is the diagonal), 3 op (device, 256-byte aligned, receives the
 * transformed kernel; op_bytes >= ccg_t3_op_bytes(m)), 4 op_bytes, 5 stream.
 * Asynchronous; the table may be freed once the stream has passed the call.
 * ccg_t3_matvec: y = A x; 1 m, 2 op, 3 x, 4 y (may equal x), 5 work (device,
 * 256-byte aligned, >= ccg_t3_workspace_bytes(CCG_WS_T3_MATVEC, m)),
 * 6 work_bytes, 7 stream.  Asynchronous.
 * ccg_t3_bicgstab_ex / ccg_t3_cocg_ex / ccg_t3_cocr_ex: the solvers of
 * ccg_bicgstab_ex / ccg_cocg_ex / ccg_cocr_ex with the structured product;
 * 1 m, 2 op, 3 y, 4 x, 5 tol, 6 maxit, 7 flags, 8 work (>=
 * ccg_t3_workspace_bytes(CCG_WS_BICGSTAB / _COCG / _COCR, m)), 9 work_bytes,
 * 10 res, 11 hist, 12 stream.  COCG and COCR need T(d) = T(-d) (A complex
 * symmetric), which the lattice kernel has.  Wait on stream.
 */
size_t ccg_t3_op_bytes(int64_t m);
size_t ccg_t3_workspace_bytes(int method, int64_t m);
int ccg_t3_setup(int64_t m, const ccg_z* table, void* op, size_t op_bytes,
                 void* stream);
int ccg_t3_matvec(int64_t m, const void* op, const ccg_z* x, ccg_z* y,
                  void* work, size_t work_bytes, void* stream);
int ccg_t3_bicgstab_ex(int64_t m, const void* op, const ccg_z* y, ccg_z* x,
                       double tol, int32_t maxit, uint32_t flags, void* work,
                       size_t work_bytes, ccg_result* res, ccg_hist* hist,
                       void* stream);
int ccg_t3_cocg_ex(int64_t m, const void* op, const ccg_z* y, ccg_z* x,
                   double tol, int32_t maxit, uint32_t flags, void* work,
                   size_t work_bytes, ccg_result* res, ccg_hist* hist,
                   void* stream);
int ccg_t3_cocr_ex(int64_t m, const void* op, const ccg_z* y, ccg_z* x,
                   double tol, int32_t maxit, uint32_t flags, void* work,
                   size_t work_bytes, ccg_result* res, ccg_hist* hist,
                   void* stream);

/*
 * Serving: many independent block systems (the ccg_bicgstab_block problem,
 * x0 = 0) solved by one server with continuous batching.  Each request is
 * A (n x n), Y and X (n x k, row-major, 1 <= k <= 16), tol and maxit.
 *
 * The server owns a device pool (given by the caller, 256-byte aligned).  A
 * request is admitted, in arrival order, when a slot is free (at most
 * max_active at once) and its footprint (A, Y, X and the block-solver
 * workspace, ccg_server_request_bytes) fits in the free pool; admission
 * copies Y, and A when it is in host memory, into the pool (hipMemcpyDefault)
 * and runs the solver set-up; an A in device memory of the server's GPU is
 * read in place (its pool region stays reserved).  Every ccg_server_step enqueues one iteration
 * of every admitted request as one batch of kernels (the grid of each kernel
 * covers all requests; each request keeps its own scalars, stop tests and
 * reduction order), so a request's result is bit for bit the result of
 * ccg_bicgstab_block_ex with CCG_X0_ZERO on the same inputs, alone or in any
 * mix.  When all columns of a request have finished (or 2 maxit + 4
 * iterations have been enqueued for it), X is copied to the caller's X and
 * the request's pool memory is released.
 *
 * Sources A, Y and destination X must stay valid and unchanged until
 * ccg_server_poll reports the request done.  A server is used from one host
 * thread at a time; its work runs on `stream`.
 */
typedef struct ccg_server ccg_server;

#define CCG_SERVER_REJECTED (-1000) /* footprint exceeds the whole pool */

enum {
    CCG_REQ_QUEUED = 0,  /* waiting for a slot or pool space */
    CCG_REQ_RUNNING = 1, /* admitted; iterating or copying out */
    CCG_REQ_DONE = 2     /* finished; res filled, ticket released */
};

typedef struct {
    int64_t ticks;           /* batched iterations enqueued */
    int64_t submitted, admitted, completed, rejected;
    int64_t admission_waits; /* steps in which the queue head did not fit */
    int32_t active, queued, peak_active, pad;
    uint64_t pool_used, pool_peak; /* bytes of request footprints */
} ccg_server_stats;

/* Creates a server on the current device.  Arguments: 1 pool (device,
 * 256-byte aligned), 2 pool_bytes, 3 max_active (1..128), 4 stream, 5 out.
 * The pool stays the caller's: it must outlive the server. */
int ccg_server_create(void* pool, size_t pool_bytes, int32_t max_active,
                      void* stream, ccg_server** out);

/* Waits for the server's stream and releases its host resources. */
int ccg_server_destroy(ccg_server* srv);

/* Bytes of pool a request of n rows and k right-hand sides occupies. */
size_t ccg_server_request_bytes(int64_t n, int64_t k);

/* Queues a request.  Arguments: 1 srv, 2 n, 3 k (1..16), 4 A, 5 lda, 6 Y,
 * 7 ldy >= k, 8 X, 9 ldx >= k, 10 tol, 11 maxit, 12 ticket (out).
 * Returns CCG_SERVER_REJECTED when the request could never fit the pool.
 * n = 0 completes at once (info 0). */
int ccg_server_submit(ccg_server* srv, int64_t n, int64_t k, const ccg_z* A,
                      int64_t lda, const ccg_z* Y, int64_t ldy, ccg_z* X,
                      int64_t ldx, double tol, int32_t maxit, int64_t* ticket);

/* A mixed-precision request (the ccg_bicgstab_block_mixed_ex problem, x0 =
 * 0): the server keeps A and a complex64 copy it rounds itself; per outer
 * step the FP64 residual and its column norms are formed for this request
 * alone, and the inner block solve (complex64 products on FP32 matrix cores)
 * joins the batched iterations with the other requests.  maxit counts outer
 * steps; tol_inner (0 < tol_inner < 1) and maxit_inner bound each inner
 * solve.  Its ccg_result per column: info as in ccg_bicgstab_block_mixed_ex,
 * iters = inner iterations, matvecs = complex64 products, confirms = FP64
 * residual products after the first, relres_rec = relres_true = the FP64
 * true relative residual.  Arguments 1-11 as ccg_server_submit, 12 tol_inner,
 * 13 maxit_inner, 14 ticket (out). */
int ccg_server_submit_mixed(ccg_server* srv, int64_t n, int64_t k,
                            const ccg_z* A, int64_t lda, const ccg_z* Y,
                            int64_t ldy, ccg_z* X, int64_t ldx, double tol,
                            int32_t maxit, double tol_inner,
                            int32_t maxit_inner, int64_t* ticket);

/* Bytes of pool a mixed-precision request occupies. */
size_t ccg_server_request_bytes_mixed(int64_t n, int64_t k);

/* One scheduling step: completes finished copy-outs, admits from the queue,
 * enqueues one batched iteration and reads the stop flags of the previous
 * one.  Blocks at most for one iteration.  Arguments: 1 srv, 2 active and
 * 3 queued (out, may be NULL). */
int ccg_server_step(ccg_server* srv, int32_t* active, int32_t* queued);

/* State of a request (CCG_REQ_*).  On CCG_REQ_DONE, res (host array of k)
 * receives the per-column results and the ticket is released; polling it
 * again returns -2.  Does not block. */
int ccg_server_poll(ccg_server* srv, int64_t ticket, int32_t* state,
                    ccg_result* res);

/* Hands out the tickets of finished requests in the order they finished
 * (ticket 0: none left); each is then read with ccg_server_poll.  Tickets
 * already released by ccg_server_poll are skipped.  Does not block. */
int ccg_server_next_done(ccg_server* srv, int64_t* ticket);

int ccg_server_get_stats(const ccg_server* srv, ccg_server_stats* out);

#ifdef __cplusplus
}
#endif

#endif /* CCG_H */
