"""Pins of the CPU oracle: checks against what mathematics fixes, not against
the oracle itself.

Each ``pin_*`` function takes an oracle handle and raises AssertionError when
the oracle disagrees with the fixed fact.  ``tests/test_oracle_*.py`` runs every
pin on the real oracle; ``tests/test_oracle_mutants.py`` plants plausible
mistakes in a copy of the oracle's C source and checks that some pin fails.

Sources of truth used here:
  * exact arithmetic (Python integers and Fractions) -- matrix products and
    the first iterations of each method;
  * dense LU solves (NumPy's LAPACK zgesv and an LU written out below);
  * closed forms (A = c I, unitary A, two-valued diagonals, 1 x 1 systems);
  * Krylov theory: CG/CGNR/BiCGSTAB terminate after m steps when the relevant
    operator has m distinct eigenvalues; CGNR's coefficients equal those of CG
    run on A^H A x = A^H y; BiCGSTAB's alpha equals CG's when A is Hermitian
    positive definite and the shadow residual is r0; omega minimises ||s - w t||
    so ||r|| <= ||s||; CGNR's residual norm never grows;
  * a third-party solver (SciPy's bicgstab);
  * for COCG / COCR (complex symmetric A): on real SPD systems the bilinear
    form is the inner product, so COCG is CG and COCR is CR, whose residual is
    the minimum over the Krylov space (checked against a brute-force least
    squares); finite termination on Q D Q^T with Q real orthogonal; exact
    bilinear-form breakdowns.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

from paper_1208_4869_amd import inputs

U = 2.0 ** -53


def gamma(k: int) -> float:
    return k * U / (1 - k * U)


# ---------------------------------------------------------------- exact tools

class Q:
    """Gaussian rational a + b i with Fraction parts (exact arithmetic)."""
    __slots__ = ("re", "im")

    def __init__(self, re, im=0):
        self.re = Fraction(re)
        self.im = Fraction(im)

    @staticmethod
    def of(z: complex) -> "Q":
        return Q(Fraction(z.real), Fraction(z.imag))

    def __add__(self, o):
        return Q(self.re + o.re, self.im + o.im)

    def __sub__(self, o):
        return Q(self.re - o.re, self.im - o.im)

    def __mul__(self, o):
        return Q(self.re * o.re - self.im * o.im, self.re * o.im + self.im * o.re)

    def __truediv__(self, o):
        d = o.re * o.re + o.im * o.im
        n = self * o.conj()
        return Q(n.re / d, n.im / d)

    def conj(self):
        return Q(self.re, -self.im)

    def abs2(self):
        return self.re * self.re + self.im * self.im

    def c(self) -> complex:
        return complex(float(self.re), float(self.im))


def qdot(a, b):
    """sum conj(a_i) b_i, exact."""
    s = Q(0)
    for u, v in zip(a, b):
        s = s + u.conj() * v
    return s


def qmatvec(A, x):
    return [sum((A[i][j] * x[j] for j in range(len(x))), Q(0))
            for i in range(len(A))]


def exact_matvec_int(A: np.ndarray, x: np.ndarray):
    """A x with Python integers (A, x Gaussian integers)."""
    n = A.shape[0]
    out = []
    for i in range(n):
        re = im = 0
        for j in range(n):
            a, b = int(A[i, j].real), int(A[i, j].imag)
            c, d = int(x[j].real), int(x[j].imag)
            re += a * c - b * d
            im += a * d + b * c
        out.append(complex(re, im))
    return np.array(out)


def lu_solve(A: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Gaussian elimination with partial pivoting, written out."""
    M = A.astype(np.complex128).copy()
    x = b.astype(np.complex128).copy()
    n = M.shape[0]
    for k in range(n):
        piv = k + int(np.argmax(np.abs(M[k:, k])))
        if piv != k:
            M[[k, piv]] = M[[piv, k]]
            x[[k, piv]] = x[[piv, k]]
        for i in range(k + 1, n):
            f = M[i, k] / M[k, k]
            M[i, k:] -= f * M[k, k:]
            x[i] -= f * x[k]
    for k in range(n - 1, -1, -1):
        x[k] = (x[k] - M[k, k + 1:] @ x[k + 1:]) / M[k, k]
    return x


def relerr(a, b) -> float:
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def hpd_with_spectrum(n: int, eigs, seed: int) -> np.ndarray:
    """Q diag(eigs) Q^H with Q a random unitary (QR of a CN(0,1) matrix)."""
    rng = np.random.default_rng(seed)
    Qm, _ = np.linalg.qr(inputs.cn01(rng, (n, n)))
    d = np.asarray(eigs, dtype=np.float64)
    A = (Qm * d) @ Qm.conj().T
    return 0.5 * (A + A.conj().T)


def dft_matrix(n: int) -> np.ndarray:
    k = np.arange(n)
    return np.exp(-2j * np.pi * np.outer(k, k) / n) / np.sqrt(n)


SOLVERS = ("bicgstab", "cgnr")


def _solve(orc, method, A, y, **kw):
    return getattr(orc, method)(np.ascontiguousarray(A), y, **kw)


# ------------------------------------------------------------ product pins

def pin_matvec_integer_exact(orc):
    """Gaussian-integer A, x: every partial sum is an integer below 2^53, so
    the product is exact whatever the order."""
    for n, seed in ((1, 0), (7, 1), (33, 2), (64, 3)):
        A = inputs.gaussian_integer_matrix(n, seed, bound=1024)
        x = inputs.gaussian_integer_vector(n, seed + 100, bound=1024)
        want = exact_matvec_int(A, x)
        assert np.array_equal(orc.matvec(A, x), want), n
        want_h = exact_matvec_int(np.ascontiguousarray(A.conj().T), x)
        assert np.array_equal(orc.matvec_h(A, x), want_h), n


def pin_matvec_rounding_bound(orc):
    """Random inputs: |fl(Ax) - Ax| <= 2 gamma_{n+2} (|A||x|) componentwise,
    against the exact product in Fractions."""
    n = 24
    rng = np.random.default_rng(7)
    A = inputs.cn01(rng, (n, n))
    x = inputs.cn01(rng, n)
    Aq = [[Q.of(A[i, j]) for j in range(n)] for i in range(n)]
    xq = [Q.of(v) for v in x]
    exact = np.array([v.c() for v in qmatvec(Aq, xq)])
    got = orc.matvec(A, x)
    bound = 2 * gamma(n + 2) * (np.abs(A) @ np.abs(x))
    assert np.all(np.abs(got - exact) <= bound)
    AH = [[Aq[j][i].conj() for j in range(n)] for i in range(n)]
    exact_h = np.array([v.c() for v in qmatvec(AH, xq)])
    got_h = orc.matvec_h(A, x)
    bound_h = 2 * gamma(n + 2) * (np.abs(A).T @ np.abs(x))
    assert np.all(np.abs(got_h - exact_h) <= bound_h)


def pin_matvec_identity_permutation(orc):
    n = 17
    rng = np.random.default_rng(3)
    x = inputs.cn01(rng, n)
    I = np.eye(n, dtype=np.complex128)
    assert np.array_equal(orc.matvec(I, x), x)
    assert np.array_equal(orc.matvec_h(I, x), x)
    perm = rng.permutation(n)
    P = np.zeros((n, n), dtype=np.complex128)
    P[np.arange(n), perm] = 1.0
    assert np.array_equal(orc.matvec(P, x), x[perm])
    out = np.empty_like(x)
    out[perm] = x
    assert np.array_equal(orc.matvec_h(P, x), out)


def pin_adjoint_identity(orc):
    """<A x, w> = <x, A^H w> up to rounding."""
    n = 96
    rng = np.random.default_rng(11)
    A = inputs.cn01(rng, (n, n))
    x = inputs.cn01(rng, n)
    w = inputs.cn01(rng, n)
    lhs = np.vdot(orc.matvec(A, x), w)
    rhs = np.vdot(x, orc.matvec_h(A, w))
    scale = np.abs(A).sum() * np.abs(x).max() * np.abs(w).max()
    assert abs(lhs - rhs) <= 4 * gamma(2 * n + 4) * scale


def pin_lattice_adjoint_symmetry(orc):
    """Complex-symmetric lattice matrix: A^H x = conj(A conj(x)), bitwise (the
    two are the same sums in the same order)."""
    A = inputs.lattice_matrix(4)
    rng = np.random.default_rng(5)
    x = inputs.cn01(rng, A.shape[0])
    assert np.array_equal(orc.matvec_h(A, x), np.conj(orc.matvec(A, np.conj(x))))


def pin_sym_upper_integer_exact(orc):
    """The upper-triangle product of a complex symmetric matrix: on Gaussian
    integers it equals, exactly, the product with the symmetric matrix whose
    upper triangle is the stored one, and NaN stored below the diagonal never
    reaches the result (so the lower triangle is not read)."""
    for n, seed in ((1, 20), (2, 21), (7, 22), (33, 23)):
        A = inputs.gaussian_integer_matrix(n, seed, bound=512)
        S = np.triu(A) + np.triu(A, 1).T
        x = inputs.gaussian_integer_vector(n, seed + 100, bound=512)
        want = exact_matvec_int(S, x)
        stored = A.copy()
        stored[np.tril_indices(n, -1)] = complex(np.nan, np.nan)
        assert np.array_equal(orc.matvec_sym_upper(stored, x), want), n


def pin_sym_upper_is_full_product_on_symmetric(orc):
    """On a matrix symmetric in full, the upper-triangle product makes the
    same sums in the same order as the dense product: equal bit for bit."""
    n = 41
    rng = np.random.default_rng(24)
    B = inputs.cn01(rng, (n, n))
    A = B + B.T
    x = inputs.cn01(rng, n)
    assert np.array_equal(orc.matvec_sym_upper(A, x), orc.matvec(A, x))
    L = inputs.lattice_matrix(3)
    xl = inputs.cn01(rng, L.shape[0])
    assert np.array_equal(orc.matvec_sym_upper(L, xl), orc.matvec(L, xl))


# ------------------------------------------------------------- solver pins

def pin_lu_dense(orc, sizes=(1, 2, 3, 4, 8, 16, 32, 64)):
    """Solutions match a dense LU solve to within the conditioning bound."""
    tol = 1e-10
    for n in sizes:
        A, _, y = inputs.dense_system(n, 40 + n)
        kappa = np.linalg.cond(A)
        x_np = np.linalg.solve(A, y)
        x_lu = lu_solve(A, y)
        assert relerr(x_lu, x_np) <= 1e-12
        for m in SOLVERS:
            r = _solve(orc, m, A, y, tol=tol, maxit=500)
            assert r.info == 0, (m, n, r.info)
            assert r.relres_true <= tol, (m, n)
            assert relerr(r.x, x_lu) <= 10 * kappa * tol, (m, n)


def pin_scaled_identity(orc):
    """A = c I: BiCGSTAB leaves at the half step of iteration 1, CGNR after
    one iteration, both with x = y / c."""
    n = 10
    c = 2.0 - 3.0j
    A = c * np.eye(n, dtype=np.complex128)
    y = inputs.cn01(np.random.default_rng(1), n)
    for m in SOLVERS:
        r = _solve(orc, m, A, y)
        assert r.info == 0 and r.iters == 1, (m, r.info, r.iters)
        assert relerr(r.x, y / c) <= 4 * U
    r = orc.bicgstab(A, y)
    assert np.isnan(r.hist[0, 7]) and r.hist[0, 6] <= 1e-15
    assert r.matvecs == 2  # v = A p, then the confirming residual


def pin_scalar_system(orc):
    """1 x 1: x = y / a after one half step."""
    a = np.array([[0.5 + 1.5j]])
    y = np.array([2.0 - 1.0j])
    for m in SOLVERS:
        r = _solve(orc, m, a, y)
        assert r.info == 0 and r.iters == 1
        assert abs(r.x[0] - y[0] / a[0, 0]) <= 4 * U * abs(y[0] / a[0, 0])


def pin_unitary(orc):
    """Normalised DFT (eigenvalues +-1, +-i): A^H A = I, so CGNR needs one
    iteration; BiCGSTAB at most 4 in exact arithmetic (one of slack)."""
    A = dft_matrix(16)
    y = inputs.cn01(np.random.default_rng(2), 16)
    r = orc.cgnr(A, y)
    assert r.info == 0 and r.iters == 1
    r = orc.bicgstab(A, y)
    assert r.info == 0 and r.iters <= 5
    assert relerr(r.x, A.conj().T @ y) <= 1e-9


def pin_two_values(orc):
    """diag with two distinct values: both methods finish in <= 2 iterations."""
    d = np.array([1.0 + 1j] * 5 + [3.0 - 2j] * 7)
    A = np.diag(d)
    y = inputs.cn01(np.random.default_rng(4), 12)
    for m in SOLVERS:
        r = _solve(orc, m, A, y)
        assert r.info == 0 and r.iters <= 2, (m, r.iters)
        assert relerr(r.x, y / d) <= 1e-9


def pin_finite_termination(orc):
    """HPD with m = 5 distinct eigenvalues: CG, CGNR (A^H A has 5 distinct
    eigenvalues) and BiCGSTAB (its BiCG part is CG here) finish in <= m
    iterations, one of slack for rounding."""
    eigs = np.repeat([1.0, 2.0, 3.5, 5.0, 7.0], [13, 13, 13, 13, 12])
    A = hpd_with_spectrum(64, eigs, 9)
    y = inputs.cn01(np.random.default_rng(10), 64)
    for name in ("cg", "cgnr", "bicgstab"):
        r = getattr(orc, name)(A, y, tol=1e-12)
        assert r.info == 0 and r.iters <= 6, (name, r.iters)
        assert r.relres_true <= 1e-12
    # generic HPD, n = 12, kappa <= 10: CG in <= n (+1)
    A = hpd_with_spectrum(12, np.linspace(1.0, 10.0, 12), 12)
    y = inputs.cn01(np.random.default_rng(13), 12)
    r = orc.cg(A, y, tol=1e-12)
    assert r.info == 0 and r.iters <= 13


def pin_cgnr_is_cg_on_normal_equations(orc):
    """CGNR's alpha_k and beta_k equal those of CG on A^H A x = A^H y."""
    A, _, y = inputs.dense_system(32, 77)
    r1 = orc.cgnr(A, y, tol=1e-13)
    N = A.conj().T @ A
    r2 = orc.cg(0.5 * (N + N.conj().T), A.conj().T @ y, tol=1e-13)
    k = min(r1.iters, r2.iters, 8)
    assert k >= 5
    a1, a2 = r1.hist[:k, 0], r2.hist[:k, 0]
    b1, b2 = r1.hist[:k - 1, 4], r2.hist[:k - 1, 4]
    assert np.allclose(a1, a2, rtol=1e-8, atol=0)
    assert np.allclose(b1, b2, rtol=1e-8, atol=0)


def pin_bicgstab_alpha_is_cg_alpha(orc):
    """A HPD, r^ = r0: BiCGSTAB's alpha_k equals CG's alpha_k."""
    A = hpd_with_spectrum(40, np.linspace(1.0, 8.0, 40), 21)
    y = inputs.cn01(np.random.default_rng(22), 40)
    rb = orc.bicgstab(A, y, tol=1e-12)
    rc = orc.cg(A, y, tol=1e-12)
    k = min(rb.iters, 6)
    assert k >= 4
    ab = rb.alpha()[:k]
    ac = rc.hist[:k, 0]
    assert np.allclose(ab.real, ac, rtol=1e-7, atol=0)
    assert np.all(np.abs(ab.imag) <= 1e-7 * np.abs(ac))


def pin_omega_minimises(orc):
    """omega minimises ||s - omega t||, so ||r_k|| <= ||s_k|| every iteration;
    the lattice and dense families give complex, non-Hermitian iterates."""
    for A, y in ((inputs.dense_system(96, 5)[0], inputs.dense_system(96, 5)[2]),
                 (inputs.lattice_matrix(4) + 0.0, None)):
        if y is None:
            y = inputs.cn01(np.random.default_rng(8), A.shape[0])
            A = A - 140.0 * np.eye(A.shape[0])  # slower convergence
        r = orc.bicgstab(np.ascontiguousarray(A), y, tol=1e-13)
        h = r.hist[:r.iters]
        full = ~np.isnan(h[:, 7])
        assert full.sum() >= 3
        assert np.all(h[full, 7] <= h[full, 6] * (1 + 1e-12))


def pin_cgnr_monotone(orc):
    """CGNR minimises ||y - A x|| over a growing space: ||r_k|| never grows."""
    A, _, y = inputs.dense_system(80, 6)
    r = orc.cgnr(A, y, tol=1e-12)
    res = r.hist[:r.iters, 7]
    assert r.iters >= 10
    assert np.all(np.diff(res) <= 1e-13 * res[:-1])


def pin_exact_first_iterations(orc):
    """First iterations in exact Gaussian-rational arithmetic on a 3 x 3
    integer system (alpha, omega, beta are rational in the data)."""
    Ai = np.array([[7 + 1j, 2 - 1j, 0 + 1j],
                   [1 + 2j, 6 - 2j, 1 + 0j],
                   [0 - 1j, 3 + 1j, 8 + 3j]])
    yi = np.array([1 + 2j, -3 + 1j, 2 - 2j])
    A = [[Q.of(Ai[i, j]) for j in range(3)] for i in range(3)]
    y = [Q.of(v) for v in yi]
    # BiCGSTAB, x0 = 0: r = r^ = y
    r = list(y)
    rh = list(y)
    p = list(r)
    v = [Q(0)] * 3
    rho_old = alpha = omega = None
    want = []
    for k in range(2):
        rho = qdot(rh, r)
        if k > 0:
            beta = (rho / rho_old) * (alpha / omega)
            p = [r[i] + beta * (p[i] - omega * v[i]) for i in range(3)]
        else:
            beta = None
        v = qmatvec(A, p)
        alpha = rho / qdot(rh, v)
        s = [r[i] - alpha * v[i] for i in range(3)]
        t = qmatvec(A, s)
        tt = qdot(t, t)
        omega = qdot(t, s) / tt
        r = [s[i] - omega * t[i] for i in range(3)]
        rho_old = rho
        want.append((alpha.c(), omega.c(), None if beta is None else beta.c()))
    res = orc.bicgstab(Ai.astype(np.complex128), yi.astype(np.complex128),
                       tol=1e-14, maxit=2)
    for k, (a, w, b) in enumerate(want):
        assert abs(res.alpha()[k] - a) <= 1e-13 * abs(a)
        assert abs(res.omega()[k] - w) <= 1e-13 * abs(w)
        if b is not None:
            assert abs(res.beta()[k] - b) <= 1e-13 * abs(b)
    # CGNR, x0 = 0: r = y, z = A^H r, p = z
    AH = [[A[j][i].conj() for j in range(3)] for i in range(3)]
    r = list(y)
    z = qmatvec(AH, r)
    p = list(z)
    g = qdot(z, z).re
    want = []
    for k in range(2):
        w = qmatvec(A, p)
        alpha = g / qdot(w, w).re
        r = [r[i] - Q(alpha) * w[i] for i in range(3)]
        z = qmatvec(AH, r)
        gn = qdot(z, z).re
        beta = gn / g
        p = [z[i] + Q(beta) * p[i] for i in range(3)]
        g = gn
        want.append((float(alpha), float(beta)))
    res = orc.cgnr(Ai.astype(np.complex128), yi.astype(np.complex128),
                   tol=1e-14, maxit=2)
    for k, (a, b) in enumerate(want):
        assert abs(res.hist[k, 0] - a) <= 1e-13 * abs(a)
        assert abs(res.hist[k, 4] - b) <= 1e-13 * abs(b)


def find_omega_zero_case():
    """Search, in exact arithmetic, for a diagonal integer A and integer y with
    s = y - alpha A y != 0 but s^H A s = 0 (so t^H s = 0 and omega = 0)."""
    vals = range(-3, 4)
    for a in vals:
        for b in vals:
            for c in vals:
                if 0 in (a, b, c):
                    continue
                for y in ((1, 1, 1), (1, 2, 1), (2, 1, 1), (1, 1, 2)):
                    yq = [Fraction(v) for v in y]
                    d = [Fraction(a), Fraction(b), Fraction(c)]
                    yy = sum(v * v for v in yq)
                    yay = sum(di * v * v for di, v in zip(d, yq))
                    if yay == 0:
                        continue
                    al = yy / yay
                    s = [v - al * di * v for di, v in zip(d, yq)]
                    if all(v == 0 for v in s):
                        continue
                    if sum(di * v * v for di, v in zip(d, s)) == 0:
                        return np.diag([a, b, c]).astype(np.complex128), \
                            np.array(y, dtype=np.complex128)
    raise AssertionError("no omega = 0 case in the search range")


def pin_breakdowns(orc):
    """sigma = 0 exactly (rotation), omega = 0 exactly (constructed case),
    non-finite input, budget exhaustion."""
    A = np.array([[0, 1], [-1, 0]], dtype=np.complex128)
    y = np.array([1, 0], dtype=np.complex128)
    r = orc.bicgstab(A, y)
    assert r.info == 2 and r.iters == 0 and np.all(r.x == 0)
    r = orc.cgnr(A, y)  # A orthogonal: one CGNR iteration solves it
    assert r.info == 0 and r.iters == 1
    assert np.allclose(r.x, A.T @ y, atol=1e-15)
    A3, y3 = find_omega_zero_case()
    r = orc.bicgstab(A3, y3)
    assert r.info == 3 and r.iters == 0
    A, _, y = inputs.dense_system(32, 3)
    ybad = y.copy()
    ybad[5] = np.nan
    x0 = np.ones(32, dtype=np.complex128)
    for m in SOLVERS:
        r = _solve(orc, m, A, ybad, x0=x0)
        assert r.info == 4 and np.array_equal(r.x, x0)
        Abad = A.copy()
        Abad[3, 4] = np.inf
        r = _solve(orc, m, Abad, y)
        assert r.info == 4
        r = _solve(orc, m, A, y, maxit=1)
        assert r.info == 1 and r.iters == 1
        r = _solve(orc, m, A, y, maxit=0)
        assert r.info == 1 and r.iters == 0


def pin_trivial_cases(orc):
    """y = 0 gives x = 0 with no work; n = 0 is a no-op."""
    A, _, _ = inputs.dense_system(8, 1)
    x0 = np.ones(8, dtype=np.complex128)
    for m in SOLVERS:
        r = _solve(orc, m, A, np.zeros(8, dtype=np.complex128), x0=x0)
        assert r.info == 0 and r.iters == 0 and r.matvecs == 0
        assert np.all(r.x == 0)
        r = _solve(orc, m, np.zeros((0, 0), dtype=np.complex128),
                   np.zeros(0, dtype=np.complex128))
        assert r.info == 0 and r.iters == 0


def pin_warm_start_and_scale(orc):
    """A warm start near the solution converges in fewer iterations; scaling
    A and y by the same c leaves x unchanged up to rounding."""
    A, xt, y = inputs.dense_system(64, 9)
    for m in SOLVERS:
        cold = _solve(orc, m, A, y)
        warm = _solve(orc, m, A, y, x0=xt + 1e-6)
        assert warm.info == 0 and warm.iters < cold.iters
        c = 0.3 - 1.7j
        sc = _solve(orc, m, c * A, c * y)
        assert sc.info == 0
        assert relerr(sc.x, cold.x) <= 1e-9


def pin_scipy_crosscheck(orc):
    """SciPy's BiCGSTAB reaches the same solution within the tolerance."""
    from scipy.sparse.linalg import bicgstab as sp_bicgstab
    for A, y in ((inputs.dense_system(256, 0)[0], inputs.dense_system(256, 0)[2]),
                 (inputs.lattice_matrix(5), None)):
        if y is None:
            y = inputs.cn01(np.random.default_rng(1), A.shape[0])
        xs, code = sp_bicgstab(A, y, rtol=1e-12, atol=0.0, maxiter=1000)
        assert code == 0
        for m in SOLVERS:
            r = _solve(orc, m, A, y)
            kappa = np.linalg.cond(A)
            assert r.info == 0
            assert relerr(r.x, xs) <= 10 * kappa * 1e-10


def pin_restart(orc):
    """A tolerance below round-off: the recursive residual keeps falling while
    the true one stalls, so confirmations fail, the true residual replaces r,
    and the budget ends the solve (info 1) with the true residual at the
    rounding floor."""
    A, _, y = inputs.dense_system(48, 2)
    for m in SOLVERS:
        r = _solve(orc, m, A, y, tol=1e-18, maxit=120)
        assert r.info == 1 and r.confirms >= 2, (m, r.info, r.confirms)
        assert r.relres_true <= 1e-14


# ------------------------------------------- complex symmetric: COCG / COCR

CS = ("cocg", "cocr")


def real_spd(n, eigs, seed):
    rng = np.random.default_rng(seed)
    Qm, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = (Qm * np.asarray(eigs, dtype=np.float64)) @ Qm.T
    return np.ascontiguousarray(0.5 * (A + A.T)).astype(np.complex128)


def complex_symmetric_with_spectrum(n, eigs, seed):
    """Q diag(eigs) Q^T with Q real orthogonal: complex symmetric, spectrum
    eigs (the bilinear form is preserved by Q, so COCG / COCR see a diagonal
    system)."""
    rng = np.random.default_rng(seed)
    Qm, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = (Qm * np.asarray(eigs)) @ Qm.T
    return np.ascontiguousarray(0.5 * (A + A.T))


def pin_cocg_is_cg_on_real_spd(orc):
    """Real symmetric positive definite A and real y: the bilinear form is the
    inner product, so COCG's alpha_k and beta_k are CG's."""
    A = real_spd(40, np.linspace(1.0, 9.0, 40), 31)
    y = np.random.default_rng(32).standard_normal(40).astype(np.complex128)
    r1 = orc.cocg(A, y, tol=1e-12)
    r2 = orc.cg(A, y, tol=1e-12)
    k = min(r1.iters, r2.iters, 8)
    assert k >= 6
    assert np.allclose(r1.hist[:k, 0], r2.hist[:k, 0], rtol=1e-9, atol=0)
    assert np.all(np.abs(r1.hist[:k, 1]) <= 1e-12 * np.abs(r1.hist[:k, 0]))
    assert np.allclose(r1.hist[:k - 1, 4], r2.hist[:k - 1, 4], rtol=1e-8, atol=0)


def krylov_min_residual(A, y, k):
    """min ||y - A x|| over x in K_k(A, y), by least squares on an
    orthonormal Krylov basis (brute force, for small k)."""
    n = A.shape[0]
    K = np.empty((n, k), dtype=np.complex128)
    v = y / np.linalg.norm(y)
    for j in range(k):
        K[:, j] = v
        v = A @ v
        v = v / np.linalg.norm(v)
    Qk, _ = np.linalg.qr(K)
    AQ = A @ Qk
    c, *_ = np.linalg.lstsq(AQ, y, rcond=None)
    return np.linalg.norm(y - AQ @ c)


def pin_cocr_is_minimal_residual_on_real_spd(orc):
    """Real SPD A, real y: COCR is CR, which minimises ||y - A x|| over the
    Krylov space K_k(A, y) -- the same residual norms as a brute-force least
    squares over that space."""
    A = real_spd(30, np.linspace(1.0, 6.0, 30), 41)
    y = np.random.default_rng(42).standard_normal(30).astype(np.complex128)
    r = orc.cocr(A, y, tol=1e-13)
    ny = np.linalg.norm(y)
    for k in range(1, 6):
        want = krylov_min_residual(A, y, k) / ny
        assert abs(r.hist[k - 1, 7] - want) <= 1e-7 * want, (k, r.hist[k - 1, 7], want)


def pin_cs_finite_termination(orc):
    """Complex symmetric A with 5 distinct eigenvalues: both methods reach
    1e-12 in at most 5 iterations (one of slack)."""
    eigs = np.repeat([2 + 1j, 3 - 0.5j, 4 + 2j, 6 + 0.2j, 7 - 1j], [10, 10, 10, 10, 8])
    A = complex_symmetric_with_spectrum(48, eigs, 43)
    y = inputs.cn01(np.random.default_rng(44), 48)
    for m in CS:
        r = getattr(orc, m)(A, y, tol=1e-12)
        assert r.info == 0 and r.iters <= 6, (m, r.info, r.iters)
        assert r.relres_true <= 1e-12


def pin_cs_lu(orc):
    """Complex symmetric systems against a dense LU solve: lattice matrices
    and a random diagonally shifted G + G^T."""
    rng = np.random.default_rng(45)
    G = inputs.cn01(rng, (40, 40))
    S = (G + G.T) / np.sqrt(80) + (5 + 1j) * np.eye(40)
    for A in (inputs.lattice_matrix(4), inputs.lattice_matrix(5), S):
        y = inputs.cn01(rng, A.shape[0])
        x_lu = lu_solve(A, y)
        kappa = np.linalg.cond(A)
        for m in CS:
            r = getattr(orc, m)(np.ascontiguousarray(A), y)
            assert r.info == 0 and r.relres_true <= 1e-10, m
            assert relerr(r.x, x_lu) <= 10 * kappa * 1e-10, m


def pin_cs_closed_forms(orc):
    """A = c I: one iteration, x = y / c.  y = (1, i) with A = I: (r, r) = 0
    and (r, A r) = 0 -- the bilinear form breaks down at once (info 2)."""
    c = 1.5 + 2.5j
    A = c * np.eye(9, dtype=np.complex128)
    y = inputs.cn01(np.random.default_rng(46), 9)
    for m in CS:
        r = getattr(orc, m)(A, y)
        assert r.info == 0 and r.iters == 1
        assert relerr(r.x, y / c) <= 16 * U
    I2 = np.eye(2, dtype=np.complex128)
    y = np.array([1.0, 1.0j])
    for m in CS:
        r = getattr(orc, m)(I2, y)
        assert r.info == 2 and r.iters == 0 and np.all(r.x == 0), m


def pin_cs_exact_first_iterations(orc):
    """First two iterations of both methods in exact Gaussian-rational
    arithmetic on a 3 x 3 complex symmetric integer system."""
    Ai = np.array([[6 + 1j, 1 - 2j, 2 + 0j],
                   [1 - 2j, 5 + 2j, -1 + 1j],
                   [2 + 0j, -1 + 1j, 7 - 1j]])
    yi = np.array([2 - 1j, 1 + 3j, -1 + 1j])
    A = [[Q.of(Ai[i, j]) for j in range(3)] for i in range(3)]
    y = [Q.of(v) for v in yi]

    def dotu_q(a, b):
        return sum((u * v for u, v in zip(a, b)), Q(0))

    # COCG
    r = list(y)
    p = list(r)
    rho = dotu_q(r, r)
    want = []
    for _ in range(2):
        q = qmatvec(A, p)
        alpha = rho / dotu_q(p, q)
        r = [r[i] - alpha * q[i] for i in range(3)]
        rho_new = dotu_q(r, r)
        beta = rho_new / rho
        p = [r[i] + beta * p[i] for i in range(3)]
        rho = rho_new
        want.append((alpha.c(), beta.c()))
    res = orc.cocg(Ai.astype(np.complex128), yi.astype(np.complex128), tol=1e-14, maxit=2)
    for k, (a, b) in enumerate(want):
        assert abs(res.hist[k, 0] + 1j * res.hist[k, 1] - a) <= 1e-13 * abs(a)
        if k == 0:
            assert abs(res.hist[k, 4] + 1j * res.hist[k, 5] - b) <= 1e-13 * abs(b)
    # COCR
    r = list(y)
    u = qmatvec(A, r)
    p, w = list(r), list(u)
    rho = dotu_q(r, u)
    want = []
    for _ in range(2):
        alpha = rho / dotu_q(w, w)
        r = [r[i] - alpha * w[i] for i in range(3)]
        u = qmatvec(A, r)
        rho_new = dotu_q(r, u)
        beta = rho_new / rho
        p = [r[i] + beta * p[i] for i in range(3)]
        w = [u[i] + beta * w[i] for i in range(3)]
        rho = rho_new
        want.append((alpha.c(), beta.c()))
    res = orc.cocr(Ai.astype(np.complex128), yi.astype(np.complex128), tol=1e-14, maxit=2)
    for k, (a, b) in enumerate(want):
        assert abs(res.hist[k, 0] + 1j * res.hist[k, 1] - a) <= 1e-13 * abs(a)
        if k == 0:
            assert abs(res.hist[k, 4] + 1j * res.hist[k, 5] - b) <= 1e-13 * abs(b)


def pin_cs_failures(orc):
    """Non-finite input, iteration budget, zero right-hand side."""
    A = inputs.lattice_matrix(3)
    y = inputs.cn01(np.random.default_rng(47), 27)
    for m in CS:
        ybad = y.copy()
        ybad[3] = np.inf
        assert getattr(orc, m)(A, ybad).info == 4
        r = getattr(orc, m)(A, y, maxit=1)
        assert r.info == 1 and r.iters == 1
        r = getattr(orc, m)(A, np.zeros(27, dtype=np.complex128), x0=y)
        assert r.info == 0 and np.all(r.x == 0) and r.matvecs == 0


# ------------------------------------------------------------ mixed precision

def pin_mixed_matvec_c64_integer_exact(orc):
    """complex64 product on small Gaussian integers: every partial sum is an
    integer below 2^24, so the FP32 sums are exact."""
    for n, seed in ((1, 0), (9, 1), (32, 2)):
        A = inputs.gaussian_integer_matrix(n, seed, bound=16)
        x = inputs.gaussian_integer_vector(n, seed + 7, bound=16)
        want = exact_matvec_int(A, x)
        got = orc.matvec_c64(A.astype(np.complex64), x.astype(np.complex64))
        assert np.array_equal(got.astype(np.complex128), want), n


def pin_mixed_solution(orc):
    """FP64 refinement reaches the FP64 tolerance: true residual <= 1e-10 and
    the LU solution within the conditioning bound."""
    systems = [inputs.lattice_matrix(5), inputs.lattice_matrix(6),
               inputs.dense_matrix(64, 12)]
    rng = np.random.default_rng(48)
    for A in systems:
        y = inputs.cn01(rng, A.shape[0])
        r = orc.bicgstab_mixed(A, y)
        assert r.info == 0 and r.relres_true <= 1e-10 and r.outer <= 4
        kappa = np.linalg.cond(A)
        assert relerr(r.x, lu_solve(A, y)) <= 10 * kappa * 1e-10


def pin_mixed_refinement_contracts(orc):
    """Each refinement step multiplies the FP64 residual by about the inner
    tolerance (plus kappa times the complex64 rounding of A): at most 1e-4
    for tol_inner = 1e-5 and 1e-2 for 1e-3 on these well-conditioned
    systems."""
    A = inputs.lattice_matrix(6)
    y = inputs.cn01(np.random.default_rng(49), A.shape[0])
    for tin, bound in ((1e-5, 1e-4), (1e-3, 1e-2)):
        r = orc.bicgstab_mixed(A, y, tol=1e-12, tol_inner=tin)
        res = r.outer_res[:r.outer + 1]
        assert r.info == 0 and len(res) >= 2
        assert np.all(res[1:] <= bound * res[:-1]), res


def pin_mixed_exact_float_system(orc):
    """A and y exactly representable in complex64 (small integers): the first
    step solves the very system A x = y in complex64, so the FP64 residual
    after it is the inner tolerance up to complex64 rounding."""
    A = inputs.gaussian_integer_matrix(24, 5, bound=4) + 40 * np.eye(24)
    y = inputs.gaussian_integer_vector(24, 6, bound=8)
    assert np.array_equal(A.astype(np.complex64).astype(np.complex128), A)
    for tin in (1e-3, 1e-5):
        r = orc.bicgstab_mixed(A, y, tol=1e-12, tol_inner=tin)
        assert r.outer_res[1] <= 1.5 * tin, (tin, r.outer_res[:3])


def pin_mixed_trivial(orc):
    A = inputs.lattice_matrix(3)
    y = inputs.cn01(np.random.default_rng(50), 27)
    x0 = np.full(27, 1.0 + 1.0j)
    ybad = y.copy()
    ybad[4] = np.nan
    r = orc.bicgstab_mixed(A, ybad, x0=x0)
    assert r.info == 4 and np.array_equal(r.x, x0)
    r = orc.bicgstab_mixed(A, np.zeros(27, dtype=np.complex128), x0=x0)
    assert r.info == 0 and np.all(r.x == 0) and r.outer == 0
    r = orc.bicgstab_mixed(A, y, maxit=0)
    assert r.info == 1 and r.outer == 0 and r.relres_true == 1.0


def pin_mixed_inner_breakdown_ends_refinement(orc):
    """Both refinement forms: an inner breakdown before the first inner update
    leaves d = 0, so the refinement ends with that inner info instead of
    repeating the same step until its budget.  The rotation A = [[0, 1],
    [-1, 0]] with y = e1 gives sigma = r^H A r = 0 exactly at the first inner
    iteration (info 2, x = 0); from x0 = (1/2, 1/2) the residual is (1, 1)/2
    and sigma is again exactly zero (x left at x0)."""
    A = np.array([[0, 1], [-1, 0]], dtype=np.complex128)
    y = np.array([1, 0], dtype=np.complex128)
    x0 = np.array([0.5, 0.5], dtype=np.complex128)
    for fn in (orc.bicgstab_mixed, orc.bicgstab_mixed_wide):
        r = fn(A, y, maxit=10)
        assert (r.info, r.outer, r.inner_iters) == (2, 1, 0) and np.all(r.x == 0)
        r = fn(A, y, x0=x0, maxit=10)
        assert (r.info, r.outer, r.inner_iters) == (2, 1, 0) and np.array_equal(r.x, x0)


def pin_mixed_scaled_identity(orc):
    """A = c I with c exact in complex64, both refinement forms: every inner
    solve leaves at the half step of its first iteration (the complex64
    product is c times the input up to FP32 rounding), so each refinement step
    gains a factor of about 2^-24: two steps reach 1e-10, with two complex64
    and two FP64 products, and x = y / c to FP64 rounding."""
    c = 2.0 - 3.0j
    A = c * np.eye(40, dtype=np.complex128)
    y = inputs.cn01(np.random.default_rng(51), 40)
    for fn in (orc.bicgstab_mixed, orc.bicgstab_mixed_wide):
        r = fn(A, y)
        assert r.info == 0 and (r.outer, r.inner_iters, r.matvecs32, r.matvecs64) == \
            (2, 2, 2, 2), (r.outer, r.inner_iters, r.matvecs32, r.matvecs64)
        assert r.outer_res[1] <= 1e-6 and r.relres_true <= 1e-13
        assert relerr(r.x, y / c) <= 1e-13


# -------------------------------- mixed precision, complex128 inner vectors

def pin_mixed_wide_matvec_integer_exact(orc):
    """The complex64 product of a complex128 vector on small Gaussian
    integers: the vector rounds to itself, every FP32 partial sum is an
    integer below 2^24, so the widened result equals the exact integer
    product (a non-symmetric A also fixes the orientation)."""
    for n, seed in ((1, 0), (9, 1), (40, 2)):
        A = inputs.gaussian_integer_matrix(n, seed, bound=16)
        x = inputs.gaussian_integer_vector(n, seed + 7, bound=16)
        want = exact_matvec_int(A, x)
        got = orc.matvec_c64_wide(A.astype(np.complex64), x)
        assert got.dtype == np.complex128 and np.array_equal(got, want), n


def pin_mixed_wide_solution(orc):
    """The complex128-vector refinement reaches the FP64 tolerance: true
    residual <= 1e-10 and the LU solution within the conditioning bound."""
    systems = [inputs.lattice_matrix(5), inputs.lattice_matrix(6),
               inputs.dense_matrix(64, 12), inputs.dense_matrix(3, 2)]
    rng = np.random.default_rng(52)
    for A in systems:
        y = inputs.cn01(rng, A.shape[0])
        r = orc.bicgstab_mixed_wide(A, y)
        assert r.info == 0 and r.relres_true <= 1e-10 and r.outer <= 4
        kappa = np.linalg.cond(A)
        assert relerr(r.x, lu_solve(A, y)) <= 10 * kappa * 1e-10


def pin_mixed_wide_refinement_contracts(orc):
    """Each refinement step multiplies the FP64 residual by about the inner
    tolerance (plus kappa times the complex64 rounding of A and of the
    product's input)."""
    A = inputs.lattice_matrix(6)
    y = inputs.cn01(np.random.default_rng(53), A.shape[0])
    for tin, bound in ((1e-5, 1e-4), (1e-3, 1e-2)):
        r = orc.bicgstab_mixed_wide(A, y, tol=1e-12, tol_inner=tin)
        res = r.outer_res[:r.outer + 1]
        assert r.info == 0 and len(res) >= 2
        assert np.all(res[1:] <= bound * res[:-1]), res


def pin_mixed_wide_trivial(orc):
    """Non-finite y: info 4 with x as given; y = 0: x = 0 with no step;
    maxit = 0: info 1 after the first check."""
    A = inputs.lattice_matrix(3)
    y = inputs.cn01(np.random.default_rng(54), 27)
    x0 = np.full(27, 1.0 + 1.0j)
    ybad = y.copy()
    ybad[4] = np.nan
    r = orc.bicgstab_mixed_wide(A, ybad, x0=x0)
    assert r.info == 4 and np.array_equal(r.x, x0)
    r = orc.bicgstab_mixed_wide(A, np.zeros(27, dtype=np.complex128), x0=x0)
    assert r.info == 0 and np.all(r.x == 0) and r.outer == 0
    r = orc.bicgstab_mixed_wide(A, y, maxit=0)
    assert r.info == 1 and r.outer == 0 and r.relres_true == 1.0


ALL_PINS = [v for k, v in sorted(globals().items()) if k.startswith("pin_")]
