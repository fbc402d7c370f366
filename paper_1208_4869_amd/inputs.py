"""Seeded synthetic inputs for the complex Krylov solvers.

This module only builds inputs (matrices, solutions, right-hand sides) and
certificates about them.  It holds none of the solvers' arithmetic, and it is
the one module that both the CPU oracle's tests and the GPU path's tests use.

The paper runs no experiment, so every workload is synthetic (section 4 says
the codes are not extensively tested; there are no tables or figures).  Two
matrix families stand in for its use case, the discrete-dipole systems of
DDSCAT named in the Introduction:

* the *dense* family, ``A = 4 I + G / sqrt(n)`` with ``G`` iid CN(0, 1);
* the *dipole-lattice* family on an ``m x m x m`` cubic lattice:
  ``A_ij = exp(i k r_ij - r_ij / L) / r_ij`` off the diagonal, with ``r_ij``
  the distance in lattice spacings, and ``A_ii = 150 + 10 i``.  It is complex
  symmetric (``A = A^T``) and three-level Toeplitz.

CN(0, 1) means real and imaginary parts independent N(0, 1/2), so that
E|z|^2 = 1.  Draw order from ``numpy.random.default_rng(seed)``: the whole real
block, then the whole imaginary block.
"""
from __future__ import annotations

import numpy as np


def cn01(rng: np.random.Generator, shape) -> np.ndarray:
    """iid CN(0, 1) samples: real block first, then imaginary block."""
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return (re + 1j * im) * np.sqrt(0.5)


# ----------------------------------------------------------------- dense family

def dense_matrix(n: int, seed: int) -> np.ndarray:
    """``A = 4 I + G / sqrt(n)``, G iid CN(0,1) drawn from ``seed``."""
    rng = np.random.default_rng(seed)
    A = cn01(rng, (n, n)) / np.sqrt(n)
    A[np.arange(n), np.arange(n)] += 4.0
    return A


def dense_system(n: int, seed: int):
    """(A, x_true, y) of the dense family; x_true drawn after G, same stream."""
    rng = np.random.default_rng(seed)
    A = cn01(rng, (n, n)) / np.sqrt(n)
    A[np.arange(n), np.arange(n)] += 4.0
    x_true = cn01(rng, n)
    y = A @ x_true
    return A, x_true, y


# --------------------------------------------------------------- lattice family

LATTICE_K = 0.5
LATTICE_L = 3.0
LATTICE_DIAG = 150.0 + 10.0j


def lattice_table(m: int, k: float = LATTICE_K, L: float = LATTICE_L,
                  diag: complex = LATTICE_DIAG) -> np.ndarray:
    """Values of A_ij for every displacement (dx, dy, dz) in (-(m-1)..m-1)^3.

    Flat index of a displacement: ((dz + m-1) * (2m-1) + (dy + m-1)) * (2m-1)
    + (dx + m-1).  The zero displacement holds the diagonal value.
    """
    w = 2 * m - 1
    d = np.arange(-(m - 1), m, dtype=np.float64)
    dz, dy, dx = np.meshgrid(d, d, d, indexing="ij")
    r = np.sqrt(dx * dx + dy * dy + dz * dz).reshape(-1)
    T = np.empty(w * w * w, dtype=np.complex128)
    nz = r > 0
    rn = r[nz]
    T[nz] = np.exp(-rn / L) / rn * (np.cos(k * rn) + 1j * np.sin(k * rn))
    T[~nz] = diag
    return T


def lattice_offsets(m: int) -> np.ndarray:
    """Per lattice point i = ix + m*iy + m*m*iz (x fastest): its offset in the
    displacement table, so that A_ij = T[center + off_i - off_j]."""
    w = 2 * m - 1
    i = np.arange(m * m * m, dtype=np.int64)
    ix, iy, iz = i % m, (i // m) % m, i // (m * m)
    return (iz * w + iy) * w + ix


def lattice_center(m: int) -> int:
    w = 2 * m - 1
    return ((m - 1) * w + (m - 1)) * w + (m - 1)


def lattice_matrix(m: int, rows: slice | None = None, **kw) -> np.ndarray:
    """Dense lattice matrix (or a block of its rows) as complex128, row-major."""
    T = lattice_table(m, **kw)
    off = lattice_offsets(m)
    c = lattice_center(m)
    n = m ** 3
    rows = rows or slice(0, n)
    r0, r1 = rows.start or 0, rows.stop if rows.stop is not None else n
    A = np.empty((r1 - r0, n), dtype=np.complex128)
    step = max(1, (1 << 22) // n)
    for a in range(r0, r1, step):
        b = min(r1, a + step)
        A[a - r0:b - r0] = T[c + off[a:b, None] - off[None, :]]
    return A


def lattice_matrix_torch(m: int, device, dtype=None, **kw):
    """The same lattice matrix, gathered on ``device`` from the host table.

    The table is computed on the host in float64 and the gather only copies
    its values, so the result is bitwise equal to ``lattice_matrix(m)``.
    """
    import torch
    dtype = dtype or torch.complex128
    T = torch.from_numpy(lattice_table(m, **kw)).to(device)
    off = torch.from_numpy(lattice_offsets(m)).to(device)
    c = lattice_center(m)
    n = m ** 3
    A = torch.empty((n, n), dtype=torch.complex128, device=device)
    step = max(1, (1 << 25) // n)
    for a in range(0, n, step):
        b = min(n, a + step)
        A[a:b] = T[c + off[a:b, None] - off[None, :]]
    if dtype != torch.complex128:
        A = A.to(dtype)
    return A


def lattice_system(m: int, seed: int, nrhs: int | None = None):
    """(A, x_true, y) of the lattice family; x_true iid CN(0,1) from ``seed``.
    With ``nrhs`` the solution and right-hand side are n x nrhs, row-major."""
    A = lattice_matrix(m)
    rng = np.random.default_rng(seed)
    n = m ** 3
    x_true = cn01(rng, n if nrhs is None else (n, nrhs))
    y = A @ x_true
    return A, x_true, y


# ------------------------------------------------------------- certificates

def gershgorin_margin(A: np.ndarray) -> float:
    """min_i |A_ii| - sum_{j != i} |A_ij|.  Positive proves A nonsingular."""
    absA = np.abs(A)
    d = np.diagonal(absA).copy()
    radius = absA.sum(axis=1) - d
    return float(np.min(d - radius))


def lattice_gershgorin_bound(m: int, **kw) -> float:
    """Lower bound of the Gershgorin margin of the m^3 lattice matrix without
    forming it: every row's off-diagonal sum is a sub-sum of the table over all
    nonzero displacements, so |A_ii| minus that total bounds every row."""
    T = lattice_table(m, **kw)
    c = lattice_center(m)
    return float(abs(T[c]) - (np.abs(T).sum() - abs(T[c])))


def sigma_extremes(A: np.ndarray):
    """(sigma_min, sigma_max) from a host LAPACK SVD.  sigma_min > 0 proves A
    nonsingular where the Gershgorin discs do not."""
    s = np.linalg.svd(A, compute_uv=False)
    return float(s[-1]), float(s[0])


# ------------------------------------------------------------ integer inputs

def gaussian_integer_matrix(n: int, seed: int, bound: int = 8) -> np.ndarray:
    """Complex matrix with integer parts in [-bound, bound]."""
    rng = np.random.default_rng(seed)
    re = rng.integers(-bound, bound + 1, size=(n, n))
    im = rng.integers(-bound, bound + 1, size=(n, n))
    return (re + 1j * im).astype(np.complex128)


def gaussian_integer_vector(n: int, seed: int, bound: int = 8) -> np.ndarray:
    rng = np.random.default_rng(seed)
    re = rng.integers(-bound, bound + 1, size=n)
    im = rng.integers(-bound, bound + 1, size=n)
    return (re + 1j * im).astype(np.complex128)
