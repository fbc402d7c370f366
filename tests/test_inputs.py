"""Properties of the seeded input generators and the nonsingularity
certificates of every matrix family the tests and the benchmark use."""
import numpy as np

from paper_1208_4869_amd import inputs


def test_cn01_moments():
    z = inputs.cn01(np.random.default_rng(0), 200000)
    assert abs(np.mean(np.abs(z) ** 2) - 1.0) < 0.01
    assert abs(np.var(z.real) - 0.5) < 0.01 and abs(np.var(z.imag) - 0.5) < 0.01


def test_dense_family_reproducible_and_shaped():
    A1, x1, y1 = inputs.dense_system(32, 5)
    A2, x2, y2 = inputs.dense_system(32, 5)
    assert np.array_equal(A1, A2) and np.array_equal(y1, y2)
    assert np.array_equal(A1, inputs.dense_matrix(32, 5))
    G = (A1 - 4 * np.eye(32)) * np.sqrt(32)
    assert abs(np.mean(np.abs(G) ** 2) - 1.0) < 0.15


def test_dense_family_certificate():
    """Gershgorin fails for A = 4 I + G / sqrt(n) at n = 256 (the disc radius
    grows like sqrt(n)); sigma_min from an SVD certifies nonsingularity."""
    for seed in range(10):
        A = inputs.dense_matrix(256, seed)
        assert inputs.gershgorin_margin(A) < 0
        smin, smax = inputs.sigma_extremes(A)
        assert 2.0 < smin and smax < 6.5


def test_dense_family_certificate_at_the_serving_sizes():
    """The serving mix draws the same family at n in {512, 1024, 2048, 4096},
    where Gershgorin fails too: sigma_min from an SVD certifies a sample of
    seeds at every size (2.6-2.7, far from zero; sigma_max about 5.5)."""
    for n, seeds in ((512, (0, 1)), (1024, (0, 1)), (2048, (0,)), (4096, (0,))):
        for seed in seeds:
            A = inputs.dense_matrix(n, 3000 + n + seed)
            assert inputs.gershgorin_margin(A) < 0
            smin, smax = inputs.sigma_extremes(A)
            assert 2.0 < smin and smax < 6.5, (n, seed, smin, smax)


def test_lattice_structure():
    m = 5
    A = inputs.lattice_matrix(m)
    n = m ** 3
    assert A.shape == (n, n)
    assert np.array_equal(A, A.T)                     # complex symmetric
    assert np.all(np.diagonal(A) == inputs.LATTICE_DIAG)
    # nearest neighbour along x: i = 0, j = 1 (x fastest), r = 1
    want = np.exp(-1 / 3.0) * (np.cos(0.5) + 1j * np.sin(0.5))
    assert abs(A[0, 1] - want) <= 1e-15
    # point (1,1,1) vs (0,0,0): r = sqrt(3)
    j = 1 + m + m * m
    r = np.sqrt(3.0)
    assert abs(A[0, j] - np.exp(-r / 3) / r * np.exp(0.5j * r)) <= 1e-15
    # three-level Toeplitz: the entry depends only on the displacement
    i2, j2 = 1 + 2 * m, 2 + 3 * m + m * m  # displacement (1, 1, 1)
    assert A[i2, j2] == A[0, j]
    # row block generation agrees with the full matrix
    assert np.array_equal(inputs.lattice_matrix(m, rows=slice(10, 20)), A[10:20])


def test_lattice_gershgorin_certificate():
    """Diagonally dominant: Gershgorin proves the lattice matrices nonsingular.
    Small lattices: the exact margin.  The benchmark lattices (20^3, 26^3):
    the table bound, which sums |A_ij| over every possible displacement and
    so bounds every row's disc radius from above."""
    for m in (4, 6, 8):
        exact = inputs.gershgorin_margin(inputs.lattice_matrix(m))
        bound = inputs.lattice_gershgorin_bound(m)
        assert exact >= bound > 40.0
    for m in (20, 26):
        assert inputs.lattice_gershgorin_bound(m) > 39.0


def test_integer_generators():
    A = inputs.gaussian_integer_matrix(9, 1, bound=3)
    assert np.all(np.abs(A.real) <= 3) and np.all(A.real == np.round(A.real))
    v = inputs.gaussian_integer_vector(9, 1, bound=3)
    assert np.all(np.abs(v.imag) <= 3)
