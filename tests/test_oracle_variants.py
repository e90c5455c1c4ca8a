"""Pins of the oracle's operator variants: the mixed-Voronoi lumped mass
(closed forms of an equilateral, a right and an obtuse triangle, the exact
partition of every triangle's area, the uniform grid's interior value h^2),
the row array of the COO export, and the conformal Laplacian of the spectral
conformal parameterization (symmetric, positive semidefinite, block diagonal
on closed surfaces, and with the similarity maps of a planar counterclockwise
mesh in its kernel: the identity and its 90 degree rotation have zero
conformal energy, Dirichlet energy equal to area)."""
import numpy as np
import scipy.sparse as sp

import meshgen


def test_voronoi_closed_forms(orc):
    F = np.array([[0, 1, 2]], np.int32)
    eq = np.array([[0, 0, 0], [1, 0, 0], [0.5, np.sqrt(3) / 2, 0]])
    np.testing.assert_allclose(orc.mass_voronoi(eq, F), np.full(3, np.sqrt(3) / 12), rtol=1e-15)
    right = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0.0]])
    np.testing.assert_allclose(orc.mass_voronoi(right, F), [0.25, 0.125, 0.125], rtol=1e-15)
    # obtuse at vertex 2 (angle 120 degrees): A/2 there, A/4 at the others
    ob = np.array([[0, 0, 0], [2, 0, 0], [1, 1 / np.sqrt(3), 0]])
    A = 0.5 * 2 / np.sqrt(3)
    np.testing.assert_allclose(orc.mass_voronoi(ob, F), [A / 4, A / 4, A / 2], rtol=1e-15)


def test_voronoi_partitions_area(orc):
    X, F = meshgen.icosphere(3, 0.05, 1)
    M = orc.mass_voronoi(X, F)
    area = 0.5 * np.linalg.norm(np.cross(X[F[:, 1]] - X[F[:, 0]], X[F[:, 2]] - X[F[:, 0]]), axis=1)
    assert abs(M.sum() - area.sum()) <= 1e-13 * area.sum()
    assert (M > 0).all()
    # per triangle, not just in total: the single-triangle sums are its area
    for t in range(0, F.shape[0], 37):
        Mt = orc.mass_voronoi(X[F[t]], np.array([[0, 1, 2]], np.int32))
        assert abs(Mt.sum() - area[t]) <= 1e-14 * area[t]


def test_voronoi_uniform_grid_interior(orc):
    n = 9
    X, F = meshgen.grid2d(n, 0.0, 0)
    h = 1.0 / (n - 1)
    M = orc.mass_voronoi(X, F)
    inner = [i * n + j for i in range(1, n - 1) for j in range(1, n - 1)]
    np.testing.assert_allclose(M[inner], h * h, rtol=1e-13)


def test_coo_rows(orc):
    X, F = meshgen.grid2d(6, 0.2, 1)
    K, M, rp, col = orc.assemble(X, F)
    rows = orc.csr_rows(rp)
    A = sp.csr_matrix((K, col, rp)).tocoo()
    np.testing.assert_array_equal(rows, A.row)
    np.testing.assert_array_equal(col, A.col)


def _planar():
    X, F = meshgen.grid2d(7, 0.2, 2)  # counterclockwise triangles in the z = 0 plane
    return X, F


def test_conformal_laplacian_similarity_kernel(orc):
    X, F = _planar()
    n = X.shape[0]
    K, M, rp, col = orc.assemble(X, F)
    L = orc.conformal_laplacian(F, n, K, rp, col)
    np.testing.assert_array_equal(L, L.T)
    x, y = X[:, 0], X[:, 1]
    for u in (np.concatenate([x, y]), np.concatenate([-y, x]), np.concatenate([np.ones(n), np.zeros(n)]),
              np.concatenate([np.zeros(n), np.ones(n)])):
        assert np.abs(L @ u).max() <= 1e-12
    # the parts: Dirichlet energy of the identity = area = shoelace area
    area = 0.5 * np.linalg.norm(np.cross(X[F[:, 1]] - X[F[:, 0]], X[F[:, 2]] - X[F[:, 0]]), axis=1).sum()
    Kd = L[:n, :n]
    assert abs(0.5 * (x @ Kd @ x + y @ Kd @ y) - area) <= 1e-12
    assert abs(x @ (-L[:n, n:]) @ y - area) <= 1e-12
    # positive semidefinite with a 4-dimensional kernel on a connected disk
    w = np.linalg.eigvalsh(L)
    assert w.min() >= -1e-12 and (np.abs(w) <= 1e-10).sum() == 4
    # a mirrored mesh (clockwise) is conformal to the reflected map instead
    Fr = F[:, ::-1].copy()
    Lr = orc.conformal_laplacian(Fr, n, K, rp, col)
    assert np.abs(Lr @ np.concatenate([x, -y])).max() <= 1e-12
    assert np.abs(Lr @ np.concatenate([x, y])).max() > 1e-3


def test_conformal_laplacian_closed_surface_is_block_diagonal(orc):
    X, F = meshgen.icosphere(1, 0.0, 0)
    K, M, rp, col = orc.assemble(X, F)
    n = X.shape[0]
    L = orc.conformal_laplacian(F, n, K, rp, col)
    assert not L[:n, n:].any() and not L[n:, :n].any()
    np.testing.assert_array_equal(L[:n, :n], L[n:, n:])
