"""Pins of the oracle's smallest generalized eigenpairs K u = lam M u: the
closed-form spectrum of a flat torus given by its edge lengths (the
periodic five-point Laplacian over h^2), the continuous spectrum l(l+1) of the
unit sphere approached by a fine icosphere, the dense definition against
ARPACK shift-invert on the same jittered grid, and invariants (residual,
M-orthonormality, one zero eigenvalue with a constant eigenvector per
connected component, canonical signs)."""
import numpy as np

import meshgen


def _torus(orc, n):
    F, ij = meshgen.flat_torus(n)
    nV = n * n
    EV, _, _ = orc.edges(nV, F)
    L = meshgen.flat_torus_lengths(n, ij, EV)
    K, M = orc.assemble_intrinsic(F, nV, L)
    rp, col = orc.csr(nV, EV)
    return K, M, rp, col


def test_flat_torus_closed_form(orc):
    n = 12
    K, M, rp, col = _torus(orc, n)
    h = 1.0 / n
    np.testing.assert_allclose(M, h * h, rtol=1e-13)
    p = np.arange(n)
    ref = np.sort(((4 * np.sin(np.pi * p[:, None] / n) ** 2 + 4 * np.sin(np.pi * p[None, :] / n) ** 2)
                   / h ** 2).ravel())
    lam, U = orc.eigs_smallest(rp, col, K, M, 25)
    np.testing.assert_allclose(lam, ref[:25], rtol=1e-10, atol=1e-9)


def test_sphere_spectrum(orc):
    X, F = meshgen.icosphere(4)
    K, M, rp, col = orc.assemble(X, F)
    lam, U = orc.eigs_smallest(rp, col, K, M, 16)
    ref = np.array([0] + [2] * 3 + [6] * 5 + [12] * 7, float)
    assert abs(lam[0]) < 1e-9
    np.testing.assert_allclose(lam[1:], ref[1:], rtol=0.02)


def test_dense_and_arpack_agree(orc):
    X, F = meshgen.grid2d(40, 0.2, 7)
    K, M, rp, col = orc.assemble(X, F)
    l1, U1 = orc.eigs_smallest(rp, col, K, M, 6)
    l2, U2 = orc.eigs_smallest(rp, col, K, M, 6, dense_max=0)
    np.testing.assert_allclose(l2, l1, rtol=1e-9, atol=1e-10)
    np.testing.assert_allclose(U2, U1, atol=1e-7)


def test_invariants(orc):
    X, F = meshgen.grid2d(30, 0.2, 3)
    K, M, rp, col = orc.assemble(X, F)
    import scipy.sparse as sp
    A = sp.csr_matrix((K, col, rp))
    lam, U = orc.eigs_smallest(rp, col, K, M, 5)
    R = A @ U - (M[:, None] * U) * lam[None, :]
    assert np.abs(R).max() <= 1e-10 * max(1.0, lam.max()) * M.max()
    np.testing.assert_allclose(U.T @ (M[:, None] * U), np.eye(5), atol=1e-12)
    assert abs(lam[0]) < 1e-10 and np.ptp(U[:, 0]) < 1e-10
    assert (np.diff(lam) >= 0).all()
    idx = np.argmax(np.abs(U), axis=0)
    assert (U[idx, np.arange(5)] > 0).all()


def test_one_zero_eigenvalue_per_component(orc):
    X1, F1 = meshgen.icosphere(2)
    X = np.vstack([X1, X1 + 3.0])
    F = np.vstack([F1, F1 + X1.shape[0]]).astype(np.int32)
    K, M, rp, col = orc.assemble(X, F)
    lam, U = orc.eigs_smallest(rp, col, K, M, 3)
    assert abs(lam[0]) < 1e-9 and abs(lam[1]) < 1e-9 and lam[2] > 1.0
