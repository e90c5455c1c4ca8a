"""Pins of the oracle's SpMV and Jacobi-PCG: dense products and dense solves
on small meshes, K 1 = 0, exactness of linear Dirichlet data, and the O(h^2)
convergence of the manufactured Poisson problem on the Kuhn cube."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import meshgen


def dense(K, rowptr, col):
    n = rowptr.size - 1
    return sp.csr_matrix((K, col, rowptr), shape=(n, n)).toarray()


@pytest.mark.parametrize("mesh", ["grid", "ico", "cube"])
def test_spmv_dense(orc, mesh):
    X, E = {"grid": lambda: meshgen.grid2d(10, 0.2, 1),
            "ico": lambda: meshgen.icosphere(2, 1e-3, 1),
            "cube": lambda: meshgen.cube_tets(5, 0.15, 1)}[mesh]()
    K, M, rp, col = orc.assemble(X, E)
    A = 0.7 * np.diag(M) + 1.3 * dense(K, rp, col)
    x = meshgen.uniform(3, X.shape[0] * 3).reshape(-1, 3) * 2 - 1
    y = orc.spmv(rp, col, 0.7, M, 1.3, K, x)
    np.testing.assert_allclose(y, A @ x, rtol=1e-13, atol=1e-14 * np.abs(A).sum(1).max())
    ones = np.ones(X.shape[0])
    assert np.abs(orc.spmv(rp, col, 0.0, M, 1.0, K, ones)).max() <= 1e-13 * np.abs(K).max()


def test_pcg_dense_solve(orc):
    X, F = meshgen.icosphere(3, 1e-3, 0)
    K, M, rp, col = orc.assemble(X, F)
    f = meshgen.normal(1, X.shape[0] * 3).reshape(-1, 3)
    b = M[:, None] * f
    A = np.diag(M) + 1e-3 * dense(K, rp, col)
    u, its, rr = orc.pcg(rp, col, 1.0, M, 1e-3, K, b, rtol=1e-12)
    ref = np.linalg.solve(A, b)
    np.testing.assert_allclose(u, ref, rtol=1e-9, atol=1e-10 * np.abs(ref).max())
    assert np.all(rr <= 1e-12)
    true_res = np.linalg.norm(b - A @ u, axis=0) / np.linalg.norm(b, axis=0)
    assert np.all(true_res <= 1e-11)


def test_pcg_dirichlet_dense(orc):
    X, T = meshgen.cube_tets(5, 0.15, 0)
    K, M, rp, col = orc.assemble(X, T)
    mask, _ = orc.boundary(X.shape[0], T)
    g = np.sin(X[:, 0]) + X[:, 1] * X[:, 2]
    f = np.cos(3 * X[:, 0])
    b = M * f
    u, its, rr = orc.pcg(rp, col, 0.0, M, 1.0, K, b, mask=mask, g=g, rtol=1e-13)
    A = dense(K, rp, col)
    I = mask == 0
    Bm = mask == 1
    ref = g.copy()
    ref[I] = np.linalg.solve(A[np.ix_(I, I)], b[I] - A[np.ix_(I, Bm)] @ g[Bm])
    np.testing.assert_allclose(u, ref, rtol=1e-10, atol=1e-12)


def test_dirichlet_linear_exact(orc):
    """Zero source with linear boundary data: the discrete solution is the
    linear function itself (linear precision of the P1 stiffness)."""
    X, T = meshgen.cube_tets(7, 0.15, 4)
    K, M, rp, col = orc.assemble(X, T)
    mask, _ = orc.boundary(X.shape[0], T)
    g = X @ np.array([1.0, 2.0, 3.0])
    u, its, rr = orc.pcg(rp, col, 0.0, M, 1.0, K, np.zeros(X.shape[0]), mask=mask, g=g,
                         rtol=1e-14, max_iter=5000)
    assert np.abs(u - g).max() <= 1e-11


def test_manufactured_poisson_rate(orc):
    """-Lap u = 3 pi^2 u* with u* = sin(pi x) sin(pi y) sin(pi z): nodal error
    falls by ~4 per halving of h."""
    errs = []
    for n in (9, 17, 33):
        X, T = meshgen.cube_tets(n, 0.15, 0)
        K, M, rp, col = orc.assemble(X, T)
        mask, _ = orc.boundary(X.shape[0], T)
        us = np.sin(math.pi * X[:, 0]) * np.sin(math.pi * X[:, 1]) * np.sin(math.pi * X[:, 2])
        b = M * (3 * math.pi ** 2 * us)
        u, its, rr = orc.pcg(rp, col, 0.0, M, 1.0, K, b, mask=mask, g=us, rtol=1e-12,
                             max_iter=20000)
        errs.append(np.sqrt(np.sum(M * (u - us) ** 2)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.0 < r1 < 5.5 and 3.0 < r2 < 5.5, errs


def test_pcg_fixed_iterations_and_freeze(orc):
    X, F = meshgen.icosphere(2, 1e-3, 0)
    K, M, rp, col = orc.assemble(X, F)
    b = meshgen.normal(2, X.shape[0] * 2).reshape(-1, 2)
    u, its, rr = orc.pcg(rp, col, 1.0, M, 1e-3, K, b, rtol=0.0, max_iter=7)
    assert list(its) == [7, 7]
    # column c alone equals column c in the pair
    u0, _, _ = orc.pcg(rp, col, 1.0, M, 1e-3, K, b[:, 0].copy(), rtol=0.0, max_iter=7)
    np.testing.assert_array_equal(u0, u[:, 0])
