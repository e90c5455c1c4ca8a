"""Pins of the oracle's operators: closed forms of single elements, the
5-point / 7-point stencils of unjittered grids, an independent second formula
for each weight (law of cosines with Kahan's Heron area; dihedral cotangents),
and invariants (row sums, symmetry, semidefiniteness, linear precision, total
measure, the energy identity u^T K u = sum_T |T| |grad u_T|^2)."""
import json
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp

import meshgen

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))


def dense(K, rowptr, col):
    n = rowptr.size - 1
    return sp.csr_matrix((K, col, rowptr), shape=(n, n)).toarray()


def test_right_isosceles(orc):
    g = GOLD["right_isosceles_triangle"]
    K, M, rp, col = orc.assemble(np.array(g["X"], float), np.array(g["F"], np.int32))
    np.testing.assert_allclose(dense(K, rp, col), g["K_dense"], atol=1e-15)
    np.testing.assert_allclose(M, g["M"], rtol=1e-15)


def test_equilateral(orc):
    g = GOLD["equilateral_triangle_unit_edge"]
    K, M, rp, col = orc.assemble(np.array(g["X"], float), np.array(g["F"], np.int32))
    A = dense(K, rp, col)
    off = A[~np.eye(3, dtype=bool)]
    np.testing.assert_allclose(off, -g["w_edge"], rtol=1e-14)
    np.testing.assert_allclose(M, g["M"], rtol=1e-14)


def test_corner_tet(orc):
    g = GOLD["corner_tet"]
    K, M, rp, col = orc.assemble(np.array(g["X"], float), np.array(g["T"], np.int32))
    np.testing.assert_allclose(dense(K, rp, col), g["K_dense"], atol=1e-15)
    np.testing.assert_allclose(M, g["M"], rtol=1e-14)


def test_regular_tet(orc):
    g = GOLD["regular_tet_unit_edge"]
    X = np.array(g["X"], float) * g["X_scale"]
    K, M, rp, col = orc.assemble(X, np.array(g["T"], np.int32))
    A = dense(K, rp, col)
    np.testing.assert_allclose(A[~np.eye(4, dtype=bool)], -g["w_edge"], rtol=1e-13)
    np.testing.assert_allclose(M, g["M"], rtol=1e-13)


def test_grid_five_point_stencil(orc):
    n = 9
    h = 1.0 / (n - 1)
    X, F = meshgen.grid2d(n)
    K, M, rp, col = orc.assemble(X, F)
    A = dense(K, rp, col)
    for i in range(1, n - 1):
        for j in range(1, n - 1):
            v = i * n + j
            row = np.zeros(n * n)
            row[v] = 4.0
            for w in (v - 1, v + 1, v - n, v + n):
                row[w] = -1.0
            np.testing.assert_allclose(A[v], row, atol=1e-14)
            assert abs(M[v] - h * h) <= 1e-15
    assert abs(M.sum() - 1.0) <= 1e-14


def test_kuhn_seven_point_stencil(orc):
    n = 6
    h = 1.0 / (n - 1)
    X, T = meshgen.cube_tets(n)
    K, M, rp, col = orc.assemble(X, T)
    A = dense(K, rp, col)
    ntet = np.bincount(T.ravel(), minlength=n ** 3)
    for i in range(1, n - 1):
        for j in range(1, n - 1):
            for k in range(1, n - 1):
                v = (i * n + j) * n + k
                row = np.zeros(n ** 3)
                row[v] = 6.0 * h
                for w in (v - 1, v + 1, v - n, v + n, v - n * n, v + n * n):
                    row[w] = -h
                np.testing.assert_allclose(A[v], row, atol=1e-14)
                assert abs(M[v] - h ** 3) <= 1e-15
                assert ntet[v] == 24
    assert abs(M.sum() - 1.0) <= 1e-13


def _kahan_heron(a, b, c):
    # Kahan, "Miscalculating area and angles of a needle-like triangle"
    s = np.sort(np.stack([a, b, c], 1), 1)[:, ::-1]
    a, b, c = s[:, 0], s[:, 1], s[:, 2]
    return 0.25 * np.sqrt((a + (b + c)) * (c - (a - b)) * (c + (a - b)) * (a + (b - c)))


def _weights_law_of_cosines(X, F, EV):
    """Per-edge 1/2 cot via cot(angle at k) = (li^2 + lj^2 - lk^2) / (4 A)."""
    idx = {tuple(e): i for i, e in enumerate(EV.tolist())}
    w = np.zeros(EV.shape[0])
    P = X[F]
    l = np.stack([np.linalg.norm(P[:, (k + 1) % 3] - P[:, (k + 2) % 3], axis=1) for k in range(3)], 1)
    A = _kahan_heron(l[:, 0], l[:, 1], l[:, 2])
    for k in range(3):
        cot = (l[:, (k + 1) % 3] ** 2 + l[:, (k + 2) % 3] ** 2 - l[:, k] ** 2) / (4.0 * A)
        for f in range(F.shape[0]):
            a, b = F[f, (k + 1) % 3], F[f, (k + 2) % 3]
            w[idx[(min(a, b), max(a, b))]] += 0.5 * cot[f]
    return w, A


@pytest.mark.parametrize("mesh", ["grid", "ico"])
def test_triangle_weights_second_formula(orc, mesh):
    X, F = meshgen.grid2d(12, 0.2, 5) if mesh == "grid" else meshgen.icosphere(2, 1e-2, 5)
    EV, ee, _ = orc.edges(X.shape[0], F)
    w = orc.edge_weights(X, F, EV, ee)
    w2, A = _weights_law_of_cosines(X, F, EV)
    np.testing.assert_allclose(w, w2, rtol=1e-11, atol=1e-12)
    K, M, rp, col = orc.assemble(X, F)
    assert abs(M.sum() - A.sum()) <= 1e-13 * A.sum()


def _dihedral_weights(X, T, EV):
    """w_ij = (1/6) l_kl cot(theta_kl), kl the edge opposite ij."""
    idx = {tuple(e): i for i, e in enumerate(EV.tolist())}
    w = np.zeros(EV.shape[0])
    pairs = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]
    for t in T.tolist():
        for a, b in pairs:
            k, l = [c for c in range(4) if c not in (a, b)]
            xk, xl, xi, xj = X[t[k]], X[t[l]], X[t[a]], X[t[b]]
            e = (xl - xk) / np.linalg.norm(xl - xk)
            u = (xi - xk) - np.dot(xi - xk, e) * e
            v = (xj - xk) - np.dot(xj - xk, e) * e
            cot = np.dot(u, v) / np.linalg.norm(np.cross(u, v))
            va, vb = t[a], t[b]
            w[idx[(min(va, vb), max(va, vb))]] += np.linalg.norm(xl - xk) * cot / 6.0
    return w


def test_tet_weights_dihedral_formula(orc):
    X, T = meshgen.cube_tets(4, 0.15, 9)
    EV, ee, _ = orc.edges(X.shape[0], T)
    w = orc.edge_weights(X, T, EV, ee)
    np.testing.assert_allclose(w, _dihedral_weights(X, T, EV), rtol=1e-11, atol=1e-13)


def _meshes():
    yield "grid", *meshgen.grid2d(14, 0.2, 0)
    yield "ico", *meshgen.icosphere(3, 1e-2, 0)
    yield "cube", *meshgen.cube_tets(6, 0.15, 0)


@pytest.mark.parametrize("name,X,E", list(_meshes()), ids=lambda v: v if isinstance(v, str) else "")
def test_invariants(orc, name, X, E):
    K, M, rp, col = orc.assemble(X, E)
    A = dense(K, rp, col)
    scale = np.abs(A).max()
    assert np.abs(A.sum(1)).max() <= 1e-13 * scale          # rows sum to zero
    assert np.array_equal(A, A.T)                            # exact symmetry
    ev = np.linalg.eigvalsh(A)
    assert ev.min() >= -1e-12 * ev.max()                     # PSD
    assert np.sum(ev < 1e-10 * ev.max()) == 1                # connected: 1-dim kernel
    assert np.all(M > 0)
    if name in ("grid", "cube"):
        # linear precision: K (a.x + c) vanishes at interior vertices
        mask, _ = orc.boundary(X.shape[0], E)
        lin = X @ np.array([0.3, -1.7, 2.2]) + 0.5
        r = A @ lin
        assert np.abs(r[mask == 0]).max() <= 1e-12 * scale
        assert abs(M.sum() - 1.0) <= 1e-13


def test_energy_identity(orc):
    """u^T K u = sum_T area_T |grad u_T|^2 with grad u_T from barycentric
    gradients (n x e_i) / (2 area), e_i the edge opposite vertex i."""
    X, F = meshgen.icosphere(3, 1e-2, 4)
    u = meshgen.normal(7, X.shape[0])
    K, M, rp, col = orc.assemble(X, F)
    A = dense(K, rp, col)
    P = X[F]
    n = np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0])
    area2 = np.linalg.norm(n, axis=1)
    nh = n / area2[:, None]
    grad = np.zeros((F.shape[0], 3))
    for i in range(3):
        e = P[:, (i + 2) % 3] - P[:, (i + 1) % 3]
        grad += u[F[:, i]][:, None] * np.cross(nh, e) / area2[:, None]
    ref = np.sum(0.5 * area2 * np.sum(grad * grad, 1))
    assert abs(u @ A @ u - ref) <= 1e-12 * ref


def test_clamp(orc):
    """Clamping replaces each summed edge weight by max(w, c) and the diagonal
    is rebuilt from the clamped weights, so rows still sum to zero."""
    X, F = meshgen.icosphere(2, 5e-2, 3)
    EV, ee, _ = orc.edges(X.shape[0], F)
    w = orc.edge_weights(X, F, EV, ee)
    c = np.quantile(w, 0.3)
    K, M, rp, col = orc.assemble(X, F, clamp_min=c)
    A = dense(K, rp, col)
    wc = np.maximum(w, c)
    np.testing.assert_allclose(-A[EV[:, 0], EV[:, 1]], wc, rtol=0, atol=0)
    assert np.abs(A.sum(1)).max() <= 1e-14 * np.abs(A).max()


def test_degenerate(orc):
    X = np.array([[0, 0, 0], [1, 0, 0], [2, 0, 0], [0, 1, 0]], float)
    F = np.array([[0, 1, 2], [0, 1, 3]], np.int32)
    with pytest.raises(orc.OracleError) as ei:
        orc.assemble(X, F)
    assert ei.value.code == 3
