"""Pins of the oracle's intrinsic assembly (edge lengths only) and of the
per-face gradient G and divergence D: closed forms of single triangles, the
extrinsic assembly (a different formula: cross and dot products of positions)
fed with lengths measured from the same positions, scale invariance of the
cotangent weights, exactness of G on linear fields (the tangential projection
of the field's gradient), D G = K against the pinned cotangent stiffness (the
sign the u-update of the geodesic ADMM loop of Sec. 7.4 needs with an SPD
Laplacian), adjointness of D and G under the area-weighted face inner product,
and the zero vertex sum of D on a closed surface."""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

import meshgen

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))


def dense(K, rowptr, col):
    n = rowptr.size - 1
    return sp.csr_matrix((K, col, rowptr), shape=(n, n)).toarray()


def lengths_of(orc, X, F):
    EV, _, _ = orc.edges(X.shape[0], F)
    return np.linalg.norm(X[EV[:, 0]] - X[EV[:, 1]], axis=1), EV


def areas_normals(X, F):
    n = np.cross(X[F[:, 1]] - X[F[:, 0]], X[F[:, 2]] - X[F[:, 0]])
    nn = np.linalg.norm(n, axis=1)
    return 0.5 * nn, n / nn[:, None]


MESHES = {
    "grid": lambda: meshgen.grid2d(9, 0.25, 3),
    "ico": lambda: meshgen.icosphere(2, 0.05, 4),
}


def test_intrinsic_right_isosceles(orc):
    g = GOLD["right_isosceles_triangle"]
    X, F = np.array(g["X"], float), np.array(g["F"], np.int32)
    L, _ = lengths_of(orc, X, F)
    K, M = orc.assemble_intrinsic(F, 3, L)
    _, _, rp, col = orc.assemble(X, F)
    np.testing.assert_allclose(dense(K, rp, col), g["K_dense"], atol=1e-15)
    np.testing.assert_allclose(M, g["M"], rtol=1e-15)


def test_intrinsic_equilateral_from_lengths_alone(orc):
    g = GOLD["equilateral_triangle_unit_edge"]
    F = np.array(g["F"], np.int32)
    K, M = orc.assemble_intrinsic(F, 3, np.ones(3))
    _, _, rp, col = orc.assemble(np.array(g["X"], float), F)
    A = dense(K, rp, col)
    np.testing.assert_allclose(A[~np.eye(3, dtype=bool)], -g["w_edge"], rtol=1e-14)
    np.testing.assert_allclose(M, g["M"], rtol=1e-14)


@pytest.mark.parametrize("name", sorted(MESHES))
def test_intrinsic_matches_extrinsic(orc, name):
    X, F = MESHES[name]()
    L, _ = lengths_of(orc, X, F)
    Ke, Me, rp, col = orc.assemble(X, F)
    Ki, Mi = orc.assemble_intrinsic(F, X.shape[0], L)
    np.testing.assert_allclose(Ki, Ke, rtol=0, atol=1e-12 * np.abs(Ke).max())
    np.testing.assert_allclose(Mi, Me, rtol=1e-12)


def test_intrinsic_scale_invariance(orc):
    X, F = MESHES["grid"]()
    L, _ = lengths_of(orc, X, F)
    K1, M1 = orc.assemble_intrinsic(F, X.shape[0], L)
    K2, M2 = orc.assemble_intrinsic(F, X.shape[0], 3.0 * L)
    np.testing.assert_allclose(K2, K1, rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(M2, 9.0 * M1, rtol=1e-13)


def test_intrinsic_rejects_triangle_inequality_violation(orc):
    F = np.array([[0, 1, 2]], np.int32)
    with pytest.raises(orc.OracleError):
        orc.assemble_intrinsic(F, 3, np.array([1.0, 1.0, 2.5]))


def test_gradient_of_hat_functions_closed_form(orc):
    X = np.array([[0, 0, 0], [2, 0, 0], [0, 1, 0]], float)
    F = np.array([[0, 1, 2]], np.int32)
    g = orc.face_gradient(X, F, np.eye(3))  # hat function j as field j
    want = np.array([[-0.5, -1, 0], [0.5, 0, 0], [0, 1, 0]])
    np.testing.assert_allclose(g[:, :, 0], want, atol=1e-15)


@pytest.mark.parametrize("name", sorted(MESHES))
def test_gradient_exact_on_linear_fields(orc, name):
    X, F = MESHES[name]()
    rng = np.random.default_rng(1)
    a = rng.standard_normal((3, 4))
    u = X @ a + rng.standard_normal(4)
    g = orc.face_gradient(X, F, u)
    _, N = areas_normals(X, F)
    for c in range(4):
        proj = a[:, c] - (N @ a[:, c])[:, None] * N
        np.testing.assert_allclose(g[c].T, proj, atol=1e-11)
    # coordinate functions: sum_j x_j (x) grad phi_j = I - N N^T
    G = orc.face_gradient(X, F, X)  # (coordinate, component, face)
    P = np.eye(3)[:, :, None] - N.T[:, None, :] * N.T[None, :, :]
    np.testing.assert_allclose(G, P, atol=1e-11)


@pytest.mark.parametrize("name", sorted(MESHES))
def test_div_grad_is_cotangent_stiffness(orc, name):
    X, F = MESHES[name]()
    K, M, rp, col = orc.assemble(X, F)
    u = meshgen.normal(11, X.shape[0] * 3).reshape(-1, 3)
    d = orc.face_divergence(X, F, orc.face_gradient(X, F, u))
    Ku = dense(K, rp, col) @ u
    np.testing.assert_allclose(d, Ku, rtol=0, atol=1e-11 * np.abs(Ku).max())


@pytest.mark.parametrize("name", sorted(MESHES))
def test_divergence_adjoint_of_gradient(orc, name):
    X, F = MESHES[name]()
    A, _ = areas_normals(X, F)
    rng = np.random.default_rng(5)
    y = rng.standard_normal((2, 3, F.shape[0]))
    u = rng.standard_normal((X.shape[0], 2))
    lhs = np.sum(orc.face_divergence(X, F, y) * u)
    rhs = np.sum(A[None, None, :] * y * orc.face_gradient(X, F, u))
    assert abs(lhs - rhs) <= 1e-11 * max(1.0, abs(rhs))


def test_divergence_sums_to_zero_on_closed_surface(orc):
    X, F = MESHES["ico"]()
    y = np.random.default_rng(9).standard_normal((3, 3, F.shape[0]))
    d = orc.face_divergence(X, F, y)
    assert np.abs(d.sum(axis=0)).max() <= 1e-12 * np.abs(d).sum()
