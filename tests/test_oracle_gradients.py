"""Pins of the oracle's derivatives of assembly with respect to the vertex
positions (the df/dx factor of the adjoint method, Sec. 3.1, for the MCF
relation of Sec. 7.1 whose matrices depend on the positions): complex-step
and central finite differences, invariance under translation, rotation and
scaling, and agreement of the direct loss gradient with the assembly VJP."""
import numpy as np
import pytest

import meshgen


def _mesh(seed=0):
    X, F = meshgen.icosphere(1, 5e-2, seed)
    u = meshgen.normal(100 + seed, X.shape[0])
    return X, F, u


def test_complex_step(orc):
    X, F, u = _mesh(1)
    L, g = orc.loss_grad_tri(X, F, u)
    for v in range(0, X.shape[0], 5):
        for c in range(3):
            d = orc.loss_cstep_tri(X, F, u, v, c)
            assert abs(d - g[v, c]) <= 1e-12 * max(1.0, np.abs(g).max()), (v, c, d, g[v, c])


def test_central_fd(orc):
    X, F, u = _mesh(2)
    L, g = orc.loss_grad_tri(X, F, u)
    h = 1e-6
    for v in range(0, X.shape[0], 7):
        for c in range(3):
            Xp, Xm = X.copy(), X.copy()
            Xp[v, c] += h
            Xm[v, c] -= h
            fd = (orc.loss_grad_tri(Xp, F, u)[0] - orc.loss_grad_tri(Xm, F, u)[0]) / (2 * h)
            assert abs(fd - g[v, c]) <= 1e-6 * np.abs(g).max()


def test_invariances(orc):
    X, F, u = _mesh(3)
    L, g = orc.loss_grad_tri(X, F, u)
    s = np.abs(g).max()
    assert np.abs(g.sum(0)).max() <= 1e-12 * s * X.shape[0]               # translation
    assert np.abs(np.cross(X, g).sum(0)).max() <= 1e-12 * s * X.shape[0]   # rotation
    # scaling: cotangents are scale invariant, area has degree 2
    K, M, rp, col = orc.assemble(X, F)
    assert abs(np.sum(X * g) - 2.0 * M.sum()) <= 1e-12 * M.sum()


def test_vjp_matches_direct_gradient(orc):
    """VJP with gK_ij = u_i u_j (d(u^T K u)/dK_ij) and gM = 1 equals the
    gradient of u^T K u + total area."""
    X, F, u = _mesh(4)
    K, M, rp, col = orc.assemble(X, F)
    rows = np.repeat(np.arange(X.shape[0]), np.diff(rp))
    gK = u[rows] * u[col]
    gX = orc.assemble_vjp_tri(X, F, rp, col, gK, np.ones(X.shape[0]))
    _, g = orc.loss_grad_tri(X, F, u)
    np.testing.assert_allclose(gX, g, rtol=1e-12, atol=1e-12 * np.abs(g).max())


def test_vjp_directional_fd(orc):
    """<gX, d> = d/dt [gK . K(X + t d) + gM . M(X + t d)] for random gK, gM."""
    X, F = meshgen.icosphere(2, 2e-2, 5)
    K, M, rp, col = orc.assemble(X, F)
    gK = meshgen.normal(11, K.size)
    gM = meshgen.normal(12, M.size)
    gX = orc.assemble_vjp_tri(X, F, rp, col, gK, gM)
    for s in range(3):
        d = meshgen.normal(20 + s, X.size).reshape(X.shape)
        h = 1e-6
        Kp, Mp, _, _ = orc.assemble(X + h * d, F, rp, col)
        Km, Mm, _, _ = orc.assemble(X - h * d, F, rp, col)
        fd = (gK @ (Kp - Km) + gM @ (Mp - Mm)) / (2 * h)
        assert abs(fd - np.sum(gX * d)) <= 1e-7 * np.abs(gX).sum()
    # only-gK and only-gM parts add up
    a = orc.assemble_vjp_tri(X, F, rp, col, gK, None)
    b = orc.assemble_vjp_tri(X, F, rp, col, None, gM)
    np.testing.assert_allclose(a + b, gX, rtol=1e-13, atol=1e-14 * np.abs(gX).max())
