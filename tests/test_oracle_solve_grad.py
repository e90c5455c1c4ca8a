"""Pins of the oracle's linear-solve gradient and of the MCF-step gradient
built on it (adjoint method, Sec. 3.1 Eq. implicit-full; MCF step, Sec. 7.1),
against dense solves, central finite differences and a translation identity."""
import numpy as np
import pytest

import meshgen
import oracle


def _dense(rp, col, vals, n):
    A = np.zeros((n, n))
    for i in range(n):
        A[i, col[rp[i]:rp[i + 1]]] = vals[rp[i]:rp[i + 1]]
    return A


@pytest.mark.parametrize("with_f", [False, True])
def test_linear_solve_vjp_matches_dense_finite_differences(with_f):
    """dl/dK_t and dl/dM_i of l = sum(W * A^-1 b), A = alpha M + beta K, by
    central differences of dense solves, against the oracle's formulas."""
    X, F = meshgen.icosphere(1, 1e-2, 4)
    K, M, rp, col = oracle.assemble(X, F)
    n, k, alpha, beta = X.shape[0], 2, 1.3, 0.7
    rng = np.random.default_rng(0)
    W = rng.standard_normal((n, k))
    f = rng.standard_normal((n, k))
    b0 = rng.standard_normal((n, k))

    def loss(Kv, Mv):
        A = alpha * np.diag(Mv) + beta * _dense(rp, col, Kv, n)
        b = Mv[:, None] * f if with_f else b0
        return float(np.sum(W * np.linalg.solve(A, b)))

    A = alpha * np.diag(M) + beta * _dense(rp, col, K, n)
    b = M[:, None] * f if with_f else b0
    u = np.linalg.solve(A, b)
    lam = np.linalg.solve(A.T, W)
    gK, gM = oracle.linear_solve_vjp(rp, col, alpha, beta, lam, u, f if with_f else None)
    h = 1e-6
    for t in rng.choice(K.size, 25, replace=False):
        e = np.zeros_like(K)
        e[t] = h
        fd = (loss(K + e, M) - loss(K - e, M)) / (2 * h)
        assert abs(fd - gK[t]) <= 1e-7 * max(1.0, abs(fd)), (t, fd, gK[t])
    for i in rng.choice(n, 10, replace=False):
        e = np.zeros_like(M)
        e[i] = h
        fd = (loss(K, M + e) - loss(K, M - e)) / (2 * h)
        assert abs(fd - gM[i]) <= 1e-7 * max(1.0, abs(fd)), (i, fd, gM[i])


def test_mcf_step_gradient_finite_differences():
    """The whole step X -> K(X), M(X) -> u = (M + tau K)^-1 M X -> sum(W * u):
    the adjoint gradient against central differences along random directions."""
    X, F = meshgen.icosphere(2, 1e-2, 5)
    tau = 1e-2
    W = meshgen.normal(6, X.size).reshape(X.shape)
    l0, gX = oracle.mcf_step_grad(X, F, tau, W)
    rng = np.random.default_rng(1)
    h = 1e-6
    for _ in range(4):
        d = rng.standard_normal(X.shape)
        lp = float(np.sum(W * oracle.mcf_step(X + h * d, F, tau)[0]))
        lm = float(np.sum(W * oracle.mcf_step(X - h * d, F, tau)[0]))
        fd = (lp - lm) / (2 * h)
        an = float(np.sum(gX * d))
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (fd, an)


def test_mcf_step_gradient_translation_identity():
    """K 1 = 0, so a uniform shift c of X shifts u by c: the gradient summed
    over the vertices equals W summed over the vertices (per coordinate)."""
    X, F = meshgen.icosphere(2, 1e-2, 7)
    W = meshgen.normal(8, X.size).reshape(X.shape)
    _, gX = oracle.mcf_step_grad(X, F, 5e-2, W)
    np.testing.assert_allclose(gX.sum(0), W.sum(0), rtol=1e-9, atol=1e-9)
