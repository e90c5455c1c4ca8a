"""GPU parity of the smallest generalized eigenpairs (subspace iteration on
the shift-invert operator with Rayleigh-Ritz) against the oracle: eigenvalues
and canonically signed, M-orthonormal eigenvectors on a jittered grid (FP64,
FP32), the closed-form spectrum of a flat torus assembled intrinsically on the
GPU, and ARPACK shift-invert on icospheres of level 6 and 7 (the eigenstudy's
162K-vertex size, with residuals, orthonormality and the sphere's spectrum
l(l+1)), plus determinism and argument errors."""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

import meshgen
import oracle

pytestmark = pytest.mark.gpu

dgo = pytest.importorskip("paper_2602_12105_amd")
DEV = "cuda:0"


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("no HIP device visible")
    import paper_2602_12105_amd._lib as L
    L.lib()  # the native library must load; there is no fallback
    yield


def _assembled(X, F, td=torch.float64):
    m = dgo.Mesh(torch.from_numpy(F).to(DEV), X.shape[0])
    K, M = dgo.assemble(m, torch.from_numpy(X).to(DEV, td))
    return m, K, M


def _check_pairs(m, K, M, lam, U, tol):
    """residual and M-orthonormality computed on the host from K, M"""
    rp, col = [t.cpu().numpy() for t in m.csr()]
    Kh, Mh = K.double().cpu().numpy(), M.double().cpu().numpy()
    A = sp.csr_matrix((Kh, col, rp))
    Uh, lh = U.double().cpu().numpy(), lam.numpy()
    R = A @ Uh - (Mh[:, None] * Uh) * lh[None, :]
    rn = np.sqrt(((R ** 2) / Mh[:, None]).sum(axis=0))
    G = Uh.T @ (Mh[:, None] * Uh)
    return rn, np.abs(G - np.eye(Uh.shape[1])).max()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_grid_against_oracle(dtype):
    print(f"[eigs] grid 30 {dtype}", flush=True)
    X, F = meshgen.grid2d(30, 0.2, 5)
    td = torch.float64 if dtype == "f64" else torch.float32
    m, K, M = _assembled(X, F, td)
    k = 6
    # FP32 vectors bound the attainable residual near eps_32 * lambda_max / lambda
    lam, U, rep = dgo.eigs_smallest(m, M, K, k, tol=1e-10 if dtype == "f64" else 2e-3)
    print(rep, flush=True)
    assert rep["converged"], rep
    rp, col = [t.cpu().numpy() for t in m.csr()]
    lo, Uo = oracle.eigs_smallest(rp, col, K.double().cpu().numpy(), M.double().cpu().numpy(), k)
    if dtype == "f64":
        np.testing.assert_allclose(lam.numpy(), lo, rtol=1e-10, atol=1e-10)
        np.testing.assert_allclose(U.cpu().numpy(), Uo, atol=1e-7)
        rn, orth = _check_pairs(m, K, M, lam, U, 1e-10)
        assert orth <= 1e-12
    else:
        np.testing.assert_allclose(lam.numpy(), lo, rtol=1e-4, atol=1e-4)
        np.testing.assert_allclose(U.double().cpu().numpy(), Uo, atol=2e-3 * np.abs(Uo).max())


def test_flat_torus_closed_form():
    print("[eigs] flat torus", flush=True)
    n = 16
    F, ij = meshgen.flat_torus(n)
    m = dgo.Mesh(torch.from_numpy(F).to(DEV), n * n)
    EV = m.edges()[0].cpu().numpy()
    L = torch.from_numpy(meshgen.flat_torus_lengths(n, ij, EV)).to(DEV)
    K, M = dgo.assemble_intrinsic(m, L)
    lam, U, rep = dgo.eigs_smallest(m, M, K, 9, tol=1e-10)
    assert rep["converged"]
    p = np.arange(n)
    ref = np.sort(((4 * np.sin(np.pi * p[:, None] / n) ** 2 + 4 * np.sin(np.pi * p[None, :] / n) ** 2)
                   * n * n).ravel())
    np.testing.assert_allclose(lam.numpy(), ref[:9], rtol=1e-9, atol=1e-8)


def test_icosphere_l6_against_arpack():
    print("[eigs] icosphere L6 vs ARPACK", flush=True)
    X, F = meshgen.icosphere(6, 1e-2, 1)
    m, K, M = _assembled(X, F)
    k = 9
    lam, U, rep = dgo.eigs_smallest(m, M, K, k, tol=1e-9)
    assert rep["converged"], rep
    rp, col = [t.cpu().numpy() for t in m.csr()]
    lo, Uo = oracle.eigs_smallest(rp, col, K.cpu().numpy(), M.cpu().numpy(), k)
    np.testing.assert_allclose(lam.numpy(), lo, rtol=1e-9, atol=1e-9)
    # eigenvectors of this noisy sphere are well separated enough to compare
    # individually, up to the canonical sign both sides apply
    Mh = M.cpu().numpy()
    cos = np.abs(np.einsum("ij,i,ij->j", U.cpu().numpy(), Mh, Uo))
    assert (cos >= 1 - 1e-6).all(), cos


def test_icosphere_l7_full_size():
    print("[eigs] icosphere L7", flush=True)
    X, F = meshgen.icosphere(7, 1e-3, 0)
    m, K, M = _assembled(X, F)
    k = 9
    lam, U, rep = dgo.eigs_smallest(m, M, K, k)
    assert rep["converged"], rep
    rn, orth = _check_pairs(m, K, M, lam, U, 1e-8)
    assert orth <= 1e-10
    assert (rn <= 1e-7 * np.maximum(np.abs(lam.numpy()), abs(rep["sigma"]))).all(), rn
    # ARPACK shift-invert on the same matrices (about 10 s of CPU)
    rp, col = [t.cpu().numpy() for t in m.csr()]
    lo, Uo = oracle.eigs_smallest(rp, col, K.cpu().numpy(), M.cpu().numpy(), k)
    np.testing.assert_allclose(lam.numpy(), lo, rtol=1e-9, atol=1e-9)
    cos = np.abs(np.einsum("ij,i,ij->j", U.cpu().numpy(), M.cpu().numpy(), Uo))
    assert (cos >= 1 - 1e-6).all(), cos
    # the unit sphere's l(l+1), lowered by the area the normal noise adds
    ref = np.array([0] + [2] * 3 + [6] * 5, float)
    assert abs(lam[0]) < 1e-8
    np.testing.assert_allclose(lam.numpy()[1:], ref[1:], rtol=0.03)
    # deterministic
    lam2, U2, _ = dgo.eigs_smallest(m, M, K, k)
    assert torch.equal(lam, lam2) and torch.equal(U, U2)


def test_eigs_errors():
    print("[eigs] errors", flush=True)
    X, F = meshgen.grid2d(6, 0.1, 1)
    m, K, M = _assembled(X, F)
    for kw in ({"k": 0}, {"k": 65}, {"k": 3, "sigma": 0.5}, {"k": 3, "block": 2}):
        k = kw.pop("k")
        with pytest.raises(dgo.DgoError) as e:
            dgo.eigs_smallest(m, M, K, k, **kw)
        assert e.value.status == "INVALID_ARG"
