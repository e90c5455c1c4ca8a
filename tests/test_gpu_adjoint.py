"""GPU checks of the hand-written adjoints against finite differences of the
GPU's own forward pass (FP64): torch.autograd.gradcheck of AssembleFn, of
LinearSolveFn (in M, f, and K perturbed symmetrically) and of the implicit
MCF step end to end, plus central differences at h = 1e-6 of config 5's loss
u^T K(x) u + total area, coordinate by coordinate on one small mesh and along
random directions on all 256 meshes of the config-5 batch (the adjoint
method, Sec. 3.1; the differentiated operators of Sec. 7.1)."""
import numpy as np
import pytest
import torch

import meshgen
import oracle

pytestmark = pytest.mark.gpu

import paper_2602_12105_amd as dgo  # noqa: E402  (no skip: a broken import fails the suite)

DEV = "cuda:0"


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("no HIP device visible")
    import paper_2602_12105_amd._lib as L
    L.lib()  # the native library must load; there is no fallback
    yield


def _loss(m, X, u, rows, cols):
    """Per-mesh loss u^T K(x) u + sum(M) from the library's K and M."""
    K, M = dgo.AssembleFn.apply(X, m)
    return (K * (u[rows] * u[cols])[None, :]).sum(1) + M.sum(1)


def _pattern(m):
    rp, col = m.csr()
    rows = torch.repeat_interleave(torch.arange(m.nV, device=DEV), (rp[1:] - rp[:-1]).long())
    return rows, col.long()


def test_assemble_fn_gradcheck():
    """The full Jacobian of (K, M) with respect to X, by VJPs, against central
    differences (eps 1e-6) of the GPU assembly, on an icosphere of level 1
    (42 vertices: 126 inputs, 324 outputs) and a jittered 5 x 5 grid."""
    print("[gradcheck] AssembleFn", flush=True)
    for X, F in (meshgen.icosphere(1, 5e-2, 3), meshgen.grid2d(5, 0.2, 4)):
        m = dgo.Mesh(torch.from_numpy(F).to(DEV), X.shape[0])
        Xd = torch.from_numpy(X).to(DEV).requires_grad_(True)
        assert torch.autograd.gradcheck(lambda x: dgo.AssembleFn.apply(x, m), (Xd,), eps=1e-6,
                                        atol=1e-8, rtol=1e-6)


def test_linear_solve_fn_gradcheck():
    """LinearSolveFn's adjoint (adjoint PCG, solve VJP, M lambda) against
    central differences of the forward PCG solved to 1e-14: in M and f
    directly, and in K through a per-edge parameter added to both CSR slots
    of its edge and subtracted from both diagonals (a perturbation that keeps
    K symmetric with zero row sums, as every assembled K is)."""
    print("[gradcheck] LinearSolveFn", flush=True)
    X, F = meshgen.icosphere(1, 5e-2, 5)
    m = dgo.Mesh(torch.from_numpy(F).to(DEV), X.shape[0])
    K0, M0 = dgo.assemble(m, torch.from_numpy(X).to(DEV))
    f0 = torch.from_numpy(meshgen.normal(31, m.nV * 2).reshape(-1, 2)).to(DEV)
    tau, rtol = 0.05, 1e-14

    def solve_mf(M, f):
        return dgo.LinearSolveFn.apply(K0, M, f, m, 1.0, tau, rtol, 10000)

    Md = M0.clone().requires_grad_(True)
    fd = f0.clone().requires_grad_(True)
    assert torch.autograd.gradcheck(solve_mf, (Md, fd), eps=1e-6, atol=1e-7, rtol=1e-5)

    EV = m.edges()[0].long()
    rows, cols = _pattern(m)
    nV = m.nV
    key = rows * nV + cols
    order = torch.argsort(key)
    ks = key[order]

    def slot(i, j):
        return order[torch.searchsorted(ks, i * nV + j)]

    s_ij, s_ji = slot(EV[:, 0], EV[:, 1]), slot(EV[:, 1], EV[:, 0])
    s_ii, s_jj = slot(EV[:, 0], EV[:, 0]), slot(EV[:, 1], EV[:, 1])

    def solve_k(theta):
        K = K0.clone()
        K = K.index_add(0, s_ij, theta).index_add(0, s_ji, theta)
        K = K.index_add(0, s_ii, -theta).index_add(0, s_jj, -theta)
        return dgo.LinearSolveFn.apply(K, M0, f0, m, 1.0, tau, rtol, 10000)

    theta = torch.zeros(m.nE, dtype=torch.float64, device=DEV, requires_grad=True)
    assert torch.autograd.gradcheck(solve_k, (theta,), eps=1e-6, atol=1e-7, rtol=1e-5)


def test_mcf_step_gradcheck():
    """The implicit MCF step u = (M(X) + tau K(X))^-1 M(X) X differentiated
    end to end (assembly VJP, adjoint solve, solve VJP) against central
    differences of the GPU forward step, icosphere level 1."""
    print("[gradcheck] mcf_step", flush=True)
    X, F = meshgen.icosphere(1, 5e-2, 7)
    m = dgo.Mesh(torch.from_numpy(F).to(DEV), X.shape[0])
    Xd = torch.from_numpy(X).to(DEV).requires_grad_(True)
    assert torch.autograd.gradcheck(lambda x: dgo.mcf_step(m, x, 0.05, rtol=1e-14, max_iter=10000),
                                    (Xd,), eps=1e-6, atol=1e-7, rtol=1e-5)


def test_loss_central_differences_per_coordinate():
    """Every coordinate of the config-5 loss gradient on an icosphere of
    level 2 (162 vertices) against central differences (h = 1e-6) of the GPU
    loss. Error budget of a central difference: truncation h^2 / 6 times the
    third derivative, plus rounding of about eps |l| / h; the bar 1e-7 of
    max |g| covers both with a wide margin."""
    print("[fd] per coordinate, icosphere L2", flush=True)
    X, F = meshgen.icosphere(2, 1e-2, 8)
    m = dgo.Mesh(torch.from_numpy(F).to(DEV), X.shape[0])
    u = torch.from_numpy(meshgen.normal(1000, m.nV)).to(DEV)
    rows, cols = _pattern(m)
    Xd = torch.from_numpy(X).to(DEV)[None].clone().requires_grad_(True)
    _loss(m, Xd, u, rows, cols).sum().backward()
    g = Xd.grad[0].cpu().numpy().ravel()
    h = 1e-6
    n = X.size
    # all 2 n perturbed copies in one batched assembly
    P = np.repeat(X[None], 2 * n, 0).reshape(2 * n, -1)
    P[np.arange(n), np.arange(n)] += h
    P[n + np.arange(n), np.arange(n)] -= h
    with torch.no_grad():
        L = _loss(m, torch.from_numpy(P.reshape(2 * n, m.nV, 3)).to(DEV), u, rows, cols)
    fd = ((L[:n] - L[n:]) / (2 * h)).cpu().numpy()
    err = np.abs(fd - g).max() / np.abs(g).max()
    print(f"  max error {err:.2e} of max |g|", flush=True)
    assert err <= 1e-7
    # and the oracle's gradient on the same mesh
    _, go = oracle.loss_grad_tri(X, F, u.cpu().numpy())
    assert np.abs(g - go.ravel()).max() <= 1e-12 * np.abs(go).max()


def test_loss_directional_differences_cfg5_batch():
    """Config 5 at full size: for each of the 256 meshes, the derivative of
    its loss along a random unit direction by central differences (h = 1e-6,
    all 512 perturbed meshes in two batched assemblies) against <g, v>, at
    1e-7 of |g| |v| (the directional derivative's own scale)."""
    print("[fd] directional, 256 x icosphere L5", flush=True)
    B = 256
    X0, F = meshgen.icosphere(5)
    m = dgo.Mesh(torch.from_numpy(F).to(DEV), X0.shape[0])
    Xs = np.stack([meshgen.icosphere(5, 1e-2, s)[0] for s in range(B)])
    u = torch.from_numpy(meshgen.normal(1000, m.nV)).to(DEV)
    rows, cols = _pattern(m)
    Xd = torch.from_numpy(Xs).to(DEV).requires_grad_(True)
    _loss(m, Xd, u, rows, cols).sum().backward()
    G = Xd.grad.reshape(B, -1)
    V = torch.from_numpy(meshgen.normal(2000, Xs.size).reshape(B, -1)).to(DEV)
    V = V / V.norm(dim=1, keepdim=True)
    h = 1e-6
    with torch.no_grad():
        Xp = (Xd + h * V.reshape(Xs.shape)).contiguous()
        Xm = (Xd - h * V.reshape(Xs.shape)).contiguous()
        fd = (_loss(m, Xp, u, rows, cols) - _loss(m, Xm, u, rows, cols)) / (2 * h)
    dd = (G * V).sum(1)
    rel = ((fd - dd).abs() / (G.norm(dim=1) * V.norm(dim=1))).max().item()
    print(f"  max error {rel:.2e} of |g| |v|", flush=True)
    assert rel <= 1e-7
