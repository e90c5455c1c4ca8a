"""GPU parity of the intrinsic assembly (edge lengths in) and of the per-face
gradient G and divergence D against the FP64 oracle, through the C ABI.

Floats use the row-scaled metric of the other parity tests: K entries within
rtol times the row's largest |K_ij|, M within rtol relative, G and D within
rtol times the scale of the exact sum (sum of |terms|), rtol = 1e-12 (FP64) or
1e-5 (FP32, the oracle in FP64 on the same FP32-rounded inputs). The meshes
span one triangle, a fan with a long row, jittered grids (several row blocks
and a ragged last one), the icosphere of the FP64/FP32 solve workload at full
size (level 7), and a tetrahedral mesh for the unsupported path.
"""
import numpy as np
import pytest
import torch

import meshgen
import oracle
from helpers import MESHES, RTOL, assert_csr_close

pytestmark = pytest.mark.gpu

import paper_2602_12105_amd as dgo  # noqa: E402  (no skip: a broken import fails the suite)
DEV = "cuda:0"
TRI = ["tri1", "fan", "fan40", "grid7", "grid64", "grid130fan", "ico3", "ico7", "fan254"]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("no HIP device visible")
    import paper_2602_12105_amd._lib as L
    L.lib()  # the native library must load; there is no fallback
    yield


def _setup(name):
    X, F = MESHES[name]()
    m = dgo.Mesh(torch.from_numpy(F).to(DEV), X.shape[0])
    return X, F, m


def _lengths(X, F):
    EV, _, _ = oracle.edges(X.shape[0], F)
    return np.linalg.norm(X[EV[:, 0]] - X[EV[:, 1]], axis=1)


def _symmetric(K, rp, col):
    rows = np.repeat(np.arange(rp.size - 1), np.diff(rp))
    order = np.lexsort((rows, col))  # (col, row) order = transposed slots
    np.testing.assert_array_equal(K[order], K)


@pytest.mark.parametrize("name", TRI)
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_intrinsic_assembly_parity(name, dtype):
    print(f"[intrinsic] {name} {dtype}", flush=True)
    X, F, m = _setup(name)
    td = torch.float64 if dtype == "f64" else torch.float32
    Ld = torch.from_numpy(_lengths(X, F)).to(DEV, td)
    K, M = dgo.assemble_intrinsic(m, Ld, check_degenerate=True)
    K, M = K.double().cpu().numpy(), M.double().cpu().numpy()
    rp, col = [t.cpu().numpy() for t in m.csr()]
    Ko, Mo = oracle.assemble_intrinsic(F, X.shape[0], Ld.double().cpu().numpy(), rp, col)
    assert_csr_close(K, Ko, rp, RTOL[dtype])
    np.testing.assert_allclose(M, Mo, rtol=RTOL[dtype], atol=0)
    _symmetric(K, rp, col)


def test_intrinsic_matches_extrinsic_batch_and_clamp():
    print("[intrinsic] batch, clamp, extrinsic", flush=True)
    X, F, m = _setup("grid64")
    L0 = _lengths(X, F)
    Lb = np.stack([L0, 2.5 * L0, L0 * (1 + 0.01 * meshgen.uniform(3, L0.size))])
    Ld = torch.from_numpy(Lb).to(DEV)
    K, M = dgo.assemble_intrinsic(m, Ld)
    rp, col = [t.cpu().numpy() for t in m.csr()]
    for b in range(3):
        Ko, Mo = oracle.assemble_intrinsic(F, X.shape[0], Lb[b], rp, col)
        assert_csr_close(K[b].cpu().numpy(), Ko, rp, RTOL["f64"], f"K[{b}]")
        np.testing.assert_allclose(M[b].cpu().numpy(), Mo, rtol=RTOL["f64"])
    # the extrinsic assembly of the same positions agrees to rounding
    Ke, Me = dgo.assemble(m, torch.from_numpy(X).to(DEV))
    assert_csr_close(K[0].cpu().numpy(), Ke.cpu().numpy(), rp, 1e-12, "K vs extrinsic")
    # the weights are scale invariant: the second batch entry has the same K
    assert_csr_close(K[1].cpu().numpy(), K[0].cpu().numpy(), rp, 1e-13, "K scaled")
    # clamp of the summed weights, as in the extrinsic path
    Kc, _ = dgo.assemble_intrinsic(m, Ld[0].contiguous(), clamp_min=0.05)
    Ko = oracle.assemble(X, F, rp, col, clamp_min=0.05)[0]
    assert_csr_close(Kc.cpu().numpy(), Ko, rp, 1e-12, "K clamped")
    # deterministic
    K2, M2 = dgo.assemble_intrinsic(m, Ld)
    assert torch.equal(K, K2) and torch.equal(M, M2)


def test_intrinsic_errors():
    print("[intrinsic] errors", flush=True)
    F = np.array([[0, 1, 2], [1, 3, 2]], np.int32)
    m = dgo.Mesh(torch.from_numpy(F).to(DEV), 4)
    L = torch.tensor([1.0, 1.0, 1.0, 1.0, 2.5], dtype=torch.float64, device=DEV)
    with pytest.raises(dgo.DgoError) as e:
        dgo.assemble_intrinsic(m, L, check_degenerate=True)
    assert e.value.status == "DEGENERATE"
    with pytest.raises(ValueError):
        dgo.assemble_intrinsic(m, L[:4].contiguous())
    X, E, mt = _setup("cube3")
    with pytest.raises(dgo.DgoError) as e:
        dgo.assemble_intrinsic(mt, torch.ones(mt.nE, dtype=torch.float64, device=DEV))
    assert e.value.status == "UNSUPPORTED"
    with pytest.raises(dgo.DgoError) as e:
        dgo.face_gradient(mt, torch.from_numpy(X).to(DEV), torch.ones(X.shape[0], dtype=torch.float64,
                                                                        device=DEV))
    assert e.value.status == "UNSUPPORTED"


def _max_grad(X, F):
    """max_j |grad phi_j| per face (= max_j |e_j| / |n|, since e_j is normal to n)."""
    n = np.cross(X[F[:, 1]] - X[F[:, 0]], X[F[:, 2]] - X[F[:, 0]])
    e = np.stack([X[F[:, 2]] - X[F[:, 1]], X[F[:, 0]] - X[F[:, 2]], X[F[:, 1]] - X[F[:, 0]]])
    return np.linalg.norm(e, axis=2).max(axis=0) / np.linalg.norm(n, axis=1)


def _grad_scale(X, F, u):
    """sum_j |u_j| max_j |grad phi_j| per field and face, (k, 1, nF): the
    error scale of G."""
    return np.abs(u)[F].sum(axis=1).T[:, None, :] * _max_grad(X, F)[None, None, :]


def _div_scale(X, F, y):
    """sum over the vertex's faces of A_f max_j |grad phi_j| |y_f|, (nV, k):
    the error scale of D."""
    A = 0.5 * np.linalg.norm(np.cross(X[F[:, 1]] - X[F[:, 0]], X[F[:, 2]] - X[F[:, 0]]), axis=1)
    w = (A * _max_grad(X, F))[None, :] * np.linalg.norm(y, axis=1)  # (k, nF)
    sc = np.zeros((X.shape[0], y.shape[0]))
    for j in range(3):
        np.add.at(sc, F[:, j], w.T)
    return sc


@pytest.mark.parametrize("name", TRI)
@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("k", [1, 3])
def test_face_gradient_and_divergence_parity(name, dtype, k):
    print(f"[grad-div] {name} {dtype} k={k}", flush=True)
    X, F, m = _setup(name)
    nV, nF = X.shape[0], F.shape[0]
    td = torch.float64 if dtype == "f64" else torch.float32
    Xd = torch.from_numpy(X).to(DEV, td)
    u = meshgen.normal(21, nV * k).reshape(nV, k)
    ud = torch.from_numpy(u).to(DEV, td)
    y = meshgen.normal(22, k * 3 * nF).reshape(k, 3, nF)
    yd = torch.from_numpy(y).to(DEV, td)
    Xr, ur, yr = [t.double().cpu().numpy() for t in (Xd, ud, yd)]
    g = dgo.face_gradient(m, Xd, ud).double().cpu().numpy()
    go = oracle.face_gradient(Xr, F, ur)
    assert np.all(np.abs(g - go) <= RTOL[dtype] * _grad_scale(Xr, F, ur)), np.abs(g - go).max()
    d = dgo.face_divergence(m, Xd, yd).double().cpu().numpy()
    do = oracle.face_divergence(Xr, F, yr)
    assert np.all(np.abs(d - do) <= RTOL[dtype] * _div_scale(Xr, F, yr)), np.abs(d - do).max()


def test_div_grad_is_stiffness_full_size():
    print("[grad-div] D G u = K u at icosphere level 7", flush=True)
    X, F, m = _setup("ico7")
    Xd = torch.from_numpy(X).to(DEV)
    ud = torch.from_numpy(meshgen.normal(31, X.shape[0] * 4).reshape(-1, 4)).to(DEV)
    K, M = dgo.assemble(m, Xd)
    Ku = dgo.spmv(m, 0.0, M, 1.0, K, ud)
    DGu = dgo.face_divergence(m, Xd, dgo.face_gradient(m, Xd, ud))
    err = (DGu - Ku).abs().max().item()
    assert err <= 1e-11 * Ku.abs().max().item(), err
    # single field in the (3, nF) layout of the geodesic loop
    g1 = dgo.face_gradient(m, Xd, ud[:, 0].contiguous())
    assert g1.shape == (1, 3, F.shape[0])
    d1 = dgo.face_divergence(m, Xd, g1[0].contiguous())
    assert d1.shape == (X.shape[0],)
    assert torch.allclose(d1, DGu[:, 0], rtol=0, atol=1e-11 * Ku.abs().max().item())


def test_face_ops_wide_k():
    print("[grad-div] k = 64", flush=True)
    X, F, m = _setup("grid7")
    Xd = torch.from_numpy(X).to(DEV)
    u = meshgen.normal(41, X.shape[0] * 64).reshape(-1, 64)
    g = dgo.face_gradient(m, Xd, torch.from_numpy(u).to(DEV)).cpu().numpy()
    np.testing.assert_allclose(g, oracle.face_gradient(X, F, u), rtol=0,
                               atol=1e-12 * np.abs(u).max() * _max_grad(X, F).max() * 3)
    with pytest.raises(dgo.DgoError):
        dgo.face_gradient(m, Xd, torch.zeros((X.shape[0], 65), dtype=torch.float64, device=DEV))
