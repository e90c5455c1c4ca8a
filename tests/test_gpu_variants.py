"""GPU parity of the operator variants against the FP64 oracle, through the
C ABI: the mixed-Voronoi lumped mass (extrinsic and intrinsic assembly; K is
unchanged by the option), the ARAP default clamp, the COO export of the
pattern (bit-exact) and the conformal Laplacian (bit-exact: its entries are
copies of K or +-1/2), including a 300 x 300 grid checked through the
similarity kernel of planar maps."""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

import meshgen
import oracle
from helpers import MESHES, RTOL

pytestmark = pytest.mark.gpu

import paper_2602_12105_amd as dgo  # noqa: E402  (no skip: a broken import fails the suite)
DEV = "cuda:0"
TRI = ["tri1", "disjoint", "fan", "fan40", "grid7", "grid64", "grid130fan", "ico3", "ico7"]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("no HIP device visible")
    import paper_2602_12105_amd._lib as L
    L.lib()  # the native library must load; there is no fallback
    yield


def _setup(name):
    X, F = MESHES[name]()
    return X, F, dgo.Mesh(torch.from_numpy(F).to(DEV), X.shape[0])


@pytest.mark.parametrize("name", TRI)
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_voronoi_mass_parity(name, dtype):
    print(f"[voronoi] {name} {dtype}", flush=True)
    X, F, m = _setup(name)
    td = torch.float64 if dtype == "f64" else torch.float32
    Xd = torch.from_numpy(X).to(DEV, td)
    Xr = Xd.double().cpu().numpy()
    K0, _ = dgo.assemble(m, Xd)
    K, M = dgo.assemble(m, Xd, mass="voronoi")
    assert torch.equal(K, K0)
    Mo = oracle.mass_voronoi(Xr, F)
    np.testing.assert_allclose(M.double().cpu().numpy(), Mo, rtol=RTOL[dtype], atol=0)
    # intrinsic: the same mass from the edge lengths
    EV = m.edges()[0].long()
    Ld = (Xd[EV[:, 0]] - Xd[EV[:, 1]]).norm(dim=1).contiguous()
    Ki, Mi = dgo.assemble_intrinsic(m, Ld, mass="voronoi")
    Ki0, _ = dgo.assemble_intrinsic(m, Ld)
    assert torch.equal(Ki, Ki0)
    tol = RTOL[dtype] if dtype == "f64" else 1e-4  # lengths rounded to FP32 before squaring
    np.testing.assert_allclose(Mi.double().cpu().numpy(), Mo, rtol=tol, atol=0)


def test_voronoi_options_and_errors():
    print("[voronoi] options", flush=True)
    X, F, m = _setup("ico3")
    Xd = torch.from_numpy(X).to(DEV)
    # batch and clamp combine with the option
    Xb = torch.stack([Xd, 1.5 * Xd])
    K, M = dgo.assemble(m, Xb, clamp_min=0.05, mass="voronoi")
    Ko = oracle.assemble(X, F, clamp_min=0.05)[0]
    np.testing.assert_allclose(K[0].cpu().numpy(), Ko, rtol=0, atol=1e-12 * np.abs(Ko).max())
    np.testing.assert_allclose(M[1].cpu().numpy(), 2.25 * oracle.mass_voronoi(X, F), rtol=1e-12)
    Xt, T, mt = _setup("cube3")
    with pytest.raises(dgo.DgoError) as e:
        dgo.assemble(mt, torch.from_numpy(Xt).to(DEV), mass="voronoi")
    assert e.value.status == "UNSUPPORTED"
    with pytest.raises(ValueError):
        dgo.assemble(m, Xd, mass="mixed")


def test_arap_default_clamp():
    print("[arap clamp]", flush=True)
    X, F, m = _setup("grid64")
    Xd = torch.from_numpy(X).to(DEV)
    Ka, Ma = dgo.arap_laplacian(m, Xd)
    Kc, Mc = dgo.assemble(m, Xd, clamp_min=1e-5)
    assert torch.equal(Ka, Kc) and torch.equal(Ma, Mc)
    Ko = oracle.assemble(X, F, clamp_min=1e-5)[0]
    np.testing.assert_allclose(Ka.cpu().numpy(), Ko, rtol=0, atol=1e-12 * np.abs(Ko).max())


@pytest.mark.parametrize("name", ["tri1", "tet1", "fan", "grid64", "ico7", "cube9"])
def test_coo_bit_exact(name):
    print(f"[coo] {name}", flush=True)
    X, E, m = _setup(name)
    EV, _, _ = oracle.edges(X.shape[0], E)
    rp, col = oracle.csr(X.shape[0], EV)
    rows, cols = [t.cpu().numpy() for t in m.coo()]
    np.testing.assert_array_equal(rows, oracle.csr_rows(rp))
    np.testing.assert_array_equal(cols, col)


@pytest.mark.parametrize("name", ["tri1", "tet1", "disjoint", "fan", "grid64", "ico7", "cube9",
                                  "cube64"])
def test_slot_map_bit_exact(name):
    print(f"[slots] {name}", flush=True)
    X, E, m = _setup(name)
    EV, _, _ = oracle.edges(X.shape[0], E)
    rp, col = oracle.csr(X.shape[0], EV)
    np.testing.assert_array_equal(m.slots().cpu().numpy(), oracle.slot_map(X.shape[0], E, rp, col))


def _dense_csr(rp, col, val, n):
    return sp.csr_matrix((val, col, rp), shape=(n, n)).toarray()


@pytest.mark.parametrize("name", ["tri1", "disjoint", "fan", "fan40", "grid7", "grid64", "ico3"])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_conformal_laplacian_bit_exact(name, dtype):
    print(f"[conformal] {name} {dtype}", flush=True)
    X, F, m = _setup(name)
    n = X.shape[0]
    td = torch.float64 if dtype == "f64" else torch.float32
    K, _ = dgo.assemble(m, torch.from_numpy(X).to(DEV, td))
    rp2, col2, v2 = dgo.conformal_laplacian(m, K)
    rp2, col2 = rp2.cpu().numpy(), col2.cpu().numpy()
    v2 = v2.double().cpu().numpy()
    assert rp2[-1] == v2.size == 2 * m.nnz + 4 * m.n_bfaces
    # sorted, unique columns per row
    for i in range(2 * n):
        c = col2[rp2[i]:rp2[i + 1]]
        assert (np.diff(c) > 0).all()
    rp, col = [t.cpu().numpy() for t in m.csr()]
    Lo = oracle.conformal_laplacian(F, n, K.double().cpu().numpy(), rp, col)
    np.testing.assert_array_equal(_dense_csr(rp2, col2, v2, 2 * n), Lo)
    # values only: the same numbers
    assert torch.equal(dgo.conformal_laplacian(m, K, pattern=False).double().cpu(),
                       torch.from_numpy(v2))


def test_conformal_laplacian_large_planar_kernel():
    print("[conformal] 300 x 300 grid", flush=True)
    X, F = meshgen.grid2d(300, 0.2, 4)
    n = X.shape[0]
    m = dgo.Mesh(torch.from_numpy(F).to(DEV), n)
    K, _ = dgo.assemble(m, torch.from_numpy(X).to(DEV))
    rp2, col2, v2 = [t.cpu().numpy() for t in dgo.conformal_laplacian(m, K)]
    L = sp.csr_matrix((v2, col2, rp2), shape=(2 * n, 2 * n))
    assert abs(L - L.T).max() == 0
    x, y = X[:, 0], X[:, 1]
    for u in (np.concatenate([x, y]), np.concatenate([-y, x])):
        r = L @ u
        assert np.abs(r).max() <= 1e-11, np.abs(r).max()
    # the boundary block carries +-1/2 on the 4 (n - 1) boundary edges
    assert m.n_bfaces == 4 * 299
    off = L[:n, n:]
    assert off.nnz == 2 * m.n_bfaces and set(np.unique(off.data)) == {-0.5, 0.5}
