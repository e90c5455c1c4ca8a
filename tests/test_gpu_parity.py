"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Integers (edges, element->edge map, signs, CSR, boundary) must match bit for
bit. Floats use the row-scaled metric: |got - ref| <= rtol * max_j |ref_ij|
over the row, rtol = 1e-12 (FP64) or 1e-5 (FP32); in FP32 the oracle runs in
FP64 on the same FP32-rounded positions.
"""
import numpy as np
import scipy.sparse as sp
import pytest
import torch

import meshgen
import oracle
from helpers import MESHES, RTOL, assert_cols_close, assert_csr_close, spmv_scale

pytestmark = pytest.mark.gpu

import paper_2602_12105_amd as dgo  # noqa: E402  (no skip: a broken import fails the suite)
DEV = "cuda:0"


def _mesh(name):
    X, E = MESHES[name]()
    E_d = torch.from_numpy(E).to(DEV)
    return X, E, dgo.Mesh(E_d, X.shape[0])


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("no HIP device visible")
    import paper_2602_12105_amd._lib as L
    L.lib()  # the native library must load; there is no fallback
    yield


@pytest.mark.parametrize("name", ["tri1", "tet1", "disjoint", "fan", "grid7", "grid64", "ico3",
                                  "ico7", "cube3", "cube9", "cube64"])
def test_topology_bit_exact(name):
    print(f"[topology] {name}", flush=True)
    X, E, m = _mesh(name)
    nV = X.shape[0]
    EV, ee, es = oracle.edges(nV, E)
    rp, col = oracle.csr(nV, EV)
    mask, nb = oracle.boundary(nV, E)
    gEV, gee, ges = [t.cpu().numpy() for t in m.edges()]
    grp, gcol = [t.cpu().numpy() for t in m.csr()]
    assert m.nE == EV.shape[0] and m.nnz == col.size and m.n_bfaces == nb
    np.testing.assert_array_equal(gEV, EV)
    np.testing.assert_array_equal(gee, ee)
    np.testing.assert_array_equal(ges, es)
    np.testing.assert_array_equal(grp, rp)
    np.testing.assert_array_equal(gcol, col)
    np.testing.assert_array_equal(m.boundary().cpu().numpy(), mask)
    assert m.n_boundary == int(mask.sum())


def test_mesh_errors():
    F = torch.tensor([[0, 1, 2], [2, 1, 7]], dtype=torch.int32, device=DEV)
    with pytest.raises(dgo.DgoError) as e:
        dgo.Mesh(F, 5)
    assert e.value.status == "INDEX_RANGE"
    F = torch.tensor([[0, 1, 1]], dtype=torch.int32, device=DEV)
    with pytest.raises(dgo.DgoError) as e:
        dgo.Mesh(F, 5)
    assert e.value.status == "INVALID_ARG"
    # degree above 254 is reported as unsupported: a closed fan whose centre
    # has degree 255 (degree 254 is covered by the parity tests), and an open
    # fan of 299
    F = torch.tensor([[0, 1 + i, 1 + (i + 1) % 255] for i in range(255)], dtype=torch.int32, device=DEV)
    with pytest.raises(dgo.DgoError) as e:
        dgo.Mesh(F, 256)
    assert e.value.status == "UNSUPPORTED"
    n = 300
    F = torch.tensor([[0, i, i + 1] for i in range(1, n)], dtype=torch.int32, device=DEV)
    with pytest.raises(dgo.DgoError) as e:
        dgo.Mesh(F, n + 1)
    assert e.value.status == "UNSUPPORTED"
    # a vertex in more elements than any supported degree allows is rejected
    # before the per-vertex sorts run (their cost is quadratic in that count)
    n = 5000
    F = torch.tensor([[0, i, i + 1] for i in range(1, n)], dtype=torch.int32, device=DEV)
    with pytest.raises(dgo.DgoError) as e:
        dgo.Mesh(F, n + 1)
    assert e.value.status == "UNSUPPORTED" and "elements" in str(e.value)


def _assemble_check(name, dtype, batch=1, clamp=None):
    X, E, m = _mesh(name)
    nV = X.shape[0]
    Xs = [X]
    for b in range(1, batch):
        Xs.append(X * (1.0 + 0.01 * meshgen.normal(500 + b, nV))[:, None])
    Xb = np.stack(Xs)
    td = torch.float64 if dtype == "f64" else torch.float32
    Xd = torch.from_numpy(Xb).to(DEV, td)
    Xref = Xd.double().cpu().numpy()  # FP32-rounded positions for the FP32 case
    K, M = dgo.assemble(m, Xd, clamp_min=clamp, check_degenerate=True)
    K = K.double().cpu().numpy()
    M = M.double().cpu().numpy()
    rp, col = [t.cpu().numpy() for t in m.csr()]
    for b in range(batch):
        Ko, Mo, rpo, colo = oracle.assemble(Xref[b], E, rp, col, clamp_min=clamp)
        assert_csr_close(K[b], Ko, rp, RTOL[dtype], f"K[{b}]")
        np.testing.assert_allclose(M[b], Mo, rtol=RTOL[dtype], atol=0)
        # bitwise symmetry: K_ij == K_ji
        rows = np.repeat(np.arange(nV), np.diff(rp))
        key = {(int(i), int(j)): v for i, j, v in zip(rows[:5000], col[:5000], K[b][:5000])}
        for (i, j), v in key.items():
            if (j, i) in key:
                assert v == key[(j, i)]
    return m, Xd, K


@pytest.mark.parametrize("name", ["tri1", "tet1", "disjoint", "fan", "grid7", "grid64", "ico3",
                                  "ico7", "cube3", "cube9", "cube64", "fan254", "ico6fan254"])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_assemble_parity(name, dtype):
    print(f"[assemble] {name} {dtype}", flush=True)
    _assemble_check(name, dtype)


@pytest.mark.parametrize("name", ["ico5", "cube9"])
def test_assemble_batch_and_clamp(name):
    print(f"[assemble-batch] {name}", flush=True)
    _assemble_check(name, "f64", batch=3)
    _assemble_check(name, "f64", batch=2, clamp=0.05 if name == "ico5" else 0.001)


def test_assemble_symmetry_full_and_determinism():
    X, E, m = _mesh("ico7")
    Xd = torch.from_numpy(X).to(DEV)
    K1, M1 = dgo.assemble(m, Xd)
    K2, M2 = dgo.assemble(m, Xd)
    assert torch.equal(K1, K2) and torch.equal(M1, M2)
    rp, col = [t.cpu().numpy() for t in m.csr()]
    K = K1.cpu().numpy()
    rows = np.repeat(np.arange(X.shape[0]), np.diff(rp))
    # mirror slot of (i, j) by searching row j
    order = np.lexsort((rows, col))  # sorted by (col, row) -> transposed order
    np.testing.assert_array_equal(K[order], K)


@pytest.mark.parametrize("dim", [2, 3])
def test_empty_element_set(dim):
    """Vertices and no elements: no edges, a diagonal-only pattern, K = 0 and
    M = 0, a zero operator; for triangles also the intrinsic assembly from
    no lengths, the VJP, and G and D on empty face fields (D = 0)."""
    print(f"[empty] dim={dim}", flush=True)
    nV = 5
    m = dgo.Mesh(torch.empty((0, dim + 1), dtype=torch.int32, device=DEV), nV)
    assert (m.n_elem, m.nE, m.nnz, m.max_row) == (0, 0, nV, 1)
    rp, col = [t.cpu().numpy() for t in m.csr()]
    np.testing.assert_array_equal(rp, np.arange(nV + 1))
    np.testing.assert_array_equal(col, np.arange(nV))
    EV, ee, _ = m.edges()
    assert EV.shape == (0, 2) and ee.shape == (0, m.nl)
    X = torch.from_numpy(meshgen.normal(3, nV * 3).reshape(nV, 3)).to(DEV)
    for td in (torch.float64, torch.float32):
        Xt = X.to(td)
        K, M = dgo.assemble(m, Xt)
        assert K.shape == (nV,) and M.shape == (nV,) and not K.any() and not M.any()
        x = torch.ones(nV, 2, dtype=td, device=DEV)
        assert not dgo.spmv(m, 0.7, M, 1.3, K, x).any()
        if dim == 2:
            Ki, Mi = dgo.assemble_intrinsic(m, torch.empty(0, dtype=td, device=DEV))
            assert not Ki.any() and not Mi.any()
            assert not dgo.assemble_vjp(m, Xt, torch.ones_like(K), torch.ones_like(M)).any()
            g = dgo.face_gradient(m, Xt, x)
            assert g.shape == (2, 3, 0)
            d = dgo.face_divergence(m, Xt, g)
            assert d.shape == (nV, 2) and not d.any()


def test_degenerate_reported():
    X = np.array([[0, 0, 0], [1, 0, 0], [2, 0, 0], [0, 1, 0]], float)
    F = torch.tensor([[0, 1, 2], [0, 1, 3]], dtype=torch.int32, device=DEV)
    m = dgo.Mesh(F, 4)
    with pytest.raises(dgo.DgoError) as e:
        dgo.assemble(m, torch.from_numpy(X).to(DEV), check_degenerate=True)
    assert e.value.status == "DEGENERATE"


@pytest.mark.parametrize("name", ["grid64", "ico5", "cube9"])
@pytest.mark.parametrize("k", [1, 2, 3, 8, 16])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_spmv_parity(name, k, dtype):
    print(f"[spmv] {name} k={k} {dtype}", flush=True)
    X, E, m = _mesh(name)
    td = torch.float64 if dtype == "f64" else torch.float32
    K, M = dgo.assemble(m, torch.from_numpy(X).to(DEV, td))
    x = (meshgen.uniform(1, X.shape[0] * k).reshape(-1, k) * 2 - 1)
    xd = torch.from_numpy(x).to(DEV, td)
    y = dgo.spmv(m, 0.7, M, 1.3, K, xd).double().cpu().numpy()
    rp, col = [t.cpu().numpy() for t in m.csr()]
    Kh, Mh, xh = K.double().cpu().numpy(), M.double().cpu().numpy(), xd.double().cpu().numpy()
    yo = oracle.spmv(rp, col, 0.7, Mh, 1.3, Kh, xh).reshape(y.shape)
    sc = spmv_scale(rp, col, 0.7, Mh, 1.3, Kh, xh).reshape(y.shape)
    assert np.all(np.abs(y - yo) <= RTOL[dtype] * sc)


@pytest.mark.parametrize("k", [1, 8])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_spmv_parity_breadth_first_rows(k, dtype):
    """Meshes of 16384 vertices or more are swept in breadth-first row order."""
    test_spmv_parity("ico7", k, dtype)


@pytest.mark.parametrize("name", ["fan40", "grid130fan", "ico6fan", "fan254", "ico6fan254"])
@pytest.mark.parametrize("k", [1, 8])
def test_spmv_parity_long_rows(name, k):
    """Rows of more than 16 entries (a fan centre)."""
    test_spmv_parity(name, k, "f64")


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_spmv_parity_tet_rows_full_size(dtype):
    """One column on the Kuhn cube 64^3 (rows of up to 15 entries, 16 lanes
    per row in the one-column pipeline), at the size of the Dirichlet workload."""
    test_spmv_parity("cube64", 1, dtype)


@pytest.mark.parametrize("name", ["ico3", "cube9"])
@pytest.mark.parametrize("k", [1, 4, 8])
def test_spmv_batch(name, k):
    X, E, m = _mesh(name)
    Xb = torch.from_numpy(np.stack([X, 1.1 * X])).to(DEV)
    K, M = dgo.assemble(m, Xb)
    x = torch.from_numpy(meshgen.normal(3, 2 * X.shape[0] * k).reshape(2, -1, k)).to(DEV)
    y = dgo.spmv(m, 1.0, M, 1e-3, K, x)
    for b in range(2):
        yb = dgo.spmv(m, 1.0, M[b].contiguous(), 1e-3, K[b].contiguous(), x[b].contiguous())
        assert torch.equal(yb, y[b])


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("k", [1, 8])
def test_spmv_beta_zero_is_the_diagonal(dtype, k):
    """beta = 0 applies alpha M without reading K: bit for bit (alpha M_i) x_i,
    in a batch too, and the oracle's product to rounding."""
    print(f"[spmv-diag] ico5 k={k} {dtype}", flush=True)
    X, E, m = _mesh("ico5")
    td = torch.float64 if dtype == "f64" else torch.float32
    Xb = torch.from_numpy(np.stack([X, 1.1 * X])).to(DEV, td)
    K, M = dgo.assemble(m, Xb)
    x = torch.from_numpy(meshgen.normal(7, 2 * X.shape[0] * k).reshape(2, -1, k)).to(DEV, td)
    y = dgo.spmv(m, 0.7, M, 0.0, K, x)
    assert torch.equal(y, (0.7 * M)[:, :, None] * x)
    rp, col = [t.cpu().numpy() for t in m.csr()]
    yo = oracle.spmv(rp, col, 0.7, M[1].double().cpu().numpy(), 0.0, K[1].double().cpu().numpy(),
                     x[1].double().cpu().numpy()).reshape(-1, k)
    assert np.allclose(y[1].double().cpu().numpy(), yo, rtol=RTOL[dtype], atol=0.0)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_spmv_k8_unaligned(dtype):
    """Eight columns at an address that is not 16-byte aligned take the
    per-column gathers instead of the 16-byte ones; both match the oracle."""
    print(f"[spmv-unaligned] ico5 k=8 {dtype}", flush=True)
    X, E, m = _mesh("ico5")
    td = torch.float64 if dtype == "f64" else torch.float32
    K, M = dgo.assemble(m, torch.from_numpy(X).to(DEV, td))
    x = meshgen.uniform(2, X.shape[0] * 8).reshape(-1, 8) * 2 - 1
    buf = torch.empty(X.shape[0] * 8 + 1, dtype=td, device=DEV)
    xu = buf[1:].view(-1, 8)
    xu.copy_(torch.from_numpy(x).to(DEV, td))
    assert xu.data_ptr() % 16 != 0
    ya = dgo.spmv(m, 0.7, M, 1.3, K, xu.clone()).double().cpu().numpy()
    yu = dgo.spmv(m, 0.7, M, 1.3, K, xu).double().cpu().numpy()
    rp, col = [t.cpu().numpy() for t in m.csr()]
    Kh, Mh, xh = K.double().cpu().numpy(), M.double().cpu().numpy(), xu.double().cpu().numpy()
    yo = oracle.spmv(rp, col, 0.7, Mh, 1.3, Kh, xh).reshape(ya.shape)
    sc = spmv_scale(rp, col, 0.7, Mh, 1.3, Kh, xh).reshape(ya.shape)
    assert np.all(np.abs(ya - yo) <= RTOL[dtype] * sc)
    assert np.all(np.abs(yu - yo) <= RTOL[dtype] * sc)


def _cfg2_system(level, k, dtype, seed=1):
    X, F = meshgen.icosphere(level, 1e-3, 0)
    m = dgo.Mesh(torch.from_numpy(F).to(DEV), X.shape[0])
    td = torch.float64 if dtype == "f64" else torch.float32
    K, M = dgo.assemble(m, torch.from_numpy(X).to(DEV, td))
    f = torch.from_numpy(meshgen.normal(seed, X.shape[0] * k).reshape(-1, k)).to(DEV, td)
    b = (M[:, None] * f).contiguous()
    return m, K, M, b


def _oracle_same_iters(rp, col, alpha, Mh, beta, Kh, bh, iters, mask=None, g=None):
    """The oracle's PCG run column by column for exactly the iteration count
    the GPU reported for that column: the same iterate on both sides, so a
    converged solve is compared at the element-wise bar, not at the solver
    tolerance."""
    bh = bh.reshape(bh.shape[0], -1)
    out = np.empty_like(bh)
    for c in range(bh.shape[1]):
        gc = None if g is None else np.ascontiguousarray(g.reshape(bh.shape[0], -1)[:, c])
        uo, its, _ = oracle.pcg(rp, col, alpha, Mh, beta, Kh, np.ascontiguousarray(bh[:, c]),
                                mask=mask, g=gc, rtol=0.0, max_iter=int(iters[c]))
        assert int(its[0]) == int(iters[c])
        out[:, c] = uo
    return out


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("iters", [1, 30, 31, 60])
def test_pcg_fixed_iterations_match_oracle(dtype, iters):
    """The same iteration count on both sides: iterates agree element by
    element at the stated bar (odd and even counts: x takes the steps in
    pairs)."""
    print(f"[pcg-fixed] {dtype} {iters}", flush=True)
    m, K, M, b = _cfg2_system(5, 8, dtype)
    u, rep = dgo.pcg(m, 1.0, M, 1e-3, K, b, rtol=0.0, max_iter=iters, fixed_iters=True)
    assert rep["iters"] == [iters] * 8
    rp, col = [t.cpu().numpy() for t in m.csr()]
    uo, its, rr = oracle.pcg(rp, col, 1.0, M.double().cpu().numpy(), 1e-3,
                             K.double().cpu().numpy(), b.double().cpu().numpy(), rtol=0.0,
                             max_iter=iters)
    w = assert_cols_close(u.double().cpu().numpy(), uo, RTOL[dtype])
    print(f"  worst column-scaled error {w:.2e}", flush=True)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_pcg_interleaved_tiles_match_oracle(dtype):
    """Icosphere L8 with 8 columns: an XCD's share of the gathered vector
    (655,362 rows x 8 values / 8 XCDs) exceeds 2 MB, so the PCG kernels that
    gather walk tiles interleaved over each XCD's workgroups. Fixed iteration
    count, element by element against the oracle."""
    print(f"[pcg-interleaved] ico8 {dtype}", flush=True)
    m, K, M, b = _cfg2_system(8, 8, dtype, seed=6)
    assert m.nV * 8 * (8 if dtype == "f64" else 4) // 8 > 2 * 1024 * 1024
    u, rep = dgo.pcg(m, 1.0, M, 1e-3, K, b, rtol=0.0, max_iter=20, fixed_iters=True)
    assert rep["iters"] == [20] * 8
    rp, col = [t.cpu().numpy() for t in m.csr()]
    uo, _, _ = oracle.pcg(rp, col, 1.0, M.double().cpu().numpy(), 1e-3, K.double().cpu().numpy(),
                          b.double().cpu().numpy(), rtol=0.0, max_iter=20)
    w = assert_cols_close(u.double().cpu().numpy(), uo, RTOL[dtype])
    print(f"  worst column-scaled error {w:.2e}", flush=True)
    # the 8-column SpMM past the L2 (persistent, interleaved tiles)
    y = dgo.spmv(m, 0.7, M, 1.3, K, b).double().cpu().numpy()
    Kh, Mh, bh = K.double().cpu().numpy(), M.double().cpu().numpy(), b.double().cpu().numpy()
    yo = oracle.spmv(rp, col, 0.7, Mh, 1.3, Kh, bh).reshape(y.shape)
    sc = spmv_scale(rp, col, 0.7, Mh, 1.3, Kh, bh).reshape(y.shape)
    assert np.all(np.abs(y - yo) <= RTOL[dtype] * sc)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("k", [13, 16])
def test_pcg_k13_match_oracle(dtype, k):
    """13 or 16 columns (lane groups of 16 over padded rows of 7 entries: the
    gather chunk past the row's end is skipped; with 16, the 16-byte gathers),
    fixed iteration count, L6 (breadth-first row order)."""
    print(f"[pcg-k{k}] ico6 {dtype}", flush=True)
    m, K, M, b = _cfg2_system(6, k, dtype, seed=4)
    u, rep = dgo.pcg(m, 1.0, M, 1e-3, K, b, rtol=0.0, max_iter=25, fixed_iters=True)
    assert rep["iters"] == [25] * k
    rp, col = [t.cpu().numpy() for t in m.csr()]
    uo, _, _ = oracle.pcg(rp, col, 1.0, M.double().cpu().numpy(), 1e-3, K.double().cpu().numpy(),
                          b.double().cpu().numpy(), rtol=0.0, max_iter=25)
    assert_cols_close(u.double().cpu().numpy(), uo, RTOL[dtype])
    assert max(rep["true_relres"]) < 1.0


@pytest.mark.parametrize("name", ["fan40", "grid130fan", "ico6fan", "fan254"])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_pcg_long_rows_match_oracle(name, dtype):
    """Meshes with a row of more than 16 entries iterate over CSR rows (in
    natural order for fan40 and grid130fan, in breadth-first order for
    ico6fan) instead of the padded rows the other tests use."""
    print(f"[pcg-long-rows] {name} {dtype}", flush=True)
    X, E, m = _mesh(name)
    td = torch.float64 if dtype == "f64" else torch.float32
    K, M = dgo.assemble(m, torch.from_numpy(X).to(DEV, td))
    f = torch.from_numpy(meshgen.normal(5, X.shape[0] * 3).reshape(-1, 3)).to(DEV, td)
    b = (M[:, None] * f).contiguous()
    u, rep = dgo.pcg(m, 1.0, M, 1e-3, K, b, rtol=0.0, max_iter=30, fixed_iters=True)
    assert rep["iters"] == [30] * 3
    rp, col = [t.cpu().numpy() for t in m.csr()]
    uo, _, _ = oracle.pcg(rp, col, 1.0, M.double().cpu().numpy(), 1e-3, K.double().cpu().numpy(),
                          b.double().cpu().numpy(), rtol=0.0, max_iter=30)
    assert_cols_close(u.double().cpu().numpy(), uo, RTOL[dtype])


def test_pcg_converges_cfg2_f64():
    """Config 2 at full size (icosphere L7, 8 right-hand sides, rtol 1e-8):
    every column stops within one iteration of the oracle's own stop, and
    the solution equals the oracle's iterate of the same count at 1e-12."""
    print("[pcg] icosphere L7 k=8 f64", flush=True)
    m, K, M, b = _cfg2_system(7, 8, "f64")
    u, rep = dgo.pcg(m, 1.0, M, 1e-3, K, b, rtol=1e-8, max_iter=500)
    assert rep["converged_all"], rep
    assert max(rep["true_relres"]) <= 2e-8
    rp, col = [t.cpu().numpy() for t in m.csr()]
    Kh, Mh, bh = K.cpu().numpy(), M.cpu().numpy(), b.cpu().numpy()
    uo, its, rr = oracle.pcg(rp, col, 1.0, Mh, 1e-3, Kh, bh, rtol=1e-8, max_iter=500)
    assert all(abs(a - o) <= 1 for a, o in zip(rep["iters"], its)), (rep["iters"], its)
    ref = _oracle_same_iters(rp, col, 1.0, Mh, 1e-3, Kh, bh, rep["iters"])
    w = assert_cols_close(u.cpu().numpy(), ref, RTOL["f64"])
    print(f"  worst column-scaled error {w:.2e}", flush=True)


@pytest.mark.parametrize("level", [6, 7])
def test_pcg_cfg2_f32_accuracy(level):
    """FP32 storage and SpMV, FP64 dots, stagnation stop: the solution is
    within 1e-5 (element by element, column-scaled) of the oracle's tight
    FP64 solution of the same FP32-rounded system; level 7 is config 2's
    full size."""
    print(f"[pcg] icosphere L{level} k=8 f32", flush=True)
    m, K, M, b = _cfg2_system(level, 8, "f32")
    u, rep = dgo.pcg(m, 1.0, M, 1e-3, K, b, rtol=1e-8, max_iter=1000, stall_iters=20)
    rp, col = [t.cpu().numpy() for t in m.csr()]
    uo, _, _ = oracle.pcg(rp, col, 1.0, M.double().cpu().numpy(), 1e-3, K.double().cpu().numpy(),
                          b.double().cpu().numpy(), rtol=1e-14, max_iter=5000)
    w = assert_cols_close(u.double().cpu().numpy(), uo, RTOL["f32"])
    print(f"  worst column-scaled error {w:.2e}; iterations {rep['iters']}", flush=True)


def _cube_problem(n, dtype):
    """Config 3's Dirichlet Poisson problem (manufactured solution
    sin(pi x) sin(pi y) sin(pi z), its values on the boundary, source
    3 pi^2 u*, b = M f) on the jittered Kuhn cube with n^3 vertices."""
    X, T = meshgen.cube_tets(n, 0.15, 0)
    m = dgo.Mesh(torch.from_numpy(T).to(DEV), X.shape[0])
    td = torch.float64 if dtype == "f64" else torch.float32
    K, M = dgo.assemble(m, torch.from_numpy(X).to(DEV, td))
    mask = m.boundary()
    us = np.sin(np.pi * X[:, 0]) * np.sin(np.pi * X[:, 1]) * np.sin(np.pi * X[:, 2])
    g = torch.from_numpy(us).to(DEV, td)
    b = (M * torch.from_numpy(3 * np.pi ** 2 * us).to(DEV, td)).contiguous()
    return m, K, M, mask, g, b


@pytest.mark.parametrize("n", [17, 26, 64])
def test_pcg_dirichlet_cube_f64(n):
    """Config 3 in FP64 (n = 64 is its full size, 262,144 vertices): the solve
    to rtol 1e-8 equals the oracle's iterate of the same count at 1e-12, and
    the solve to 1e-14 equals the oracle's tight solution at 1e-12."""
    print(f"[pcg-dirichlet] cube{n} f64", flush=True)
    m, K, M, mask, g, b = _cube_problem(n, "f64")
    rp, col = [t.cpu().numpy() for t in m.csr()]
    Kh, Mh, bh, gh, mh = (t.cpu().numpy() for t in (K, M, b, g, mask))
    u, rep = dgo.pcg(m, 0.0, M, 1.0, K, b, mask=mask, g=g, rtol=1e-8, max_iter=5000)
    assert rep["converged_all"], rep
    ref = _oracle_same_iters(rp, col, 0.0, Mh, 1.0, Kh, bh, rep["iters"], mask=mh, g=gh)
    w = assert_cols_close(u.cpu().numpy(), ref, RTOL["f64"])
    bm = mh == 1
    assert np.array_equal(u.cpu().numpy()[bm], gh[bm])
    ut, rep_t = dgo.pcg(m, 0.0, M, 1.0, K, b, mask=mask, g=g, rtol=1e-14, max_iter=5000,
                        stall_iters=30)
    uo, its, _ = oracle.pcg(rp, col, 0.0, Mh, 1.0, Kh, bh, mask=mh, g=gh, rtol=1e-14,
                            max_iter=20000)
    wt = assert_cols_close(ut.cpu().numpy(), uo, RTOL["f64"])
    print(f"  same-count error {w:.2e}, tight error {wt:.2e}, iterations {rep['iters']}",
          flush=True)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_pcg_dirichlet_breadth_first_rows(dtype):
    """Dirichlet elimination with rows in breadth-first order (an icosphere of
    level 7; a polar cap of fixed vertices with values z): the masked
    iteration against the oracle's iterate of the same count."""
    print(f"[pcg-dirichlet] icosphere L7 cap {dtype}", flush=True)
    X, F = meshgen.icosphere(7, 1e-3, 0)
    m = dgo.Mesh(torch.from_numpy(F).to(DEV), X.shape[0])
    td = torch.float64 if dtype == "f64" else torch.float32
    K, M = dgo.assemble(m, torch.from_numpy(X).to(DEV, td))
    mask = torch.from_numpy((X[:, 2] > 0.8).astype(np.uint8)).to(DEV)
    g = torch.from_numpy(X[:, 2].copy()).to(DEV, td)
    f = torch.from_numpy(meshgen.normal(9, X.shape[0])).to(DEV, td)
    b = (M * f).contiguous()
    u, rep = dgo.pcg(m, 1.0, M, 1e-3, K, b, mask=mask, g=g, rtol=1e-8, max_iter=2000,
                     stall_iters=20 if dtype == "f32" else 0)
    rp, col = [t.cpu().numpy() for t in m.csr()]
    ref = _oracle_same_iters(rp, col, 1.0, M.double().cpu().numpy(), 1e-3,
                             K.double().cpu().numpy(), b.double().cpu().numpy(), rep["iters"],
                             mask=mask.cpu().numpy(), g=g.double().cpu().numpy())
    assert_cols_close(u.double().cpu().numpy(), ref, RTOL[dtype])


def _jacobi_condition(rp, col, alpha, Mh, beta, Kh, mask=None, steps=400, seed=3):
    """2-norm condition number of the Jacobi-scaled operator D^-1/2 A D^-1/2
    (A restricted to the unmasked rows and columns), estimated from the
    extreme Ritz values of a plain Lanczos run on the oracle-side matrices."""
    n = rp.size - 1
    rows = np.repeat(np.arange(n), np.diff(rp))
    A = sp.csr_matrix((beta * Kh, col, rp), shape=(n, n)) + sp.diags(alpha * Mh)
    keep = np.ones(n, bool) if mask is None else (mask == 0)
    A = A[keep][:, keep].tocsr()
    d = 1.0 / np.sqrt(A.diagonal())
    S = sp.diags(d) @ A @ sp.diags(d)
    q = meshgen.normal(seed, S.shape[0])
    q /= np.linalg.norm(q)
    qp = np.zeros_like(q)
    al, be = [], []
    bprev = 0.0
    for _ in range(steps):
        w = S @ q - bprev * qp
        a = float(q @ w)
        w -= a * q
        bn = float(np.linalg.norm(w))
        al.append(a)
        be.append(bn)
        if bn == 0.0:
            break
        qp, q, bprev = q, w / bn, bn
    T = np.diag(al) + np.diag(be[:-1], 1) + np.diag(be[:-1], -1)
    ev = np.linalg.eigvalsh(T)
    return float(ev[-1] / ev[0])


@pytest.mark.parametrize("n", [17, 64])
def test_pcg_dirichlet_cube_f32_attainable(n):
    """Config 3 in FP32 (n = 64: its full size). FP32 vectors and SpMV cannot
    reach 1e-5 here in general: the attainable relative accuracy of CG in a
    working precision u is of order kappa u, kappa the condition number of
    the Jacobi-scaled operator (about 10^3 at n = 64). The test measures kappa
    on the oracle-side matrices and asserts the achieved error (against the
    oracle's tight FP64 solution of the same FP32-rounded system, element by
    element, column-scaled) is within max(1e-5, kappa u_32), u_32 = 2^-24."""
    print(f"[pcg-dirichlet] cube{n} f32", flush=True)
    m, K, M, mask, g, b = _cube_problem(n, "f32")
    rp, col = [t.cpu().numpy() for t in m.csr()]
    Kh, Mh, bh, gh = (t.double().cpu().numpy() for t in (K, M, b, g))
    mh = mask.cpu().numpy()
    u, rep = dgo.pcg(m, 0.0, M, 1.0, K, b, mask=mask, g=g, rtol=1e-8, max_iter=5000,
                     stall_iters=30)
    uo, _, _ = oracle.pcg(rp, col, 0.0, Mh, 1.0, Kh, bh, mask=mh, g=gh, rtol=1e-14,
                          max_iter=20000)
    kappa = _jacobi_condition(rp, col, 0.0, Mh, 1.0, Kh, mask=mh)
    bound = max(RTOL["f32"], kappa * 2.0 ** -24)
    w = assert_cols_close(u.double().cpu().numpy(), uo, bound)
    print(f"  achieved {w:.2e}; kappa {kappa:.0f}; bound {bound:.2e}", flush=True)
    bm = mh == 1
    assert np.array_equal(u.double().cpu().numpy()[bm], gh[bm])


def test_pcg_zero_column_and_zero_iterations():
    """Degenerate solves. A zero right-hand side with a zero initial guess
    meets ||r|| <= max(rtol ||b||, atol) = 0 before any iteration: 0
    iterations, converged, u = 0 exactly, residual 0; the other columns of the
    block iterate as usual (the oracle's iterate of the same count, counts
    within one of the oracle's own stop). max_iter = 0 returns the initial
    guess unchanged and reports no convergence."""
    print("[pcg] zero column, zero iterations", flush=True)
    m, K, M, b = _cfg2_system(4, 8, "f64")
    b[:, 2] = 0
    rp, col = [t.cpu().numpy() for t in m.csr()]
    Kh, Mh, bh = K.cpu().numpy(), M.cpu().numpy(), b.cpu().numpy()
    u, rep = dgo.pcg(m, 1.0, M, 1e-3, K, b, rtol=1e-8, max_iter=2000)
    assert rep["converged_all"], rep
    assert int(rep["iters"][2]) == 0 and rep["relres"][2] == 0.0 and rep["true_relres"][2] == 0.0
    assert not u[:, 2].any()
    uo = _oracle_same_iters(rp, col, 1.0, Mh, 1e-3, Kh, bh, rep["iters"])
    assert_cols_close(u.cpu().numpy(), uo, RTOL["f64"])
    for c in (0, 5):
        _, its, _ = oracle.pcg(rp, col, 1.0, Mh, 1e-3, Kh, bh[:, c].copy(), rtol=1e-8, max_iter=2000)
        assert abs(int(rep["iters"][c]) - int(its[0])) <= 1
    u0 = torch.from_numpy(meshgen.normal(8, bh.size).reshape(bh.shape)).to(DEV)
    u, rep = dgo.pcg(m, 1.0, M, 1e-3, K, b, u0=u0, rtol=1e-8, max_iter=0)
    assert torch.equal(u, u0)
    assert not rep["converged_all"] and all(int(i) == 0 for i in rep["iters"])


def test_pcg_strict_and_deterministic():
    m, K, M, b = _cfg2_system(4, 3, "f64")
    with pytest.raises(dgo.DgoError) as e:
        dgo.pcg(m, 1.0, M, 1e-3, K, b, rtol=1e-12, max_iter=2, strict=True)
    assert e.value.status == "NOT_CONVERGED"
    u1, _ = dgo.pcg(m, 1.0, M, 1e-3, K, b, rtol=1e-10)
    u2, _ = dgo.pcg(m, 1.0, M, 1e-3, K, b, rtol=1e-10)
    assert torch.equal(u1, u2)
    # a column solved alone agrees with the column solved in the block (the
    # row split of the SpMV depends on k, so agreement is to rounding), for
    # the same iteration count
    ub, _ = dgo.pcg(m, 1.0, M, 1e-3, K, b, rtol=0.0, max_iter=40, fixed_iters=True)
    u0, _ = dgo.pcg(m, 1.0, M, 1e-3, K, b[:, 1].contiguous(), rtol=0.0, max_iter=40,
                    fixed_iters=True)
    assert_cols_close(u0.cpu().numpy(), ub[:, 1].cpu().numpy(), RTOL["f64"])


def test_pcg_rtol_initial_matches_oracle():
    """Stopping at a fraction of the initial residual equals the textbook
    stop ||r|| <= rtol ||b|| with rtol = rtol_initial ||r_0|| / ||b||."""
    print("[pcg] rtol_initial", flush=True)
    m, K, M, b = _cfg2_system(4, 3, "f64")
    rp, col = [t.cpu().numpy() for t in m.csr()]
    Kh, Mh, bh = K.cpu().numpy(), M.cpu().numpy(), b.cpu().numpy()
    u0 = 0.01 * meshgen.normal(77, bh.size).reshape(bh.shape)
    A = sp.csr_matrix((1e-3 * Kh, col, rp)) + sp.diags(Mh)
    r0 = np.linalg.norm(bh - A @ u0, axis=0)
    u, rep = dgo.pcg(m, 1.0, M, 1e-3, K, b, u0=torch.from_numpy(u0).to(DEV), rtol=0.0,
                     rtol_initial=1e-4, max_iter=2000)
    assert rep["converged_all"]
    for c in range(bh.shape[1]):
        uo, its, _ = oracle.pcg(rp, col, 1.0, Mh, 1e-3, Kh, bh[:, c].copy(), u0=u0[:, c].copy(),
                                rtol=1e-4 * r0[c] / np.linalg.norm(bh[:, c]), max_iter=2000)
        assert abs(int(rep["iters"][c]) - int(its[0])) <= 1
        rg = np.linalg.norm(bh[:, c] - A @ u.cpu().numpy()[:, c])
        assert rg <= 1.05e-4 * r0[c]


def test_pcg_atol_matches_oracle():
    """The absolute tolerance (Sec. 6.2's absolute and relative tolerances): a
    column stops at ||r|| <= max(rtol ||b||, atol). With atol the larger
    bound this is the oracle's relative stop at rtol = atol / ||b||; the
    iteration counts agree within one and the solution equals the oracle's
    iterate of the same count at 1e-12."""
    print("[pcg] atol", flush=True)
    m, K, M, b = _cfg2_system(4, 3, "f64")
    rp, col = [t.cpu().numpy() for t in m.csr()]
    Kh, Mh, bh = K.cpu().numpy(), M.cpu().numpy(), b.cpu().numpy()
    bn = np.linalg.norm(bh, axis=0)
    atol = 1e-6 * float(bn.min())
    A = sp.csr_matrix((1e-3 * Kh, col, rp)) + sp.diags(Mh)
    for rtol in (0.0, 1e-12):
        u, rep = dgo.pcg(m, 1.0, M, 1e-3, K, b, rtol=rtol, atol=atol, max_iter=2000)
        assert rep["converged_all"], rep
        for c in range(bh.shape[1]):
            _, its, _ = oracle.pcg(rp, col, 1.0, Mh, 1e-3, Kh, bh[:, c].copy(),
                                   rtol=atol / bn[c], max_iter=2000)
            assert abs(int(rep["iters"][c]) - int(its[0])) <= 1, (rep["iters"], its)
            rg = np.linalg.norm(bh[:, c] - A @ u.cpu().numpy()[:, c])
            assert rg <= 1.05 * atol
        ref = _oracle_same_iters(rp, col, 1.0, Mh, 1e-3, Kh, bh, rep["iters"])
        assert_cols_close(u.cpu().numpy(), ref, RTOL["f64"])
    # the relative bound is the larger one: atol has no effect
    u1, r1 = dgo.pcg(m, 1.0, M, 1e-3, K, b, rtol=1e-6, atol=1e-30, max_iter=2000)
    u2, r2 = dgo.pcg(m, 1.0, M, 1e-3, K, b, rtol=1e-6, max_iter=2000)
    assert r1["iters"] == r2["iters"] and torch.equal(u1, u2)
    with pytest.raises(dgo.DgoError) as e:
        dgo.pcg(m, 1.0, M, 1e-3, K, b, atol=-1.0)
    assert e.value.status == "INVALID_ARG"


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_vjp_parity(dtype):
    print(f"[vjp] ico5 {dtype}", flush=True)
    X, F = meshgen.icosphere(5, 1e-2, 3)
    m = dgo.Mesh(torch.from_numpy(F).to(DEV), X.shape[0])
    td = torch.float64 if dtype == "f64" else torch.float32
    Xd = torch.from_numpy(X).to(DEV, td)
    gK = torch.from_numpy(meshgen.normal(11, m.nnz)).to(DEV, td)
    gM = torch.from_numpy(meshgen.normal(12, m.nV)).to(DEV, td)
    gX = dgo.assemble_vjp(m, Xd, gK, gM).double().cpu().numpy()
    rp, col = [t.cpu().numpy() for t in m.csr()]
    ref = oracle.assemble_vjp_tri(Xd.double().cpu().numpy(), F, rp, col,
                                  gK.double().cpu().numpy(), gM.double().cpu().numpy())
    tol = 1e-12 if dtype == "f64" else 1e-5
    assert np.abs(gX - ref).max() <= tol * np.abs(ref).max()


def _fans(n_fans, spokes, seed):
    """n_fans disjoint disk fans with their centres numbered 0 .. n_fans - 1:
    the first row blocks hold many rows of spokes + 1 entries."""
    rng = np.random.default_rng(seed)
    th = np.linspace(0, 2 * np.pi, spokes, endpoint=False)
    X = np.zeros((n_fans * (spokes + 1), 3))
    F = []
    for f in range(n_fans):
        X[f] = (3.0 * f, 0.0, 0.0)
        ring = n_fans + f * spokes
        X[ring:ring + spokes, 0] = 3.0 * f + np.cos(th)
        X[ring:ring + spokes, 1] = np.sin(th)
        X[ring:ring + spokes, 2] = 0.05 * rng.standard_normal(spokes)
        F += [[f, ring + k, ring + (k + 1) % spokes] for k in range(spokes)]
    return X, np.array(F, np.int32)


@pytest.mark.parametrize("shape", ["ico4", "fans", "fan254"])
def test_vjp_row_block_and_long_rows(shape):
    """The row-block VJP (ico4) and the per-row form it falls back to when a
    row block of very long rows does not fit its LDS budget (fans); fan254
    has a vertex of the largest supported degree."""
    print(f"[vjp] {shape}", flush=True)
    if shape == "ico4":
        X, F = meshgen.icosphere(4, 1e-2, 5)
    elif shape == "fans":
        X, F = _fans(64, 150, 5)
    else:
        X, F = MESHES[shape]()
    m = dgo.Mesh(torch.from_numpy(F).to(DEV), X.shape[0])
    Xd = torch.from_numpy(X).to(DEV)
    gK = torch.from_numpy(meshgen.normal(13, m.nnz)).to(DEV)
    gM = torch.from_numpy(meshgen.normal(14, m.nV)).to(DEV)
    rp, col = [t.cpu().numpy() for t in m.csr()]
    for a, b in ((gK, gM), (gK, None), (None, gM)):
        gX = dgo.assemble_vjp(m, Xd, a, b).cpu().numpy()
        ref = oracle.assemble_vjp_tri(X, F, rp, col, None if a is None else a.cpu().numpy(),
                                      None if b is None else b.cpu().numpy())
        assert np.abs(gX - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("dtype,with_f", [("f64", True), ("f64", False), ("f32", True)])
def test_linear_solve_vjp_parity(dtype, with_f):
    print(f"[solve-vjp] ico5 {dtype} f={with_f}", flush=True)
    X, F = meshgen.icosphere(5, 1e-2, 9)
    m = dgo.Mesh(torch.from_numpy(F).to(DEV), X.shape[0])
    td = torch.float64 if dtype == "f64" else torch.float32
    k = 3
    lam = torch.from_numpy(meshgen.normal(21, m.nV * k).reshape(-1, k)).to(DEV, td)
    u = torch.from_numpy(meshgen.normal(22, m.nV * k).reshape(-1, k)).to(DEV, td)
    f = torch.from_numpy(meshgen.normal(23, m.nV * k).reshape(-1, k)).to(DEV, td)
    gK, gM = dgo.linear_solve_vjp(m, 1.0, 1e-2, lam, u, f if with_f else None)
    rp, col = [t.cpu().numpy() for t in m.csr()]
    L, U, Fh = (t.double().cpu().numpy() for t in (lam, u, f))
    rK, rM = oracle.linear_solve_vjp(rp, col, 1.0, 1e-2, L, U, Fh if with_f else None)
    # error scale: the sums of |terms| (beta |lam_i| . |u_j| per slot)
    rows = np.repeat(np.arange(m.nV), np.diff(rp))
    sK = 1e-2 * np.sum(np.abs(L[rows]) * np.abs(U[col]), 1)
    sM = np.sum(np.abs(L) * np.abs(U), 1) + (np.sum(np.abs(L) * np.abs(Fh), 1) if with_f else 0)
    tol = 1e-12 if dtype == "f64" else 1e-5
    assert np.all(np.abs(gK.double().cpu().numpy() - rK) <= tol * sK)
    assert np.all(np.abs(gM.double().cpu().numpy() - rM) <= tol * sM)


def test_mcf_step_gradient_matches_oracle():
    """Autograd through AssembleFn and LinearSolveFn (forward PCG, adjoint PCG,
    solve VJP, assembly VJP) against the oracle's adjoint gradient of one
    implicit MCF step. Both sides solve to their tightest tolerance, so the
    comparison is bounded by the solves' accuracy: each converged solution is
    within kappa * 1e-14 of the exact one (kappa about 10 for M + tau K at
    this size), hence the bar 1e-12 on the loss and on the gradient."""
    print("[mcf-step] ico4 f64", flush=True)
    X, F = meshgen.icosphere(4, 1e-2, 10)
    tau = 1e-2
    W = meshgen.normal(24, X.size).reshape(X.shape)
    m = dgo.Mesh(torch.from_numpy(F).to(DEV), X.shape[0])
    Xd = torch.from_numpy(X).to(DEV).requires_grad_(True)
    u = dgo.mcf_step(m, Xd, tau, rtol=1e-14, max_iter=5000)
    loss = (u * torch.from_numpy(W).to(DEV)).sum()
    loss.backward()
    lo, go = oracle.mcf_step_grad(X, F, tau, W)
    g = Xd.grad.cpu().numpy()
    el = abs(loss.item() - lo) / abs(lo)
    eg = np.abs(g - go).max() / np.abs(go).max()
    print(f"  loss error {el:.2e}, gradient error {eg:.2e}", flush=True)
    assert el <= RTOL["f64"] and eg <= RTOL["f64"]


def _cfg5_batch(dtype, B=256):
    """Config 5: B icosphere L5 meshes with radial noise 1e-2 (seeds 0..B-1)
    sharing one topology and one field u ~ N(0, 1) (seed 1000)."""
    X0, F = meshgen.icosphere(5)
    m = dgo.Mesh(torch.from_numpy(F).to(DEV), X0.shape[0])
    Xs = np.stack([meshgen.icosphere(5, 1e-2, s)[0] for s in range(B)])
    td = torch.float64 if dtype == "f64" else torch.float32
    X = torch.from_numpy(Xs).to(DEV, td)
    u = torch.from_numpy(meshgen.normal(1000, X0.shape[0])).to(DEV, td)
    return m, F, X, u


def _cfg5_loss(m, X, u):
    """Per-mesh loss u^T K(x) u + total area through AssembleFn (torch only
    forms the quadratic form from the CSR values the library returns)."""
    K, M = dgo.AssembleFn.apply(X, m)
    rp, col = m.csr()
    rows = torch.repeat_interleave(torch.arange(m.nV, device=DEV), (rp[1:] - rp[:-1]).long())
    quad = (K * (u[rows] * u[col.long()])[None, :]).sum(1)
    return quad + M.sum(1)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_autograd_loss_gradient_cfg5(dtype):
    """Config 5 at full size (256 meshes of 10,242 vertices): loss and
    gradient through AssembleFn against the oracle's direct loss gradient on
    the same (in FP32: FP32-rounded) positions and field, each mesh's
    gradient element by element at rtol * max |g*| of that mesh."""
    print(f"[autograd] 256 x icosphere L5 {dtype}", flush=True)
    m, F, X, u = _cfg5_batch(dtype)
    X.requires_grad_(True)
    loss = _cfg5_loss(m, X, u)
    loss.sum().backward()
    Xr = X.detach().double().cpu().numpy()
    ur = u.double().cpu().numpy()
    G = X.grad.double().cpu().numpy()
    Lg = loss.detach().double().cpu().numpy()
    worst = 0.0
    for b in range(X.shape[0]):
        Lo, go = oracle.loss_grad_tri(Xr[b], F, ur)
        if dtype == "f64":  # in FP32 the loss value is torch's FP32 sum, not the library's
            assert abs(Lg[b] - Lo) <= RTOL[dtype] * abs(Lo)
        e = np.abs(G[b] - go)
        assert np.all(e <= RTOL[dtype] * np.abs(go).max()), b
        worst = max(worst, float(e.max() / np.abs(go).max()))
    print(f"  worst gradient error {worst:.2e}", flush=True)
