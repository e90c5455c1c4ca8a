"""Pins of the oracle's topology (edges, element->edge map, CSR pattern,
boundary) against brute force on tiny meshes, exact counts and Euler
characteristics. Notation of Sec. 4.1 (EV, VV) and Sec. 6.1 (face-subface
tensors with subface j opposite vertex j)."""
import itertools

import numpy as np
import pytest

import meshgen

pytestmark = pytest.mark.filterwarnings("ignore")


def _tiny_meshes():
    yield "grid4", *meshgen.grid2d(4, 0.2, 3)
    yield "grid5", *meshgen.grid2d(5)
    for L in range(3):
        yield f"ico{L}", *meshgen.icosphere(L, 1e-3, 1)
    yield "cube3", *meshgen.cube_tets(3, 0.15, 2)
    yield "cube4", *meshgen.cube_tets(4)
    # two disjoint triangles and an isolated vertex (index 6)
    X = np.random.default_rng(0).normal(size=(7, 3))
    yield "disjoint", X, np.array([[0, 1, 2], [5, 4, 3]], np.int32)
    # a fan around vertex 0 (degree 6, open)
    X = np.random.default_rng(1).normal(size=(8, 3))
    yield "fan", X, np.array([[0, i, i + 1] for i in range(1, 7)], np.int32)


def _local_pairs(nl):
    if nl == 3:
        return [(1, 2), (2, 0), (0, 1)]
    return [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]


@pytest.mark.parametrize("name,X,E", list(_tiny_meshes()), ids=lambda v: v if isinstance(v, str) else "")
def test_edges_brute_force(orc, name, X, E):
    nV = X.shape[0]
    edge_set = set()
    for el in E:
        for a, b in itertools.combinations(el.tolist(), 2):
            edge_set.add((min(a, b), max(a, b)))
    ref_EV = np.array(sorted(edge_set), np.int32)
    EV, ee, es = orc.edges(nV, E)
    np.testing.assert_array_equal(EV, ref_EV)
    rank = {tuple(e): i for i, e in enumerate(ref_EV.tolist())}
    nl = 3 if E.shape[1] == 3 else 6
    for f, el in enumerate(E.tolist()):
        for s, (a, b) in enumerate(_local_pairs(nl)):
            va, vb = el[a], el[b]
            assert ee[f, s] == rank[(min(va, vb), max(va, vb))]
            assert es[f, s] == (1 if va < vb else -1)
    # CSR = {(i,i)} U VV, rows and columns ascending
    rowptr, col = orc.csr(nV, EV)
    ent = sorted({(i, i) for i in range(nV)} | edge_set | {(b, a) for a, b in edge_set})
    ref_rowptr = np.zeros(nV + 1, np.int64)
    for i, _ in ent:
        ref_rowptr[i + 1] += 1
    np.testing.assert_array_equal(rowptr, np.cumsum(ref_rowptr))
    np.testing.assert_array_equal(col, [j for _, j in ent])


@pytest.mark.parametrize("name,X,E", list(_tiny_meshes()), ids=lambda v: v if isinstance(v, str) else "")
def test_boundary_brute_force(orc, name, X, E):
    nV = X.shape[0]
    count = {}
    sub = 2 if E.shape[1] == 3 else 3
    for el in E.tolist():
        for c in itertools.combinations(sorted(el), sub):
            count[c] = count.get(c, 0) + 1
    bf = [c for c, n in count.items() if n == 1]
    ref = np.zeros(nV, np.uint8)
    for c in bf:
        ref[list(c)] = 1
    mask, nb = orc.boundary(nV, E)
    np.testing.assert_array_equal(mask, ref)
    assert nb == len(bf)


@pytest.mark.parametrize("L", range(6))
def test_icosphere_counts_and_orientation(orc, L):
    X, F = meshgen.icosphere(L)
    nV = X.shape[0]
    EV, ee, es = orc.edges(nV, F)
    assert nV == 10 * 4 ** L + 2 and F.shape[0] == 20 * 4 ** L and EV.shape[0] == 30 * 4 ** L
    assert nV - EV.shape[0] + F.shape[0] == 2
    # closed, consistently oriented surface: every edge in exactly two faces,
    # once in each direction
    cnt = np.bincount(ee.ravel(), minlength=EV.shape[0])
    assert np.all(cnt == 2)
    signed = np.zeros(EV.shape[0], np.int64)
    np.add.at(signed, ee.ravel(), es.ravel().astype(np.int64))
    assert np.all(signed == 0)
    # FE[f, j] is the edge opposite vertex j: its endpoints are F[f] minus F[f, j]
    for j in range(3):
        ends = EV[ee[:, j]]
        others = np.sort(np.stack([F[:, (j + 1) % 3], F[:, (j + 2) % 3]], 1), 1)
        np.testing.assert_array_equal(ends, others)
    mask, nb = orc.boundary(nV, F)
    assert nb == 0 and mask.sum() == 0


@pytest.mark.parametrize("n", [2, 3, 7, 64])
def test_grid_counts(orc, n):
    X, F = meshgen.grid2d(n, 0.2, 0)
    EV, _, _ = orc.edges(n * n, F)
    assert EV.shape[0] == 2 * n * (n - 1) + (n - 1) ** 2
    assert n * n - EV.shape[0] + F.shape[0] == 1
    mask, nb = orc.boundary(n * n, F)
    assert nb == 4 * (n - 1) and mask.sum() == 4 * (n - 1)
    if n == 64:
        rowptr, col = orc.csr(n * n, EV)
        assert rowptr[-1] == 28162 and F.shape[0] == 7938


@pytest.mark.parametrize("n", [2, 3, 5, 9])
def test_cube_counts(orc, n):
    X, T = meshgen.cube_tets(n, 0.15, 0)
    m = n - 1
    EV, ee, _ = orc.edges(n ** 3, T)
    assert EV.shape[0] == 3 * m * n * n + 3 * m * m * n + m ** 3
    tris = set()
    for el in T.tolist():
        tris.update(itertools.combinations(sorted(el), 3))
    # V - E + F - T = 1 for a ball
    assert n ** 3 - EV.shape[0] + len(tris) - T.shape[0] == 1
    mask, nb = orc.boundary(n ** 3, T)
    assert nb == 12 * m * m
    assert mask.sum() == n ** 3 - max(0, n - 2) ** 3


def test_cube64_counts(orc):
    X, T = meshgen.cube_tets(64, 0.15, 0)
    EV, _, _ = orc.edges(64 ** 3, T)
    assert T.shape[0] == 1_500_282 and EV.shape[0] == 1_786_239
    rowptr, col = orc.csr(64 ** 3, EV)
    assert rowptr[-1] == 3_834_622


def test_validate(orc):
    F = np.array([[0, 1, 2], [2, 1, 3]], np.int32)
    assert orc.validate(4, F) == 0
    assert orc.validate(3, F) == 2  # index out of range
    assert orc.validate(4, np.array([[0, 1, 1]], np.int32)) == 1  # repeated vertex
    assert orc.validate(4, np.array([[0, -1, 2]], np.int32)) == 2
    T = np.array([[0, 1, 2, 3]], np.int32)
    assert orc.validate(4, T) == 0 and orc.validate(4, np.array([[0, 1, 2, 0]], np.int32)) == 1


def test_slot_map_brute_force(orc):
    """Every element-local pair's two CSR slots, against a dictionary of the
    pattern built in Python (local pair order: triangle slot j is the edge
    opposite vertex j, tet pairs 01 02 03 12 13 23)."""
    import meshgen
    pairs = {2: [(1, 2), (2, 0), (0, 1)], 3: [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]}
    for X, E in (meshgen.grid2d(5, 0.1, 1), meshgen.icosphere(1), meshgen.cube_tets(3, 0.1, 2)):
        nV = X.shape[0]
        EV, _, _ = orc.edges(nV, E)
        rp, col = orc.csr(nV, EV)
        where = {}
        for i in range(nV):
            for s in range(rp[i], rp[i + 1]):
                where[(i, int(col[s]))] = s
        sm = orc.slot_map(nV, E, rp, col)
        dim = 2 if E.shape[1] == 3 else 3
        for e in range(E.shape[0]):
            for j, (a, b) in enumerate(pairs[dim]):
                va, vb = int(E[e, a]), int(E[e, b])
                assert sm[e, j, 0] == where[(va, vb)] and sm[e, j, 1] == where[(vb, va)]
