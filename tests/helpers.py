"""Shared helpers of the tests: the row-scaled comparison metrics and mesh
recipes. No arithmetic of the method lives here."""
import numpy as np

import meshgen

RTOL = {"f64": 1e-12, "f32": 1e-5}


def rows_of(rowptr):
    rowptr = np.asarray(rowptr)
    return np.repeat(np.arange(rowptr.size - 1), np.diff(rowptr))


def assert_csr_close(got, ref, rowptr, rtol, what="K"):
    """|got - ref| <= rtol * max_j |ref_ij| over the row (row-scaled)."""
    got, ref = np.asarray(got, np.float64), np.asarray(ref, np.float64)
    rowptr = np.asarray(rowptr)
    srow = np.maximum.reduceat(np.abs(ref), rowptr[:-1])
    lim = rtol * srow[rows_of(rowptr)]
    err = np.abs(got - ref)
    bad = np.nonzero(~(err <= lim))[0]
    assert bad.size == 0, (f"{what}: {bad.size} entries off; worst at {bad[:5]}: "
                           f"got {got[bad[:5]]} ref {ref[bad[:5]]} lim {lim[bad[:5]]}")


def assert_vec_close(got, ref, rtol, scale=None, what="v"):
    got, ref = np.asarray(got, np.float64), np.asarray(ref, np.float64)
    s = np.abs(ref) if scale is None else scale
    err = np.abs(got - ref)
    bad = np.nonzero(~(err <= rtol * s))[0] if np.ndim(s) else np.nonzero(~(err <= rtol * s))
    assert np.size(bad) == 0, f"{what}: max err {err.max()} vs scale {np.max(s)}"


def assert_cols_close(got, ref, rtol, what="u"):
    """Element by element, |got_ic - ref_ic| <= rtol * max_i |ref_ic|: every
    column of a solution block is an independent system, scaled by its own
    largest entry (the vector form of the row-scaled metric)."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    n = ref.shape[0]
    got, ref = got.reshape(n, -1), ref.reshape(n, -1)
    sc = np.abs(ref).max(axis=0)
    err = np.abs(got - ref)
    bad = ~(err <= rtol * sc[None, :])
    worst = float((err / np.where(sc > 0, sc, 1.0)[None, :]).max()) if err.size else 0.0
    assert not bad.any(), f"{what}: {int(bad.sum())} entries off; worst scaled error {worst:.3e} > {rtol}"
    return worst


def spmv_scale(rowptr, col, alpha, M, beta, K, x):
    """sum_j |A_ij| |x_j| per row and column, the SpMV error scale."""
    rowptr, col = np.asarray(rowptr), np.asarray(col)
    rows = rows_of(rowptr)
    a = np.abs(beta * K) + np.where(col == rows, np.abs(alpha * M[rows]), 0.0)
    x = np.abs(x.reshape(rowptr.size - 1, -1))
    out = np.zeros_like(x)
    np.add.at(out, rows, a[:, None] * x[col])
    return out


def _fan(n, seed):
    """A disk fan: center 0 and a ring of n vertices (row 0 has n + 1 entries)."""
    th = np.linspace(0, 2 * np.pi, n, endpoint=False)
    rng = np.random.default_rng(seed)
    X = np.zeros((n + 1, 3))
    X[1:, 0], X[1:, 1] = np.cos(th), np.sin(th)
    X[1:, 2] = 0.05 * rng.standard_normal(n)
    F = np.array([[0, 1 + i, 1 + (i + 1) % n] for i in range(n)], np.int32)
    return X, F


def _grid_with_fan(n, m, seed):
    """grid2d(n) plus one vertex below the bottom row joined to its first m + 1
    vertices by m triangles (a row of m + 2 entries in a mesh of n^2 + 1
    vertices)."""
    X, F = meshgen.grid2d(n, 0.2, seed)
    c = X.shape[0]
    Xc = np.array([[0.5 * m / (n - 1), -0.3, 0.0]])
    Ff = np.array([[c, i + 1, i] for i in range(m)], np.int32)
    return np.vstack([X, Xc]), np.vstack([F, Ff]).astype(np.int32)


def _icosphere_with_fan(level, m, seed):
    """icosphere(level) plus one vertex above the north pole joined by m
    triangles to m + 1 consecutive vertices (a row of m + 2 entries in a mesh
    whose rows are swept in breadth-first order)."""
    X, F = meshgen.icosphere(level, 1e-3, seed)
    c = X.shape[0]
    Xc = np.array([[0.0, 0.0, 1.5]])
    Ff = np.array([[c, i, i + 1] for i in range(m)], np.int32)
    return np.vstack([X, Xc]), np.vstack([F, Ff]).astype(np.int32)


MESHES = {
    "tri1": lambda: (np.array([[0.0, 0, 0], [1, 0, 0], [0.2, 0.9, 0]]), np.array([[0, 1, 2]], np.int32)),
    "tet1": lambda: (np.array([[0.0, 0, 0], [1, 0, 0], [0.1, 1, 0], [0.2, 0.3, 1]]),
                     np.array([[0, 1, 2, 3]], np.int32)),
    "disjoint": lambda: (np.random.default_rng(0).normal(size=(7, 3)),
                         np.array([[0, 1, 2], [5, 4, 3]], np.int32)),
    "fan": lambda: (np.random.default_rng(1).normal(size=(9, 3)),
                    np.array([[0, i, i + 1] for i in range(1, 8)], np.int32)),
    "grid64": lambda: meshgen.grid2d(64, 0.2, 0),
    "grid7": lambda: meshgen.grid2d(7, 0.2, 1),
    "ico3": lambda: meshgen.icosphere(3, 1e-3, 0),
    "ico5": lambda: meshgen.icosphere(5, 1e-2, 0),
    "ico7": lambda: meshgen.icosphere(7, 1e-3, 0),
    "cube3": lambda: meshgen.cube_tets(3, 0.15, 0),
    "cube9": lambda: meshgen.cube_tets(9, 0.15, 0),
    "cube64": lambda: meshgen.cube_tets(64, 0.15, 0),
    "fan40": lambda: _fan(40, 2),
    "grid130fan": lambda: _grid_with_fan(130, 30, 3),
    "ico6fan": lambda: _icosphere_with_fan(6, 30, 3),
    # the largest supported vertex degree, 254 (row-local ranks of 8 bits):
    # a closed fan, and a vertex joined to 254 vertices of a mesh swept in
    # breadth-first row order
    "fan254": lambda: _fan(254, 4),
    "ico6fan254": lambda: _icosphere_with_fan(6, 253, 6),
}
