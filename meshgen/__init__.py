"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module holds no arithmetic of the method (no cotangents, no areas, no
operators): it only produces vertex positions, element connectivity and
right-hand sides, all from one counter-based generator (splitmix64, Steele,
Lea and Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014).

The meshes stand in for the paper's inputs (a triangle surface for the
cotangent Laplacian of the geometry module, Sec. 5.1 and the MCF application,
Sec. 7.1; tetrahedra for the d=3 level of the simplex hierarchy, Sec. 4.1 and
Sec. 6.1). The paper's own meshes are not used.

Conventions
-----------
* Element arrays are int32, shape (n_elem, 3) for triangles and (n_elem, 4)
  for tetrahedra; positions are float64, shape (nV, 3).
* ``uniform(seed, n)`` is the n first draws of the seed's stream, each
  ``(u64 >> 11) * 2**-53`` in [0, 1).
* Jitter draws are taken for every vertex in id order (x, then y, then z) and
  applied to interior vertices only, so the draw for a vertex does not depend
  on which vertices are interior.
"""
from __future__ import annotations

import hashlib
import math

import numpy as np

__all__ = [
    "splitmix64", "uniform", "normal", "grid2d", "icosphere", "cube_tets",
    "sha256", "serving_requests",
]

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, n: int) -> np.ndarray:
    """The first ``n`` outputs of splitmix64 seeded with ``seed`` (uint64)."""
    with np.errstate(over="ignore"):
        ctr = np.arange(1, n + 1, dtype=np.uint64)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + ctr * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform(seed: int, n: int) -> np.ndarray:
    """``n`` uniform draws in [0, 1) (float64, 53 random bits each)."""
    return (splitmix64(seed, n) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def normal(seed: int, n: int) -> np.ndarray:
    """``n`` standard normal draws by Box-Muller, two uniforms per draw."""
    u = uniform(seed, 2 * n)
    u1 = 1.0 - u[0::2]  # in (0, 1]
    u2 = u[1::2]
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * math.pi * u2)


def sha256(*arrays: np.ndarray) -> str:
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def grid2d(n: int, jitter: float = 0.0, seed: int = 0):
    """Regular n x n vertex grid on the unit square, two triangles per cell.

    Vertex id = i*n + j at (i*h, j*h, 0), h = 1/(n-1). Cell (i, j) with
    corners a=(i,j), b=(i+1,j), c=(i+1,j+1), d=(i,j+1) is split into the
    triangles (a, b, c) and (a, c, d). Interior vertices move by
    U(-jitter*h, +jitter*h) in x and y.
    Returns (X float64 (n*n, 3), F int32 (2(n-1)^2, 3)).
    """
    if n < 2:
        raise ValueError("grid2d needs n >= 2")
    h = 1.0 / (n - 1)
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    X = np.zeros((n * n, 3))
    X[:, 0] = (i * h).ravel()
    X[:, 1] = (j * h).ravel()
    if jitter:
        u = uniform(seed, 2 * n * n).reshape(n * n, 2)
        interior = ((i > 0) & (i < n - 1) & (j > 0) & (j < n - 1)).ravel()
        X[interior, 0:2] += (2.0 * u[interior] - 1.0) * (jitter * h)
    ci, cj = np.meshgrid(np.arange(n - 1), np.arange(n - 1), indexing="ij")
    a = (ci * n + cj).ravel()
    b = ((ci + 1) * n + cj).ravel()
    c = ((ci + 1) * n + cj + 1).ravel()
    d = (ci * n + cj + 1).ravel()
    F = np.empty((2 * a.size, 3), dtype=np.int32)
    F[0::2] = np.stack([a, b, c], 1)
    F[1::2] = np.stack([a, c, d], 1)
    return X, F


def flat_torus(n: int):
    """Periodic n x n grid (a flat torus, given intrinsically by its edge
    lengths): vertex id = i*n + j; cell (i, j) split like grid2d with indices
    taken mod n. Returns (F int32 (2 n^2, 3), ij int64 (n^2, 2)); the length
    of an edge (a, b) is h * |wrap(ij[a] - ij[b])| with h = 1/n and each
    difference wrapped into {-1, 0, 1}.
    """
    if n < 3:
        raise ValueError("flat_torus needs n >= 3")
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    ij = np.stack([i.ravel(), j.ravel()], 1)
    a = (i * n + j).ravel()
    b = (((i + 1) % n) * n + j).ravel()
    c = (((i + 1) % n) * n + (j + 1) % n).ravel()
    d = (i * n + (j + 1) % n).ravel()
    F = np.empty((2 * a.size, 3), dtype=np.int32)
    F[0::2] = np.stack([a, b, c], 1)
    F[1::2] = np.stack([a, c, d], 1)
    return F, ij


def flat_torus_lengths(n: int, ij: np.ndarray, EV: np.ndarray) -> np.ndarray:
    """Edge lengths of flat_torus(n) for the edge list EV (nE x 2)."""
    dd = ij[EV[:, 0]] - ij[EV[:, 1]]
    dd = (dd + 1) % n - 1  # wrap into {-1, 0, 1}
    return np.sqrt((dd.astype(np.float64) ** 2).sum(axis=1)) / n


_PHI = (1.0 + math.sqrt(5.0)) / 2.0
_ICO_V = np.array([
    [-1, _PHI, 0], [1, _PHI, 0], [-1, -_PHI, 0], [1, -_PHI, 0],
    [0, -1, _PHI], [0, 1, _PHI], [0, -1, -_PHI], [0, 1, -_PHI],
    [_PHI, 0, -1], [_PHI, 0, 1], [-_PHI, 0, -1], [-_PHI, 0, 1],
], dtype=np.float64)
_ICO_F = np.array([
    [0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
    [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
    [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
    [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1],
], dtype=np.int64)


def icosphere(level: int, noise: float = 0.0, seed: int = 0):
    """Subdivided icosahedron on the unit sphere.

    Each level splits every face (a, b, c) into (a, ab, ca), (b, bc, ab),
    (c, ca, bc), (ab, bc, ca); the new midpoint vertices are numbered in order
    of first encounter (faces in order, edges ab, bc, ca within a face) and
    projected to the unit sphere. Noise moves every vertex radially:
    x <- x * (1 + noise * xi), xi ~ N(0, 1).
    Returns (X float64 (10*4^L+2, 3), F int32 (20*4^L, 3)).
    """
    V = _ICO_V / np.linalg.norm(_ICO_V, axis=1, keepdims=True)
    F = _ICO_F.copy()
    for _ in range(level):
        nv = V.shape[0]
        e = np.stack([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]], 1).reshape(-1, 2)
        lo = e.min(1)
        hi = e.max(1)
        key = lo * nv + hi
        uniq, first, inv = np.unique(key, return_index=True, return_inverse=True)
        order = np.argsort(first, kind="stable")  # unique edges by first encounter
        rank = np.empty_like(order)
        rank[order] = np.arange(order.size)
        mid_id = nv + rank[inv].reshape(-1, 3)
        ulo = uniq[order] // nv
        uhi = uniq[order] % nv
        M = 0.5 * (V[ulo] + V[uhi])
        M /= np.linalg.norm(M, axis=1, keepdims=True)
        V = np.concatenate([V, M], 0)
        a, b, c = F[:, 0], F[:, 1], F[:, 2]
        ab, bc, ca = mid_id[:, 0], mid_id[:, 1], mid_id[:, 2]
        F = np.stack([
            np.stack([a, ab, ca], 1), np.stack([b, bc, ab], 1),
            np.stack([c, ca, bc], 1), np.stack([ab, bc, ca], 1)], 1).reshape(-1, 3)
    X = V.copy()
    if noise:
        xi = normal(seed, X.shape[0])
        X *= (1.0 + noise * xi)[:, None]
    return X, F.astype(np.int32)


_PERMS = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]


def cube_tets(n: int, jitter: float = 0.0, seed: int = 0):
    """Unit cube as an n^3 vertex grid, each cell split into 6 Kuhn tetrahedra.

    Vertex id = (i*n + j)*n + k at (i, j, k)*h, h = 1/(n-1). Cell with corner
    c yields, for each axis permutation s (in lexicographic order), the tet
    (c, c+e_s0, c+e_s0+e_s1, c+(1,1,1)). Interior vertices move by
    U(-jitter*h, +jitter*h) per coordinate.
    Returns (X float64 (n^3, 3), T int32 (6(n-1)^3, 4)).
    """
    if n < 2:
        raise ValueError("cube_tets needs n >= 2")
    h = 1.0 / (n - 1)
    i, j, k = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    X = np.stack([i.ravel() * h, j.ravel() * h, k.ravel() * h], 1).astype(np.float64)
    if jitter:
        u = uniform(seed, 3 * n ** 3).reshape(-1, 3)
        interior = ((i > 0) & (i < n - 1) & (j > 0) & (j < n - 1)
                    & (k > 0) & (k < n - 1)).ravel()
        X[interior] += (2.0 * u[interior] - 1.0) * (jitter * h)
    m = n - 1
    ci, cj, ck = [a.ravel() for a in
                  np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")]
    stride = np.array([n * n, n, 1])
    base = ci * n * n + cj * n + ck
    tets = []
    for p in _PERMS:
        v1 = base + stride[p[0]]
        v2 = v1 + stride[p[1]]
        v3 = base + stride.sum()
        tets.append(np.stack([base, v1, v2, v3], 1))
    T = np.stack(tets, 1).reshape(-1, 4).astype(np.int32)
    return X, T


def serving_requests(n_req: int, seed: int = 0, vmin: float = 1e3, vmax: float = 2e5,
                     kmax: int = 16):
    """Descriptors of a stream of solve requests of uneven size.

    Each request draws a vertex count N ~ logU[vmin, vmax], a kind (grid or
    icosphere, p = 1/2 each) and a right-hand-side count k ~ U{1..kmax}. A grid
    gets round(sqrt(N)) vertices per side; an icosphere gets the level in
    4..7 nearest to N in log scale. Returns a list of dicts with keys
    kind, size (side or level), k, mesh_seed, rhs_seed.
    """
    u = uniform(seed, 3 * n_req).reshape(n_req, 3)
    out = []
    ico_nv = np.array([10 * 4 ** L + 2 for L in range(4, 8)], dtype=np.float64)
    for r in range(n_req):
        N = math.exp(math.log(vmin) + u[r, 0] * (math.log(vmax) - math.log(vmin)))
        kind = "grid" if u[r, 1] < 0.5 else "ico"
        k = 1 + min(kmax - 1, int(u[r, 2] * kmax))
        if kind == "grid":
            size = max(2, int(round(math.sqrt(N))))
        else:
            size = 4 + int(np.argmin(np.abs(np.log(ico_nv) - math.log(N))))
        out.append({"kind": kind, "size": size, "k": k,
                    "mesh_seed": 10_000 + r, "rhs_seed": 20_000 + r})
    return out
