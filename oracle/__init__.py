"""Python access to the FP64 C oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by the
benchmark's CPU-baseline leg. The library and its Python binding never import
this module. Nothing here shares code with the HIP path.

Every wrapper takes numpy arrays, converts them to contiguous float64 / int32
and returns freshly allocated numpy results.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-fPIC", "-shared"]


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (single-threaded, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        P = C.c_void_p
        i32, i64, f64 = C.c_int32, C.c_int64, C.c_double
        sig = {
            "orc_validate": [C.c_int, i32, i64, P],
            "orc_edges": [C.c_int, i32, i64, P, P, P, P, P],
            "orc_csr": [i32, i64, P, P, P],
            "orc_boundary": [C.c_int, i32, i64, P, P, P],
            "orc_assemble": [C.c_int, i32, i64, P, P, P, P, f64, P, P],
            "orc_edge_weights": [C.c_int, i32, i64, P, P, i64, P, P],
            "orc_spmv": [i32, P, P, f64, P, f64, P, i32, P, P],
            "orc_pcg": [i32, P, P, f64, P, f64, P, P, P, i32, P, P, f64, i32, P, P],
            "orc_loss_grad_tri": [i32, i64, P, P, P, P, P],
            "orc_loss_cstep_tri": [i32, i64, P, P, P, i32, i32, f64, P],
            "orc_assemble_vjp_tri": [i32, i64, P, P, P, P, P, P, P],
            "orc_linear_solve_vjp": [i32, P, P, f64, f64, i32, P, P, P, P, P],
            "orc_assemble_intrinsic": [i32, i64, P, P, P, P, P, P],
            "orc_face_gradient": [i32, i64, P, P, i32, P, P],
            "orc_face_divergence": [i32, i64, P, P, i32, P, P],
            "orc_mass_voronoi": [i32, i64, P, P, P],
            "orc_slot_map": [C.c_int, i32, i64, P, P, P, P],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = C.c_int
        _lib = L
    return _lib


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        names = {1: "INVALID_ARG", 2: "INDEX_RANGE", 3: "DEGENERATE", 4: "NOMEM"}
        super().__init__(f"oracle {what}: {names.get(code, code)}")
        self.code = code


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _check(code, what):
    if code:
        raise OracleError(code, what)


def _dim(elem):
    return 2 if elem.shape[1] == 3 else 3


def validate(nV, elem):
    elem = _i32(elem)
    return lib().orc_validate(_dim(elem), nV, elem.shape[0], _p(elem))


def edges(nV, elem):
    """-> (EV (nE,2), elem_edge (n,nl), elem_sign (n,nl))"""
    elem = _i32(elem)
    dim = _dim(elem)
    nl = 3 if dim == 2 else 6
    cap = max(1, elem.shape[0] * nl)
    EV = np.empty((cap, 2), np.int32)
    ee = np.empty((elem.shape[0], nl), np.int32)
    es = np.empty((elem.shape[0], nl), np.int8)
    nE = C.c_int64(0)
    _check(lib().orc_edges(dim, nV, elem.shape[0], _p(elem), _p(EV), C.byref(nE),
                           _p(ee), _p(es)), "edges")
    return EV[: nE.value].copy(), ee, es


def csr(nV, EV):
    EV = _i32(EV)
    rowptr = np.empty(nV + 1, np.int32)
    col = np.empty(nV + 2 * EV.shape[0], np.int32)
    _check(lib().orc_csr(nV, EV.shape[0], _p(EV), _p(rowptr), _p(col)), "csr")
    return rowptr, col


def boundary(nV, elem):
    elem = _i32(elem)
    mask = np.empty(nV, np.uint8)
    nb = C.c_int64(0)
    _check(lib().orc_boundary(_dim(elem), nV, elem.shape[0], _p(elem), _p(mask),
                              C.byref(nb)), "boundary")
    return mask, nb.value


def topology(nV, elem):
    EV, ee, es = edges(nV, elem)
    rowptr, col = csr(nV, EV)
    return {"EV": EV, "elem_edge": ee, "elem_sign": es, "rowptr": rowptr, "col": col}


def edge_weights(X, elem, EV=None, elem_edge=None):
    X, elem = _f64(X), _i32(elem)
    nV = X.shape[0]
    if EV is None:
        EV, elem_edge, _ = edges(nV, elem)
    w = np.empty(EV.shape[0])
    _check(lib().orc_edge_weights(_dim(elem), nV, elem.shape[0], _p(elem), _p(X),
                                  EV.shape[0], _p(_i32(elem_edge)), _p(w)), "edge_weights")
    return w


def assemble(X, elem, rowptr=None, col=None, clamp_min=None):
    """-> (Kvals (nnz,), Mdiag (nV,), rowptr, col)"""
    X, elem = _f64(X), _i32(elem)
    nV = X.shape[0]
    if rowptr is None:
        EV, _, _ = edges(nV, elem)
        rowptr, col = csr(nV, EV)
    rowptr, col = _i32(rowptr), _i32(col)
    K = np.empty(int(rowptr[-1]))
    M = np.empty(nV)
    cm = -np.inf if clamp_min is None else float(clamp_min)
    _check(lib().orc_assemble(_dim(elem), nV, elem.shape[0], _p(elem), _p(X), _p(rowptr),
                              _p(col), cm, _p(K), _p(M)), "assemble")
    return K, M, rowptr, col


def spmv(rowptr, col, alpha, M, beta, K, x):
    rowptr, col, M, K = _i32(rowptr), _i32(col), _f64(M), _f64(K)
    x = _f64(x)
    nV = rowptr.size - 1
    k = 1 if x.ndim == 1 else x.shape[1]
    y = np.empty_like(x)
    _check(lib().orc_spmv(nV, _p(rowptr), _p(col), alpha, _p(M), beta, _p(K), k, _p(x),
                          _p(y)), "spmv")
    return y


def pcg(rowptr, col, alpha, M, beta, K, b, u0=None, mask=None, g=None, rtol=1e-8,
        max_iter=10000):
    """-> (u, iters (k,), relres (k,))"""
    rowptr, col, M, K = _i32(rowptr), _i32(col), _f64(M), _f64(K)
    b = _f64(b)
    nV = rowptr.size - 1
    k = 1 if b.ndim == 1 else b.shape[1]
    u = np.zeros_like(b) if u0 is None else _f64(u0).copy()
    if mask is not None:
        mask = np.ascontiguousarray(mask, dtype=np.uint8)
        g = _f64(g).reshape(b.shape)
    its = np.empty(k, np.int32)
    rr = np.empty(k)
    _check(lib().orc_pcg(nV, _p(rowptr), _p(col), alpha, _p(M), beta, _p(K), _p(mask),
                         _p(g), k, _p(b), _p(u), rtol, max_iter, _p(its), _p(rr)), "pcg")
    return u, its, rr


def loss_grad_tri(X, F, u):
    X, F, u = _f64(X), _i32(F), _f64(u)
    g = np.empty_like(X)
    L = C.c_double(0)
    _check(lib().orc_loss_grad_tri(X.shape[0], F.shape[0], _p(F), _p(X), _p(u), C.byref(L),
                                   _p(g)), "loss_grad_tri")
    return L.value, g


def loss_cstep_tri(X, F, u, v, c, h=1e-30):
    X, F, u = _f64(X), _i32(F), _f64(u)
    d = C.c_double(0)
    _check(lib().orc_loss_cstep_tri(X.shape[0], F.shape[0], _p(F), _p(X), _p(u), v, c, h,
                                    C.byref(d)), "loss_cstep_tri")
    return d.value


def assemble_vjp_tri(X, F, rowptr, col, gK=None, gM=None):
    X, F = _f64(X), _i32(F)
    gX = np.empty_like(X)
    _check(lib().orc_assemble_vjp_tri(X.shape[0], F.shape[0], _p(F), _p(X), _p(_i32(rowptr)),
                                      _p(_i32(col)), _p(None if gK is None else _f64(gK)),
                                      _p(None if gM is None else _f64(gM)), _p(gX)),
           "assemble_vjp_tri")
    return gX


def linear_solve_vjp(rowptr, col, alpha, beta, lam, u, f=None):
    """-> (gK (nnz,), gM (nV,)) of a solve (alpha M + beta K) u = b (b = M f when f is given)."""
    rowptr, col = _i32(rowptr), _i32(col)
    nV = rowptr.size - 1
    lam, u = _f64(lam).reshape(nV, -1), _f64(u).reshape(nV, -1)
    k = lam.shape[1]
    f = None if f is None else _f64(f).reshape(nV, k)
    gK = np.empty(int(rowptr[-1]))
    gM = np.empty(nV)
    _check(lib().orc_linear_solve_vjp(nV, _p(rowptr), _p(col), float(alpha), float(beta), k,
                                      _p(lam), _p(u), _p(f), _p(gK), _p(gM)), "linear_solve_vjp")
    return gK, gM


def mcf_step(X, F, tau, rtol=1e-14, max_iter=20000):
    """One implicit mean-curvature-flow step (Sec. 7.1) with the PSD stiffness:
    u = (M + tau K)^{-1} M X, K and M assembled from X. -> (u, K, M, rowptr, col)."""
    K, M, rp, col = assemble(X, F)
    b = M[:, None] * _f64(X)
    u, _, _ = pcg(rp, col, 1.0, M, tau, K, b, rtol=rtol, max_iter=max_iter)
    return u, K, M, rp, col


def mcf_step_grad(X, F, tau, W, rtol=1e-14, max_iter=20000):
    """Gradient of l = sum(W * u) over one MCF step with respect to X, by the
    adjoint method: lambda solves the same system with W on the right-hand
    side; X enters through K(X), M(X) (assembly VJP) and through b = M X
    (the term M lambda). -> (l, gX)."""
    X = _f64(X)
    u, K, M, rp, col = mcf_step(X, F, tau, rtol, max_iter)
    lam, _, _ = pcg(rp, col, 1.0, M, tau, K, _f64(W), rtol=rtol, max_iter=max_iter)
    gK, gM = linear_solve_vjp(rp, col, 1.0, tau, lam, u, X)
    gX = assemble_vjp_tri(X, F, rp, col, gK, gM) + M[:, None] * lam
    return float(np.sum(_f64(W) * u)), gX


def assemble_intrinsic(F, nV, lengths, rowptr=None, col=None):
    """(Kvals, Mdiag) from edge lengths indexed like EV."""
    F = _i32(F)
    if rowptr is None:
        EV, _, _ = edges(nV, F)
        rowptr, col = csr(nV, EV)
    rowptr, col = _i32(rowptr), _i32(col)
    K = np.empty(int(rowptr[-1]))
    M = np.empty(nV)
    _check(lib().orc_assemble_intrinsic(nV, F.shape[0], _p(F), _p(_f64(lengths)), _p(rowptr),
                                        _p(col), _p(K), _p(M)), "assemble_intrinsic")
    return K, M


def face_gradient(X, F, u):
    """(G u) per face, component-major: (k, 3, nF) for u of shape (nV,) or (nV, k)."""
    X, F = _f64(X), _i32(F)
    u = _f64(u).reshape(X.shape[0], -1)
    k = u.shape[1]
    g = np.empty((k, 3, F.shape[0]))
    _check(lib().orc_face_gradient(X.shape[0], F.shape[0], _p(F), _p(X), k, _p(u), _p(g)),
           "face_gradient")
    return g


def face_divergence(X, F, y):
    """(D y) per vertex: (nV, k) for y of shape (k, 3, nF) or (3, nF)."""
    X, F = _f64(X), _i32(F)
    y = _f64(y).reshape(-1, 3, F.shape[0])
    k = y.shape[0]
    d = np.empty((X.shape[0], k))
    _check(lib().orc_face_divergence(X.shape[0], F.shape[0], _p(F), _p(X), k, _p(y), _p(d)),
           "face_divergence")
    return d


def mass_voronoi(X, F):
    """Mixed-Voronoi lumped mass (nV,) of a triangle mesh."""
    X, F = _f64(X), _i32(F)
    M = np.empty(X.shape[0])
    _check(lib().orc_mass_voronoi(X.shape[0], F.shape[0], _p(F), _p(X), _p(M)), "mass_voronoi")
    return M


def csr_rows(rowptr):
    """Row index of every CSR slot (the row array of the COO form)."""
    rowptr = np.asarray(rowptr)
    return np.repeat(np.arange(rowptr.size - 1, dtype=np.int32), np.diff(rowptr))


def conformal_laplacian(F, nV, K, rowptr, col):
    """Conformal Laplacian L_C of the spectral conformal parameterization
    (Sec. 7.2), dense (2 nV x 2 nV), unknowns ordered (all x, then all y):
    L_C = [[K, -S], [S, K]], where the conformal energy of a planar map
    (x, y) is 1/2 u^T L_C u = E_D - A: E_D = 1/2 (x^T K x + y^T K y) its
    Dirichlet energy and A = x^T S y its signed area by the shoelace formula
    over the boundary edges (i -> j in the orientation of their one face):
    S_ij = 1/2, S_ji = -1/2."""
    F = np.asarray(F)
    n = int(nV)
    Kd = np.zeros((n, n))
    for i in range(n):
        for s in range(rowptr[i], rowptr[i + 1]):
            Kd[i, col[s]] = K[s]
    count = {}
    for f in F:
        for j in range(3):
            a, b = int(f[(j + 1) % 3]), int(f[(j + 2) % 3])
            key = (min(a, b), max(a, b))
            count[key] = count.get(key, 0) + 1
    S = np.zeros((n, n))
    for f in F:
        for j in range(3):
            a, b = int(f[(j + 1) % 3]), int(f[(j + 2) % 3])
            if count[(min(a, b), max(a, b))] == 1:
                S[a, b] += 0.5
                S[b, a] -= 0.5
    L = np.zeros((2 * n, 2 * n))
    L[:n, :n] = Kd
    L[n:, n:] = Kd
    L[:n, n:] = -S
    L[n:, :n] = S
    return L


def canonical_sign(U):
    """Flip each column so that its entry of largest magnitude (the first
    such entry on ties) is positive: the canonical sign of the orthonormalized
    eigenvector blocks of Sec. 5.2 (Eq. eigiter)."""
    U = np.array(U, dtype=np.float64, copy=True)
    idx = np.argmax(np.abs(U), axis=0)
    s = np.sign(U[idx, np.arange(U.shape[1])])
    s[s == 0] = 1.0
    return U * s


def eigs_smallest(rowptr, col, K, M, k, dense_max=4000, sigma=-1e-3):
    """The k smallest eigenpairs of the generalized problem K u = lam M u
    (Sec. 5.2, spectral implicit layers: A U = B U diag(lam), U^T B U = I,
    with A = K and B = M diagonal and positive). Up to dense_max vertices the
    definition is evaluated directly: a dense symmetric eigendecomposition of
    M^-1/2 K M^-1/2 (LAPACK through numpy); above, ARPACK in shift-invert
    mode about sigma (scipy eigsh; the CPU eigensolver the paper names).
    Returns (lam ascending (k,), U (nV, k) M-orthonormal with canonical signs)."""
    import scipy.sparse as sps
    rowptr, col = np.asarray(rowptr), np.asarray(col)
    K, M = np.asarray(K, np.float64), np.asarray(M, np.float64)
    n = rowptr.size - 1
    A = sps.csr_matrix((K, col, rowptr), shape=(n, n))
    if n <= dense_max:
        d = 1.0 / np.sqrt(M)
        S = (A.toarray() * d[:, None]) * d[None, :]
        S = 0.5 * (S + S.T)
        lam, V = np.linalg.eigh(S)
        lam, V = lam[:k], V[:, :k] * d[:, None]
    else:
        from scipy.sparse.linalg import eigsh
        lam, V = eigsh(A.tocsc(), k=k, M=sps.diags(M).tocsc(), sigma=sigma, which="LM", tol=1e-14)
        o = np.argsort(lam)
        lam, V = lam[o], V[:, o]
    # M-normalize (eigsh and eigh both return B-orthonormal vectors up to
    # rounding; normalize again so the comparison metric is exact)
    V = V / np.sqrt(np.einsum("ij,i,ij->j", V, M, V))[None, :]
    return lam, canonical_sign(V)


def slot_map(nV, elem, rowptr, col):
    """(n_elem, nl, 2) CSR slots of each element-local pair: (a, b) in row a,
    (b, a) in row b."""
    elem = _i32(elem)
    dim = _dim(elem)
    nl = 3 if dim == 2 else 6
    out = np.empty((elem.shape[0], nl, 2), np.int32)
    _check(lib().orc_slot_map(dim, nV, elem.shape[0], _p(elem), _p(_i32(rowptr)), _p(_i32(col)),
                              _p(out)), "slot_map")
    return out
