"""dgo: discrete geometry operators on simplicial meshes for MI355X (gfx950).

Thin Python binding over the C ABI of libdgo.so (include/dgo.h). It only
marshals arguments: PyTorch supplies device memory and the current HIP stream,
and every step of the computation runs in the library's HIP kernels.

    mesh = Mesh(faces_cuda_int32, nV)            # topology on the device
    K, M = assemble(mesh, X)                     # cotangent stiffness + mass
    y = spmv(mesh, 1.0, M, 1e-3, K, x)           # (M + 1e-3 K) x
    u, rep = pcg(mesh, 1.0, M, 1e-3, K, b)       # Jacobi PCG
    K, M = AssembleFn.apply(X, mesh)             # differentiable in X
"""
from __future__ import annotations

import ctypes as C

import torch

from ._lib import (ARAP_CLAMP_MIN, DGO_F32, DGO_F64, AssembleOpts, CgOpts, CgReport, DgoError,
                   EigOpts, EigReport, Sizes, check, lib)

__all__ = ["Mesh", "assemble", "assemble_vjp", "spmv", "pcg", "linear_solve_vjp", "AssembleFn",
           "LinearSolveFn", "mcf_step", "DgoError", "library_path", "build", "trace_enable",
           "trace_read", "trace_reset", "assemble_intrinsic", "face_gradient", "face_divergence",
           "arap_laplacian", "conformal_laplacian", "eigs_smallest", "pcg_fixed_noalloc",
           "pcg_fixed_noalloc_bytes"]


def build():
    from .build import build as _b
    return _b()


def library_path():
    from ._lib import LIB_PATH
    return LIB_PATH


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _dtype_code(dt):
    if dt == torch.float64:
        return DGO_F64
    if dt == torch.float32:
        return DGO_F32
    raise TypeError(f"dgo: unsupported dtype {dt} (float32 or float64)")


def _need(t, name, dtype=None, shape=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"dgo: {name} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"dgo: {name} must be on a HIP device")
    if not t.is_contiguous():
        raise ValueError(f"dgo: {name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"dgo: {name} must be {dtype}, got {t.dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"dgo: {name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return t


class Mesh:
    """Topology of a triangle (elem: n x 3) or tetrahedral (n x 4) mesh."""

    def __init__(self, elem: torch.Tensor, nV: int):
        _need(elem, "elem", torch.int32)
        if elem.dim() != 2 or elem.shape[1] not in (3, 4):
            raise ValueError("dgo: elem must be (n, 3) or (n, 4)")
        self.device = elem.device
        h = C.c_void_p()
        dim = 2 if elem.shape[1] == 3 else 3
        check(lib().dgo_mesh_create(dim, int(nV), elem.shape[0], _ptr(elem), None, _stream(),
                                    C.byref(h)), "dgo_mesh_create")
        self._h = h
        s = Sizes()
        check(lib().dgo_mesh_sizes(h, C.byref(s)), "dgo_mesh_sizes")
        self.dim, self.nV, self.n_elem = s.dim, s.nV, s.n_elem
        self.nE, self.nnz, self.n_bfaces = s.nE, s.nnz, s.n_bfaces
        self.n_boundary, self.max_row = s.n_boundary, s.max_row
        self.nl = 3 if dim == 2 else 6

    @property
    def handle(self):
        return self._h

    def edges(self):
        EV = torch.empty((self.nE, 2), dtype=torch.int32, device=self.device)
        ee = torch.empty((self.n_elem, self.nl), dtype=torch.int32, device=self.device)
        es = torch.empty((self.n_elem, self.nl), dtype=torch.int8, device=self.device)
        check(lib().dgo_mesh_edges(self._h, _ptr(EV), _ptr(ee), _ptr(es), _stream()),
              "dgo_mesh_edges")
        return EV, ee, es

    def csr(self):
        rowptr = torch.empty(self.nV + 1, dtype=torch.int32, device=self.device)
        col = torch.empty(self.nnz, dtype=torch.int32, device=self.device)
        check(lib().dgo_mesh_csr(self._h, _ptr(rowptr), _ptr(col), _stream()), "dgo_mesh_csr")
        return rowptr, col

    def coo(self):
        """(rows, cols) of the CSR pattern in CSR slot order (COO form)."""
        rows = torch.empty(self.nnz, dtype=torch.int32, device=self.device)
        cols = torch.empty(self.nnz, dtype=torch.int32, device=self.device)
        check(lib().dgo_mesh_coo(self._h, _ptr(rows), _ptr(cols), _stream()), "dgo_mesh_coo")
        return rows, cols

    def slots(self):
        """(n_elem, nl, 2) CSR slots of each element-local pair: (a, b) in row
        a and (b, a) in row b."""
        out = torch.empty((self.n_elem, self.nl, 2), dtype=torch.int32, device=self.device)
        check(lib().dgo_mesh_slots(self._h, _ptr(out), _stream()), "dgo_mesh_slots")
        return out

    def boundary(self):
        m = torch.empty(self.nV, dtype=torch.uint8, device=self.device)
        check(lib().dgo_mesh_boundary(self._h, _ptr(m), _stream()), "dgo_mesh_boundary")
        return m

    def close(self):
        if getattr(self, "_h", None):
            torch.cuda.current_stream(self.device).synchronize()
            lib().dgo_mesh_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _batched(X, nV, name="X", last=3):
    if X.dim() == 2:
        return 1, False
    if X.dim() == 3 and X.shape[1] == nV and X.shape[2] == last:
        return X.shape[0], True
    raise ValueError(f"dgo: {name} must be (nV, {last}) or (batch, nV, {last})")


_MASS = {"barycentric": 0, "voronoi": 1}


def _assemble_opts(clamp_min, mass):
    if mass not in _MASS:
        raise ValueError(f"dgo: mass must be one of {sorted(_MASS)}")
    if clamp_min is None and mass == "barycentric":
        return None
    return C.byref(AssembleOpts(0 if clamp_min is None else 1,
                                0.0 if clamp_min is None else float(clamp_min), _MASS[mass]))


def assemble(mesh: Mesh, X: torch.Tensor, clamp_min=None, check_degenerate=False,
             out=None, mass="barycentric"):
    """Cotangent stiffness K (CSR values, PSD) and lumped mass diag M
    (mass: "barycentric" or "voronoi", the mixed-Voronoi vertex areas)."""
    _need(X, "X")
    b, batched = _batched(X, mesh.nV)
    if not batched:
        _need(X, "X", shape=(mesh.nV, 3))
    dt = _dtype_code(X.dtype)
    if out is None:
        K = torch.empty((b, mesh.nnz) if batched else (mesh.nnz,), dtype=X.dtype, device=X.device)
        M = torch.empty((b, mesh.nV) if batched else (mesh.nV,), dtype=X.dtype, device=X.device)
    else:
        K, M = out
    opts = _assemble_opts(clamp_min, mass)
    nd = C.c_int64(0)
    check(lib().dgo_assemble(mesh.handle, dt, b, _ptr(X), opts, _ptr(K), _ptr(M),
                             C.byref(nd) if check_degenerate else None, _stream()), "dgo_assemble")
    return K, M


def assemble_intrinsic(mesh: Mesh, lengths: torch.Tensor, clamp_min=None,
                       check_degenerate=False, out=None, mass="barycentric"):
    """K (CSR values) and lumped M of a triangle mesh from its edge lengths,
    (nE,) or (batch, nE) in the mesh's edge order."""
    _need(lengths, "lengths")
    if lengths.dim() == 1:
        b, batched = 1, False
        _need(lengths, "lengths", shape=(mesh.nE,))
    else:
        b, batched = lengths.shape[0], True
        _need(lengths, "lengths", shape=(b, mesh.nE))
    dt = _dtype_code(lengths.dtype)
    if out is None:
        dev, ty = lengths.device, lengths.dtype
        K = torch.empty((b, mesh.nnz) if batched else (mesh.nnz,), dtype=ty, device=dev)
        M = torch.empty((b, mesh.nV) if batched else (mesh.nV,), dtype=ty, device=dev)
    else:
        K, M = out
    opts = _assemble_opts(clamp_min, mass)
    nd = C.c_int64(0)
    check(lib().dgo_assemble_intrinsic(mesh.handle, dt, b, _ptr(lengths), opts, _ptr(K), _ptr(M),
                                       C.byref(nd) if check_degenerate else None, _stream()),
          "dgo_assemble_intrinsic")
    return K, M


def face_gradient(mesh: Mesh, X: torch.Tensor, u: torch.Tensor, out=None):
    """Per-face gradients of vertex fields u ((nV,) or (nV, k)): a (k, 3, nF)
    tensor (component-major face fields)."""
    _need(X, "X", shape=(mesh.nV, 3))
    _need(u, "u", X.dtype)
    k = 1 if u.dim() == 1 else u.shape[1]
    if u.shape[0] != mesh.nV:
        raise ValueError("u must have nV rows")
    g = torch.empty((k, 3, mesh.n_elem), dtype=X.dtype, device=X.device) if out is None else out
    _need(g, "out", X.dtype, shape=(k, 3, mesh.n_elem))
    check(lib().dgo_face_gradient(mesh.handle, _dtype_code(X.dtype), _ptr(X), k, _ptr(u), _ptr(g),
                                  _stream()), "dgo_face_gradient")
    return g


def face_divergence(mesh: Mesh, X: torch.Tensor, y: torch.Tensor, out=None):
    """Divergence D = G^T diag(A) of face fields y ((3, nF) or (k, 3, nF)):
    an (nV, k) tensor, (nV,) for a (3, nF) input."""
    _need(X, "X", shape=(mesh.nV, 3))
    _need(y, "y", X.dtype)
    k = 1 if y.dim() == 2 else y.shape[0]
    if tuple(y.shape[-2:]) != (3, mesh.n_elem):
        raise ValueError("y must be (3, nF) or (k, 3, nF)")
    d = torch.empty((mesh.nV, k), dtype=X.dtype, device=X.device) if out is None else out
    _need(d, "out", X.dtype, shape=(mesh.nV, k))
    check(lib().dgo_face_divergence(mesh.handle, _dtype_code(X.dtype), _ptr(X), k, _ptr(y), _ptr(d),
                                    _stream()), "dgo_face_divergence")
    return d[:, 0] if y.dim() == 2 and out is None else d


def conformal_laplacian(mesh: Mesh, K: torch.Tensor, pattern=True):
    """Conformal Laplacian L_C = [[K, -S], [S, K]] of a triangle mesh as CSR
    (rowptr2, col2, vals2) over 2 nV rows (all x, then all y); with
    pattern=False only vals2 is returned."""
    _need(K, "K", shape=(mesh.nnz,))
    nnz2 = 2 * mesh.nnz + 4 * mesh.n_bfaces
    vals = torch.empty(nnz2, dtype=K.dtype, device=K.device)
    rp = col = None
    if pattern:
        rp = torch.empty(2 * mesh.nV + 1, dtype=torch.int32, device=K.device)
        col = torch.empty(nnz2, dtype=torch.int32, device=K.device)
    check(lib().dgo_conformal_laplacian(mesh.handle, _dtype_code(K.dtype), _ptr(K),
                                        _ptr(rp) if pattern else None,
                                        _ptr(col) if pattern else None, _ptr(vals), _stream()),
          "dgo_conformal_laplacian")
    return (rp, col, vals) if pattern else vals


def eigs_smallest(mesh: Mesh, M: torch.Tensor, K: torch.Tensor, k: int, sigma=0.0, tol=0.0,
                  block=0, max_iter=0, inner_rtol=0.0, inner_max_iter=0, seed=0,
                  inner_rtol_initial=0.0):
    """The k smallest eigenpairs of K u = lam M u (spectral implicit layer
    forward): returns (lam (k,) float64 on the host, U (nV, k) M-orthonormal
    with canonical signs, report dict). sigma = 0 picks -1 / sum(M)."""
    _need(M, "M", shape=(mesh.nV,))
    _need(K, "K", M.dtype, shape=(mesh.nnz,))
    U = torch.empty((mesh.nV, k), dtype=M.dtype, device=M.device)
    lam = (C.c_double * k)()
    o = EigOpts(float(sigma), float(tol), float(inner_rtol), float(inner_rtol_initial), int(block),
                int(max_iter), int(inner_max_iter), 0, int(seed))
    r = EigReport()
    check(lib().dgo_eigs_smallest(mesh.handle, _dtype_code(M.dtype), _ptr(M), _ptr(K), int(k),
                                  C.byref(o), _ptr(U), lam, C.byref(r), _stream()),
          "dgo_eigs_smallest")
    rep = {"k": r.k, "block": r.block, "iters": r.iters, "converged": bool(r.converged),
           "inner_iters": r.inner_iters, "sigma": r.sigma, "resid": list(r.resid[:k])}
    return torch.tensor(list(lam), dtype=torch.float64), U, rep


def arap_laplacian(mesh: Mesh, X: torch.Tensor, clamp_min=ARAP_CLAMP_MIN, out=None):
    """Cotangent stiffness and mass with the ARAP example's default weight
    clamp (Sec. 4.2: weights clamped from below at 1e-5)."""
    return assemble(mesh, X, clamp_min=clamp_min, out=out)


def assemble_vjp(mesh: Mesh, X, gK=None, gM=None):
    _need(X, "X")
    b, batched = _batched(X, mesh.nV)
    dt = _dtype_code(X.dtype)
    if gK is not None:
        _need(gK, "gK", X.dtype)
    if gM is not None:
        _need(gM, "gM", X.dtype)
    gX = torch.empty_like(X)
    check(lib().dgo_assemble_vjp(mesh.handle, dt, b, _ptr(X), _ptr(gK), _ptr(gM), _ptr(gX),
                                 _stream()), "dgo_assemble_vjp")
    return gX


def spmv(mesh: Mesh, alpha, M, beta, K, x, out=None):
    """y = (alpha M + beta K) x; x is (nV,), (nV, k) or (batch, nV, k)."""
    _need(M, "M")
    _need(K, "K", M.dtype)
    _need(x, "x", M.dtype)
    if x.dim() == 1:
        b, k = 1, 1
    elif x.dim() == 2:
        b, k = 1, x.shape[1]
    else:
        b, k = x.shape[0], x.shape[2]
    y = torch.empty_like(x) if out is None else out
    check(lib().dgo_spmv(mesh.handle, _dtype_code(M.dtype), b, float(alpha), _ptr(M), float(beta),
                         _ptr(K), k, _ptr(x), _ptr(y), _stream()), "dgo_spmv")
    return y


def pcg(mesh: Mesh, alpha, M, beta, K, b, u0=None, mask=None, g=None, rtol=1e-8,
        max_iter=1000, fixed_iters=False, check_every=8, stall_iters=0, strict=False,
        rtol_initial=0.0, atol=0.0):
    """Jacobi PCG on (alpha M + beta K) u = b; returns (u, report dict).
    A column stops at ||r|| <= max(rtol ||b||, atol); rtol_initial > 0 also
    stops it at that fraction of its initial residual."""
    _need(M, "M")
    _need(K, "K", M.dtype)
    _need(b, "b", M.dtype)
    k = 1 if b.dim() == 1 else b.shape[1]
    u = torch.zeros_like(b) if u0 is None else u0.clone()
    if mask is not None:
        _need(mask, "mask", torch.uint8)
        _need(g, "g", M.dtype, b.shape)
    opts = CgOpts(float(rtol), int(max_iter), int(bool(fixed_iters)), int(check_every),
                  int(stall_iters), int(bool(strict)), float(rtol_initial), float(atol))
    rep = CgReport()
    check(lib().dgo_pcg(mesh.handle, _dtype_code(M.dtype), float(alpha), _ptr(M), float(beta),
                        _ptr(K), _ptr(mask), _ptr(g), k, _ptr(b), _ptr(u), C.byref(opts),
                        C.byref(rep), _stream()), "dgo_pcg")
    report = {"converged_all": bool(rep.converged_all), "iters": list(rep.iters[:k]),
              "relres": list(rep.relres[:k]), "true_relres": list(rep.true_relres[:k])}
    return u, report


def pcg_fixed_noalloc(mesh: Mesh, alpha, M, beta, K, b, u, iters, mask=None, g=None):
    """Exactly `iters` PCG iterations on (alpha M + beta K) u = b into the
    caller's u (initial guess on entry), with the library's static workspace:
    no allocation and no host synchronisation (graph capture, serving loops).
    Calls on one GPU must not overlap."""
    _need(M, "M")
    _need(K, "K", M.dtype)
    _need(b, "b", M.dtype)
    _need(u, "u", M.dtype, b.shape)
    k = 1 if b.dim() == 1 else b.shape[1]
    if mask is not None:
        _need(mask, "mask", torch.uint8)
        _need(g, "g", M.dtype, b.shape)
    check(lib().dgo_pcg_fixed_noalloc(mesh.handle, _dtype_code(M.dtype), float(alpha), _ptr(M),
                                      float(beta), _ptr(K), _ptr(mask), _ptr(g), k, _ptr(b),
                                      _ptr(u), int(iters), _stream()), "dgo_pcg_fixed_noalloc")
    return u


def pcg_fixed_noalloc_bytes(mesh: Mesh, dtype, k):
    """(bytes this solve needs, bytes the static workspace holds)."""
    return (int(lib().dgo_pcg_fixed_noalloc_bytes(mesh.handle, _dtype_code(dtype), int(k))),
            int(lib().dgo_pcg_fixed_noalloc_max_bytes()))


def linear_solve_vjp(mesh: Mesh, alpha, beta, lam, u, f=None):
    """Gradients (gK, gM) of a solve (alpha M + beta K) u = b with respect to K
    and M, given the adjoint solution lam (b = M f when f is given)."""
    _need(lam, "lam")
    _need(u, "u", lam.dtype, lam.shape)
    if f is not None:
        _need(f, "f", lam.dtype, lam.shape)
    k = 1 if lam.dim() == 1 else lam.shape[1]
    gK = torch.empty(mesh.nnz, dtype=lam.dtype, device=lam.device)
    gM = torch.empty(mesh.nV, dtype=lam.dtype, device=lam.device)
    check(lib().dgo_linear_solve_vjp(mesh.handle, _dtype_code(lam.dtype), float(alpha),
                                     float(beta), k, _ptr(lam), _ptr(u), _ptr(f), _ptr(gK),
                                     _ptr(gM), _stream()), "dgo_linear_solve_vjp")
    return gK, gM


class LinearSolveFn(torch.autograd.Function):
    """u = (alpha M + beta K)^-1 (M f) by PCG, differentiable in K, M and f by
    the adjoint method: the backward solves the same (symmetric) system with
    the incoming gradient, then forms gK, gM on the CSR pattern and gf = M lam."""

    @staticmethod
    def forward(ctx, K, M, f, mesh, alpha, beta, rtol, max_iter):
        f = f.contiguous()
        b = spmv(mesh, 1.0, M, 0.0, K, f)  # b = M f
        u, _ = pcg(mesh, alpha, M, beta, K, b, rtol=rtol, max_iter=max_iter)
        ctx.save_for_backward(K, M, f, u)
        ctx.args = (mesh, alpha, beta, rtol, max_iter)
        return u

    @staticmethod
    def backward(ctx, gu):
        K, M, f, u = ctx.saved_tensors
        mesh, alpha, beta, rtol, max_iter = ctx.args
        lam, _ = pcg(mesh, alpha, M, beta, K, gu.contiguous(), rtol=rtol, max_iter=max_iter)
        gK, gM = linear_solve_vjp(mesh, alpha, beta, lam, u, f)
        gf = spmv(mesh, 1.0, M, 0.0, K, lam)  # M lam
        return gK, gM, gf, None, None, None, None, None


def mcf_step(mesh: Mesh, X, tau, rtol=1e-10, max_iter=10000):
    """One implicit mean-curvature-flow step (Sec. 7.1), u = (M + tau K)^-1 M X
    with K(X), M(X) assembled from X, differentiable in X (triangle meshes)."""
    K, M = AssembleFn.apply(X, mesh)
    return LinearSolveFn.apply(K, M, X, mesh, 1.0, tau, rtol, max_iter)


class AssembleFn(torch.autograd.Function):
    """(K, M) = assemble(mesh, X) with a hand-written adjoint in X (triangles)."""

    @staticmethod
    def forward(ctx, X, mesh):
        K, M = assemble(mesh, X.detach().contiguous())
        ctx.mesh = mesh
        ctx.save_for_backward(X)
        return K, M

    @staticmethod
    def backward(ctx, gK, gM):
        (X,) = ctx.saved_tensors
        gK = None if gK is None else gK.contiguous()
        gM = None if gM is None else gM.contiguous()
        gX = assemble_vjp(ctx.mesh, X.detach().contiguous(), gK, gM)
        return gX, None


def trace_enable(on=True, name_filter=None):
    """Bracket the library's kernel launches with hipEvents (measurement aid)."""
    f = None if name_filter is None else name_filter.encode()
    check(lib().dgo_trace_enable(int(bool(on)), f), "dgo_trace_enable")


def trace_read():
    """-> {kernel name: {count, total_ms, min_ms, max_ms, avg_ms}} (consumes pending records)."""
    from ._lib import TraceEntry
    cap = 64
    arr = (TraceEntry * cap)()
    n = C.c_int32(0)
    check(lib().dgo_trace_read(arr, cap, C.byref(n)), "dgo_trace_read")
    out = {}
    for i in range(min(cap, n.value)):
        e = arr[i]
        out[e.name.decode()] = {"count": e.count, "total_ms": e.total_ms, "min_ms": e.min_ms,
                                "max_ms": e.max_ms, "avg_ms": e.total_ms / max(1, e.count)}
    return out


def trace_reset():
    lib().dgo_trace_reset()
