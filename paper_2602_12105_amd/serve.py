"""Python access to the serving loop (include/dgo_serve.h): argument
marshalling only; the scheduler, admission and batched kernels are native."""
from __future__ import annotations

import ctypes as C

import numpy as np

from ._lib import ReqStats, Request, ServerCounters, ServerOpts, check, lib

__all__ = ["Server", "footprint"]


def footprint(nV, nF, k):
    return int(lib().dgo_server_footprint(int(nV), int(nF), int(k)))


class Server:
    """Continuous-batching server of assemble-and-solve requests (FP32).

    Each request: faces F (nF x 3 int32), positions X (nV x 3 float32) and
    right-hand sides f (nV x k float32); result u after `cg_iters` Jacobi-PCG
    iterations on (alpha M + beta K) u = M f.
    """

    def __init__(self, hbm_budget_bytes=8 << 30, max_slots=64, cg_iters=50, cg_chunk=10,
                 batched=True, alpha=1.0, beta=1e-3, prep_threads=2):
        o = ServerOpts(int(max_slots), int(cg_iters), int(cg_chunk), int(bool(batched)),
                       int(hbm_budget_bytes), float(alpha), float(beta), int(prep_threads), 0)
        h = C.c_void_p()
        check(lib().dgo_server_create(C.byref(o), C.byref(h)), "dgo_server_create")
        self._h = h
        self._live = {}

    def submit(self, F, X, f, user=0):
        """Queue a request; returns its ticket. The arrays are kept alive until wait."""
        F = np.ascontiguousarray(F, dtype=np.int32)
        X = np.ascontiguousarray(X, dtype=np.float32)
        f = np.ascontiguousarray(f, dtype=np.float32)
        if f.ndim == 1:
            f = f[:, None]
        u = np.empty_like(f)
        r = Request(X.shape[0], f.shape[1], F.shape[0], F.ctypes.data_as(C.c_void_p),
                    X.ctypes.data_as(C.c_void_p), f.ctypes.data_as(C.c_void_p),
                    u.ctypes.data_as(C.c_void_p), int(user))
        t = C.c_uint64(0)
        check(lib().dgo_server_submit(self._h, C.byref(r), C.byref(t)), "dgo_server_submit")
        self._live[t.value] = (F, X, f, u)
        return t.value

    def wait(self, ticket, timeout=60.0):
        """-> (u (nV x k float32), stats dict); raises DgoError if the request failed."""
        st = ReqStats()
        code = lib().dgo_server_wait(self._h, C.c_uint64(ticket), float(timeout), C.byref(st))
        arrays = self._live.get(ticket)
        if code != 9:  # keep the buffers while the request may still run (timeout)
            self._live.pop(ticket, None)
        check(code, "dgo_server_wait")
        stats = {"status": st.status, "slot": st.slot, "t_submit": st.t_submit,
                 "t_admit": st.t_admit, "t_start": st.t_start, "t_done": st.t_done,
                 "iters": st.iters, "footprint": st.footprint}
        return arrays[3], stats

    def stats(self):
        c = ServerCounters()
        check(lib().dgo_server_stats(self._h, C.byref(c)), "dgo_server_stats")
        return {n: getattr(c, n) for n, _ in ServerCounters._fields_}

    def close(self):
        if getattr(self, "_h", None):
            lib().dgo_server_destroy(self._h)
            self._h = None
            self._live.clear()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
