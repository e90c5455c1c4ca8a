"""The allocation-free PCG entry point (dgo_pcg_fixed_noalloc) through the C
ABI against dgo_pcg with the same fixed iteration count and against the
oracle: two calls in a row on one GPU, the second with a smaller input, in
FP64 and FP32, with and without Dirichlet data, and the size limit of its
static workspace."""
import numpy as np
import pytest
import torch

import meshgen
import oracle
from helpers import RTOL, assert_cols_close

pytestmark = pytest.mark.gpu

import paper_2602_12105_amd as dgo  # noqa: E402

DEV = "cuda:0"


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("no HIP device visible")
    import paper_2602_12105_amd._lib as L
    L.lib()
    yield


def _icosphere_system(level, k, dtype, seed):
    X, F = meshgen.icosphere(level, 1e-3, seed)
    m = dgo.Mesh(torch.from_numpy(F).to(DEV), X.shape[0])
    td = torch.float64 if dtype == "f64" else torch.float32
    K, M = dgo.assemble(m, torch.from_numpy(X).to(DEV, td))
    f = torch.from_numpy(meshgen.normal(seed + 1, X.shape[0] * k).reshape(-1, k)).to(DEV, td)
    b = (M[:, None] * f).contiguous()
    return m, K, M, b


def _check(m, K, M, b, iters, dtype, alpha=1.0, beta=1e-3, mask=None, g=None):
    u0 = torch.zeros_like(b)
    u = dgo.pcg_fixed_noalloc(m, alpha, M, beta, K, b, u0.clone(), iters, mask=mask, g=g)
    ref, rep = dgo.pcg(m, alpha, M, beta, K, b, mask=mask, g=g, rtol=0.0, max_iter=iters,
                       fixed_iters=True)
    torch.cuda.synchronize()
    # the same kernels in the same order: the same bits as dgo_pcg
    assert torch.equal(u, ref)
    rp, col = [t.cpu().numpy() for t in m.csr()]
    uo, _, _ = oracle.pcg(rp, col, alpha, M.double().cpu().numpy(), beta,
                          K.double().cpu().numpy(), b.double().cpu().numpy(),
                          mask=None if mask is None else mask.cpu().numpy(),
                          g=None if g is None else g.double().cpu().numpy(), rtol=0.0,
                          max_iter=iters)
    assert_cols_close(u.double().cpu().numpy(), uo, RTOL[dtype])


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_noalloc_matches_pcg_twice_second_smaller(dtype):
    print(f"[noalloc] icosphere L6 k=8 then L4 k=3, {dtype}", flush=True)
    big = _icosphere_system(6, 8, dtype, 3)
    small = _icosphere_system(4, 3, dtype, 5)
    need, cap = dgo.pcg_fixed_noalloc_bytes(big[0], big[1].dtype, 8)
    assert 0 < need <= cap
    _check(*big, 30, dtype)
    _check(*small, 17, dtype)


def test_noalloc_dirichlet_and_zero_iterations():
    print("[noalloc] Kuhn cube 12, Dirichlet", flush=True)
    X, T = meshgen.cube_tets(12, 0.15, 0)
    m = dgo.Mesh(torch.from_numpy(T).to(DEV), X.shape[0])
    K, M = dgo.assemble(m, torch.from_numpy(X).to(DEV))
    mask = m.boundary()
    us = np.sin(np.pi * X[:, 0]) * np.sin(np.pi * X[:, 1]) * np.sin(np.pi * X[:, 2])
    g = torch.from_numpy(us).to(DEV)
    b = (M * torch.from_numpy(3 * np.pi ** 2 * us).to(DEV)).contiguous()
    _check(m, K, M, b, 25, "f64", alpha=0.0, beta=1.0, mask=mask, g=g)
    _check(m, K, M, b, 0, "f64", alpha=0.0, beta=1.0, mask=mask, g=g)


def test_noalloc_rejects_workspace_above_the_limit():
    print("[noalloc] size limit", flush=True)
    m, K, M, b = _icosphere_system(7, 1, "f64", 7)
    need, cap = dgo.pcg_fixed_noalloc_bytes(m, torch.float64, 64)
    assert need > cap  # 163,842 vertices x 64 FP64 columns: about 0.5 GB
    b64 = b.repeat(1, 64).contiguous()
    u = torch.zeros_like(b64)
    with pytest.raises(dgo.DgoError) as e:
        dgo.pcg_fixed_noalloc(m, 1.0, M, 1e-3, K, b64, u, 10)
    assert e.value.status == "UNSUPPORTED"
    assert torch.count_nonzero(u).item() == 0  # nothing was enqueued
