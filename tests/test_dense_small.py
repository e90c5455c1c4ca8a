"""Host test of the eigensolver's small dense algebra (Cholesky, cyclic
Jacobi, Rayleigh-Ritz on H c = theta G c), compiled with g++ and run on the
CPU, plus the same generalized problems solved by LAPACK through scipy: the
eigenvalues agree. The random matrices are rebuilt here from the same
splitmix64 stream."""
import os
import subprocess

import numpy as np
import scipy.linalg

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cpp", "test_dense_small.cpp")
INC = os.path.join(HERE, "..", "paper_2602_12105_amd", "csrc")


def _stream(seed):
    state = seed
    M = (1 << 64) - 1
    while True:
        state = (state + 0x9E3779B97F4A7C15) & M
        z = state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
        z ^= z >> 31
        yield 2.0 * (z >> 11) * 2.0 ** -53 - 1.0


def test_dense_small(tmp_path):
    exe = tmp_path / "dense_small"
    subprocess.run(["g++", "-std=c++17", "-O1", "-I", INC, SRC, "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "dense tests passed" in r.stdout
    got = {}
    for line in r.stdout.splitlines():
        if line.startswith("theta p="):
            head, vals = line.split(":", 1)
            got[int(head.split("=")[1])] = np.array([float(v) for v in vals.split()])
    g = _stream(12345)
    for p in (1, 2, 5, 16, 33, 64):
        B = np.array([next(g) for _ in range(p * p)]).reshape(p, p)
        G = B @ B.T + 0.5 * np.eye(p)
        H = np.zeros((p, p))
        for i in range(p):
            for j in range(i + 1):
                H[i, j] = H[j, i] = next(g)
        ref = scipy.linalg.eigh(H, G, eigvals_only=True)
        np.testing.assert_allclose(got[p], ref, rtol=1e-9, atol=1e-9 * np.abs(ref).max())
