// Small dense symmetric algebra on the host for the eigensolver's
// Rayleigh-Ritz step (blocks of at most 64 columns): Cholesky, cyclic Jacobi
// eigendecomposition and the generalized problem H c = theta G c. Plain C++,
// no device code, so it is also built and tested on the CPU alone.
#pragma once

#include <algorithm>
#include <cmath>
#include <vector>

namespace dgo {
namespace dense {

// Cholesky G = L L^T in place (lower triangle); false if G is not positive
// definite to working precision.
inline bool cholesky(std::vector<double> &A, int p) {
    for (int j = 0; j < p; ++j) {
        double d = A[j * p + j];
        for (int k = 0; k < j; ++k) d -= A[j * p + k] * A[j * p + k];
        if (!(d > 0.0)) return false;
        const double l = std::sqrt(d);
        A[j * p + j] = l;
        for (int i = j + 1; i < p; ++i) {
            double s = A[i * p + j];
            for (int k = 0; k < j; ++k) s -= A[i * p + k] * A[j * p + k];
            A[i * p + j] = s / l;
        }
    }
    for (int i = 0; i < p; ++i)
        for (int j = i + 1; j < p; ++j) A[i * p + j] = 0.0;
    return true;
}

// Symmetric eigendecomposition by cyclic Jacobi rotations (Golub and Van
// Loan, Sec. 8.5): A = V diag(w) V^T, eigenvalues ascending.
inline void jacobi_eig(std::vector<double> A, int p, std::vector<double> &w, std::vector<double> &V) {
    V.assign((size_t)p * p, 0.0);
    for (int i = 0; i < p; ++i) V[i * p + i] = 1.0;
    double norm = 0.0;
    for (double a : A) norm += a * a;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int i = 0; i < p; ++i)
            for (int j = i + 1; j < p; ++j) off += A[i * p + j] * A[i * p + j];
        if (off <= 1e-32 * norm) break;
        for (int a = 0; a < p; ++a)
            for (int b = a + 1; b < p; ++b) {
                const double apq = A[a * p + b];
                if (apq == 0.0) continue;
                const double th = (A[b * p + b] - A[a * p + a]) / (2.0 * apq);
                const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < p; ++k) {  // columns a, b
                    const double x = A[k * p + a], y = A[k * p + b];
                    A[k * p + a] = c * x - s * y;
                    A[k * p + b] = s * x + c * y;
                }
                for (int k = 0; k < p; ++k) {  // rows a, b
                    const double x = A[a * p + k], y = A[b * p + k];
                    A[a * p + k] = c * x - s * y;
                    A[b * p + k] = s * x + c * y;
                }
                for (int k = 0; k < p; ++k) {
                    const double x = V[k * p + a], y = V[k * p + b];
                    V[k * p + a] = c * x - s * y;
                    V[k * p + b] = s * x + c * y;
                }
            }
    }
    std::vector<int> ord(p);
    for (int i = 0; i < p; ++i) ord[i] = i;
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return A[x * p + x] < A[y * p + y]; });
    std::vector<double> Vs((size_t)p * p);
    w.resize(p);
    for (int j = 0; j < p; ++j) {
        w[j] = A[ord[j] * p + ord[j]];
        for (int i = 0; i < p; ++i) Vs[i * p + j] = V[i * p + ord[j]];
    }
    V.swap(Vs);
}

// Rayleigh-Ritz: H c = theta G c. Columns are first scaled to unit G-norm
// (D = diag(G)^-1/2), then G' = L L^T, W = L^-1 H' L^-T = V Theta V^T and
// C = D L^-T V, so that C^T G C = I and C^T H C = Theta.
inline bool rayleigh_ritz(const std::vector<double> &G, const std::vector<double> &H, int p,
                   std::vector<double> &theta, std::vector<double> &C) {
    std::vector<double> D(p);
    for (int i = 0; i < p; ++i) {
        if (!(G[i * p + i] > 0.0)) return false;
        D[i] = 1.0 / std::sqrt(G[i * p + i]);
    }
    std::vector<double> L((size_t)p * p), Hs((size_t)p * p);
    for (int i = 0; i < p; ++i)
        for (int j = 0; j < p; ++j) {
            L[i * p + j] = 0.5 * (G[i * p + j] + G[j * p + i]) * D[i] * D[j];
            Hs[i * p + j] = 0.5 * (H[i * p + j] + H[j * p + i]) * D[i] * D[j];
        }
    if (!cholesky(L, p)) return false;
    // X = L^-1 Hs (forward substitution per column), W = X L^-T = L^-1 X^T
    std::vector<double> X((size_t)p * p), W((size_t)p * p);
    for (int c = 0; c < p; ++c)
        for (int i = 0; i < p; ++i) {
            double s = Hs[i * p + c];
            for (int k = 0; k < i; ++k) s -= L[i * p + k] * X[k * p + c];
            X[i * p + c] = s / L[i * p + i];
        }
    for (int c = 0; c < p; ++c)
        for (int i = 0; i < p; ++i) {
            double s = X[c * p + i];
            for (int k = 0; k < i; ++k) s -= L[i * p + k] * W[k * p + c];
            W[i * p + c] = s / L[i * p + i];
        }
    for (int i = 0; i < p; ++i)
        for (int j = i + 1; j < p; ++j) W[i * p + j] = W[j * p + i] = 0.5 * (W[i * p + j] + W[j * p + i]);
    std::vector<double> V;
    jacobi_eig(W, p, theta, V);
    // C = D L^-T V: back substitution L^T Z = V, then scale rows by D
    C.assign((size_t)p * p, 0.0);
    for (int c = 0; c < p; ++c)
        for (int i = p - 1; i >= 0; --i) {
            double s = V[i * p + c];
            for (int k = i + 1; k < p; ++k) s -= L[k * p + i] * C[k * p + c];
            C[i * p + c] = s / L[i * p + i];
        }
    for (int i = 0; i < p; ++i)
        for (int c = 0; c < p; ++c) C[i * p + c] *= D[i];
    return true;
}

}  // namespace dense
}  // namespace dgo
