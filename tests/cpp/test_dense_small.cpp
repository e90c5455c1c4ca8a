// Host test of the eigensolver's small dense algebra: for random symmetric
// positive definite G and symmetric H (fixed seeds) the Rayleigh-Ritz result
// satisfies C^T G C = I and C^T H C = diag(theta) with theta ascending, and
// Cholesky rejects an indefinite matrix. Prints theta for an independent
// check of the eigenvalues in Python.
#include <cmath>
#include <cstdio>
#include <cstdint>
#include <vector>

#include "dense_small.hpp"

static uint64_t state = 12345;
static double urand() {  // splitmix64 -> [-1, 1)
    uint64_t z = (state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return 2.0 * (double)(z >> 11) * 0x1.0p-53 - 1.0;
}

int main() {
    int fails = 0;
    for (int p : {1, 2, 5, 16, 33, 64}) {
        std::vector<double> B((size_t)p * p), G((size_t)p * p, 0.0), H((size_t)p * p);
        for (auto &b : B) b = urand();
        for (int i = 0; i < p; ++i)
            for (int j = 0; j < p; ++j) {
                double s = 0.0;
                for (int k = 0; k < p; ++k) s += B[i * p + k] * B[j * p + k];
                G[i * p + j] = s + (i == j ? 0.5 : 0.0);
            }
        for (int i = 0; i < p; ++i)
            for (int j = 0; j <= i; ++j) H[i * p + j] = H[j * p + i] = urand();
        std::vector<double> theta, C;
        if (!dgo::dense::rayleigh_ritz(G, H, p, theta, C)) {
            std::printf("p=%d: rayleigh_ritz failed\n", p);
            ++fails;
            continue;
        }
        double e1 = 0.0, e2 = 0.0, hn = 0.0;
        for (double h : H) hn = std::fmax(hn, std::fabs(h));
        for (int a = 0; a < p; ++a)
            for (int b = 0; b < p; ++b) {
                double g = 0.0, h = 0.0;
                for (int i = 0; i < p; ++i)
                    for (int j = 0; j < p; ++j) {
                        g += C[i * p + a] * G[i * p + j] * C[j * p + b];
                        h += C[i * p + a] * H[i * p + j] * C[j * p + b];
                    }
                e1 = std::fmax(e1, std::fabs(g - (a == b ? 1.0 : 0.0)));
                e2 = std::fmax(e2, std::fabs(h - (a == b ? theta[a] : 0.0)));
            }
        bool asc = true;
        for (int a = 1; a < p; ++a) asc = asc && theta[a - 1] <= theta[a];
        if (!(e1 < 1e-10 && e2 < 1e-9 * std::fmax(1.0, hn * p) && asc)) {
            std::printf("p=%d: orthonormality %g, diagonalization %g, ascending %d\n", p, e1, e2, asc);
            ++fails;
        }
        std::printf("theta p=%d:", p);
        for (double t : theta) std::printf(" %.17g", t);
        std::printf("\n");
    }
    std::vector<double> I2 = {1.0, 2.0, 2.0, 1.0};  // eigenvalues 3 and -1
    if (dgo::dense::cholesky(I2, 2)) {
        std::printf("cholesky accepted an indefinite matrix\n");
        ++fails;
    }
    if (fails) return 1;
    std::printf("dense tests passed\n");
    return 0;
}
