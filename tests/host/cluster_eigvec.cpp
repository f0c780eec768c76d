#include <cstdio>
#include <random>
#include <algorithm>
#include "dense.h"
using namespace bgcr;
using namespace bgcr::dense;
// Host eigenvectors for clustered eigenvalues: K = X diag(lam) X^{-1} (n = 60)
// with a 10-fold eigenvalue among the 16 of smallest modulus.  Prints the
// ratio of the smallest to the largest diagonal entry of the R factor of the
// 16 computed vectors (near 0: nearly dependent vectors) and the largest
// eigen-residual |K v - lambda v| of a vector.
int main() {
    const int n = 60;
    std::mt19937_64 g(3);
    std::normal_distribution<double> d(0.0, 1.0);
    Mat X(n, n), Li(n, n);
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) X(i, j) = cd(d(g), d(g)) + (i == j ? cd(8.0, 0.0) : cd(0.0, 0.0));
    std::vector<cd> lam(n);
    for (int i = 0; i < n; ++i) lam[i] = cd(10.0 + i, 0.5 * i);
    for (int i = 3; i < 13; ++i) lam[i] = cd(6.0, 0.4);  // 10-fold
    Mat D(n, n);
    for (int i = 0; i < n; ++i) D(i, i) = lam[i];
    // K = X D X^{-1}: solve X^T K^T = (X D)^T via inverse of X
    Mat I(n, n);
    for (int i = 0; i < n; ++i) I(i, i) = 1.0;
    Mat Xi;
    solve_lu(X, I, Xi);
    Mat K = matmul(matmul(X, D), Xi);
    EigSolver E;
    E.compute(K, false);
    std::vector<int> idx;
    // the 16 eigenvalues of smallest modulus
    std::vector<int> ord(n);
    for (int i = 0; i < n; ++i) ord[i] = i;
    std::sort(ord.begin(), ord.end(), [&](int a, int b) { return std::abs(E.lam[a]) < std::abs(E.lam[b]); });
    for (int i = 0; i < 16; ++i) idx.push_back(ord[i]);
    auto v = E.vectors_for(idx);
    Mat V(n, 16);
    for (int c = 0; c < 16; ++c)
        for (int i = 0; i < n; ++i) V(i, c) = v[c][i];
    Mat Q, R;
    qr_pos(V, Q, R);
    double mx = 0, mn = 1e300;
    for (int i = 0; i < 16; ++i) { mx = std::max(mx, std::abs(R(i, i))); mn = std::min(mn, std::abs(R(i, i))); }
    // eigen-residual of each vector
    double res = 0;
    for (int c = 0; c < 16; ++c) {
        double r = 0;
        for (int i = 0; i < n; ++i) { cd s = 0; for (int l = 0; l < n; ++l) s += K(i, l) * V(l, c); r += std::norm(s - E.lam[idx[c]] * V(i, c)); }
        res = std::max(res, std::sqrt(r));
    }
    std::printf("R diag ratio %.2e, max eigen-residual %.2e\n", mn / mx, res);
}
