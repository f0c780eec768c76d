// Small dense FP64 linear algebra on the host (see dense.h).
#include "dense.h"

#include <functional>

#include <omp.h>

#include <algorithm>
#include <cmath>
#include <limits>
#include <numeric>

namespace bgcr {
namespace dense {

static const double EPS = std::numeric_limits<double>::epsilon();

// Host threads for the independent loops of one small problem (output
// columns of a product, columns of Q, eigenvectors); a team only pays off
// above ~1e5 flops of work.
static int team(double work) {
    if (work < 2e5) return 1;
    return std::max(1, std::min(4, omp_get_max_threads()));
}

// sum of x[i] y[i] with eight independent partial sums (two AVX2 vectors),
// combined in a fixed order: the result depends only on the inputs
static inline double dotr(const double* __restrict__ x, const double* __restrict__ y, int len) {
    double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int i = 0;
    for (; i + 8 <= len; i += 8)
        for (int u = 0; u < 8; ++u) s[u] += x[i + u] * y[i + u];
    for (int u = 0; i < len; ++i, ++u) s[u] += x[i] * y[i];
    return ((s[0] + s[4]) + (s[1] + s[5])) + ((s[2] + s[6]) + (s[3] + s[7]));
}

Mat Mat::block(int i0, int j0, int nr, int nc) const {
    Mat B(nr, nc);
    for (int j = 0; j < nc; ++j)
        for (int i = 0; i < nr; ++i) B(i, j) = (*this)(i0 + i, j0 + j);
    return B;
}

void Mat::set_block(int i0, int j0, const Mat& B) {
    for (int j = 0; j < B.c; ++j)
        for (int i = 0; i < B.r; ++i) (*this)(i0 + i, j0 + j) = B(i, j);
}

// Real-arithmetic fast paths: the refresh problems of real systems are real
// (only eigenvectors of complex-conjugate pairs are complex), and real
// arithmetic does a quarter of the work of complex arithmetic.
static bool all_real(const Mat& A) {
    for (const cd& v : A.a)
        if (v.imag() != 0.0) return false;
    return true;
}
static std::vector<double> real_part(const Mat& A) {
    std::vector<double> r(A.a.size());
    for (size_t e = 0; e < r.size(); ++e) r[e] = A.a[e].real();
    return r;
}
static Mat from_real(int r, int c, const std::vector<double>& a) {
    Mat M(r, c);
    for (size_t e = 0; e < a.size(); ++e) M.a[e] = cd(a[e], 0.0);
    return M;
}

Mat matmul(const Mat& A, const Mat& B) {
    if (all_real(A) && all_real(B)) {
        const std::vector<double> a = real_part(A), b = real_part(B);
        std::vector<double> c((size_t)A.r * B.c, 0.0);
#pragma omp parallel for schedule(static) num_threads(team(2.0 * A.r * A.c * B.c))
        for (int j = 0; j < B.c; ++j)
            for (int l = 0; l < A.c; ++l) {
                const double bl = b[(size_t)j * A.c + l];
                if (bl == 0.0) continue;
                const double* al = &a[(size_t)l * A.r];
                double* cj = &c[(size_t)j * A.r];
                for (int i = 0; i < A.r; ++i) cj[i] += al[i] * bl;
            }
        return from_real(A.r, B.c, c);
    }
    Mat C(A.r, B.c);
#pragma omp parallel for schedule(static) num_threads(team(8.0 * A.r * A.c * B.c))
    for (int j = 0; j < B.c; ++j)
        for (int l = 0; l < A.c; ++l) {
            const cd b = B(l, j);
            if (b == cd(0.0, 0.0)) continue;
            const cd* a = &A.a[(size_t)l * A.r];
            cd* c = &C.a[(size_t)j * C.r];
            for (int i = 0; i < A.r; ++i) c[i] += a[i] * b;
        }
    return C;
}

Mat matmul_upper(const Mat& A, const Mat& B) {
    if (all_real(A) && all_real(B)) {
        const std::vector<double> a = real_part(A), b = real_part(B);
        std::vector<double> c((size_t)A.r * B.c, 0.0);
#pragma omp parallel for schedule(dynamic, 4) num_threads(team(1.0 * A.r * A.c * B.c))
        for (int j = 0; j < B.c; ++j)
            for (int l = 0; l <= std::min(j, A.c - 1); ++l) {
                const double bl = b[(size_t)j * A.c + l];
                if (bl == 0.0) continue;
                const double* al = &a[(size_t)l * A.r];
                double* cj = &c[(size_t)j * A.r];
                for (int i = 0; i < A.r; ++i) cj[i] += al[i] * bl;
            }
        return from_real(A.r, B.c, c);
    }
    Mat C(A.r, B.c);
#pragma omp parallel for schedule(dynamic, 4) num_threads(team(4.0 * A.r * A.c * B.c))
    for (int j = 0; j < B.c; ++j)
        for (int l = 0; l <= std::min(j, A.c - 1); ++l) {
            const cd b = B(l, j);
            if (b == cd(0.0, 0.0)) continue;
            const cd* a = &A.a[(size_t)l * A.r];
            cd* c = &C.a[(size_t)j * C.r];
            for (int i = 0; i < A.r; ++i) c[i] += a[i] * b;
        }
    return C;
}

Mat adjoint(const Mat& A) {
    Mat B(A.c, A.r);
    for (int j = 0; j < A.c; ++j)
        for (int i = 0; i < A.r; ++i) B(j, i) = std::conj(A(i, j));
    return B;
}

double fro(const Mat& A) {
    double s = 0.0;
    for (const cd& v : A.a) s += std::norm(v);
    return std::sqrt(s);
}

bool chol_upper(const Mat& G, Mat& R) {
    const int n = G.r;
    R = Mat(n, n);
    double maxd = 0.0;
    for (int i = 0; i < n; ++i) maxd = std::max(maxd, G(i, i).real());
    if (!(maxd > 0.0) || !std::isfinite(maxd)) return false;
    for (int i = 0; i < n; ++i) {
        double d = G(i, i).real();
        for (int l = 0; l < i; ++l) d -= std::norm(R(l, i));
        if (!(d > 1e-24 * maxd) || !std::isfinite(d)) return false;
        const double rii = std::sqrt(d);
        R(i, i) = rii;
        for (int j = i + 1; j < n; ++j) {
            cd s = G(i, j);
            for (int l = 0; l < i; ++l) s -= std::conj(R(l, i)) * R(l, j);
            R(i, j) = s / rii;
        }
    }
    return true;
}

int chol_pivoted(const Mat& G, double tau, std::vector<int>& piv, Mat& R) {
    const int n = G.r;
    Mat W = G, Rf(n, n);  // W: Schur complement, in the current column order
    piv.resize(n);
    for (int i = 0; i < n; ++i) piv[i] = i;
    double gmax = 0.0;
    for (int i = 0; i < n; ++i) gmax = std::max(gmax, G(i, i).real());
    int r = 0;
    if (gmax > 0.0 && std::isfinite(gmax)) {
        for (int j = 0; j < n; ++j) {
            int q = j;
            for (int i = j + 1; i < n; ++i)
                if (W(i, i).real() > W(q, q).real()) q = i;
            if (q != j) {
                for (int c = 0; c < n; ++c) std::swap(W(j, c), W(q, c));
                for (int c = 0; c < n; ++c) std::swap(W(c, j), W(c, q));
                for (int l = 0; l < j; ++l) std::swap(Rf(l, j), Rf(l, q));
                std::swap(piv[j], piv[q]);
            }
            const double d = W(j, j).real();
            if (!(d > tau * gmax) || !std::isfinite(d)) break;
            const double rjj = std::sqrt(d);
            Rf(j, j) = rjj;
            for (int i = j + 1; i < n; ++i) Rf(j, i) = W(j, i) / rjj;
            for (int i = j + 1; i < n; ++i)
                for (int l = j + 1; l < n; ++l) W(i, l) -= std::conj(Rf(j, i)) * Rf(j, l);
            r = j + 1;
        }
    }
    R = Mat(r, r);
    for (int i = 0; i < r; ++i)
        for (int j = i; j < r; ++j) R(i, j) = Rf(i, j);
    return r;
}

Mat tri_inv_upper(const Mat& R) {
    const int n = R.r;
    if (all_real(R)) {
        // rows of R contiguous (rt[i][l] = R(i, l)) for the row-times-column sums
        std::vector<double> rt((size_t)n * n);
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) rt[(size_t)i * n + j] = R.a[(size_t)i + (size_t)j * R.r].real();
        std::vector<double> x((size_t)n * n, 0.0);
        for (int j = 0; j < n; ++j) {
            double* xj = &x[(size_t)j * n];
            xj[j] = 1.0 / rt[(size_t)j * n + j];
            for (int i = j - 1; i >= 0; --i) {
                const double s = dotr(&rt[(size_t)i * n + i + 1], xj + i + 1, j - i);
                xj[i] = -s / rt[(size_t)i * n + i];
            }
        }
        return from_real(n, n, x);
    }
    // rows of R contiguous; the columns of the inverse are independent
    std::vector<cd> rt((size_t)n * n);
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) rt[(size_t)i * n + j] = R(i, j);
    Mat X(n, n);
#pragma omp parallel for schedule(dynamic, 4) num_threads(team(4.0 * n * n * n / 6.0))
    for (int j = 0; j < n; ++j) {
        cd* xj = &X.a[(size_t)j * n];
        xj[j] = 1.0 / rt[(size_t)j * n + j];
        for (int i = j - 1; i >= 0; --i) {
            const cd* ri = &rt[(size_t)i * n];
            cd s = 0.0;
            for (int l = i + 1; l <= j; ++l) s += ri[l] * xj[l];
            xj[i] = -s / ri[i];
        }
    }
    return X;
}

Mat solve_upper(const Mat& R, const Mat& B) {
    const int n = B.r;
    Mat X = B;
    for (int j = 0; j < B.c; ++j)
        for (int i = n - 1; i >= 0; --i) {
            cd s = X(i, j);
            for (int l = i + 1; l < n; ++l) s -= R(i, l) * X(l, j);
            X(i, j) = s / R(i, i);
        }
    return X;
}

bool solve_lu(const Mat& A0, const Mat& B, Mat& X) {
    const int n = A0.r;
    Mat A = A0;
    X = B;
    double amax = 0.0;
    for (const cd& v : A.a) amax = std::max(amax, std::abs(v));
    for (int k = 0; k < n; ++k) {
        int piv = k;
        double best = std::abs(A(k, k));
        for (int i = k + 1; i < n; ++i)
            if (std::abs(A(i, k)) > best) {
                best = std::abs(A(i, k));
                piv = i;
            }
        if (!(best > 1e-300) || !(best > EPS * 1e-4 * amax)) return false;
        if (piv != k) {
            for (int j = 0; j < n; ++j) std::swap(A(k, j), A(piv, j));
            for (int j = 0; j < X.c; ++j) std::swap(X(k, j), X(piv, j));
        }
        for (int i = k + 1; i < n; ++i) {
            const cd f = A(i, k) / A(k, k);
            if (f == cd(0.0, 0.0)) continue;
            for (int j = k; j < n; ++j) A(i, j) -= f * A(k, j);
            for (int j = 0; j < X.c; ++j) X(i, j) -= f * X(k, j);
        }
    }
    X = solve_upper(A, X);
    return true;
}

// Householder vector v (v[0..] over rows i0..m-1 of column x) with
// (I - 2 v v^H / v^H v) x = beta e_1; returns v^H v (0 for the identity).
static double house(const cd* x, int len, std::vector<cd>& v) {
    v.assign(x, x + len);
    double al = 0.0;
    for (int i = 0; i < len; ++i) al += std::norm(x[i]);
    al = std::sqrt(al);
    if (al == 0.0) return 0.0;
    const double ax = std::abs(x[0]);
    const cd ph = ax > 0.0 ? x[0] / ax : cd(1.0, 0.0);
    const cd beta = -al * ph;
    v[0] = x[0] - beta;
    double s = 0.0;
    for (int i = 0; i < len; ++i) s += std::norm(v[i]);
    return s;
}

// real Householder QR with positive diagonal (column-major, m x n); with
// lower bandwidth bw >= 0 (A(i, j) = 0 for i > j + bw, a band Householder
// preserves) the reflector of column k spans rows k .. k + bw only
static void qr_pos_real(const Mat& A0, Mat& Q, Mat& R, int bw) {
    const int m = A0.r, n = A0.c;
    auto rows_of = [&](int k) { return bw < 0 ? m - k : std::min(m - k, bw + 1); };
    std::vector<double> a = real_part(A0);
    auto col = [&](int j) { return &a[(size_t)j * m]; };
    const int kk = std::min(m, n);
    std::vector<std::vector<double>> vs(kk);
    std::vector<double> vvs(kk, 0.0);
    for (int k = 0; k < kk; ++k) {
        double* ck = col(k);
        const int len = rows_of(k);
        const double al = std::sqrt(dotr(ck + k, ck + k, len));
        if (al == 0.0) continue;
        const double beta = ck[k] >= 0.0 ? -al : al;
        std::vector<double>& v = vs[k];
        v.assign(ck + k, ck + k + len);
        v[0] = ck[k] - beta;
        const double vv = dotr(v.data(), v.data(), len);
        vvs[k] = vv;
        if (vv == 0.0) continue;
        const double f = 2.0 / vv;
        for (int j = k; j < n; ++j) {
            double* cj = col(j) + k;
            const double w = f * dotr(v.data(), cj, len);
            for (int i = 0; i < len; ++i) cj[i] -= w * v[i];
        }
    }
    std::vector<double> r((size_t)kk * n, 0.0), q((size_t)m * kk, 0.0);
    for (int j = 0; j < n; ++j)
        for (int i = 0; i <= std::min(j, kk - 1); ++i) r[(size_t)i + (size_t)j * kk] = col(j)[i];
    for (int i = 0; i < kk; ++i) q[(size_t)i + (size_t)i * m] = 1.0;
#pragma omp parallel for schedule(static) num_threads(team(4.0 * m * kk * kk))
    for (int j = 0; j < kk; ++j) {
        for (int k = std::min(j, kk - 1); k >= 0; --k) {  // reflectors k > j leave column j unchanged
            if (vvs[k] == 0.0) continue;
            const std::vector<double>& v = vs[k];
            const int len = (int)v.size();
            double* qj = &q[(size_t)j * m + k];
            const double w = 2.0 / vvs[k] * dotr(v.data(), qj, len);
            for (int i = 0; i < len; ++i) qj[i] -= w * v[i];
        }
    }
    for (int i = 0; i < kk; ++i)
        if (r[(size_t)i + (size_t)i * kk] < 0.0) {
            for (int j = 0; j < n; ++j) r[(size_t)i + (size_t)j * kk] = -r[(size_t)i + (size_t)j * kk];
            for (int rr = 0; rr < m; ++rr) q[(size_t)rr + (size_t)i * m] = -q[(size_t)rr + (size_t)i * m];
        }
    R = from_real(kk, n, r);
    Q = from_real(m, kk, q);
}

void qr_pos(const Mat& A0, Mat& Q, Mat& R, int bw) {
    if (all_real(A0)) {
        qr_pos_real(A0, Q, R, bw);
        return;
    }
    const int m = A0.r, n = A0.c;
    auto end_of = [&](int k) { return bw < 0 ? m : std::min(m, k + bw + 1); };
    Mat A = A0;
    std::vector<std::vector<cd>> vs(n);
    std::vector<double> vvs(n, 0.0);
    for (int k = 0; k < n && k < m; ++k) {
        const int ke = end_of(k);
        vvs[k] = house(&A(k, k), ke - k, vs[k]);
        if (vvs[k] == 0.0) continue;
        const double f = 2.0 / vvs[k];
        for (int j = k; j < n; ++j) {
            cd w = 0.0;
            for (int i = k; i < ke; ++i) w += std::conj(vs[k][i - k]) * A(i, j);
            w *= f;
            for (int i = k; i < ke; ++i) A(i, j) -= vs[k][i - k] * w;
        }
    }
    const int kk = std::min(m, n);
    R = Mat(kk, n);
    for (int j = 0; j < n; ++j)
        for (int i = 0; i <= std::min(j, kk - 1); ++i) R(i, j) = A(i, j);
    // Q = H_0 H_1 ... applied to the first kk columns of the identity
    Q = Mat(m, kk);
    for (int i = 0; i < kk; ++i) Q(i, i) = 1.0;
    for (int k = kk - 1; k >= 0; --k) {
        if (vvs[k] == 0.0) continue;
        const double f = 2.0 / vvs[k];
        const int ke = end_of(k);
        for (int j = 0; j < kk; ++j) {
            cd w = 0.0;
            for (int i = k; i < ke; ++i) w += std::conj(vs[k][i - k]) * Q(i, j);
            w *= f;
            for (int i = k; i < ke; ++i) Q(i, j) -= vs[k][i - k] * w;
        }
    }
    // positive real diagonal
    for (int i = 0; i < kk; ++i) {
        const double a = std::abs(R(i, i));
        if (a == 0.0) continue;
        const cd ph = R(i, i) / a;
        for (int j = 0; j < n; ++j) R(i, j) *= std::conj(ph);
        for (int r = 0; r < m; ++r) Q(r, i) *= ph;
    }
}

// Givens rotation G = [c s; -conj(s) c] with G [f; g] = [r; 0], c real.
static void givens(cd f, cd g, double& c, cd& s) {
    const double af = std::abs(f), ag = std::abs(g);
    if (ag == 0.0) {
        c = 1.0;
        s = 0.0;
        return;
    }
    if (af == 0.0) {
        c = 0.0;
        s = std::conj(g) / ag;
        return;
    }
    const double r = std::hypot(af, ag);
    c = af / r;
    s = (f / af) * std::conj(g) / r;
}

// Complex Schur form by Householder reduction to Hessenberg form and the
// explicitly shifted QR iteration (Wilkinson shift, exceptional shift every
// 11th iteration without deflation).  T is kept row-major and Z transposed so
// that every long loop runs over contiguous memory.
Schur schur(const Mat& A0) {
    const int n = A0.r;
    Schur S;
    S.lam.assign(n, cd(0.0, 0.0));
    S.T = Mat(n, n);
    S.Z = Mat(n, n);
    if (n == 0) {
        S.ok = true;
        return S;
    }
    std::vector<cd> T((size_t)n * n), Zt((size_t)n * n, cd(0.0, 0.0));  // T[i*n+j], Zt[j*n+i] = Z(i, j)
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            const cd v = A0(i, j);
            if (!std::isfinite(v.real()) || !std::isfinite(v.imag())) return S;
            T[(size_t)i * n + j] = v;
        }
    for (int i = 0; i < n; ++i) Zt[(size_t)i * n + i] = 1.0;
    auto Tr = [&](int i) { return &T[(size_t)i * n]; };
    auto Zr = [&](int j) { return &Zt[(size_t)j * n]; };
    std::vector<cd> v, w(n);
    for (int k = 0; k + 2 < n; ++k) {
        const int len = n - k - 1;
        std::vector<cd> x(len);
        for (int i = 0; i < len; ++i) x[i] = Tr(k + 1 + i)[k];
        const double vv = house(x.data(), len, v);
        if (vv == 0.0) continue;
        const double f = 2.0 / vv;
        // left: rows k+1.., w = v^H T_sub, T_sub -= f v w
        std::fill(w.begin(), w.end(), cd(0.0, 0.0));
        for (int i = 0; i < len; ++i) {
            const cd cv = std::conj(v[i]);
            const cd* row = Tr(k + 1 + i);
            for (int j = k; j < n; ++j) w[j] += cv * row[j];
        }
        for (int i = 0; i < len; ++i) {
            const cd fv = f * v[i];
            cd* row = Tr(k + 1 + i);
            for (int j = k; j < n; ++j) row[j] -= fv * w[j];
        }
        // right: columns k+1.. of every row, and of Z
        for (int i = 0; i < n; ++i) {
            cd* row = Tr(i) + k + 1;
            cd dot = 0.0;
            for (int l = 0; l < len; ++l) dot += row[l] * v[l];
            dot *= f;
            for (int l = 0; l < len; ++l) row[l] -= dot * std::conj(v[l]);
        }
        // Z <- Z H: Zt rows k+1.. updated with Zt_sub -= f v^* (v^T Zt_sub)
        std::fill(w.begin(), w.end(), cd(0.0, 0.0));
        for (int l = 0; l < len; ++l) {
            const cd vl = v[l];
            const cd* zr = Zr(k + 1 + l);
            for (int i = 0; i < n; ++i) w[i] += vl * zr[i];
        }
        for (int l = 0; l < len; ++l) {
            const cd fc = f * std::conj(v[l]);
            cd* zr = Zr(k + 1 + l);
            for (int i = 0; i < n; ++i) zr[i] -= fc * w[i];
        }
        for (int i = k + 2; i < n; ++i) Tr(i)[k] = 0.0;
    }
    int hi = n - 1, iter = 0, total = 0;
    std::vector<double> cs(n);
    std::vector<cd> ss(n);
    while (hi > 0) {
        int lo = hi;
        while (lo > 0) {
            const double tst = std::abs(Tr(lo - 1)[lo - 1]) + std::abs(Tr(lo)[lo]);
            if (std::abs(Tr(lo)[lo - 1]) <= EPS * (tst > 0.0 ? tst : 1.0)) {
                Tr(lo)[lo - 1] = 0.0;
                break;
            }
            --lo;
        }
        if (lo == hi) {
            --hi;
            iter = 0;
            continue;
        }
        if (++total > 60 * n) return S;
        ++iter;
        cd mu;
        if (iter % 11 == 0) {
            mu = Tr(hi)[hi] + 0.75 * std::abs(Tr(hi)[hi - 1]);
        } else {
            const cd a = Tr(hi - 1)[hi - 1], b = Tr(hi - 1)[hi], c = Tr(hi)[hi - 1], d = Tr(hi)[hi];
            const cd half = 0.5 * (a - d);
            const cd disc = std::sqrt(half * half + b * c);
            const cd m1 = 0.5 * (a + d) + disc, m2 = 0.5 * (a + d) - disc;
            mu = std::abs(m1 - d) < std::abs(m2 - d) ? m1 : m2;
        }
        for (int k = lo; k <= hi; ++k) Tr(k)[k] -= mu;
        for (int k = lo; k < hi; ++k) {
            double c;
            cd s;
            givens(Tr(k)[k], Tr(k + 1)[k], c, s);
            cs[k] = c;
            ss[k] = s;
            cd* r0 = Tr(k);
            cd* r1 = Tr(k + 1);
            const cd sc = -std::conj(s);
            for (int j = k; j < n; ++j) {
                const cd x = r0[j], y = r1[j];
                r0[j] = c * x + s * y;
                r1[j] = sc * x + c * y;
            }
            r1[k] = 0.0;
        }
        for (int k = lo; k < hi; ++k) {
            const double c = cs[k];
            const cd s = ss[k], scj = std::conj(s);
            const int rmax = std::min(k + 2, hi);
            for (int i = 0; i <= rmax; ++i) {
                cd* row = Tr(i);
                const cd x = row[k], y = row[k + 1];
                row[k] = c * x + scj * y;
                row[k + 1] = -s * x + c * y;
            }
            cd* z0 = Zr(k);
            cd* z1 = Zr(k + 1);
            for (int i = 0; i < n; ++i) {
                const cd x = z0[i], y = z1[i];
                z0[i] = c * x + scj * y;
                z1[i] = -s * x + c * y;
            }
        }
        for (int k = lo; k <= hi; ++k) Tr(k)[k] += mu;
    }
    for (int i = 0; i < n; ++i) {
        S.lam[i] = Tr(i)[i];
        for (int j = 0; j < n; ++j) {
            S.T(i, j) = Tr(i)[j];
            S.Z(i, j) = Zr(j)[i];
        }
    }
    S.ok = true;
    return S;
}

std::vector<cd> schur_eigvec(const Schur& S, int idx) {
    const int n = S.T.r;
    const Mat& T = S.T;
    double tn = 0.0;
    for (const cd& v : T.a) tn = std::max(tn, std::abs(v));
    const double small = std::max(EPS * tn, 1e-300);
    std::vector<cd> x(n, cd(0.0, 0.0));
    const cd lam = T(idx, idx);
    x[idx] = 1.0;
    for (int r = idx - 1; r >= 0; --r) {
        cd s = T(r, idx);
        for (int l = r + 1; l < idx; ++l) s += T(r, l) * x[l];
        cd d = T(r, r) - lam;
        if (std::abs(d) < small) d = small;
        x[r] = -s / d;
    }
    std::vector<cd> y(n, cd(0.0, 0.0));
    for (int l = 0; l <= idx; ++l) {
        const cd xl = x[l];
        if (xl == cd(0.0, 0.0)) continue;
        for (int i = 0; i < n; ++i) y[i] += S.Z(i, l) * xl;
    }
    double nr = 0.0;
    for (const cd& v : y) nr += std::norm(v);
    nr = std::sqrt(nr);
    if (nr > 0.0)
        for (cd& v : y) v /= nr;
    return y;
}

// ---------------------------------------------------------------------------
// eigenvalues (window-restricted QR) + inverse iteration
// ---------------------------------------------------------------------------
static bool eig_real_francis(std::vector<double>& H, int n, std::vector<cd>& lam) {
    auto h = [&](int i, int j) -> double& { return H[(size_t)i * n + j]; };
    double anorm = 0.0;
    for (double v : H) anorm = std::max(anorm, std::fabs(v));
    if (anorm == 0.0) anorm = 1.0;
    int hi = n - 1, iter = 0, total = 0;
    while (hi >= 0) {
        if (hi == 0) {
            lam[0] = h(0, 0);
            break;
        }
        int lo = hi;
        while (lo > 0) {
            double s = std::fabs(h(lo - 1, lo - 1)) + std::fabs(h(lo, lo));
            if (s == 0.0) s = anorm;
            if (std::fabs(h(lo, lo - 1)) <= EPS * s) {
                h(lo, lo - 1) = 0.0;
                break;
            }
            --lo;
        }
        if (lo == hi) {
            lam[hi] = h(hi, hi);
            --hi;
            iter = 0;
            continue;
        }
        if (lo == hi - 1) {
            const double a = h(hi - 1, hi - 1), b = h(hi - 1, hi), c = h(hi, hi - 1), d = h(hi, hi);
            const double p = 0.5 * (a - d), disc = p * p + b * c;
            if (disc >= 0.0) {
                const double r = std::sqrt(disc);
                const double z = p >= 0.0 ? p + r : p - r;
                lam[hi - 1] = d + z;
                lam[hi] = z != 0.0 ? d - b * c / z : d + z;
            } else {
                const double r = std::sqrt(-disc);
                lam[hi - 1] = cd(d + p, r);
                lam[hi] = cd(d + p, -r);
            }
            hi -= 2;
            iter = 0;
            continue;
        }
        if (++total > 40 * n) return false;
        ++iter;
        double s, t;
        if (iter % 10 == 0) {
            // exceptional shift: a perturbed quadratic from the last subdiagonal entries
            const double x = std::fabs(h(hi, hi - 1)) + std::fabs(h(hi - 1, hi - 2));
            s = 1.5 * x + h(hi, hi);
            t = x * x + h(hi, hi) * (1.5 * x);
        } else {
            s = h(hi - 1, hi - 1) + h(hi, hi);
            t = h(hi - 1, hi - 1) * h(hi, hi) - h(hi - 1, hi) * h(hi, hi - 1);
        }
        // first column of H^2 - s H + t I at rows lo, lo+1, lo+2
        double x = h(lo, lo) * h(lo, lo) + h(lo, lo + 1) * h(lo + 1, lo) - s * h(lo, lo) + t;
        double y = h(lo + 1, lo) * (h(lo, lo) + h(lo + 1, lo + 1) - s);
        double z = h(lo + 1, lo) * h(lo + 2, lo + 1);
        for (int k = lo; k <= hi - 1; ++k) {
            const int nr = (k < hi - 1) ? 3 : 2;  // reflector length
            double v0 = x, v1 = y, v2 = nr == 3 ? z : 0.0;
            const double al = std::sqrt(v0 * v0 + v1 * v1 + v2 * v2);
            if (al > 0.0) {
                const double alpha = v0 >= 0.0 ? -al : al;
                v0 -= alpha;
                const double vv = v0 * v0 + v1 * v1 + v2 * v2;
                if (vv > 0.0) {
                    const double tau = 2.0 / vv;
                    const int c0 = std::max(lo, k - 1);
                    for (int j = c0; j <= hi; ++j) {
                        double w = v0 * h(k, j) + v1 * h(k + 1, j) + (nr == 3 ? v2 * h(k + 2, j) : 0.0);
                        w *= tau;
                        h(k, j) -= w * v0;
                        h(k + 1, j) -= w * v1;
                        if (nr == 3) h(k + 2, j) -= w * v2;
                    }
                    const int r1 = std::min(k + 3, hi);
                    for (int i = lo; i <= r1; ++i) {
                        double w = v0 * h(i, k) + v1 * h(i, k + 1) + (nr == 3 ? v2 * h(i, k + 2) : 0.0);
                        w *= tau;
                        h(i, k) -= w * v0;
                        h(i, k + 1) -= w * v1;
                        if (nr == 3) h(i, k + 2) -= w * v2;
                    }
                }
            }
            if (k > lo) {
                h(k + 1, k - 1) = 0.0;
                if (nr == 3) h(k + 2, k - 1) = 0.0;
            }
            if (k < hi - 1) {
                x = h(k + 1, k);
                y = h(k + 2, k);
                z = (k < hi - 2) ? h(k + 3, k) : 0.0;
            }
        }
    }
    return true;
}

static bool eig_complex_window(std::vector<cd>& T, int n, std::vector<cd>& lam) {
    auto Tr = [&](int i) { return &T[(size_t)i * n]; };
    int hi = n - 1, iter = 0, total = 0;
    std::vector<double> cs(n);
    std::vector<cd> ss(n);
    while (hi > 0) {
        int lo = hi;
        while (lo > 0) {
            const double tst = std::abs(Tr(lo - 1)[lo - 1]) + std::abs(Tr(lo)[lo]);
            if (std::abs(Tr(lo)[lo - 1]) <= EPS * (tst > 0.0 ? tst : 1.0)) {
                Tr(lo)[lo - 1] = 0.0;
                break;
            }
            --lo;
        }
        if (lo == hi) {
            lam[hi] = Tr(hi)[hi];
            --hi;
            iter = 0;
            continue;
        }
        if (++total > 60 * n) return false;
        ++iter;
        cd mu;
        if (iter % 11 == 0) {
            mu = Tr(hi)[hi] + 0.75 * std::abs(Tr(hi)[hi - 1]);
        } else {
            const cd a = Tr(hi - 1)[hi - 1], b = Tr(hi - 1)[hi], c = Tr(hi)[hi - 1], d = Tr(hi)[hi];
            const cd half = 0.5 * (a - d);
            const cd disc = std::sqrt(half * half + b * c);
            const cd m1 = 0.5 * (a + d) + disc, m2 = 0.5 * (a + d) - disc;
            mu = std::abs(m1 - d) < std::abs(m2 - d) ? m1 : m2;
        }
        for (int k = lo; k <= hi; ++k) Tr(k)[k] -= mu;
        for (int k = lo; k < hi; ++k) {
            double c;
            cd s;
            givens(Tr(k)[k], Tr(k + 1)[k], c, s);
            cs[k] = c;
            ss[k] = s;
            cd* r0 = Tr(k);
            cd* r1 = Tr(k + 1);
            const cd sc = -std::conj(s);
            for (int j = k; j <= hi; ++j) {
                const cd x = r0[j], y = r1[j];
                r0[j] = c * x + s * y;
                r1[j] = sc * x + c * y;
            }
            r1[k] = 0.0;
        }
        for (int k = lo; k < hi; ++k) {
            const double c = cs[k];
            const cd s = ss[k], scj = std::conj(s);
            const int rmax = std::min(k + 2, hi);
            for (int i = lo; i <= rmax; ++i) {
                cd* row = Tr(i);
                const cd x = row[k], y = row[k + 1];
                row[k] = c * x + scj * y;
                row[k + 1] = -s * x + c * y;
            }
        }
        for (int k = lo; k <= hi; ++k) Tr(k)[k] += mu;
    }
    if (n > 0) lam[0] = Tr(0)[0];
    return true;
}

// Hessenberg reduction of a real row-major matrix by Householder reflectors
// (reflector k acts on rows/columns k+1 .. n-1)
static void hessenberg_real(std::vector<double>& H, int n, std::vector<std::vector<double>>& refl,
                            std::vector<double>& vvs) {
    refl.assign(n, {});
    vvs.assign(n, 0.0);
    std::vector<double> w(n);
    for (int k = 0; k + 2 < n; ++k) {
        const int len = n - k - 1;
        std::vector<double>& v = refl[k];
        v.resize(len);
        double al = 0.0;
        for (int i = 0; i < len; ++i) {
            v[i] = H[(size_t)(k + 1 + i) * n + k];
            al += v[i] * v[i];
        }
        al = std::sqrt(al);
        if (al == 0.0) continue;
        const double beta = v[0] >= 0.0 ? -al : al;
        v[0] -= beta;
        double vv = 0.0;
        for (double x : v) vv += x * x;
        vvs[k] = vv;
        if (vv == 0.0) continue;
        const double f = 2.0 / vv;
        // left: rows k+1.. of columns k..
        std::fill(w.begin(), w.end(), 0.0);
        for (int i = 0; i < len; ++i) {
            const double vi = v[i];
            const double* row = &H[(size_t)(k + 1 + i) * n];
            for (int j = k; j < n; ++j) w[j] += vi * row[j];
        }
        for (int i = 0; i < len; ++i) {
            const double fv = f * v[i];
            double* row = &H[(size_t)(k + 1 + i) * n];
            for (int j = k; j < n; ++j) row[j] -= fv * w[j];
        }
        // right: columns k+1.. of every row
        for (int i = 0; i < n; ++i) {
            double* row = &H[(size_t)i * n + k + 1];
            const double dot = f * dotr(row, v.data(), len);
            for (int l = 0; l < len; ++l) row[l] -= dot * v[l];
        }
        for (int i = k + 2; i < n; ++i) H[(size_t)i * n + k] = 0.0;
    }
}

void EigSolver::compute(const Mat& A, bool real_input) {
    n = A.r;
    real = real_input;
    ok = false;
    lam.assign(n, cd(0.0, 0.0));
    if (real) {
        Hd.assign((size_t)n * n, 0.0);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                const double v = A(i, j).real();
                if (!std::isfinite(v)) return;
                Hd[(size_t)i * n + j] = v;
            }
        hessenberg_real(Hd, n, reflr, reflvv);
        hnorm = 0.0;
        for (double v : Hd) hnorm = std::max(hnorm, std::abs(v));
        std::vector<double> H = Hd;
        ok = eig_real_francis(H, n, lam);
        return;
    }
    Hh.assign((size_t)n * n, cd(0.0, 0.0));
    refl.assign(n, {});
    reflvv.assign(n, 0.0);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            const cd v = A(i, j);
            if (!std::isfinite(v.real()) || !std::isfinite(v.imag())) return;
            Hh[(size_t)i * n + j] = real ? cd(v.real(), 0.0) : v;
        }
    auto Hr = [&](int i) { return &Hh[(size_t)i * n]; };
    std::vector<cd> w(n);
    for (int k = 0; k + 2 < n; ++k) {
        const int len = n - k - 1;
        std::vector<cd> x(len);
        for (int i = 0; i < len; ++i) x[i] = Hr(k + 1 + i)[k];
        std::vector<cd>& v = refl[k];
        const double vv = house(x.data(), len, v);
        reflvv[k] = vv;
        if (vv == 0.0) continue;
        const double f = 2.0 / vv;
        std::fill(w.begin(), w.end(), cd(0.0, 0.0));
        for (int i = 0; i < len; ++i) {
            const cd cv = std::conj(v[i]);
            const cd* row = Hr(k + 1 + i);
            for (int j = k; j < n; ++j) w[j] += cv * row[j];
        }
        for (int i = 0; i < len; ++i) {
            const cd fv = f * v[i];
            cd* row = Hr(k + 1 + i);
            for (int j = k; j < n; ++j) row[j] -= fv * w[j];
        }
        for (int i = 0; i < n; ++i) {
            cd* row = Hr(i) + k + 1;
            cd dot = 0.0;
            for (int l = 0; l < len; ++l) dot += row[l] * v[l];
            dot *= f;
            for (int l = 0; l < len; ++l) row[l] -= dot * std::conj(v[l]);
        }
        for (int i = k + 2; i < n; ++i) Hr(i)[k] = 0.0;
    }
    hnorm = 0.0;
    for (const cd& v : Hh) hnorm = std::max(hnorm, std::abs(v));
    std::vector<cd> T = Hh;
    ok = eig_complex_window(T, n, lam);
}

// inverse iteration with a real shift on the real Hessenberg matrix
static void inverse_iteration_real(const std::vector<double>& Hd, int n, double sh, double pert,
                                   std::vector<double>& x) {
    std::vector<double> U = Hd;
    for (int i = 0; i < n; ++i) U[(size_t)i * n + i] -= sh;
    std::vector<int> swp(n, 0);
    std::vector<double> mult(n, 0.0);
    for (int k = 0; k + 1 < n; ++k) {
        double* rk = &U[(size_t)k * n];
        double* rk1 = &U[(size_t)(k + 1) * n];
        if (std::abs(rk1[k]) > std::abs(rk[k])) {
            for (int j = k; j < n; ++j) std::swap(rk[j], rk1[j]);
            swp[k] = 1;
        }
        if (rk[k] == 0.0) rk[k] = pert;
        const double l = rk1[k] / rk[k];
        mult[k] = l;
        if (l != 0.0)
            for (int j = k; j < n; ++j) rk1[j] -= l * rk[j];
    }
    if (U[(size_t)(n - 1) * n + n - 1] == 0.0) U[(size_t)(n - 1) * n + n - 1] = pert;
    auto nrm = [&](std::vector<double>& v) {
        double s = 0.0;
        for (double a : v) s += a * a;
        s = std::sqrt(s);
        if (s > 0.0)
            for (double& a : v) a /= s;
    };
    nrm(x);
    for (int it = 0; it < 3; ++it) {
        for (int k = 0; k + 1 < n; ++k) {
            if (swp[k]) std::swap(x[k], x[k + 1]);
            x[k + 1] -= mult[k] * x[k];
        }
        for (int i = n - 1; i >= 0; --i) {
            const double* row = &U[(size_t)i * n];
            x[i] = (x[i] - dotr(row + i + 1, x.data() + i + 1, n - i - 1)) / row[i];
        }
        nrm(x);
    }
}

// back to the basis of A: x <- H_0 H_1 ... H_{n-3} x
std::vector<cd> EigSolver::to_basis(std::vector<cd> x) const {
    auto back = [&](std::vector<cd>& x) {
        for (int k = n - 3; k >= 0; --k) {
            if (reflvv[k] == 0.0) continue;
            const double f = 2.0 / reflvv[k];
            const int len = n - k - 1;
            cd d = 0.0;
            if (real) {
                const std::vector<double>& v = reflr[k];
                for (int l = 0; l < len; ++l) d += v[l] * x[k + 1 + l];
                d *= f;
                for (int l = 0; l < len; ++l) x[k + 1 + l] -= d * v[l];
            } else {
                const std::vector<cd>& v = refl[k];
                for (int l = 0; l < len; ++l) d += std::conj(v[l]) * x[k + 1 + l];
                d *= f;
                for (int l = 0; l < len; ++l) x[k + 1 + l] -= d * v[l];
            }
        }
    };
    back(x);
    return x;
}

std::vector<cd> EigSolver::hess_vector(cd lambda, const std::vector<std::vector<cd>>& against) const {
    // inverse iteration on the Hessenberg matrix with a slightly perturbed shift
    const double pert = std::max(hnorm, 1e-300) * 1e-13;
    const cd sh = lambda + cd(pert, 0.0);
    std::vector<cd> x(n);
    uint64_t st = 0x9E3779B97F4A7C15ull;
    std::vector<double> x0(n);
    for (int i = 0; i < n; ++i) {
        st ^= st << 13;
        st ^= st >> 7;
        st ^= st << 17;
        x0[i] = 0.5 + (double)(st % 1000003) / 1000003.0;
    }
    if (real && lambda.imag() == 0.0 && against.empty()) {
        inverse_iteration_real(Hd, n, sh.real(), pert, x0);
        for (int i = 0; i < n; ++i) x[i] = cd(x0[i], 0.0);
        return x;
    }
    std::vector<cd> U((size_t)n * n);
    if (real)
        for (size_t e = 0; e < U.size(); ++e) U[e] = cd(Hd[e], 0.0);
    else
        for (size_t e = 0; e < U.size(); ++e) U[e] = Hh[e];
    for (int i = 0; i < n; ++i) U[(size_t)i * n + i] -= sh;
    // Hessenberg LU with partial pivoting (only rows k, k+1 compete); record ops
    std::vector<int> swp(n, 0);
    std::vector<cd> mult(n, cd(0.0, 0.0));
    for (int k = 0; k + 1 < n; ++k) {
        cd* rk = &U[(size_t)k * n];
        cd* rk1 = &U[(size_t)(k + 1) * n];
        if (std::abs(rk1[k]) > std::abs(rk[k])) {
            for (int j = k; j < n; ++j) std::swap(rk[j], rk1[j]);
            swp[k] = 1;
        }
        if (std::abs(rk[k]) == 0.0) rk[k] = pert;
        const cd l = rk1[k] / rk[k];
        mult[k] = l;
        if (l != cd(0.0, 0.0))
            for (int j = k; j < n; ++j) rk1[j] -= l * rk[j];
    }
    if (std::abs(U[(size_t)(n - 1) * n + n - 1]) == 0.0) U[(size_t)(n - 1) * n + n - 1] = pert;
    auto solve = [&](std::vector<cd>& b) {
        for (int k = 0; k + 1 < n; ++k) {
            if (swp[k]) std::swap(b[k], b[k + 1]);
            b[k + 1] -= mult[k] * b[k];
        }
        for (int i = n - 1; i >= 0; --i) {
            const cd* row = &U[(size_t)i * n];
            cd s = b[i];
            for (int j = i + 1; j < n; ++j) s -= row[j] * b[j];
            b[i] = s / row[i];
        }
    };
    auto orth_normalize = [&](std::vector<cd>& x) {
        for (const auto& a : against) {
            cd d = 0.0;
            for (int i = 0; i < n; ++i) d += std::conj(a[i]) * x[i];
            for (int i = 0; i < n; ++i) x[i] -= d * a[i];
        }
        double nr = 0.0;
        for (const cd& v : x) nr += std::norm(v);
        nr = std::sqrt(nr);
        if (nr > 0.0)
            for (cd& v : x) v /= nr;
    };
    for (int i = 0; i < n; ++i) x[i] = cd(x0[i], 0.0);
    orth_normalize(x);
    for (int it = 0; it < 3; ++it) {
        solve(x);
        orth_normalize(x);
    }
    return x;
}

std::vector<std::vector<cd>> EigSolver::vectors_for(const std::vector<int>& idx) const {
    // clusters: eigenvalues closer than 1e-10 |H| (a thousand times the
    // shift perturbation), joined transitively.  Inverse iteration cannot
    // tell such eigenvalues apart and would return nearly the same vector for
    // each; within a cluster the vectors are computed in turn, each kept
    // orthogonal to the earlier ones (for a multiple eigenvalue an orthonormal
    // basis of its eigenspace).  Clusters run concurrently.
    const int k = (int)idx.size();
    const double tol = 1e-10 * std::max(hnorm, 1e-300);
    std::vector<int> root(k);
    for (int i = 0; i < k; ++i) root[i] = i;
    std::function<int(int)> find = [&](int i) { return root[i] == i ? i : root[i] = find(root[i]); };
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < i; ++j)
            if (std::abs(lam[idx[i]] - lam[idx[j]]) <= tol) root[find(i)] = find(j);
    std::vector<std::vector<int>> groups;
    std::vector<int> gof(k, -1);
    for (int i = 0; i < k; ++i) {
        const int r = find(i);
        if (gof[r] < 0) {
            gof[r] = (int)groups.size();
            groups.emplace_back();
        }
        groups[gof[r]].push_back(i);
    }
    std::vector<std::vector<cd>> out(k);
#pragma omp parallel for schedule(dynamic, 1) num_threads(team(20.0 * n * n * k))
    for (int g = 0; g < (int)groups.size(); ++g) {
        std::vector<std::vector<cd>> hv;
        for (int i : groups[g]) {
            hv.push_back(hess_vector(lam[idx[i]], hv));
            out[i] = to_basis(hv.back());
        }
    }
    return out;
}

Selection select_ritz(const std::vector<cd>& theta, int k, bool largest, bool real) {
    Selection sel;
    std::vector<int> order;
    for (int i = 0; i < (int)theta.size(); ++i)
        if (std::isfinite(theta[i].real()) && std::isfinite(theta[i].imag())) order.push_back(i);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        const double ma = std::abs(theta[a]), mb = std::abs(theta[b]);
        if (ma != mb) return largest ? ma > mb : ma < mb;
        if (theta[a].real() != theta[b].real()) return theta[a].real() < theta[b].real();
        if (theta[a].imag() != theta[b].imag()) return theta[a].imag() < theta[b].imag();
        return a < b;
    });
    if (!real) {
        for (int i = 0; i < (int)order.size() && (int)sel.idx.size() < k; ++i) {
            sel.idx.push_back(order[i]);
            sel.pair_first.push_back(0);
        }
        sel.ncols = (int)sel.idx.size();
        return sel;
    }
    std::vector<char> used(theta.size(), 0);
    for (int oi = 0; oi < (int)order.size() && sel.ncols < k; ++oi) {
        const int i = order[oi];
        if (used[i]) continue;
        const cd th = theta[i];
        if (std::abs(th.imag()) <= 1e-9 * std::max(std::abs(th), 1e-300)) {
            sel.idx.push_back(i);
            sel.pair_first.push_back(0);
            used[i] = 1;
            sel.ncols += 1;
        } else {
            int jp = -1;
            double best = 0.0;
            for (int oj = 0; oj < (int)order.size(); ++oj) {
                const int j = order[oj];
                if (used[j] || j == i) continue;
                const double dd = std::abs(theta[j] - std::conj(th));
                if (jp < 0 || dd < best) {
                    best = dd;
                    jp = j;
                }
            }
            if (jp < 0) continue;
            const int ip = th.imag() > 0 ? i : jp;
            sel.idx.push_back(ip);
            sel.pair_first.push_back(1);
            used[i] = 1;
            used[jp] = 1;
            sel.ncols += 2;
        }
    }
    return sel;
}

}  // namespace dense
}  // namespace bgcr
