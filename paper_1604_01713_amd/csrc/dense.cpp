// Small dense FP64 linear algebra on the host (see dense.h).
#include "dense.h"

#include <algorithm>
#include <cmath>
#include <limits>
#include <numeric>

namespace bgcr {
namespace dense {

static const double EPS = std::numeric_limits<double>::epsilon();

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

Mat matmul(const Mat& A, const Mat& B) {
    Mat C(A.r, B.c);
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

Mat tri_inv_upper(const Mat& R) {
    const int n = R.r;
    Mat X(n, n);
    for (int j = 0; j < n; ++j) {
        X(j, j) = 1.0 / R(j, j);
        for (int i = j - 1; i >= 0; --i) {
            cd s = 0.0;
            for (int l = i + 1; l <= j; ++l) s += R(i, l) * X(l, j);
            X(i, j) = -s / R(i, i);
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

void qr_pos(const Mat& A0, Mat& Q, Mat& R) {
    const int m = A0.r, n = A0.c;
    Mat A = A0;
    std::vector<std::vector<cd>> vs(n);
    std::vector<double> vvs(n, 0.0);
    for (int k = 0; k < n && k < m; ++k) {
        vvs[k] = house(&A(k, k), m - k, vs[k]);
        if (vvs[k] == 0.0) continue;
        const double f = 2.0 / vvs[k];
        for (int j = k; j < n; ++j) {
            cd w = 0.0;
            for (int i = k; i < m; ++i) w += std::conj(vs[k][i - k]) * A(i, j);
            w *= f;
            for (int i = k; i < m; ++i) A(i, j) -= vs[k][i - k] * w;
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
        for (int j = 0; j < kk; ++j) {
            cd w = 0.0;
            for (int i = k; i < m; ++i) w += std::conj(vs[k][i - k]) * Q(i, j);
            w *= f;
            for (int i = k; i < m; ++i) Q(i, j) -= vs[k][i - k] * w;
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

Schur schur(const Mat& A0) {
    const int n = A0.r;
    Schur S;
    S.T = A0;
    S.Z = Mat::eye(n);
    Mat& T = S.T;
    Mat& Z = S.Z;
    S.lam.assign(n, cd(0.0, 0.0));
    if (n == 0) {
        S.ok = true;
        return S;
    }
    for (const cd& v : T.a)
        if (!std::isfinite(v.real()) || !std::isfinite(v.imag())) return S;
    // Hessenberg reduction by Householder reflections
    std::vector<cd> v;
    for (int k = 0; k + 2 < n; ++k) {
        const int len = n - k - 1;
        std::vector<cd> x(len);
        for (int i = 0; i < len; ++i) x[i] = T(k + 1 + i, k);
        const double vv = house(x.data(), len, v);
        if (vv == 0.0) continue;
        const double f = 2.0 / vv;
        for (int j = k; j < n; ++j) {
            cd w = 0.0;
            for (int i = 0; i < len; ++i) w += std::conj(v[i]) * T(k + 1 + i, j);
            w *= f;
            for (int i = 0; i < len; ++i) T(k + 1 + i, j) -= v[i] * w;
        }
        for (int i = 0; i < n; ++i) {
            cd w = 0.0;
            for (int l = 0; l < len; ++l) w += T(i, k + 1 + l) * v[l];
            w *= f;
            for (int l = 0; l < len; ++l) T(i, k + 1 + l) -= w * std::conj(v[l]);
        }
        for (int i = 0; i < n; ++i) {
            cd w = 0.0;
            for (int l = 0; l < len; ++l) w += Z(i, k + 1 + l) * v[l];
            w *= f;
            for (int l = 0; l < len; ++l) Z(i, k + 1 + l) -= w * std::conj(v[l]);
        }
        for (int i = k + 2; i < n; ++i) T(i, k) = 0.0;
    }
    // shifted QR iteration (Wilkinson shift, exceptional shifts on stagnation)
    int hi = n - 1, iter = 0, total = 0;
    std::vector<double> cs(n);
    std::vector<cd> ss(n);
    while (hi > 0) {
        int lo = hi;
        while (lo > 0) {
            const double tst = std::abs(T(lo - 1, lo - 1)) + std::abs(T(lo, lo));
            if (std::abs(T(lo, lo - 1)) <= EPS * (tst > 0.0 ? tst : 1.0)) {
                T(lo, lo - 1) = 0.0;
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
            mu = T(hi, hi) + 0.75 * std::abs(T(hi, hi - 1));
        } else {
            const cd a = T(hi - 1, hi - 1), b = T(hi - 1, hi), c = T(hi, hi - 1), d = T(hi, hi);
            const cd half = 0.5 * (a - d);
            const cd disc = std::sqrt(half * half + b * c);
            const cd m1 = 0.5 * (a + d) + disc, m2 = 0.5 * (a + d) - disc;
            mu = std::abs(m1 - d) < std::abs(m2 - d) ? m1 : m2;
        }
        for (int k = lo; k <= hi; ++k) T(k, k) -= mu;
        for (int k = lo; k < hi; ++k) {
            double c;
            cd s;
            givens(T(k, k), T(k + 1, k), c, s);
            cs[k] = c;
            ss[k] = s;
            for (int j = k; j < n; ++j) {
                const cd x = T(k, j), y = T(k + 1, j);
                T(k, j) = c * x + s * y;
                T(k + 1, j) = -std::conj(s) * x + c * y;
            }
            T(k + 1, k) = 0.0;
        }
        for (int k = lo; k < hi; ++k) {
            const double c = cs[k];
            const cd s = ss[k];
            const int rmax = std::min(k + 2, hi);
            for (int i = 0; i <= rmax; ++i) {
                const cd x = T(i, k), y = T(i, k + 1);
                T(i, k) = c * x + std::conj(s) * y;
                T(i, k + 1) = -s * x + c * y;
            }
            for (int i = 0; i < n; ++i) {
                const cd x = Z(i, k), y = Z(i, k + 1);
                Z(i, k) = c * x + std::conj(s) * y;
                Z(i, k + 1) = -s * x + c * y;
            }
        }
        for (int k = lo; k <= hi; ++k) T(k, k) += mu;
    }
    for (int i = 0; i < n; ++i) S.lam[i] = T(i, i);
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
