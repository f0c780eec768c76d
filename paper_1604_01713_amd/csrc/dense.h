// Small dense FP64 linear algebra on the host for the per-cycle problems of
// block GCRO-DR: back substitution for the block GMRES least-squares solution,
// thin QR with positive diagonal, Cholesky, and the harmonic-Ritz eigenproblem
// (a complex Schur form by Hessenberg reduction and shifted QR iteration).
// Everything works on column-major std::complex<double> matrices; real
// problems are embedded.
#pragma once

#include <complex>
#include <vector>

namespace bgcr {
namespace dense {

using cd = std::complex<double>;

struct Mat {
    int r = 0, c = 0;
    std::vector<cd> a;
    Mat() = default;
    Mat(int r_, int c_) : r(r_), c(c_), a((size_t)r_ * c_, cd(0.0, 0.0)) {}
    cd& operator()(int i, int j) { return a[(size_t)i + (size_t)j * r]; }
    const cd& operator()(int i, int j) const { return a[(size_t)i + (size_t)j * r]; }
    static Mat eye(int n) {
        Mat I(n, n);
        for (int i = 0; i < n; ++i) I(i, i) = 1.0;
        return I;
    }
    Mat block(int i0, int j0, int nr, int nc) const;
    void set_block(int i0, int j0, const Mat& B);
};

Mat matmul(const Mat& A, const Mat& B);
// A B with B upper triangular (entries below its diagonal not read)
Mat matmul_upper(const Mat& A, const Mat& B);
Mat adjoint(const Mat& A);
double fro(const Mat& A);

// G = R^H R, R upper triangular with real positive diagonal; false if G is
// not numerically positive definite.
bool chol_upper(const Mat& G, Mat& R);
// Pivoted Cholesky of a Hermitian positive semidefinite G: with the column
// order piv, G(piv, piv) = R^H R on the leading r rows, stopping at the first
// pivot at or below tau times the largest diagonal entry.  Returns r (piv[0..r)
// are the numerically independent columns); R is r x r upper triangular.
int chol_pivoted(const Mat& G, double tau, std::vector<int>& piv, Mat& R);
Mat tri_inv_upper(const Mat& R);
// X with R X = B, R upper triangular (leading n x n of R is used)
Mat solve_upper(const Mat& R, const Mat& B);
// X with A X = B, Gaussian elimination with partial pivoting; false if singular
bool solve_lu(const Mat& A, const Mat& B, Mat& X);
// thin Householder QR, A = Q R with diag(R) real and >= 0; lower_bw >= 0
// declares A(i, j) = 0 for i > j + lower_bw (the reflectors then span
// lower_bw + 1 rows; a band Householder preserves)
void qr_pos(const Mat& A, Mat& Q, Mat& R, int lower_bw = -1);

// complex Schur form A = Z T Z^H (T upper triangular)
struct Schur {
    Mat T, Z;
    std::vector<cd> lam;
    bool ok = false;
};
Schur schur(const Mat& A);
// eigenvector of A for eigenvalue index i of the Schur form (unit 2-norm)
std::vector<cd> schur_eigvec(const Schur& S, int i);

// Eigenvalues by Hessenberg reduction and shifted QR restricted to the active
// window (real Francis double shift for real input, complex single shift
// otherwise), then eigenvectors for chosen eigenvalues only, by inverse
// iteration on the Hessenberg matrix.
struct EigSolver {
    int n = 0;
    bool real = true;
    std::vector<cd> Hh;                 // Hessenberg form, row-major
    std::vector<std::vector<cd>> refl;  // Householder vectors of the reduction
    std::vector<double> reflvv;
    std::vector<double> Hd;                  // real input: Hessenberg form, row-major
    std::vector<std::vector<double>> reflr;  // real input: Householder vectors
    std::vector<cd> lam;
    double hnorm = 0.0;
    bool ok = false;
    // A: n x n; real selects the real double-shift path (A must be real)
    void compute(const Mat& A, bool real_input);
    // eigenvector for eigenvalue lambda in the Hessenberg basis (unit 2-norm),
    // orthogonal to `against` (vectors in that basis already chosen for
    // eigenvalues of the same cluster)
    std::vector<cd> hess_vector(cd lambda, const std::vector<std::vector<cd>>& against) const;
    // a Hessenberg-basis vector in the basis of A
    std::vector<cd> to_basis(std::vector<cd> x) const;
    // eigenvectors for lam[i], i in idx, in the basis of A; eigenvalues that
    // inverse iteration cannot separate are taken as one cluster whose vectors
    // are mutually orthogonal
    std::vector<std::vector<cd>> vectors_for(const std::vector<int>& idx) const;
};

// harmonic Ritz selection rules (Section 4.1): k values of smallest modulus
// (largest with `largest`), order (|theta|, Re, Im, index), infinite or NaN
// values never kept; `real` keeps a conjugate pair whole (k may grow by one)
// and returns the basis [Re t, Im t] for it.  Returns the selected indices in
// `idx` and, for real problems, whether index is the first of a pair.
struct Selection {
    std::vector<int> idx;        // eigenvalue indices, in selection order
    std::vector<int> pair_first; // 1 if idx[i] opens a conjugate pair (real case)
    int ncols = 0;               // columns of the real/complex basis
};
Selection select_ritz(const std::vector<cd>& theta, int k, bool largest, bool real);

}  // namespace dense
}  // namespace bgcr
