"""ILU(0) and right preconditioning for the block GCRO-DR oracle.

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the CPU
baseline of the benchmark, never by the product path.  Shares no code with the
HIP library.

The paper preconditions every system of its convergence experiments with an
incomplete LU factorization: ILU(0) for each Newton system (Section 6.1) and
ILU with a drop tolerance for each convection-diffusion system (Section 6.2).
Algorithm 1 itself is stated without a preconditioner.  Readings taken here:

  * ILU(0) is the zero-fill incomplete LU factorization of the literature
    (Meijerink and van der Vorst; Saad, Iterative Methods for Sparse Linear
    Systems, Section 10.3): L unit lower triangular and U upper triangular,
    both restricted to the sparsity pattern of A, such that (L U)_ij = A_ij for
    every (i, j) in that pattern.  It is computed by Gaussian elimination in
    row order (the IKJ form) with every update that would fall outside the
    pattern dropped.
  * Preconditioning is from the right, with a factorization per system:
    Algorithm 1 runs on A^[i] M_i^{-1}, M_i = L_i U_i, in the variable
    Xhat = M_i X, and returns X = M_i^{-1} Xhat.  The residual B - A X, hence
    the stopping test, is the unpreconditioned one.  The recycled U lives in
    the preconditioned variable and is carried to the next system unchanged;
    its recycle import forms C from the next system's A M^{-1} U.

Pins (tests/test_oracle_ilu.py, -m "not gpu"): (L U)_ij = A_ij on the pattern
and nothing outside it; exact LU (no pivoting, as scipy.linalg.lu gives with
P = I) where elimination makes no fill (tridiagonal and dense matrices); one
block step per system when the factorization is exact (A M^{-1} = I); the
preconditioned sequence against dense LU; the block Arnoldi relation of the
explicit operator A M^{-1}.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spl


def ilu0(A):
    """ILU(0) of a square CSR matrix with sorted column indices and a nonzero
    diagonal in every row: returns (L, U) as CSR, L with a unit diagonal.

    Row i is eliminated against the finished rows k < i of its own pattern,
    in increasing k: l_ik = a_ik / u_kk, then a_ij -= l_ik u_kj for every
    j > k that row i holds in its pattern (updates to positions outside the
    pattern are dropped)."""
    A = sp.csr_matrix(A)
    A.sort_indices()
    n = A.shape[0]
    rows = []
    for i in range(n):
        lo, hi = A.indptr[i], A.indptr[i + 1]
        rows.append(dict(zip(A.indices[lo:hi].tolist(), A.data[lo:hi].tolist())))
    for i in range(n):
        ri = rows[i]
        if i not in ri:
            raise ValueError(f"ILU(0) needs a diagonal entry in row {i}")
        cols = sorted(ri)
        for k in cols:
            if k >= i:
                break
            rk = rows[k]
            lik = ri[k] / rk[k]
            ri[k] = lik
            for j in cols:
                if j > k and j in rk:
                    ri[j] = ri[j] - lik * rk[j]
    dt = A.dtype
    lower = [(i, j, v) for i, ri in enumerate(rows) for j, v in ri.items() if j < i]
    upper = [(i, j, v) for i, ri in enumerate(rows) for j, v in ri.items() if j >= i]

    def csr_of(entries):
        if not entries:
            return sp.csr_matrix((n, n), dtype=dt)
        ii, jj, vv = zip(*entries)
        return sp.csr_matrix((np.array(vv, dtype=dt), (ii, jj)), shape=(n, n))

    L = csr_of(lower) + sp.identity(n, dtype=dt, format="csr")
    U = csr_of(upper)
    L.sort_indices()
    U.sort_indices()
    return L.tocsr(), U.tocsr()


def apply_inverse(L, U, V):
    """M^{-1} V = U^{-1} (L^{-1} V), two sparse triangular solves."""
    Y = spl.spsolve_triangular(L, V, lower=True, unit_diagonal=True)
    return spl.spsolve_triangular(U, Y, lower=False)


def right_preconditioned(A, L, U):
    """The operator A M^{-1} (M = L U) as a LinearOperator."""
    n = A.shape[0]
    dt = np.result_type(A.dtype, L.dtype)

    def mv(v):
        return A @ apply_inverse(L, U, v)

    def mm(V):
        return A @ apply_inverse(L, U, V)

    return spl.LinearOperator((n, n), matvec=mv, matmat=mm, dtype=dt)
