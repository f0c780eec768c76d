"""Pins of the oracle's ILU(0) and of right preconditioning (the paper
preconditions each system with an incomplete LU factorization, Sections 6.1
and 6.2), against facts that do not depend on the oracle's own code: the
defining property of ILU(0), exact LU where elimination makes no fill
(scipy.linalg.lu), dense LU solutions, and the block Arnoldi relation of the
explicit operator A M^{-1}.  Mistakes planted in the oracle on the CPU must
fail one of them."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import oracle as O
import problems as P
from oracle import bgcrodr as OB
from oracle import ilu as OI


def _random_pattern(n, density, seed, cplx=False):
    """Nonsymmetric random pattern with a full diagonal (diagonally dominant)."""
    rng = np.random.default_rng(seed)
    A = sp.random(n, n, density=density, random_state=rng, format="csr")
    A.data = rng.uniform(-1, 1, A.nnz)
    if cplx:
        A = A.astype(np.complex128)
        A.data = A.data + 1j * rng.uniform(-1, 1, A.nnz)
    rowsum = np.asarray(abs(A).sum(axis=1)).ravel()
    A = (A + sp.diags(rowsum + 1.0)).tocsr()
    A.sort_indices()
    return A


def _matrices():
    # (name, A, whether elimination creates fill outside the pattern)
    yield "convdiff2d", P.convdiff(9, 2, conv=(12.0, -5.0, 0.0)), True
    yield "convdiff3d", P.convdiff(5, 3, diff=(1.0, 0.1, 0.01), conv=(5.0, 5.0, 5.0)), True
    yield "banded", P.banded(60, 4, seed=3), False   # a full band: LU stays inside it
    yield "random", _random_pattern(80, 0.06, 4), True
    yield "random_complex", _random_pattern(70, 0.08, 5, cplx=True), True


def _pattern(A):
    A = A.tocoo()
    return set(zip(A.row.tolist(), A.col.tolist()))


@pytest.mark.parametrize("name,A,fill", list(_matrices()))
def test_ilu0_reproduces_A_on_its_pattern(name, A, fill):
    """Defining property of ILU(0): L unit lower and U upper triangular, both
    inside the pattern of A, with (L U)_ij = A_ij on that pattern."""
    L, U = O.ilu0(A)
    n = A.shape[0]
    assert np.allclose(L.diagonal(), 1.0)
    assert sp.triu(L, 1).nnz == 0 and sp.tril(U, -1).nnz == 0
    pat = _pattern(A)
    assert _pattern(sp.tril(L, -1)) <= pat and _pattern(U) <= pat
    LU = (L @ U).tocsr()
    Ad, LUd = A.toarray(), LU.toarray()
    rows, cols = zip(*sorted(pat))
    rows, cols = np.array(rows), np.array(cols)
    err = np.abs(LUd[rows, cols] - Ad[rows, cols]).max()
    assert err <= 1e-13 * np.abs(Ad).max(), (name, err)
    # it is an incomplete factorization: where elimination creates fill, the
    # product has entries off the pattern; a full band has none (exact LU)
    off = np.ones((n, n), dtype=bool)
    off[rows, cols] = False
    if fill:
        assert np.abs(LUd[off]).max() > 1e-8 * np.abs(Ad).max()
    else:
        assert np.abs(LUd[off]).max() <= 1e-13 * np.abs(Ad).max()


@pytest.mark.parametrize("kind", ["tridiagonal", "dense"])
def test_ilu0_is_exact_lu_without_fill(kind):
    """Where elimination creates no fill (tridiagonal) or the pattern is full
    (dense), ILU(0) is the LU factorization without pivoting: compared with
    scipy.linalg.lu on matrices for which partial pivoting keeps P = I
    (column diagonally dominant)."""
    rng = np.random.default_rng(11)
    n = 40
    if kind == "tridiagonal":
        A = P.convdiff(n, 1, conv=(15.0, 0.0, 0.0))
    else:
        D = rng.uniform(-1, 1, (n, n))
        D += np.diag(np.abs(D).sum(axis=0) + 1.0)
        A = sp.csr_matrix(D)
    Pm, Ld, Ud = sla.lu(A.toarray())
    assert np.array_equal(Pm, np.eye(n))
    L, U = O.ilu0(A)
    assert np.linalg.norm(L.toarray() - Ld) <= 1e-13 * np.linalg.norm(Ld)
    assert np.linalg.norm(U.toarray() - Ud) <= 1e-13 * np.linalg.norm(Ud)


def test_exact_factorization_solves_in_one_block_step():
    """When ILU(0) is exact (tridiagonal A), A M^{-1} = I: every system of a
    recycling sequence is solved by its first block step."""
    A0 = P.convdiff(200, 1, conv=(30.0, 0.0, 0.0))
    rng = np.random.default_rng(2)
    systems = []
    for i in range(3):
        A = (A0 + sp.diags(0.1 * i * rng.uniform(0, 1, A0.shape[0]))).tocsr()
        B = rng.uniform(-1, 1, (A.shape[0], 3))
        systems.append((A, B, np.zeros_like(B)))
    out, U = O.solve_sequence(systems, 1e-10, 5, 2, precond="ilu0")
    for (X, st), (A, B, _) in zip(out, systems):
        assert st["block_steps"] == 1
        assert np.linalg.norm(B - A @ X) <= 1e-10 * np.linalg.norm(B)


@pytest.mark.parametrize("cplx", [False, True])
def test_preconditioned_sequence_matches_dense_lu(cplx):
    w = P.cfg1()
    U = None
    for i, s in enumerate(w.systems):
        A, B = s.A, s.B
        if cplx:
            A = (A.astype(np.complex128) + sp.identity(A.shape[0]) * (5.0 - 40.0j)).tocsr()
            B = B + 0.5j * B[::-1]
        X, U, st = O.solve(A, B, np.zeros_like(B), w.tol, w.m, w.k, U=U, precond="ilu0")
        Ad = A.toarray()
        Xs = np.linalg.solve(Ad, B)
        rel = np.linalg.norm(X - Xs) / np.linalg.norm(Xs)
        assert st["rel_res"] <= w.tol
        assert rel <= np.linalg.cond(Ad) * st["rel_res"] * 1.01 and rel < 1e-6
        # the true (unpreconditioned) residual is what the stopping test used
        assert np.linalg.norm(B - A @ X) / np.linalg.norm(B) <= w.tol


def test_preconditioned_arnoldi_relation_with_explicit_operator():
    """Every traced cycle satisfies the block modified Arnoldi relation of the
    explicit dense A M^{-1} (right preconditioning), with orthonormal [C V];
    and the stored recycled pair satisfies (A M^{-1}) U = C."""
    A = P.convdiff(10, 2, conv=(9.0, 4.0, 0.0))
    rng = np.random.default_rng(6)
    B = rng.uniform(-1, 1, (A.shape[0], 3))
    X, U, st = O.solve(A, B, np.zeros_like(B), 1e-12, 4, 4, max_cycles=3, trace=True, precond="ilu0")
    L, Uf = st["precond_factors"]
    Ahat = A.toarray() @ np.linalg.inv((L @ Uf).toarray())
    assert len(st["trace"]) >= 2
    for tr in st["trace"][1:]:
        cyc, C = tr["cyc"], tr["C_in"]
        me = cyc["m_eff"]
        Wm1 = np.hstack(cyc["V"])
        Wm = Wm1[:, : me * B.shape[1]]
        lhs = Ahat @ Wm
        assert np.linalg.norm(lhs - C @ cyc["F"] - Wm1 @ cyc["H"]) <= 1e-11 * np.linalg.norm(lhs)
        assert np.linalg.norm(C.T @ Wm1) < 1e-10
    for tr in st["trace"]:
        assert np.linalg.norm(Ahat @ tr["U"] - tr["C"]) <= 1e-10 * np.linalg.norm(tr["C"])


# ---- mistakes planted in the oracle must fail a pin -------------------------

def _no_update_ilu(A):
    """ILU(0) with the row update dropped: L = tril(A) D^{-1}, U = triu(A)."""
    A = sp.csr_matrix(A)
    d = A.diagonal()
    L = (sp.tril(A, -1) @ sp.diags(1.0 / d) + sp.identity(A.shape[0])).tocsr()
    return L, sp.triu(A, 0).tocsr()


_true_ilu0 = OI.ilu0


def _lower_diag_ilu(A):
    """The diagonal kept in L instead of U (U with a unit diagonal)."""
    L, U = _true_ilu0(A)
    return (L @ sp.diags(U.diagonal())).tocsr(), (sp.diags(1.0 / U.diagonal()) @ U).tocsr()


def test_mutation_ilu_without_row_update_fails_the_pattern_pin(monkeypatch):
    monkeypatch.setattr(OI, "ilu0", _no_update_ilu)
    monkeypatch.setattr(O, "ilu0", _no_update_ilu)
    with pytest.raises(AssertionError):
        test_ilu0_reproduces_A_on_its_pattern("convdiff2d", P.convdiff(9, 2, conv=(12.0, -5.0, 0.0)), True)


def test_mutation_diagonal_in_L_fails_the_unit_diagonal_pin(monkeypatch):
    monkeypatch.setattr(O, "ilu0", _lower_diag_ilu)
    with pytest.raises(AssertionError):
        test_ilu0_reproduces_A_on_its_pattern("banded", P.banded(60, 4, seed=3), False)


def test_mutation_left_preconditioning_fails_the_arnoldi_pin(monkeypatch):
    """Left preconditioning (Algorithm 1 on M^{-1} A with M^{-1} B) builds the
    Krylov space of another operator: the relation of A M^{-1} fails."""
    real_solve = OB.solve

    def left_solve(A, B, X0, tol, m, k, U=None, precond=None, **kw):
        if precond is None:
            return real_solve(A, B, X0, tol, m, k, U=U, **kw)
        Lf, Uf = _true_ilu0(A)
        import scipy.sparse.linalg as spl
        n = A.shape[0]
        op = spl.LinearOperator((n, n), matvec=lambda v: OI.apply_inverse(Lf, Uf, A @ v),
                                matmat=lambda V: OI.apply_inverse(Lf, Uf, A @ V), dtype=A.dtype)
        X, U, st = real_solve(op, OI.apply_inverse(Lf, Uf, B), X0, tol, m, k, U=U, **kw)
        st["precond_factors"] = (Lf, Uf)
        return X, U, st

    monkeypatch.setattr(OB, "solve", left_solve)
    monkeypatch.setattr(O, "solve", left_solve)
    with pytest.raises(AssertionError):
        test_preconditioned_arnoldi_relation_with_explicit_operator()
