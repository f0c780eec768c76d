"""Pins of the FP64 oracle against facts the paper and the mathematics fix.

Each test names the relation it checks.  None of them re-types the oracle's
own formula: they use dense LU, scipy's GMRES, closed-form eigenvalues,
brute-force least squares and exact invariants of the method.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle as O
import pinlib
import problems as P


def _small(N=12, conv=(6.0, 3.0, 0.0), p=3, seed=0, cplx=False):
    A = P.convdiff(N, 2, conv=conv)
    if cplx:
        A = (A.astype(np.complex128) + sp.identity(A.shape[0]) * (-30.0 + 15.0j)).tocsr()
    rng = np.random.default_rng(seed)
    B = rng.uniform(-1, 1, (A.shape[0], p))
    if cplx:
        B = B + 1j * rng.uniform(-1, 1, B.shape)
    return A, B


# ---- P1: dense LU (the plain definition X* = A^{-1} B) ---------------------

def test_cfg1_sequence_matches_dense_lu():
    w = P.cfg1()
    U = None
    for s in w.systems:
        X, U, st = O.solve(s.A, s.B, s.X0, w.tol, w.m, w.k, U=U)
        Ad = s.A.toarray()
        Xs = np.linalg.solve(Ad, s.B)
        kappa = np.linalg.cond(Ad)
        assert st["rel_res"] <= w.tol
        rel_err = np.linalg.norm(X - Xs) / np.linalg.norm(Xs)
        # forward error bound: ||dx||/||x|| <= kappa ||r||/||b||
        assert rel_err <= kappa * st["rel_res"] * 1.01
        assert rel_err < 1e-6


def test_complex_matches_dense_lu():
    A, B = _small(N=10, cplx=True, p=2)
    X, U, st = O.solve(A, B, np.zeros_like(B), 1e-10, 6, 4)
    Xs = np.linalg.solve(A.toarray(), B)
    assert np.linalg.norm(X - Xs) / np.linalg.norm(Xs) < 1e-7
    X2, U2, st2 = O.solve(A, B * 0.5, np.zeros_like(B), 1e-10, 6, 4, U=U)
    assert np.linalg.norm(X2 - 0.5 * Xs) / np.linalg.norm(0.5 * Xs) < 1e-7


# ---- P2/P3/P4: block modified Arnoldi relation, orthonormality, A U = C ----

@pytest.mark.parametrize("cplx", [False, True])
def test_modified_arnoldi_relation_and_orthonormality(cplx):
    A, B = _small(cplx=cplx)
    X, U, st = O.solve(A, B, np.zeros_like(B), 1e-10, 5, 4, max_cycles=4, trace=True)
    assert len(st["trace"]) >= 3
    Ad = A.toarray()
    for tr in st["trace"][1:]:
        cyc, C = tr["cyc"], tr["C_in"]
        V = cyc["V"]
        me = cyc["m_eff"]
        Wm1 = np.hstack(V)
        Wm = Wm1[:, : me * B.shape[1]]
        lhs = Ad @ Wm
        rhs = C @ cyc["F"] + Wm1 @ cyc["H"]
        # eq. block-modified-arnoldi: A W_m = C F_m + W_{m+1} H_m
        assert np.linalg.norm(lhs - rhs) <= 1e-12 * np.linalg.norm(lhs)
        I = np.eye(Wm1.shape[1])
        assert np.linalg.norm(Wm1.conj().T @ Wm1 - I) < 1e-13
        assert np.linalg.norm(C.conj().T @ C - np.eye(C.shape[1])) < 1e-13
        assert np.linalg.norm(C.conj().T @ Wm1) < 1e-13
        # subdiagonal blocks are upper triangular (Section 3.1)
        p = B.shape[1]
        H = cyc["H"]
        for j in range(me):
            blk = H[(j + 1) * p:(j + 2) * p, j * p:(j + 1) * p]
            assert np.allclose(np.tril(blk, -1), 0)
            # and every block below the subdiagonal is zero
            assert np.allclose(H[(j + 2) * p:, j * p:(j + 1) * p], 0)
    for tr in st["trace"]:
        U_, C_ = tr["U"], tr["C"]
        # A U = C with orthonormal C (Algorithm 1: C <- A U orthonormal)
        assert np.linalg.norm(Ad @ U_ - C_) <= 1e-11 * np.linalg.norm(C_)
        assert np.linalg.norm(C_.conj().T @ C_ - np.eye(C_.shape[1])) < 1e-12


def test_recycle_import_gives_AU_equals_C():
    A, B = _small()
    X, U, st = O.solve(A, B, np.zeros_like(B), 1e-9, 5, 4)
    A2 = (A + sp.diags(np.linspace(0, 1, A.shape[0]))).tocsr()
    U2, C2, X0, R0 = O.recycle_import(A2, U, np.zeros_like(B), B.copy())
    assert np.linalg.norm(A2 @ U2 - C2) < 1e-11 * np.linalg.norm(C2)
    assert np.linalg.norm(C2.T @ C2 - np.eye(C2.shape[1])) < 1e-13
    # R0 <- (I - Phi) R0 is orthogonal to C and equals B - A X0
    assert np.linalg.norm(C2.T @ R0) < 1e-12 * np.linalg.norm(B)
    assert np.linalg.norm(R0 - (B - A2 @ X0)) < 1e-12 * np.linalg.norm(B)


# ---- P5: residual equivalence (Proposition residual-equiv) ----------------

@pytest.mark.parametrize("cplx", [False, True])
def test_recurrence_residual_equals_true_residual(cplx):
    A, B = _small(cplx=cplx, p=4)
    X, U, st = O.solve(A, B, np.zeros_like(B), 1e-10, 4, 5, max_cycles=8)
    assert max(st["recur_drift"]) < 1e-12


# ---- P6: monotone LSQ residual within a cycle (nested spaces) -------------

def test_rho_monotone_within_cycle():
    w = P.cfg1()
    s = w.systems[0]
    X, U, st = O.solve(s.A, s.B, s.X0, w.tol, w.m, w.k)
    for rh in st["rho"]:
        assert all(b <= a * (1 + 1e-12) for a, b in zip(rh, rh[1:]))


# ---- P7: minimal residual over U + K_m by brute force ----------------------

@pytest.mark.parametrize("cplx", [False, True])
def test_cycle_is_minimal_residual_over_augmented_space(cplx):
    A, B = _small(N=9, p=2, cplx=cplx)
    X, U, st = O.solve(A, B, np.zeros_like(B), 1e-12, 4, 3, max_cycles=4, trace=True)
    Ad = A.toarray()
    for i in range(1, len(st["trace"])):
        prev, tr = st["trace"][i - 1], st["trace"][i]
        R_prev = prev["R"]
        U_in = tr["U_in"]
        cyc = tr["cyc"]
        Wm = np.hstack(cyc["V"][: cyc["m_eff"]])
        basis = np.hstack([U_in, Wm])
        AB = Ad @ basis
        # columnwise min over span(basis) -- the block residual minimisation decouples
        Zb, *_ = np.linalg.lstsq(AB, R_prev, rcond=None)
        best = R_prev - AB @ Zb
        assert np.linalg.norm(tr["R"]) == pytest.approx(np.linalg.norm(best), rel=1e-8)
        assert np.linalg.norm(tr["R"] - best) < 1e-9 * np.linalg.norm(R_prev)


# ---- P8: k = 0, p = 1 reduces to restarted GMRES(m) (scipy) ----------------

@pytest.mark.parametrize("cycles", [1, 2, 4])
def test_k0_p1_is_gmres_m(cycles):
    A = P.convdiff(10, 2, conv=(5.0, 3.0, 0.0))
    n = A.shape[0]
    b = np.random.default_rng(1).uniform(-1, 1, (n, 1))
    x, _ = spla.gmres(A, b[:, 0], x0=np.zeros(n), rtol=1e-300, atol=0.0, restart=7, maxiter=cycles)
    X, U, st = O.solve(A, b, np.zeros((n, 1)), 1e-300, 7, 0, max_cycles=cycles)
    assert st["cycles"] == cycles
    assert np.linalg.norm(X[:, 0] - x) <= 1e-12 * np.linalg.norm(x)


def test_k0_block_is_block_gmres_over_block_krylov_space():
    """k=0, one cycle: the correction is the column-wise minimal residual over
    blspan{R0, A R0, ..., A^{m-1} R0} (eq. block-Krylov-sum-space), built here
    from explicit powers."""
    A, B = _small(N=8, p=3)
    m = 3
    X, U, st = O.solve(A, B, np.zeros_like(B), 1e-300, m, 0, max_cycles=1)
    Ad = A.toarray()
    K = [B]
    for _ in range(m - 1):
        K.append(Ad @ K[-1])
    K = np.hstack(K)
    Qk, _ = np.linalg.qr(K)
    Zb, *_ = np.linalg.lstsq(Ad @ Qk, B, rcond=None)
    Xb = Qk @ Zb
    assert np.linalg.norm(X - Xb) < 1e-9 * np.linalg.norm(Xb)


# ---- enlarged block (p = 1, block size L > 1; Section 3.1) ------------------

def test_splitmix64_matches_published_outputs():
    """The enlarging vectors come from SplitMix64; its first three outputs from
    seed 0 (states golden, 2 golden, 3 golden) are published test values."""
    g = int(0x9E3779B97F4A7C15)
    out = O.splitmix64(np.array([0, g, (2 * g) % 2**64], dtype=np.uint64))
    assert [int(v) for v in out] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    Z = O.enlarging_vectors(1000, 4, seed=0)
    assert Z.shape == (1000, 3) and Z.min() >= -1.0 and Z.max() < 1.0
    assert abs(Z.mean()) < 0.05 and abs(Z.std() - 1 / np.sqrt(3)) < 0.02


def test_enlarged_block_cycle_is_min_residual_over_block_krylov_space():
    """p = 1, L = 3, k = 0, one cycle: the correction minimises the single
    residual over blspan{[r Z], A [r Z], ..., A^{m-1} [r Z]} (eq.
    1rhs-block-gmres-min), built here from explicit powers."""
    A, B = _small(N=9, p=1)
    m, L = 3, 3
    X, U, st = O.solve(A, B, np.zeros_like(B), 1e-300, m, 0, max_cycles=1, block_size=L)
    Ad = A.toarray()
    K = [np.hstack([B, O.enlarging_vectors(A.shape[0], L)])]
    for _ in range(m - 1):
        K.append(Ad @ K[-1])
    Qk, _ = np.linalg.qr(np.hstack(K))
    zb, *_ = np.linalg.lstsq(Ad @ Qk, B, rcond=None)
    xb = Qk @ zb
    assert np.linalg.norm(X - xb) < 1e-9 * np.linalg.norm(xb)
    # the enlarged space is richer: a smaller residual than one GMRES(m) cycle
    Xg, _, _ = O.solve(A, B, np.zeros_like(B), 1e-300, m, 0, max_cycles=1)
    assert np.linalg.norm(B - A @ X) < np.linalg.norm(B - A @ Xg)


def test_enlarged_block_sequence_with_recycling_matches_dense_lu():
    A, B = _small(N=10, p=1)
    systems = [(A, B, np.zeros_like(B)),
               ((A + 0.05 * sp.identity(A.shape[0])).tocsr(), B[::-1].copy(), np.zeros_like(B))]
    out, U = O.solve_sequence(systems, 1e-10, 4, 5, block_size=4)
    for (Ai, Bi, _), (X, st) in zip(systems, out):
        Xd = np.linalg.solve(Ai.toarray(), Bi)
        assert np.linalg.norm(X - Xd) <= 1e-8 * np.linalg.norm(Xd)
        assert st["rel_res"] <= 1e-10
    assert U.shape[1] in (5, 6)


def test_enlarged_block_basis_is_orthogonal_to_C():
    """With a recycled space the enlarged start block is (I - C C^H) [r, Z]:
    the basis of every cycle is orthogonal to C, as the modified Arnoldi
    relation (eq. block-modified-arnoldi) needs."""
    A, B = _small(N=10, p=1)
    X, U, st = O.solve(A, B, np.zeros_like(B), 1e-10, 4, 5, block_size=4, trace=True)
    assert st["cycles"] >= 3
    for tr in st["trace"][1:]:
        C = tr["C_in"]
        Wm1 = np.hstack(tr["cyc"]["V"])
        assert np.linalg.norm(C.conj().T @ Wm1) < 1e-12
        assert np.linalg.norm(Wm1.conj().T @ Wm1 - np.eye(Wm1.shape[1])) < 1e-12


def _augmented_min_residual(Ad, U, C, r, Z, m):
    """Brute force: the smallest ||r - A S y|| over S = [U, K], K the Krylov
    space of (I - C C^H) A from the start block (I - C C^H) [r, Z] (Z may have
    no columns), built from explicit powers."""
    proj = (lambda M: M - C @ (C.conj().T @ M)) if C is not None else (lambda M: M)
    blk = proj(np.hstack([r, Z]))
    K = [blk]
    for _ in range(m - 1):
        K.append(proj(Ad @ K[-1]))
    S = np.hstack(([U] if U is not None else []) + K)
    Q, _ = np.linalg.qr(S)
    z, *_ = np.linalg.lstsq(Ad @ Q, r, rcond=None)
    return Q @ z


def test_hybrid_enlarged_then_single_cycles_are_min_residual():
    """Section 4.1.3 hybrid: the first cycles of the sequence enlarge the block
    (p = 1, L = 4), every later one is non-block GCRO-DR.  Each traced cycle's
    correction equals the brute-force minimiser over span(U) plus the Krylov
    space of its own block size; the final X matches dense LU."""
    A, B = _small(N=10, p=1)
    A2 = (A + 0.05 * sp.identity(A.shape[0])).tocsr()
    m, k, L, E = 4, 5, 4, 3
    n = A.shape[0]
    Z = O.enlarging_vectors(n, L)
    sizes, checked = [], 0
    U = None
    left = E
    for Ai, Bi in ((A, B), (A2, B[::-1].copy())):
        Ad = Ai.toarray()
        X, U, st = O.solve(Ai, Bi, np.zeros_like(Bi), 1e-10, m, k, U=U, block_size=L, trace=True,
                           enlarged_cycles=left)
        left = max(0, left - st["cycles"])
        sizes += st["block_size"]
        # cycles after the first of a system: the previous trace holds X, R before it
        for prev, tr in zip(st["trace"], st["trace"][1:]):
            r = Bi - Ad @ prev["X"]
            Lc = tr["cyc"]["V"][0].shape[1]
            d = _augmented_min_residual(Ad, tr["U_in"], tr["C_in"], r, Z if Lc == L else Z[:, :0], m)
            if tr["cyc"]["m_eff"] == m:
                # relative to the correction, plus rounding of X itself
                tol_d = 1e-8 * np.linalg.norm(d) + 1e-13 * np.linalg.norm(tr["X"])
                assert np.linalg.norm(tr["X"] - prev["X"] - d) < tol_d
                checked += 1
        Xd = np.linalg.solve(Ad, Bi)
        assert np.linalg.norm(X - Xd) <= 1e-8 * np.linalg.norm(Xd)
    assert sizes[:E] == [L] * E and all(b == 1 for b in sizes[E:]) and len(sizes) > E
    assert checked >= 3
    # the sequence driver counts the enlarged cycles over the whole sequence
    out, _ = O.solve_sequence([(A, B, np.zeros_like(B)), (A2, B[::-1].copy(), np.zeros_like(B))], 1e-10, m, k,
                              block_size=L, enlarge_cycles=E)
    assert sum((st["block_size"] for _, st in out), []) == sizes


# ---- P10: harmonic Ritz ----------------------------------------------------

def _toeplitz_tridiag(n, a, b, c):
    return sp.diags([b * np.ones(n - 1), a * np.ones(n), c * np.ones(n - 1)], [-1, 0, 1]).tocsr()


def test_harmonic_ritz_exact_when_krylov_space_is_whole_space():
    """n = m p: the block Krylov space is C^n, harmonic Ritz values are the
    eigenvalues of A (closed form for a tridiagonal Toeplitz matrix) and one
    cycle solves exactly."""
    n, p, m = 12, 3, 4
    a, b, c = 4.0, 1.5, 0.6           # eigenvalues a + 2 sqrt(bc) cos(j pi/(n+1))
    A = _toeplitz_tridiag(n, a, b, c)
    B = np.random.default_rng(3).uniform(-1, 1, (n, p))
    cyc = O.block_arnoldi_cycle(A, B, None, m, 0.0)
    theta, T = O.harmonic_ritz_first(cyc["H"], p)
    exact = a + 2 * np.sqrt(b * c) * np.cos(np.arange(1, n + 1) * np.pi / (n + 1))
    assert np.allclose(np.sort(theta.real), np.sort(exact), atol=1e-9)
    assert np.max(np.abs(theta.imag)) < 1e-9
    X, U, st = O.solve(A, B, np.zeros_like(B), 1e-300, m, 2, max_cycles=1)
    Xs = np.linalg.solve(A.toarray(), B)
    assert np.linalg.norm(X - Xs) < 1e-10 * np.linalg.norm(Xs)


# ---- NEXT-3: Ritz vectors as the recycled space (Section 4.1.3) -------------

def _galerkin_check(Ad, Wh, Y, k_sel, largest=False):
    """Y spans Ritz vectors of A on range(Wh): Wh^H (A Y - Y S) = 0 for the
    small S, and S's eigenvalues are the k_sel Ritz values of smallest modulus
    of the pencil (Wh^H A Wh, Wh^H Wh), all formed from the explicit A."""
    Qh, _ = np.linalg.qr(Wh)
    S, *_ = np.linalg.lstsq(Qh.conj().T @ Y, Qh.conj().T @ (Ad @ Y), rcond=None)
    res = Qh.conj().T @ (Ad @ Y - Y @ S)
    assert np.linalg.norm(res) < 1e-8 * np.linalg.norm(Ad) * np.linalg.norm(Y)
    allv = np.linalg.eigvals(Qh.conj().T @ Ad @ Qh)
    mags = np.sort(np.abs(allv))
    if largest:
        mags = mags[::-1]
    got = np.sort(np.abs(np.linalg.eigvals(S)))
    want = np.sort(mags[: len(got)])
    assert len(got) >= k_sel
    assert np.allclose(got, want, rtol=1e-7, atol=1e-9)


@pytest.mark.parametrize("largest", [False, True])
def test_ritz_selection_satisfies_galerkin_condition(largest):
    """Every cycle's new U (first cycle: from the block Krylov space; later:
    from U + K_m) spans the selected Ritz vectors of A on the searched space."""
    A, B = _small(N=10, p=2)
    Ad = A.toarray()
    m, k = 4, 4
    X, U, st = O.solve(A, B, np.zeros_like(B), 1e-10, m, k, ritz=True, trace=True, select_largest=largest,
                       max_cycles=4)
    assert len(st["trace"]) >= 3
    for i, tr in enumerate(st["trace"]):
        me = tr["cyc"]["m_eff"]
        Wm = np.hstack(tr["cyc"]["V"][:me])
        Wh = Wm if tr["U_in"] is None else np.hstack([tr["U_in"], Wm])
        _galerkin_check(Ad, Wh, tr["U"], k, largest)
    # and U is not the harmonic choice (whose vectors fail the check above)
    Xh, Uh, sth = O.solve(A, B, np.zeros_like(B), 1e-10, m, k, trace=True, max_cycles=1, select_largest=largest)
    Y1, Y2 = st["trace"][0]["U"], sth["trace"][0]["U"]
    Q1, _ = np.linalg.qr(Y1)
    Q2, _ = np.linalg.qr(Y2)
    assert np.linalg.norm(Q2 - Q1 @ (Q1.T @ Q2)) > 1e-6


def test_ritz_values_exact_when_krylov_space_is_whole_space():
    """n = m p: W_m spans C^n, so H_m is similar to A and the Ritz values are the
    eigenvalues of A (closed form for a tridiagonal Toeplitz matrix)."""
    n, p, m, k = 12, 3, 4, 4
    a, b, c = 4.0, 1.5, 0.6
    A = _toeplitz_tridiag(n, a, b, c)
    B = np.random.default_rng(3).uniform(-1, 1, (n, p))
    cyc = O.block_arnoldi_cycle(A, B, None, m, 0.0)
    exact = a + 2 * np.sqrt(b * c) * np.cos(np.arange(1, n + 1) * np.pi / (n + 1))
    U, C, vals = O.refresh_first(cyc, k, ritz=True)
    assert np.allclose(np.sort(vals.real), np.sort(exact)[:k], atol=1e-9)
    # A U = C holds for the Ritz choice as well (C = A U orthonormal)
    assert np.linalg.norm(A @ U - C) < 1e-10 * np.linalg.norm(C)
    assert np.linalg.norm(C.T @ C - np.eye(C.shape[1])) < 1e-12


def test_ritz_recycling_sequence_matches_dense_lu():
    A, B = _small(N=10, p=2)
    systems = [(A, B, np.zeros_like(B)),
               ((A + 0.05 * sp.identity(A.shape[0])).tocsr(), B[::-1].copy(), np.zeros_like(B))]
    out, U = O.solve_sequence(systems, 1e-10, 4, 5, ritz=True)
    for (Ai, Bi, _), (X, st) in zip(systems, out):
        Xd = np.linalg.solve(Ai.toarray(), Bi)
        assert np.linalg.norm(X - Xd) <= 1e-8 * np.linalg.norm(Xd)
    assert U.shape[1] in (5, 6)


def test_harmonic_ritz_standard_equals_generalized_at_k0():
    """Proposition block-harm-ritz vs eq. harm-ritz-gen-eig with no recycled space."""
    A, B = _small(N=10, p=3)
    cyc = O.block_arnoldi_cycle(A, B, None, 5, 0.0)
    th1, _ = O.harmonic_ritz_first(cyc["H"], 3)
    W = np.hstack(cyc["V"])
    th2, _ = O.harmonic_ritz_augmented(cyc["H"], W, W[:, : cyc["H"].shape[1]])
    th2 = th2[np.isfinite(th2)]
    k1 = np.sort_complex(np.round(th1, 6))
    k2 = np.sort_complex(np.round(th2, 6))
    assert len(k1) == len(k2)
    assert np.allclose(k1, k2, rtol=1e-6, atol=1e-6)


@pytest.mark.parametrize("cplx", [False, True])
def test_harmonic_ritz_petrov_galerkin_bruteforce(cplx):
    """(A y - theta y) orthogonal to A * span(W^_m) (harmonic Ritz condition,
    Section 4.1), checked with explicit products for the augmented problem."""
    A, B = _small(N=9, p=2, cplx=cplx)
    X, U, st = O.solve(A, B, np.zeros_like(B), 1e-12, 4, 3, max_cycles=3, trace=True)
    tr = st["trace"][1]
    Uin, Cin, cyc = tr["U_in"], tr["C_in"], tr["cyc"]
    Ad = A.toarray()
    d = 1.0 / np.linalg.norm(Uin, axis=0)
    Ut = Uin * d
    kk = Uin.shape[1]
    H, F = cyc["H"], cyc["F"]
    G = np.zeros((kk + H.shape[0], kk + H.shape[1]), dtype=H.dtype)
    G[:kk, :kk] = np.diag(d)
    G[:kk, kk:] = F
    G[kk:, kk:] = H
    Wh = np.hstack([Ut] + cyc["V"][:-1])
    Wt = np.hstack([Cin] + cyc["V"])
    # the compact relation A W^ = W~ G (eq. mod-arn-rel)
    assert np.linalg.norm(Ad @ Wh - Wt @ G) < 1e-11 * np.linalg.norm(Ad @ Wh)
    theta, T = O.harmonic_ritz_augmented(G, Wt, Wh)
    AW = Ad @ Wh
    ok = np.isfinite(theta)
    for th, t in zip(theta[ok], T[:, ok].T):
        y = Wh @ t
        r = Ad @ y - th * y
        assert np.linalg.norm(AW.conj().T @ r) <= 1e-8 * np.linalg.norm(AW) * np.linalg.norm(y) * max(1, abs(th))


@pytest.mark.parametrize("cplx,largest,p,m,k", [
    (False, False, 3, 5, 4), (False, True, 3, 5, 4), (False, False, 1, 8, 5), (False, True, 1, 8, 5),
    (False, False, 2, 4, 3), (True, False, 2, 4, 3), (True, True, 3, 5, 4)])
def test_harmonic_selection_spans_selected_pairs_of_explicit_problem(cplx, largest, p, m, k):
    """Which harmonic Ritz vectors are recycled (Section 4.1.2: the refresh
    after Proposition block-harm-ritz in the first cycle and after eq.
    harm-ritz-gen-eig later; smallest modulus by default, largest as in
    Section 6.2).  For every traced cycle the harmonic problem is formed again
    from explicit dense products of A on the searched space What = [U, W_m]
    (W_m in the first cycle):  (A What)^H (A What) t = theta (A What)^H What t,
    the k values of smallest (largest) modulus are taken, conjugate pairs whole,
    and the refreshed U must span What t_sel: sine of the largest principal
    angle <= 1e-8."""
    A, B = _small(p=p, cplx=cplx)
    X, U, st = O.solve(A, B, np.zeros_like(B), 1e-10, m, k, max_cycles=5, trace=True, select_largest=largest)
    worst, checked = pinlib.recycle_selection_violation(A.toarray(), st["trace"], k, largest, real=not cplx)
    assert checked >= 4 and checked >= len(st["trace"]) - 1
    assert st["trace"][0]["U_in"] is None            # the first-cycle (no U) refresh is among them
    assert worst <= 1e-8


def test_harmonic_selection_after_recycle_import():
    """The same pin on the second system of a sequence, whose first cycle
    refreshes a U that came from the previous system and was imported
    (A U = C S, Algorithm 1)."""
    A, B = _small(p=2)
    A2 = (A + 0.05 * sp.identity(A.shape[0])).tocsr()
    X, U, st = O.solve(A, B, np.zeros_like(B), 1e-10, 4, 3)
    X2, U2, st2 = O.solve(A2, B[::-1].copy(), np.zeros_like(B), 1e-10, 4, 3, U=U, trace=True, max_cycles=4)
    assert st2["trace"][0]["U_in"] is not None
    worst, checked = pinlib.recycle_selection_violation(A2.toarray(), st2["trace"], 3)
    assert checked >= 3 and worst <= 1e-8


def test_select_ritz_keeps_conjugate_pairs_whole():
    theta = np.array([1.0 + 0j, 2 + 1j, 2 - 1j, 5.0 + 0j, 0.5 + 0j])
    T = np.eye(5, dtype=complex)
    T[:, 1] = [0, 1, 1j, 0, 0]
    T[:, 2] = [0, 1, -1j, 0, 0]
    Pm, vals = O.select_ritz(theta, T, 2)
    assert Pm.shape[1] == 2 and set(np.round(vals.real, 6)) == {0.5, 1.0}
    Pm, vals = O.select_ritz(theta, T, 3)
    # the third smallest |theta| is a member of a pair: both are kept, k_eff = 4
    assert Pm.shape[1] == 4
    assert np.isrealobj(Pm)
    Pl, vl = O.select_ritz(theta, T, 1, largest=True)
    assert vl[0] == 5.0
    # infinite values are never kept
    Pm, vals = O.select_ritz(np.array([np.inf, 3.0, 1.0]), np.eye(3), 2)
    assert set(vals.real) == {1.0, 3.0}


# ---- P11: Vital containment (Section 5) ------------------------------------

def test_block_cycle_beats_single_vector_gmres_per_column():
    A, B = _small(N=14, p=4, seed=5)
    m = 5
    X, U, st = O.solve(A, B, np.zeros_like(B), 1e-300, m, 0, max_cycles=1)
    Rb = B - A @ X
    for i in range(B.shape[1]):
        x, _ = spla.gmres(A, B[:, i], x0=np.zeros(A.shape[0]), rtol=1e-300, atol=0.0, restart=m, maxiter=1)
        rs = np.linalg.norm(B[:, i] - A @ x)
        assert np.linalg.norm(Rb[:, i]) <= rs * (1 + 1e-10)


# ---- P12: equivariance -----------------------------------------------------

def test_column_permutation_and_scaling_equivariance():
    A, B = _small(N=10, p=4, seed=7)
    X, U, st = O.solve(A, B, np.zeros_like(B), 1e-10, 5, 4, max_cycles=3)
    perm = [2, 0, 3, 1]
    Xp, _, stp = O.solve(A, B[:, perm], np.zeros_like(B), 1e-10, 5, 4, max_cycles=3)
    assert stp["block_steps"] == st["block_steps"]
    assert np.linalg.norm(Xp - X[:, perm]) < 1e-8 * np.linalg.norm(X)
    Xs, _, sts = O.solve(A, 3.0 * B, np.zeros_like(B), 1e-10, 5, 4, max_cycles=3)
    assert np.linalg.norm(Xs - 3.0 * X) < 1e-8 * np.linalg.norm(3.0 * X)


# ---- P13: degenerate inputs --------------------------------------------------

def test_zero_rhs_and_exact_initial_guess():
    A, B = _small(N=8, p=2)
    X, U, st = O.solve(A, np.zeros_like(B), np.ones_like(B), 1e-8, 4, 3)
    assert np.all(X == 0) and st["cycles"] == 0
    Xs = np.linalg.solve(A.toarray(), B)
    X, U, st = O.solve(A, B, Xs, 1e-8, 4, 3)
    assert st["cycles"] == 0 and np.array_equal(X, Xs)


def test_duplicate_rhs_columns_still_converge():
    """A rank-deficient block R_0: the Householder QR gives an orthonormal V_1
    whose extra column is an arbitrary direction; the solve still converges."""
    A, B = _small(N=10, p=3)
    B[:, 2] = B[:, 0]
    X, U, st = O.solve(A, B, np.zeros_like(B), 1e-9, 5, 4)
    assert st["rel_res"] <= 1e-9
    assert np.linalg.norm(X[:, 2] - X[:, 0]) < 1e-6 * np.linalg.norm(X[:, 0])


# ---- NEXT-2: projected operator of the data-movement study (Section 6.3) ----

def test_projected_operator_against_explicit_projector():
    """(I - C C^H) A V: the result is orthogonal to C, equals the explicit
    n x n projector times the dense product on a small case, and a block is
    the columns applied one at a time."""
    A = P.banded(200, 4, seed=11)
    rng = np.random.default_rng(12)
    C, _ = np.linalg.qr(rng.uniform(-1, 1, (200, 10)))
    V = rng.uniform(-1, 1, (200, 8))
    W = O.apply_projected(A, C, V)
    assert np.linalg.norm(C.T @ W) < 1e-12 * np.linalg.norm(W)
    Pi = np.eye(200) - C @ C.T
    Wd = Pi @ (A.toarray() @ V)
    assert np.linalg.norm(W - Wd) < 1e-12 * np.linalg.norm(Wd)
    for j in range(8):
        wj = O.apply_projected(A, C, V[:, j:j + 1])
        assert np.linalg.norm(wj[:, 0] - W[:, j]) < 1e-12 * np.linalg.norm(W[:, j])


def test_banded_generator_recipe():
    A = P.banded(300, 5, seed=4)
    Ad = A.toarray()
    i, j = np.nonzero(Ad)
    assert np.max(np.abs(i - j)) == 5 and A.nnz == 300 * 11 - 5 * 6
    off = np.abs(Ad).sum(axis=1) - np.abs(np.diag(Ad))
    assert np.allclose(np.diag(Ad), off + 1.0)
