"""Block GCRO-DR oracle: Algorithm 1 (block RGMRES) of Parks, Soodhalter and Szyld,
written step by step in plain NumPy/SciPy, FP64 (complex128 for complex input).

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the CPU
baseline of the benchmark, never by the product path.  Shares no code with the
HIP library.

Every pin for this module lives in tests/test_oracle_*.py (run with
`-m "not gpu"`): dense LU solutions, the block modified Arnoldi relation
(eq. block-modified-arnoldi), orthonormality, A U = C, residual equivalence
(Proposition residual-equiv), monotone LSQ residual within a cycle, minimal
residual over U + K_m by brute force, reduction to restarted GMRES at k=0, p=1
(against scipy's gmres), harmonic-Ritz checks (Proposition block-harm-ritz vs
the generalized form eq. harm-ritz-gen-eig, exact eigenvalues when the block
Krylov space is the whole space, the Petrov-Galerkin condition by brute
force), which vectors every refresh recycles (the refreshed U spans the
selected pairs of the harmonic problem formed again from explicit products of
A on [U, W_m], smallest or largest modulus), the Vital containment bound
(Section 5) and equivariance.

Readings of points the paper leaves open:
  * E in Algorithm 1 is the first p columns of the identity of order (m+1)p
    (the block GMRES right-hand side E_1 F_0 of eq. true-block-gmres-min).
  * The stopping test is relative: ||B - A X||_F <= tol ||B||_F.  Inside a cycle
    the LSQ residual rho_j is checked after every block step and the cycle ends
    at m_eff = j when rho_j <= tol ||B||_F; the loop condition then confirms
    with the true residual.
  * The residual carried between cycles is the recurrence R_i = R_{i-1} -
    W_{m+1} H_m Y_i of Algorithm 1; the true residual is used only in the test.
  * Reduced QR factors are unique with a positive real diagonal (Householder
    QR followed by a sign fix).
  * The Arnoldi step orthogonalises twice against [C, V_1 .. V_j] (block MGS
    per pass here); the new block is then QR-factored.
  * Harmonic Ritz selection keeps the k values of smallest |theta| (largest
    with select_largest), stable order (|theta|, Re, Im, index); infinite or
    NaN values are never kept.  For real arithmetic a conjugate pair split by
    the cut is kept whole (k_eff = k + 1) and represented by [Re t, Im t].
  * k_eff = min(k, size of the space the Ritz problem lives in).
  * U is refreshed after every cycle, including the last one, so the stored U
    reflects the final cycle.
  * The first-cycle selection uses Proposition block-harm-ritz; if the square
    part H_m is numerically singular it falls back to the generalized form with
    no recycled space.
  * Enlarged block (p = 1, block size L > 1, Section 3.1): every cycle starts
    from (I - C C^H) [r, Z] (the Krylov space of the augmented method is built
    from (I - Phi) R_0) with the same L - 1 vectors Z, drawn once by a
    counter-based SplitMix64 (entry (i, c) of the n x L block, c = 1 .. L-1),
    and solves the single-vector problem eq. 1rhs-block-gmres-min (right-hand
    side E_1 F_0 e_1).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import ilu


# ----------------------------------------------------------------------------
# small dense helpers
# ----------------------------------------------------------------------------

def qr_pos(M):
    """Reduced QR  M = Q R  with diag(R) real and >= 0 (Householder via LAPACK,
    then a column sign/phase fix).  Used for R_0 = V_1 Z (Algorithm 1),
    A U = C S (Algorithm 1, recycle import) and the new Arnoldi block."""
    Q, R = np.linalg.qr(M, mode="reduced")
    d = np.diag(R).copy()
    mag = np.abs(d)
    ph = np.ones_like(d)
    nz = mag > 0
    ph[nz] = d[nz] / mag[nz]
    Q = Q * ph[None, :]
    R = np.conj(ph)[:, None] * R
    return Q, R


_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_MIX1 = np.uint64(0xBF58476D1CE4E5B9)
_MIX2 = np.uint64(0x94D049BB133111EB)


def splitmix64(counter):
    """SplitMix64 (Steele, Lea and Flood, OOPSLA 2014; the finaliser of
    Vigna's splitmix64.c) applied to a uint64 counter array: the output for
    state x is mix(x + golden gamma).  counter 0 gives 0xE220A8397B1DCDAF, the
    generator's first output from seed 0."""
    z = np.asarray(counter, dtype=np.uint64) + _GOLDEN
    z = (z ^ (z >> np.uint64(30))) * _MIX1
    z = (z ^ (z >> np.uint64(27))) * _MIX2
    return z ^ (z >> np.uint64(31))


def enlarging_vectors(n, L, seed=0):
    """The L - 1 extra start vectors of the enlarged block: entry (i, c) for
    c = 1 .. L-1 is 2 u - 1 with u the top 53 bits of
    splitmix64(i + 2^40 c + 2^56 seed) scaled to [0, 1)."""
    i = np.arange(n, dtype=np.uint64)[:, None]
    c = np.arange(1, L, dtype=np.uint64)[None, :]
    ctr = i + (c << np.uint64(40)) + (np.uint64(seed) << np.uint64(56))
    u = (splitmix64(ctr) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    return 2.0 * u - 1.0


def _bj(j, p):
    """Row/column slice of block j (0-based) with block size p."""
    return slice(j * p, (j + 1) * p)


# ----------------------------------------------------------------------------
# the block Arnoldi cycle (Section 3.1, Section 4 eq. block-modified-arnoldi,
# Algorithm 1 cycle body)
# ----------------------------------------------------------------------------

def block_arnoldi_cycle(A, R, C, m, thresh, extra=None):
    """Block Arnoldi on (I - C C^H) A started from the block residual R, with the
    block GMRES least-squares problem solved after every block step.  With
    `extra` (enlarged block, p = 1) the start block is [R, extra] and only R's
    column is a right-hand side (eq. 1rhs-block-gmres-min).

    Returns a dict with
      V   : list of m_eff+1 orthonormal n x p blocks (W_{m_eff+1} = [V_1 .. V_{m_eff+1}])
      H   : (m_eff+1)p x m_eff p block upper Hessenberg, upper-triangular subdiagonal blocks
      F   : k x m_eff p, F = C^H A W_m (called B_m in eq. block-modified-arnoldi)
      Z   : p x p, R = V_1 Z
      Y   : m_eff p x p least-squares solution of min ||H Y - E Z||_F
      rho : list of the LSQ residual norms after each block step
      m_eff
    """
    nrhs = R.shape[1]
    if extra is not None:
        # the start block of the augmented method is (I - C C^H) [R, Z]; R is
        # already orthogonal to C, the enlarging vectors are projected here
        # (twice, as in the block Gram-Schmidt passes)
        Zx = extra.astype(np.result_type(R.dtype, extra.dtype))
        if C is not None:
            for _ in range(2):
                Zx = Zx - C @ (C.conj().T @ Zx)
        R = np.hstack([R, Zx])
    n, p = R.shape                                   # p: block size (L when enlarged)
    k = 0 if C is None else C.shape[1]
    dt = np.result_type(R.dtype, A.dtype, np.float64)
    V1, Z = qr_pos(R.astype(dt))
    V = [V1]
    H = np.zeros(((m + 1) * p, m * p), dtype=dt)
    F = np.zeros((k, m * p), dtype=dt)
    EZ = np.zeros(((m + 1) * p, nrhs), dtype=dt)
    EZ[:p, :] = Z[:, :nrhs]                          # E Z (E = I_{(m+1)p}[:, :p]), or E_1 F_0 e_1
    rho = []
    Y = None
    m_eff = 0
    for j in range(m):
        W = A @ V[j]
        for _ in range(2):                           # orthogonalise twice
            if k:
                S = C.conj().T @ W
                W = W - C @ S
                F[:, _bj(j, p)] += S
            for i in range(j + 1):
                S = V[i].conj().T @ W
                W = W - V[i] @ S
                H[_bj(i, p), _bj(j, p)] += S
        Vn, Rj = qr_pos(W)
        H[_bj(j + 1, p), _bj(j, p)] = Rj
        V.append(Vn)
        jj = j + 1
        Hj = H[:(jj + 1) * p, :jj * p]
        rhs = EZ[:(jj + 1) * p]
        Y, *_ = np.linalg.lstsq(Hj, rhs, rcond=None)
        rho.append(float(np.linalg.norm(Hj @ Y - rhs)))
        m_eff = jj
        if rho[-1] <= thresh:
            break
    return {
        "V": V[: m_eff + 1],
        "H": H[: (m_eff + 1) * p, : m_eff * p].copy(),
        "F": F[:, : m_eff * p].copy(),
        "Z": Z,
        "Y": Y,
        "rho": rho,
        "m_eff": m_eff,
    }


# ----------------------------------------------------------------------------
# harmonic Ritz selection (Section 4.1, Proposition block-harm-ritz and
# eq. harm-ritz-gen-eig)
# ----------------------------------------------------------------------------

def select_ritz(theta, T, k, largest=False, real=True, rtol_real=1e-9):
    """Pick k harmonic Ritz vectors.  Returns (P, chosen theta values).

    Smallest |theta| by default (largest with `largest`); infinite/NaN values
    are skipped.  With `real`, a conjugate pair is always taken whole, so P may
    have k+1 columns, and a pair (t, conj t) is represented by [Re t, Im t]."""
    theta = np.asarray(theta)
    idx = np.nonzero(np.isfinite(theta))[0]
    mag = np.abs(theta[idx])
    primary = -mag if largest else mag
    order = idx[np.lexsort((idx, theta.imag[idx], theta.real[idx], primary))]
    if not real:
        sel = order[:k]
        return T[:, sel], theta[sel]
    cols, vals, used = [], [], set()
    for i in order:
        if len(cols) >= k:
            break
        if i in used:
            continue
        th = theta[i]
        if abs(th.imag) <= rtol_real * max(abs(th), 1e-300):
            v = T[:, i]
            j = int(np.argmax(np.abs(v)))
            v = v * (np.conj(v[j]) / abs(v[j]))        # make it real
            cols.append(np.real(v))
            vals.append(th)
            used.add(i)
        else:
            cand = [c for c in order if c not in used and c != i]
            if not cand:
                continue
            cand = np.array(cand)
            jpart = int(cand[np.argmin(np.abs(theta[cand] - np.conj(th)))])
            ip = i if th.imag > 0 else jpart
            v = T[:, ip]
            cols.append(np.real(v))
            cols.append(np.imag(v))
            vals.extend([theta[i], theta[jpart]])
            used.add(i)
            used.add(jpart)
    return np.column_stack(cols), np.array(vals)


def harmonic_ritz_first(H, p):
    """Proposition block-harm-ritz: eigenpairs of
    H_m + H_m^{-H} Ehat (H_{m+1,m}^H H_{m+1,m}) Ehat^H  (order mp).
    Only the last p columns of H_m are modified."""
    mp = H.shape[1]
    Hm = H[:mp, :]
    Hs = H[mp:mp + p, mp - p:]
    K = Hm.astype(np.result_type(Hm.dtype, np.float64)).copy()
    rhs = np.zeros((mp, p), dtype=K.dtype)
    rhs[mp - p:, :] = Hs.conj().T @ Hs
    K[:, mp - p:] += np.linalg.solve(Hm.conj().T, rhs)
    theta, T = sla.eig(K)
    return theta, T


def harmonic_ritz_augmented(G, Wt, Wh):
    """eq. harm-ritz-gen-eig: G^H G t = theta G^H (Wt^H Wh) t, with Wt = [C W_{m+1}]
    and Wh = [U~ W_m]; Wt^H Wh is formed explicitly."""
    M = Wt.conj().T @ Wh
    GhG = G.conj().T @ G
    GhM = G.conj().T @ M
    theta, T = sla.eig(GhG, GhM)
    return theta, T


def ritz_augmented(G, Wt, Wh):
    """Ritz pairs on range(Wh) (Section 4.1.3 alternative to harmonic Ritz
    vectors): Galerkin condition (A y - theta y) orthogonal to range(Wh) for
    y = Wh t, with A Wh = Wt G, i.e. (Wh^H Wt G) t = theta (Wh^H Wh) t; both
    products are formed explicitly."""
    theta, T = sla.eig(Wh.conj().T @ Wt @ G, Wh.conj().T @ Wh)
    return theta, T


def refresh_first(cyc, k, largest=False, real=True, ritz=False):
    """First system, no U given (Algorithm 1, else-branch): select U in the block
    Krylov space from the first cycle, with C = A U orthonormal.
    [Q, rho] = qr(H P), C = W_{m+1} Q, U = W_m P rho^{-1}.  With `ritz` the
    selected vectors are Ritz vectors of the block Krylov space: the
    eigenvectors of its square Hessenberg block H_m = W_m^H A W_m."""
    V, H = cyc["V"], cyc["H"]
    p = V[0].shape[1]
    mp = H.shape[1]
    k_t = min(k, mp)
    if k_t == 0:
        return None, None, np.array([])
    Hm = H[:mp, :]
    if ritz:
        theta, T = sla.eig(Hm)
    elif np.linalg.cond(Hm) > 1e14:
        W = np.hstack(V)
        theta, T = harmonic_ritz_augmented(H, W, W[:, :mp])
    else:
        theta, T = harmonic_ritz_first(H, p)
    P, vals = select_ritz(theta, T, k_t, largest=largest, real=real)
    Q, rho = qr_pos(H @ P)
    Wm1 = np.hstack(V)
    C = Wm1 @ Q
    U = (Wm1[:, :mp] @ P) @ np.linalg.inv(rho)
    return U, C, vals


def refresh_augmented(U, C, cyc, k, largest=False, real=True, ritz=False):
    """Algorithm 1, end of a cycle: D scales U to unit columns, G = [[D, F],[0, H]],
    harmonic Ritz on U + K_m (eq. harm-ritz-gen-eig; Ritz pairs with `ritz`),
    then [Q, rho] = qr(G P), C = [C W_{m+1}] Q, U = [U D  W_m] P rho^{-1}."""
    V, H, F = cyc["V"], cyc["H"], cyc["F"]
    kk = U.shape[1]
    mp = H.shape[1]
    d = 1.0 / np.linalg.norm(U, axis=0)
    Ut = U * d[None, :]
    dt = np.result_type(H.dtype, U.dtype, np.float64)
    G = np.zeros((kk + H.shape[0], kk + mp), dtype=dt)
    G[:kk, :kk] = np.diag(d)
    G[:kk, kk:] = F
    G[kk:, kk:] = H
    Wt = np.hstack([C] + V)
    Wh = np.hstack([Ut] + V[:-1])
    theta, T = (ritz_augmented if ritz else harmonic_ritz_augmented)(G, Wt, Wh)
    k_t = min(k, kk + mp)
    P, vals = select_ritz(theta, T, k_t, largest=largest, real=real)
    Q, rho = qr_pos(G @ P)
    C_new = Wt @ Q
    U_new = (Wh @ P) @ np.linalg.inv(rho)
    return U_new, C_new, vals


# ----------------------------------------------------------------------------
# Algorithm 1
# ----------------------------------------------------------------------------

def recycle_import(A, U, X, R):
    """Algorithm 1, U available: A U = C S (reduced QR), U <- U S^{-1},
    X_0 <- X_0 + U C^H R_0, R_0 <- R_0 - C C^H R_0."""
    AU = A @ U
    C, S = qr_pos(AU)
    U = U @ np.linalg.inv(S)
    T = C.conj().T @ R
    return U, C, X + U @ T, R - C @ T


def solve(A, B, X0, tol, m, k, U=None, max_cycles=1000, select_largest=False, trace=False, block_size=None,
          seed=0, enlarged_cycles=None, ritz=False, precond=None):
    """Algorithm 1 (block RGMRES / block GCRO-DR) for one system A X = B.

    Returns (X, U, stats).  stats holds per-cycle block-step counts, the LSQ
    residual history, true relative residuals and (with trace=True) the cycle
    internals used by the pins.  block_size L > 1 with one right-hand side
    enlarges the block with enlarging_vectors(n, L, seed).  enlarged_cycles:
    with an enlarged block, only the first enlarged_cycles cycles of this
    call use it and every later cycle is non-block (L = 1), the hybrid of
    Section 4.1.3; None: every cycle uses it.  ritz: recycle Ritz instead of
    harmonic Ritz vectors (Section 4.1.3).  precond="ilu0": right
    preconditioning with the ILU(0) of this A (oracle/ilu.py): the same
    algorithm on A M^{-1} in the variable M X, X returned unpreconditioned,
    U in the preconditioned variable.
    """
    if precond is not None:
        if precond != "ilu0":
            raise ValueError(f"unknown preconditioner {precond!r}")
        Lf, Uf = ilu.ilu0(A)
        X0 = np.asarray(X0)
        Xh, U, stats = solve(ilu.right_preconditioned(A, Lf, Uf), B, Lf @ (Uf @ X0), tol, m, k, U=U,
                             max_cycles=max_cycles, select_largest=select_largest, trace=trace,
                             block_size=block_size, seed=seed, enlarged_cycles=enlarged_cycles, ritz=ritz)
        X = ilu.apply_inverse(Lf, Uf, Xh)
        bn = float(np.linalg.norm(B))
        stats["rel_res"] = float(np.linalg.norm(B - A @ X)) / bn if bn > 0 else 0.0
        if trace:
            stats["precond_factors"] = (Lf, Uf)
        return X, U, stats
    A = A.tocsr() if hasattr(A, "tocsr") else A
    B = np.asarray(B)
    n, p = B.shape
    cplx = np.iscomplexobj(B) or np.iscomplexobj(A.data if hasattr(A, "data") else A) \
        or (U is not None and np.iscomplexobj(U))
    dt = np.complex128 if cplx else np.float64
    real = not cplx
    B = B.astype(dt)
    X = np.array(X0, dtype=dt, copy=True)
    bn = float(np.linalg.norm(B))
    stats = {"cycles": 0, "block_steps": 0, "steps_per_cycle": [], "rho": [],
             "true_rel_res": [], "recur_drift": [], "trace": [], "k_eff": []}
    if bn == 0.0:
        X[:] = 0
        stats["rel_res"] = 0.0
        return X, U, stats
    thresh = tol * bn
    extra = None
    if block_size is not None and block_size > p:
        if p != 1:
            raise ValueError("an enlarged block needs a single right-hand side")
        extra = enlarging_vectors(n, block_size, seed).astype(dt)
    R = B - A @ X
    if np.linalg.norm(R) <= thresh:
        stats["rel_res"] = float(np.linalg.norm(R)) / bn
        return X, U, stats
    def extra_now():
        if enlarged_cycles is None or stats["cycles"] < enlarged_cycles:
            return extra
        return None

    C = None
    if U is not None:
        U, C, X, R = recycle_import(A, U.astype(dt), X, R)
    else:
        cyc = block_arnoldi_cycle(A, R, None, m, thresh, extra_now())
        me = cyc["m_eff"]
        Wm = np.hstack(cyc["V"][:me])
        Wm1 = np.hstack(cyc["V"])
        X = X + Wm @ cyc["Y"]
        R = R - Wm1 @ (cyc["H"] @ cyc["Y"])
        U, C, _ = refresh_first(cyc, k, largest=select_largest, real=real, ritz=ritz)
        _log(stats, cyc, A, B, X, R, bn, trace, U, C)
    while True:
        Rt = B - A @ X
        if np.linalg.norm(Rt) <= thresh or stats["cycles"] >= max_cycles:
            break
        Uold, Cold = U, C
        cyc = block_arnoldi_cycle(A, R, C, m, thresh, extra_now())
        me = cyc["m_eff"]
        Wm = np.hstack(cyc["V"][:me])
        Wm1 = np.hstack(cyc["V"])
        Y = cyc["Y"]
        if C is not None:
            X = X + Wm @ Y - U @ (cyc["F"] @ Y)
        else:
            X = X + Wm @ Y
        R = R - Wm1 @ (cyc["H"] @ Y)
        if C is not None:
            U, C, _ = refresh_augmented(U, C, cyc, k, largest=select_largest, real=real, ritz=ritz)
        elif k > 0:
            U, C, _ = refresh_first(cyc, k, largest=select_largest, real=real, ritz=ritz)
        _log(stats, cyc, A, B, X, R, bn, trace, U, C, Uold, Cold)
    stats["rel_res"] = float(np.linalg.norm(B - A @ X)) / bn
    return X, U, stats


def _log(stats, cyc, A, B, X, R, bn, trace, U, C, Uold=None, Cold=None):
    stats["cycles"] += 1
    stats["block_steps"] += cyc["m_eff"]
    stats["steps_per_cycle"].append(cyc["m_eff"])
    stats["rho"].append(list(cyc["rho"]))
    Rt = B - A @ X
    stats["true_rel_res"].append(float(np.linalg.norm(Rt)) / bn)
    stats["recur_drift"].append(float(np.linalg.norm(R - Rt)) / bn)
    stats["k_eff"].append(0 if U is None else U.shape[1])
    stats.setdefault("block_size", []).append(cyc["V"][0].shape[1])
    if trace:
        stats["trace"].append({"cyc": cyc, "U": U, "C": C, "U_in": Uold, "C_in": Cold,
                               "X": X.copy(), "R": R.copy()})


def solve_sequence(systems, tol, m, k, max_cycles=1000, select_largest=False, block_size=None, seed=0,
                   enlarge_cycles=None, ritz=False, precond=None):
    """Solve a sequence A^[i] X = B^[i], carrying U from each system to the next
    (Algorithm 1, last line).  `systems` is a list of (A, B, X0).
    enlarge_cycles (with block_size L > p = 1): the first enlarge_cycles
    cycles of the whole sequence use the enlarged block, every later cycle
    L = 1 (Section 4.1.3: inflate the block for the first cycles to obtain a
    good recycled space quickly, then switch at a restart to non-block
    GCRO-DR); None: every cycle is enlarged."""
    U = None
    out = []
    left = enlarge_cycles
    for (A, B, X0) in systems:
        X, U, st = solve(A, B, X0, tol, m, k, U=U, max_cycles=max_cycles,
                         select_largest=select_largest, block_size=block_size, seed=seed,
                         enlarged_cycles=left, ritz=ritz, precond=precond)
        if left is not None:
            left = max(0, left - st["cycles"])
        out.append((X, st))
    return out, U


# ----------------------------------------------------------------------------
# Projected operator of the data-movement study (Section 6.3)
# ----------------------------------------------------------------------------

def apply_projected(A, C, V):
    """(I - C C^H) A V for a C with orthonormal columns (Section 6.3 applies
    the projected operator (I - Phi) A with Phi = C C^H to blocks of vectors):
    the plain definition, one product after the other."""
    W = A @ V
    return W - C @ (C.conj().T @ W)

