"""Checks shared by the oracle pins and the mutation tests.

They are written from the definitions in the paper with explicit dense
products of A, never with the oracle's own small matrices (G, W~^H W^, the
block Hessenberg H), so that a mistake in how the oracle forms those matrices
cannot also hide in the check.
"""
import numpy as np
import scipy.linalg as sla


def orth(M, rtol=1e-12):
    """Orthonormal basis of range(M) from an SVD (rank by relative threshold)."""
    Uu, s, _ = np.linalg.svd(M, full_matrices=False)
    r = int(np.sum(s > rtol * s[0])) if s.size and s[0] > 0 else 0
    return Uu[:, :r]


def sin_largest_angle(Y1, Y2):
    """Sine of the largest principal angle between range(Y1) and range(Y2);
    1.0 when the dimensions differ."""
    Q1, Q2 = orth(Y1), orth(Y2)
    if Q1.shape[1] != Q2.shape[1]:
        return 1.0
    if Q1.shape[1] == 0:
        return 0.0
    return float(np.linalg.norm(Q2 - Q1 @ (Q1.conj().T @ Q2), 2))


def harmonic_pairs_explicit(Ad, What):
    """Harmonic Ritz pairs of A on range(What) with respect to A range(What)
    (Section 4.1: y = What t with (A y - theta y) orthogonal to A range(What)),
    from the explicit dense products:
        (A What)^H (A What) t = theta (A What)^H What t.
    Returns (theta, Y) with Y = What T; infinite or NaN theta are dropped."""
    AW = Ad @ What
    theta, T = sla.eig(AW.conj().T @ AW, AW.conj().T @ What)
    ok = np.isfinite(theta)
    return theta[ok], What @ T[:, ok]


def ritz_pairs_explicit(Ad, What):
    """Ritz pairs of A on range(What) (Galerkin: What^H (A y - theta y) = 0)."""
    Q = orth(What)
    theta, T = np.linalg.eig(Q.conj().T @ Ad @ Q)
    return theta, Q @ T


def select_by_modulus(theta, k, largest=False, real=True, tol=1e-8):
    """Indices of the k values of smallest (largest) modulus; with real data a
    complex value whose conjugate falls outside the cut brings its conjugate
    along, so the kept set is closed under conjugation."""
    order = np.argsort(-np.abs(theta) if largest else np.abs(theta), kind="stable")
    sel = list(order[:k])
    if real:
        for i in list(sel):
            th = theta[i]
            if abs(th.imag) > tol * max(abs(th), 1e-300):
                partner = int(np.argmin(np.abs(theta - np.conj(th))))
                if partner not in sel:
                    sel.append(partner)
    return sel


def cut_gap(theta, sel):
    """Relative gap in modulus between the kept values `sel` and the nearest
    value left out (a small gap makes the kept space ill-determined)."""
    rest = np.setdiff1d(np.arange(len(theta)), sel)
    if rest.size == 0:
        return np.inf
    kept = np.abs(theta[sel])
    out = np.abs(theta[rest])
    d = np.min(np.abs(out[:, None] - kept[None, :]))
    return d / max(np.max(kept), 1e-300)


def searched_space(tr):
    """What of a traced cycle: [U_in, W_m], or W_m in a cycle without U."""
    cyc = tr["cyc"]
    Wm = np.hstack(cyc["V"][: cyc["m_eff"]])
    return Wm if tr["U_in"] is None else np.hstack([tr["U_in"], Wm])


def recycle_selection_violation(Ad, trace, k, largest=False, ritz=False, real=True, min_gap=1e-6):
    """Worst sine of the largest principal angle, over the traced cycles,
    between the refreshed U and the span of the selected (harmonic) Ritz
    vectors of the explicit problem on the searched space.  Cycles whose cut
    falls in a near-tie of moduli are skipped (the kept space is then not
    determined).  Returns (worst, cycles checked)."""
    worst, checked = 0.0, 0
    for tr in trace:
        What = searched_space(tr)
        theta, Y = (ritz_pairs_explicit if ritz else harmonic_pairs_explicit)(Ad, What)
        k_t = min(k, What.shape[1])
        sel = select_by_modulus(theta, k_t, largest, real)
        if cut_gap(theta, sel) < min_gap:
            continue
        worst = max(worst, sin_largest_angle(tr["U"], Y[:, sel]))
        checked += 1
    return worst, checked
