"""Plant plausible mistakes in the oracle (on the CPU only) and check that the
pins catch each one: a dropped term, a wrong sign, a transposed operand, a
wrong index, the wrong end of the harmonic Ritz selection and a pencil without
the metric W~^H W^.  This shows the pins are strong enough to be trusted."""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle.bgcrodr as ob
import pinlib
import problems as P


def _invariants(A, B, m=4, k=3, cycles=4):
    """Run the oracle and return the worst violations of the pinned invariants."""
    X, U, st = ob.solve(A, B, np.zeros_like(B), 1e-12, m, k, max_cycles=cycles, trace=True)
    Ad = A.toarray()
    au_c = max(np.linalg.norm(Ad @ tr["U"] - tr["C"]) / np.linalg.norm(tr["C"]) for tr in st["trace"])
    drift = max(st["recur_drift"])
    minres = 0.0
    for i in range(1, len(st["trace"])):
        prev, tr = st["trace"][i - 1], st["trace"][i]
        Wm = np.hstack(tr["cyc"]["V"][: tr["cyc"]["m_eff"]])
        AB = Ad @ np.hstack([tr["U_in"], Wm])
        Zb, *_ = np.linalg.lstsq(AB, prev["R"], rcond=None)
        best = np.linalg.norm(prev["R"] - AB @ Zb)
        minres = max(minres, abs(np.linalg.norm(B - Ad @ tr["X"]) - best) / np.linalg.norm(B))
    return au_c, drift, minres


def _problem():
    A = P.convdiff(9, 2, conv=(6.0, 3.0, 0.0))
    B = np.random.default_rng(0).uniform(-1, 1, (A.shape[0], 2))
    return A, B


def _caught(viol):
    au_c, drift, minres = viol
    return au_c > 1e-9 or drift > 1e-9 or minres > 1e-9


def test_unmutated_oracle_passes():
    assert not _caught(_invariants(*_problem()))


def test_dropped_F_block_in_G_is_caught(monkeypatch):
    orig = ob.refresh_augmented

    def bad(U, C, cyc, k, largest=False, real=True, ritz=False):
        cyc = dict(cyc)
        cyc["F"] = np.zeros_like(cyc["F"])          # G = [[D, 0], [0, H]]
        return orig(U, C, cyc, k, largest, real, ritz)

    monkeypatch.setattr(ob, "refresh_augmented", bad)
    assert _caught(_invariants(*_problem()))


def test_wrong_sign_of_pi_term_is_caught(monkeypatch):
    orig_cycle = ob.block_arnoldi_cycle

    def bad_cycle(A, R, C, m, thresh, extra=None):
        cyc = orig_cycle(A, R, C, m, thresh, extra)
        cyc["F"] = -cyc["F"]                          # X += W Y + U F Y instead of - U F Y
        return cyc

    monkeypatch.setattr(ob, "block_arnoldi_cycle", bad_cycle)
    assert _caught(_invariants(*_problem()))


def test_transposed_hessenberg_in_first_ritz_is_caught():
    """H_m^{-1} in place of H_m^{-H} in Proposition block-harm-ritz breaks the
    Petrov-Galerkin condition."""
    A, B = _problem()
    cyc = ob.block_arnoldi_cycle(A, B, None, 5, 0.0)
    H = cyc["H"]
    p = B.shape[1]
    mp = H.shape[1]
    Hm, Hs = H[:mp], H[mp:, mp - p:]
    rhs = np.zeros((mp, p))
    rhs[mp - p:] = Hs.T @ Hs
    W = np.hstack(cyc["V"])
    Ad = A.toarray()
    AW = Ad @ W[:, :mp]

    def pg_violation(K):
        th, T = sla.eig(K)
        worst = 0.0
        for t_, v in zip(th, T.T):
            y = W[:, :mp] @ v
            r = Ad @ y - t_ * y
            worst = max(worst, np.linalg.norm(AW.T @ r) / (np.linalg.norm(AW) * np.linalg.norm(y) * max(1, abs(t_))))
        return worst

    good = Hm.copy()
    good[:, mp - p:] += np.linalg.solve(Hm.T, rhs)
    bad = Hm.copy()
    bad[:, mp - p:] += np.linalg.solve(Hm, rhs)
    assert pg_violation(good) < 1e-9
    assert pg_violation(bad) > 1e-6


def test_wrong_rhs_block_index_is_caught(monkeypatch):
    """E Z placed in the second block row instead of the first."""
    orig_lstsq = np.linalg.lstsq

    def bad_lstsq(a, b, rcond=None):
        b2 = np.roll(b, b.shape[1], axis=0)
        return orig_lstsq(a, b2, rcond=rcond)

    monkeypatch.setattr(ob.np.linalg, "lstsq", bad_lstsq)
    A, B = _problem()
    try:
        viol = _invariants(A, B)
    finally:
        monkeypatch.setattr(ob.np.linalg, "lstsq", orig_lstsq)
    assert _caught(viol)


# ---- which harmonic Ritz vectors are recycled (Section 4.1.2) ---------------

def _selection_violation(largest=False):
    A, B = _problem()
    X, U, st = ob.solve(A, B, np.zeros_like(B), 1e-12, 4, 3, max_cycles=4, trace=True, select_largest=largest)
    return pinlib.recycle_selection_violation(A.toarray(), st["trace"], 3, largest)


def test_unmutated_selection_passes():
    for largest in (False, True):
        worst, checked = _selection_violation(largest)
        assert checked >= 3 and worst <= 1e-8


@pytest.mark.parametrize("largest", [False, True])
def test_flipped_selection_in_augmented_refresh_is_caught(monkeypatch, largest):
    """refresh_augmented keeping the other end of the spectrum."""
    orig = ob.refresh_augmented

    def bad(U, C, cyc, k, largest=False, real=True, ritz=False):
        return orig(U, C, cyc, k, not largest, real, ritz)

    monkeypatch.setattr(ob, "refresh_augmented", bad)
    assert _selection_violation(largest)[0] > 1e-3


@pytest.mark.parametrize("largest", [False, True])
def test_flipped_selection_in_first_refresh_is_caught(monkeypatch, largest):
    """refresh_first (Proposition block-harm-ritz) keeping the other end."""
    orig = ob.refresh_first

    def bad(cyc, k, largest=False, real=True, ritz=False):
        return orig(cyc, k, not largest, real, ritz)

    monkeypatch.setattr(ob, "refresh_first", bad)
    assert _selection_violation(largest)[0] > 1e-3


def test_pencil_without_metric_is_caught(monkeypatch):
    """eq. harm-ritz-gen-eig solved as G^H G t = theta G^H [I; 0] t, i.e. with
    W~^H W^ replaced by the identity it would be for an orthonormal W^."""
    def bad(G, Wt, Wh):
        M = np.eye(Wt.shape[1], Wh.shape[1], dtype=G.dtype)
        return sla.eig(G.conj().T @ G, G.conj().T @ M)

    monkeypatch.setattr(ob, "harmonic_ritz_augmented", bad)
    assert _selection_violation()[0] > 1e-3
