"""GPU checks at the full sizes of the benchmark configurations, in the launch
configuration bench.py times (default parameters of the sequence).

At these sizes the oracle cannot run a whole solve, so the checks are:
* the headline 128^3 sequence (p = 8, m = 10, k = 20): the iterate after
  exactly one restart cycle against the oracle's first cycle (the parity bar);
* every GPU configuration (128^3 FP64, complex 1024^2 Helmholtz, 192^3 FP32 in
  FP64 refinement) for a few cycles, by properties that hold at any size:
  the reported residual is the FP64 true residual recomputed on the host, the
  true residual does not grow from cycle to cycle (each cycle minimises it
  over a space that contains the zero correction), and the stored recycle
  pair satisfies C = A U with orthonormal C.
"""
import numpy as np
import pytest

import oracle
import problems

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

PARITY = 1e-6


def _bg():
    import paper_1604_01713_amd as bg
    bg.lib()
    return bg


def _dev():
    assert torch.cuda.is_available(), "GPU test without a GPU"
    return torch.device("cuda:0")


def _solve(bg, dev, A, B, p, m, k, tol, max_cycles, precision=0):
    cplx = np.iscomplexobj(B) or np.iscomplexobj(A.data)
    seq = bg.Sequence(A.shape[0], p, m, k, dtype=bg.BGCR_C128 if cplx else bg.BGCR_F64, precision=precision,
                      max_cycles=max_cycles)
    dA = bg.DeviceCSR.from_scipy(A, dev)
    dB = torch.from_numpy(np.ascontiguousarray(B)).to(dev)
    dX = torch.zeros_like(dB)
    st = seq.solve(dA, dB, dX, tol)
    torch.cuda.synchronize()
    return seq, dX.cpu().numpy(), st.as_dict(), seq.cycle_log()


def _properties(bg, dev, seq, A, B, X, st, log, pair_tol):
    rel_host = np.linalg.norm(B - A @ X) / np.linalg.norm(B)
    print(f"  reported rel.res {st['rel_res']:.6e}, host FP64 {rel_host:.6e}; per-cycle "
          f"{[f'{r:.2e}' for r in log[1]]}", flush=True)
    assert abs(st["rel_res"] - rel_host) <= 1e-9 * rel_host
    res = log[1]
    assert len(res) == st["cycles"] >= 2
    assert all(b <= a * (1 + 1e-10) for a, b in zip(res, res[1:]))
    ke = seq.recycle_dim()
    n = A.shape[0]
    dt = torch.complex128 if np.iscomplexobj(X) else torch.float64
    U = torch.zeros((n, ke), dtype=dt, device=dev)
    C = torch.zeros_like(U)
    seq.get_recycle(U, C)
    torch.cuda.synchronize()
    U, C = U.cpu().numpy(), C.cpu().numpy()
    E = np.linalg.norm(A @ U - C)
    au = E / np.linalg.norm(C)
    # normwise backward error of the relation: C = A U holds to rounding in
    # forming U and C, i.e. |AU - C| <= c u (|A| |U| + |C|); its plain relative
    # form grows with |A| |U|, which the shifted Helmholtz operator makes large
    # (|A| ~ 8 / h^2 and U spans the slowest directions)
    anorm = float(abs(A).sum(axis=1).max())
    bw = E / (anorm * np.linalg.norm(U) + np.linalg.norm(C))
    orth = np.linalg.norm(C.conj().T @ C - np.eye(ke))
    print(f"  k_eff {ke}: |AU - C|/|C| {au:.2e} (backward error {bw:.2e}), |C^H C - I| {orth:.2e}", flush=True)
    assert orth <= pair_tol
    assert au <= pair_tol or bw <= 1e-13


def test_headline_first_cycle_matches_oracle_at_full_size():
    """128^3 (n = 2,097,152), p = 8, m = 10, k = 20: one block GMRES(m) cycle
    (the first system's, Algorithm 1 without U) against the oracle's."""
    bg = _bg()
    dev = _dev()
    w = problems.cfg2(nsys=1)
    s = w.systems[0]
    seq, Xg, st, log = _solve(bg, dev, s.A, s.B, w.p, w.m, w.k, w.tol, max_cycles=1)
    seq.release()
    Xo, _, so = oracle.solve(s.A, s.B, s.X0, w.tol, w.m, w.k, max_cycles=1)
    rel = np.linalg.norm(Xg - Xo) / np.linalg.norm(Xo)
    print(f"cfg2 full size, one cycle: gpu steps {st['block_steps']} rel.res {st['rel_res']:.4e} | oracle steps "
          f"{so['block_steps']} rel.res {so['rel_res']:.4e} | rel diff {rel:.2e}", flush=True)
    assert st["cycles"] == 1 and st["block_steps"] == so["block_steps"]
    assert abs(st["rel_res"] - so["rel_res"]) <= 1e-8 * so["rel_res"]
    assert rel <= PARITY


def test_helmholtz_two_cycles_match_oracle_at_full_size():
    """Complex 1024^2 Helmholtz (n = 1,048,576, complex128), p = 16, m = 8,
    k = 16: two restart cycles of the first system against the oracle's, the
    second one augmented with the recycled pair of the first (Algorithm 1 with
    C in the projections).  These are the matrix-core complex sweeps in the
    launch configuration the benchmark times."""
    bg = _bg()
    dev = _dev()
    w = problems.cfg3(nsys=1)
    s = w.systems[0]
    seq, Xg, st, log = _solve(bg, dev, s.A, s.B, w.p, w.m, w.k, w.tol, max_cycles=2)
    seq.release()
    Xo, _, so = oracle.solve(s.A, s.B, s.X0, w.tol, w.m, w.k, max_cycles=2)
    rel = np.linalg.norm(Xg - Xo) / np.linalg.norm(Xo)
    col = max(np.linalg.norm(Xg[:, j] - Xo[:, j]) / np.linalg.norm(Xo[:, j]) for j in range(Xo.shape[1]))
    print(f"cfg3 full size, two cycles: gpu steps {st['block_steps']} rel.res {st['rel_res']:.6e} | oracle steps "
          f"{so['block_steps']} rel.res {so['rel_res']:.6e} | rel diff {rel:.2e}, worst column {col:.2e}", flush=True)
    assert st["cycles"] == 2 and st["block_steps"] == so["block_steps"]
    assert abs(st["rel_res"] - so["rel_res"]) <= 1e-8 * so["rel_res"]
    assert col <= 1e-10


@pytest.mark.parametrize("name", ["cfg2_128^3_fp64", "cfg3_1024^2_complex", "cfg4_192^3_fp32_in_fp64"])
def test_full_size_properties(name):
    bg = _bg()
    dev = _dev()
    if name.startswith("cfg2"):
        w, prec, pair_tol = problems.cfg2(nsys=1), 0, 1e-10
    elif name.startswith("cfg3"):
        w, prec, pair_tol = problems.cfg3(nsys=1), 0, 1e-10
    else:
        w, prec, pair_tol = problems.cfg4(nsys=1), 1, 1e-4
    s = w.systems[0]
    print(f"{name}: n = {s.A.shape[0]}, nnz = {s.A.nnz}, p = {w.p}, m = {w.m}, k = {w.k}", flush=True)
    seq, X, st, log = _solve(bg, dev, s.A, s.B, w.p, w.m, w.k, w.tol, max_cycles=3, precision=prec)
    _properties(bg, dev, seq, s.A, s.B, X, st, log, pair_tol)
    seq.release()
