"""Seeded synthetic workloads for block GCRO-DR sequences.

This module builds the matrices and right-hand sides that both the GPU path and
the FP64 oracle are fed.  It holds no arithmetic of the solver itself: only
finite-difference stencil assembly and seeded random draws.

The paper measures on sherman5, Tramonto, IFISS and SuiteSparse matrices that
are not available here; these PDE sequences stand in for them (sequences of
slowly changing non-Hermitian systems, Section 1 eq. (1.1), Section 2).

Conventions (one reading, used everywhere):
  * unit square / cube, N interior nodes per side, h = 1/(N+1), zero Dirichlet
    boundary, lexicographic ordering with x fastest;
  * operator -div(a grad u) + b . grad u, first-order upwind convection,
    entries keep the 1/h^2 and 1/h factors (no h^2 rescaling);
  * an x-dependent factor is evaluated at the node x_i = (i+1) h;
  * CSR with int32 row_ptr/col_idx, column indices sorted within each row.
"""
from __future__ import annotations

import dataclasses
import numpy as np
import scipy.sparse as sp

__all__ = [
    "convdiff", "helmholtz2d", "Workload", "System",
    "cfg1", "cfg2", "cfg3", "cfg4", "serving_requests", "reduced",
]


def _stencil(shape, diag, offdiag):
    """Assemble a CSR matrix from per-node diagonal and per-direction neighbour
    coefficients.  `offdiag` maps (axis, +1/-1) to an array over the grid (or a
    scalar).  Nodes outside the grid are dropped (Dirichlet)."""
    dims = len(shape)
    n = int(np.prod(shape))
    idx = np.arange(n, dtype=np.int64).reshape(shape[::-1])  # [z][y][x] with x fastest
    rows = [idx.ravel()]
    cols = [idx.ravel()]
    vals = [np.broadcast_to(diag, shape[::-1]).ravel()]
    for (axis, sgn), coef in offdiag.items():
        # axis 0 = x (last numpy axis), 1 = y, 2 = z
        ax = dims - 1 - axis
        c = np.broadcast_to(coef, shape[::-1])
        sl_src = [slice(None)] * dims
        sl_dst = [slice(None)] * dims
        if sgn > 0:
            sl_src[ax] = slice(0, shape[axis] - 1)
            sl_dst[ax] = slice(1, shape[axis])
        else:
            sl_src[ax] = slice(1, shape[axis])
            sl_dst[ax] = slice(0, shape[axis] - 1)
        r = idx[tuple(sl_src)].ravel()
        cc = idx[tuple(sl_dst)].ravel()
        v = c[tuple(sl_src)].ravel()
        rows.append(r)
        cols.append(cc)
        vals.append(v)
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    A = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    A.sum_duplicates()
    A.sort_indices()
    A.indices = A.indices.astype(np.int32)
    A.indptr = A.indptr.astype(np.int32)
    return A


def convdiff(N, dims, diff=(1.0, 1.0, 1.0), conv=(0.0, 0.0, 0.0), xfactor=None, dtype=np.float64):
    """Upwind finite-difference convection-diffusion on an N^dims interior grid.

    diff:  diffusivities (a_x, a_y, a_z) (constant).
    conv:  convection vector (b_x, b_y, b_z).
    xfactor: optional callable f(x) multiplying the convection vector, evaluated
             at node coordinate x_i = (i+1) h.
    """
    h = 1.0 / (N + 1)
    shape = (N,) * dims
    x = (np.arange(N) + 1) * h
    fx = np.ones(N) if xfactor is None else np.asarray(xfactor(x), dtype=np.float64)
    # broadcast f(x) over the grid, x fastest ([z][y][x] numpy order)
    fgrid = fx.reshape((1,) * (dims - 1) + (N,))
    diag = np.zeros((N,) * dims)
    off = {}
    for axis in range(dims):
        a = float(diff[axis])
        b = float(conv[axis]) * fgrid
        diag = diag + 2.0 * a / h**2
        bp = np.maximum(b, 0.0)  # upwind from the minus side
        bm = np.minimum(b, 0.0)  # upwind from the plus side
        diag = diag + (bp - bm) / h
        off[(axis, -1)] = -a / h**2 - bp / h + 0.0 * fgrid
        off[(axis, +1)] = -a / h**2 + bm / h + 0.0 * fgrid
    A = _stencil(shape, diag, off)
    return A.astype(dtype)


def helmholtz2d(N, kappa, damping=0.5):
    """(1/h^2) L_5pt - kappa^2 (1 - damping*i) I on an N x N grid (complex128)."""
    h = 1.0 / (N + 1)
    L = convdiff(N, 2, diff=(1.0, 1.0, 1.0), conv=(0.0, 0.0, 0.0))
    shift = -(kappa**2) * (1.0 - 1j * damping)
    A = (L.astype(np.complex128) + shift * sp.identity(L.shape[0], format="csr", dtype=np.complex128)).tocsr()
    A.sort_indices()
    A.indices = A.indices.astype(np.int32)
    A.indptr = A.indptr.astype(np.int32)
    return A


@dataclasses.dataclass
class System:
    A: sp.csr_matrix
    B: np.ndarray
    X0: np.ndarray


@dataclasses.dataclass
class Workload:
    name: str
    systems: list
    p: int
    m: int
    k: int
    tol: float
    dtype: str          # "f64" or "c128"
    precision: str      # "plain" or "mixed"
    meta: dict


def _rhs(rng, n, p):
    return rng.uniform(-1.0, 1.0, size=(n, p))


def cfg1(seed=1, N=32, nsys=3):
    """2D convection-diffusion, 32x32 interior, unit diffusion, convection (20,10);
    A_i = A + 0.01 i D, D diagonal U[0,1]; B U[-1,1] with p=4; X0=0; m=20, k=10."""
    rng = np.random.default_rng(seed)
    A = convdiff(N, 2, diff=(1.0, 1.0, 1.0), conv=(20.0, 10.0, 0.0))
    n = A.shape[0]
    D = rng.uniform(0.0, 1.0, size=n)
    systems = []
    for i in range(nsys):
        Ai = (A + sp.diags(0.01 * i * D)).tocsr()
        Ai.sort_indices()
        Ai.indices = Ai.indices.astype(np.int32)
        Ai.indptr = Ai.indptr.astype(np.int32)
        B = _rhs(rng, n, 4)
        systems.append(System(Ai, B, np.zeros_like(B)))
    return Workload("convdiff2d_32x32_p4_m20_k10", systems, 4, 20, 10, 1e-8, "f64", "plain",
                    {"grid": f"{N}x{N}", "n": n})


def _xfac(x):
    return 1.0 + 0.5 * np.sin(2.0 * np.pi * x)


def cfg2(seed=2, N=128, nsys=10, p=8, m=10, k=20):
    """3D convection-diffusion 7-point upwind on N^3, convection (10,5,2)(1+0.5 sin 2 pi x),
    diffusion scaled by (1+0.02 i); p RHS U[-1,1]; m=10, k=20, tol 1e-8."""
    rng = np.random.default_rng(seed)
    systems = []
    for i in range(nsys):
        s = 1.0 + 0.02 * i
        A = convdiff(N, 3, diff=(s, s, s), conv=(10.0, 5.0, 2.0), xfactor=_xfac)
        B = _rhs(rng, A.shape[0], p)
        systems.append(System(A, B, np.zeros_like(B)))
    return Workload(f"convdiff3d_{N}^3_p{p}_m{m}_k{k}", systems, p, m, k, 1e-8, "f64", "plain",
                    {"grid": f"{N}^3", "n": N**3})


def cfg3(seed=3, N=1024, nsys=8, p=16, m=8, k=16, kappa0=20.0):
    """2D shifted-Laplacian Helmholtz (complex128), kappa = kappa0 + i; B = p unit point sources."""
    rng = np.random.default_rng(seed)
    systems = []
    n = N * N
    for i in range(nsys):
        A = helmholtz2d(N, kappa0 + i)
        B = np.zeros((n, p), dtype=np.complex128)
        loc = rng.choice(n, size=p, replace=False)
        B[loc, np.arange(p)] = 1.0
        systems.append(System(A, B, np.zeros_like(B)))
    return Workload(f"helmholtz2d_{N}^2_p{p}_m{m}_k{k}", systems, p, m, k, 1e-8, "c128", "plain",
                    {"grid": f"{N}^2", "n": n})


def cfg4(seed=4, N=192, nsys=6, p=16, m=10, k=24):
    """Anisotropic 3D convection-diffusion, diffusivities (1,0.1,0.01)(1+0.02 i), convection (5,5,5);
    p=16 U[-1,1]; m=10, k=24; target 1e-10; mixed precision."""
    rng = np.random.default_rng(seed)
    systems = []
    for i in range(nsys):
        s = 1.0 + 0.02 * i
        A = convdiff(N, 3, diff=(1.0 * s, 0.1 * s, 0.01 * s), conv=(5.0, 5.0, 5.0))
        B = _rhs(rng, A.shape[0], p)
        systems.append(System(A, B, np.zeros_like(B)))
    return Workload(f"aniso_convdiff3d_{N}^3_p{p}_m{m}_k{k}", systems, p, m, k, 1e-10, "f64", "mixed",
                    {"grid": f"{N}^3", "n": N**3})


def serving_requests(seed=5, nreq=256, sides=tuple(range(64, 161, 16)), ps=(1, 4, 8, 16),
                     nsys_range=(4, 16), rate=None):
    """Request descriptors for the served stream: each request is a sequence of
    related 3D convection-diffusion systems.  Matrices are built lazily by
    `request_system` so that a large stream does not sit in host memory."""
    rng = np.random.default_rng(seed)
    reqs = []
    t = 0.0
    for r in range(nreq):
        side = int(rng.choice(sides))
        p = int(rng.choice(ps))
        nsys = int(rng.integers(nsys_range[0], nsys_range[1] + 1))
        mag = float(rng.uniform(1.0, 20.0))
        d = rng.normal(size=3)
        d = d / np.linalg.norm(d)
        rseed = int(rng.integers(0, 2**31 - 1))
        gap = float(rng.exponential(1.0 / rate)) if rate else 0.0
        t += gap
        reqs.append({"id": r, "side": side, "p": p, "nsys": nsys, "conv": tuple(mag * d),
                     "seed": rseed, "arrival": t})
    return reqs


def request_system(req, i):
    """System i of a served request (diffusion scaled by 1+0.02 i)."""
    s = 1.0 + 0.02 * i
    A = convdiff(req["side"], 3, diff=(s, s, s), conv=req["conv"])
    rng = np.random.default_rng(req["seed"] + 7919 * i)
    B = _rhs(rng, A.shape[0], req["p"])
    return System(A, B, np.zeros_like(B))


def banded(n, bw, seed):
    """Synthetic banded matrix of the data-movement study (Section 6.3 used
    rand/spdiags-built banded matrices): 2 bw + 1 diagonals with seeded
    U[-1, 1] entries, the diagonal replaced by the row's off-diagonal
    magnitude sum plus 1 (diagonally dominant); CSR with sorted indices."""
    rng = np.random.default_rng(seed)
    offs = list(range(-bw, bw + 1))
    diags = [rng.uniform(-1.0, 1.0, n - abs(o)) for o in offs]
    A = sp.diags(diags, offs, shape=(n, n), format="csr")
    off = np.asarray(abs(A).sum(axis=1)).ravel() - np.abs(A.diagonal())
    A.setdiag(off + 1.0)
    A = A.tocsr()
    A.sort_indices()
    return A
