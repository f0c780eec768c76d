"""CPU-side checks of the C ABI: the library loads, exports every symbol the
header declares, validates arguments without a GPU, and the input generators
produce what their recipes say."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1604_01713_amd as bg
import problems

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    txt = open(os.path.join(ROOT, "include", "bgcr.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|size_t|const char\*)\s+(bgcr_\w+)\s*\(", txt, re.M)))


def test_header_declares_the_binding_symbols():
    assert _header_functions() == sorted(bg.EXPORTED_SYMBOLS)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(bg.LIB_PATH):
        from paper_1604_01713_amd.build import build
        build()
    return bg.lib()


def test_library_exports_every_declared_symbol(lib):
    for name in _header_functions():
        assert hasattr(lib, name), name


def test_library_resolves_every_symbol_at_load(lib):
    """Loaded with immediate binding, the library has no undefined symbol (a
    kernel launcher declared but never instantiated would only fail at its
    first call otherwise)."""
    ctypes.CDLL(bg.LIB_PATH, mode=os.RTLD_NOW | os.RTLD_LOCAL)


def test_ilu0_parameters_without_gpu(lib):
    """Right preconditioning with ILU(0): plain FP64 (real or complex), no
    enlarged block or hybrid; its footprint adds the M^{-1} work block, the
    level orders and the factors on A's pattern."""
    n, nnz = 32**3, 7 * 32**3
    P = lambda pc, **kw: bg.bgcr_params(kw.get("p", 8), 10, 20, kw.get("dtype", bg.BGCR_F64),
                                        kw.get("prec", bg.BGCR_PLAIN_FP64), 100, 0, kw.get("bs", 0), 0, 0, pc)
    f0 = bg.bgcr_footprint_bytes(P(0), n, nnz)
    f1 = bg.bgcr_footprint_bytes(P(1), n, nnz)
    # two n x p solve blocks, diagonal positions, row pointers, flag and
    # tickets, two level orders, the factors and column indices
    assert f1 - f0 == 2 * n * 8 * 8 + 4 * (2 * n + 4) + 8 * n + nnz * (8 + 4)
    fc = bg.bgcr_footprint_bytes(P(1, dtype=bg.BGCR_C128, p=16), n, nnz)
    assert fc - bg.bgcr_footprint_bytes(P(0, dtype=bg.BGCR_C128, p=16), n, nnz) == \
        2 * n * 16 * 16 + 4 * (2 * n + 4) + 8 * n + nnz * (16 + 4)
    h = ctypes.c_void_p()
    for bad in (P(1, prec=bg.BGCR_MIXED_FP32), P(1, p=1, bs=8), P(2)):
        assert bg.bgcr_footprint_bytes(bad, n, nnz) == 0
        assert lib.bgcr_create_sequence(ctypes.byref(bad), n, None, ctypes.byref(h)) == bg.BGCR_ERR_INVALID


def test_strerror_and_footprint_without_gpu(lib):
    assert bg.bgcr_strerror(0) == "ok"
    assert "invalid" in bg.bgcr_strerror(-1)
    prm = bg.bgcr_params(8, 10, 20, bg.BGCR_F64, bg.BGCR_PLAIN_FP64, 100, 0, 0)
    n = 128**3
    fb = bg.bgcr_footprint_bytes(prm, n, 7 * n)
    # at least the basis (m blocks), U and C (double buffered) and W2, Wb, R, X
    assert fb >= (10 + 4 * 3 + 4) * n * 8 * 8
    assert fb < 8 * 1024**3
    bad = bg.bgcr_params(3, 10, 20, bg.BGCR_F64, bg.BGCR_PLAIN_FP64, 100, 0, 0)
    assert bg.bgcr_footprint_bytes(bad, n, 7 * n) == 0
    mixed_c = bg.bgcr_params(8, 10, 20, bg.BGCR_C128, bg.BGCR_MIXED_FP32, 100, 0, 0)
    assert bg.bgcr_footprint_bytes(mixed_c, n, 7 * n) == 0
    fm = bg.bgcr_footprint_bytes(bg.bgcr_params(8, 10, 20, bg.BGCR_F64, bg.BGCR_MIXED_FP32, 100, 0, 0), n, 7 * n)
    assert fm < fb


def test_bf16_basis_footprint_and_limits_without_gpu(lib):
    n = 64**3
    fm = bg.bgcr_footprint_bytes(bg.bgcr_params(8, 10, 20, bg.BGCR_F64, bg.BGCR_MIXED_FP32, 100, 0, 0), n, 7 * n)
    fh = bg.bgcr_footprint_bytes(bg.bgcr_params(8, 10, 20, bg.BGCR_F64, bg.BGCR_MIXED_FP32_BF16, 100, 0, 0), n,
                                 7 * n)
    # only the basis blocks shrink: V_1..V_{m+1} and two copies each of U and C
    # (k + 1 = 21 columns -> 3 blocks of 8), 4 -> 2 bytes per value
    assert fm - fh == (11 + 4 * 3) * n * 8 * 2
    for bad in (bg.bgcr_params(4, 10, 20, bg.BGCR_F64, bg.BGCR_MIXED_FP32_BF16, 100, 0, 0),
                bg.bgcr_params(16, 10, 20, bg.BGCR_C128, bg.BGCR_MIXED_FP32_BF16, 100, 0, 0),
                bg.bgcr_params(8, 10, 20, bg.BGCR_F64, 3, 100, 0, 0)):
        assert bg.bgcr_footprint_bytes(bad, n, 7 * n) == 0
        h = ctypes.c_void_p()
        assert lib.bgcr_create_sequence(ctypes.byref(bad), n, None, ctypes.byref(h)) == bg.BGCR_ERR_INVALID


def test_enlarged_block_parameters_without_gpu(lib):
    n = 32**3
    f1 = bg.bgcr_footprint_bytes(bg.bgcr_params(1, 10, 20, bg.BGCR_F64, bg.BGCR_PLAIN_FP64, 100, 0, 0), n, 7 * n)
    f8 = bg.bgcr_footprint_bytes(bg.bgcr_params(1, 10, 20, bg.BGCR_F64, bg.BGCR_PLAIN_FP64, 100, 0, 8), n, 7 * n)
    assert 0 < f1 < f8   # n x 8 blocks instead of n x 1, plus B padded
    h = ctypes.c_void_p()
    for bad in (bg.bgcr_params(1, 10, 20, bg.BGCR_F64, bg.BGCR_PLAIN_FP64, 100, 0, 3),
                bg.bgcr_params(2, 10, 20, bg.BGCR_F64, bg.BGCR_PLAIN_FP64, 100, 0, 8),
                bg.bgcr_params(1, 10, 20, bg.BGCR_F64, bg.BGCR_PLAIN_FP64, 100, 0, 32)):
        assert bg.bgcr_footprint_bytes(bad, n, 7 * n) == 0
        assert lib.bgcr_create_sequence(ctypes.byref(bad), n, None, ctypes.byref(h)) == bg.BGCR_ERR_INVALID
    same = bg.bgcr_params(4, 10, 20, bg.BGCR_F64, bg.BGCR_PLAIN_FP64, 100, 0, 4)   # block_size = p: no enlargement
    assert bg.bgcr_footprint_bytes(same, n, 7 * n) == bg.bgcr_footprint_bytes(
        bg.bgcr_params(4, 10, 20, bg.BGCR_F64, bg.BGCR_PLAIN_FP64, 100, 0, 0), n, 7 * n)


def test_hybrid_parameters_without_gpu(lib):
    """enlarge_cycles > 0 (Section 4.1.3 hybrid) holds an L-block and an
    L = 1 sequence plus one n x k' FP64 hand-over buffer; it needs an
    enlarged block and a basis type the L = 1 sequence has."""
    n = 32**3
    P = lambda bs, ec, prec=bg.BGCR_PLAIN_FP64, p=1: bg.bgcr_params(p, 10, 20, bg.BGCR_F64, prec, 100, 0, bs, ec)
    f1 = bg.bgcr_footprint_bytes(P(0, 0), n, 7 * n)
    f8 = bg.bgcr_footprint_bytes(P(8, 0), n, 7 * n)
    fh = bg.bgcr_footprint_bytes(P(8, 3), n, 7 * n)
    assert fh == f1 + f8 + n * 24 * 8   # ceil(21 / 8) * 8 = 24 hand-over columns
    fm = bg.bgcr_footprint_bytes(P(8, 3, bg.BGCR_MIXED_FP32), n, 7 * n)
    assert fm == (bg.bgcr_footprint_bytes(P(0, 0, bg.BGCR_MIXED_FP32), n, 7 * n)
                  + bg.bgcr_footprint_bytes(P(8, 0, bg.BGCR_MIXED_FP32), n, 7 * n) + n * 24 * 8)
    h = ctypes.c_void_p()
    for bad in (P(0, 3), P(1, 3), P(4, 3, p=4), P(8, -1), P(8, 3, bg.BGCR_MIXED_FP32_BF16)):
        assert bg.bgcr_footprint_bytes(bad, n, 7 * n) == 0
        assert lib.bgcr_create_sequence(ctypes.byref(bad), n, None, ctypes.byref(h)) == bg.BGCR_ERR_INVALID


def test_projected_operator_arguments_without_gpu(lib):
    """bgcr_apply_projected validates before touching the device; its workspace
    holds S (kc p^2) and one launch's partials."""
    wb = bg.bgcr_apply_projected_work_bytes
    assert wb(1000, 3, 4) == 0 and wb(1000, 8, -1) == 0
    assert wb(1000, 8, 13) == 8 * (13 * 64 + 512 * 14 * 64)
    assert wb(1000, 1, 100) == 8 * (100 + 512 * 33)
    csr = bg.bgcr_csr(100, 0, None, None, None)
    assert lib.bgcr_apply_projected(ctypes.byref(csr), 8, 0, None, None, None, 0, None, 0, None) == bg.BGCR_ERR_INVALID
    # the allocation-free variant checks its size limit before anything else
    # touches the device: p = 16 fits 1536 blocks of C in its 20 MiB
    assert wb(1000, 16, 1536) <= bg.BGCR_NOALLOC_SCRATCH_BYTES < wb(1000, 16, 1537)
    na = lib.bgcr_apply_projected_noalloc
    assert na(ctypes.byref(csr), 16, 1537, None, None, None, 0, None) == bg.BGCR_ERR_INVALID
    assert na(ctypes.byref(csr), 3, 1, None, None, None, 0, None) == bg.BGCR_ERR_INVALID
    assert na(None, 8, 1, None, None, None, 0, None) == bg.BGCR_ERR_INVALID


def test_invalid_arguments_are_rejected_without_a_gpu(lib):
    h = ctypes.c_void_p()
    # the recycle refresh combines [U, C, V_1 .. V_{m+1}]: 2 ceil((k+1)/p) + m + 1 <= 64 blocks
    assert bg.bgcr_footprint_bytes(bg.bgcr_params(1, 21, 20, bg.BGCR_F64, bg.BGCR_PLAIN_FP64, 100, 0, 0), 4096, 0) > 0
    ritz = bg.bgcr_params(8, 10, 20, bg.BGCR_F64, bg.BGCR_PLAIN_FP64, 100, 0, 0, 0, 1)
    assert bg.bgcr_footprint_bytes(ritz, 4096, 0) == bg.bgcr_footprint_bytes(
        bg.bgcr_params(8, 10, 20, bg.BGCR_F64, bg.BGCR_PLAIN_FP64, 100, 0, 0), 4096, 0)
    bad_ritz = bg.bgcr_params(8, 10, 20, bg.BGCR_F64, bg.BGCR_PLAIN_FP64, 100, 0, 0, 0, 2)
    assert bg.bgcr_footprint_bytes(bad_ritz, 4096, 0) == 0
    too_wide = bg.bgcr_params(1, 22, 20, bg.BGCR_F64, bg.BGCR_PLAIN_FP64, 100, 0, 0)
    assert bg.bgcr_footprint_bytes(too_wide, 4096, 0) == 0
    assert lib.bgcr_create_sequence(ctypes.byref(too_wide), 4096, None, ctypes.byref(h)) == bg.BGCR_ERR_INVALID
    assert lib.bgcr_create_sequence(None, 10, None, ctypes.byref(h)) == bg.BGCR_ERR_INVALID
    prm = bg.bgcr_params(5, 10, 20, bg.BGCR_F64, bg.BGCR_PLAIN_FP64, 100, 0, 0)
    assert lib.bgcr_create_sequence(ctypes.byref(prm), 10, None, ctypes.byref(h)) == bg.BGCR_ERR_INVALID
    assert lib.bgcr_solve(None, None, None, 0, None, 0, 1e-8, None) == bg.BGCR_ERR_INVALID
    assert lib.bgcr_release(None) == 0
    assert lib.bgcr_spmm(None, 0, 4, None, None, None) == bg.BGCR_ERR_INVALID


def test_generators_follow_their_recipes():
    A = problems.convdiff(4, 3, diff=(1.0, 0.1, 0.01), conv=(5.0, -5.0, 5.0))
    n = 64
    assert A.shape == (n, n) and A.nnz == 7 * 4**3 - 6 * 4**2
    h = 1.0 / 5
    # interior node (1,1,1): diagonal 2(a_x+a_y+a_z)/h^2 + (|b_x|+|b_y|+|b_z|)/h
    i = 1 + 4 * 1 + 16 * 1
    assert A[i, i] == pytest.approx(2 * 1.11 / h**2 + 15.0 / h)
    assert A[i, i - 1] == pytest.approx(-1.0 / h**2 - 5.0 / h)     # upwind from -x for b_x > 0
    assert A[i, i + 1] == pytest.approx(-1.0 / h**2)
    assert A[i, i + 4] == pytest.approx(-0.1 / h**2 - 5.0 / h)     # b_y < 0: upwind from +y
    assert A[i, i - 4] == pytest.approx(-0.1 / h**2)
    w = problems.cfg1()
    assert w.systems[0].A.shape == (1024, 1024) and w.systems[0].A.nnz == 5 * 32**2 - 4 * 32
    d = (w.systems[1].A - w.systems[0].A).diagonal()
    assert np.all(d >= 0) and np.all(d <= 0.01)
    H = problems.helmholtz2d(8, 20.0)
    assert H.dtype == np.complex128
    assert H[0, 0] == pytest.approx(4 * 81 - 400 * (1 - 0.5j))


def test_stream_probe_arguments_without_gpu(lib):
    """The streaming-rate probe validates its arguments before any device call:
    1..16 inputs, 0..4 outputs, an even element count, 16-byte alignment."""
    sp = lib.bgcr_stream_probe
    P = ctypes.c_void_p
    ins = (P * 2)(P(0x1000), P(0x2000))
    outs = (P * 1)(P(0x3000))
    assert sp(None, 1, None, 0, 16, 0, None) == bg.BGCR_ERR_INVALID
    assert sp(ins, 0, None, 0, 16, 0, None) == bg.BGCR_ERR_INVALID
    assert sp(ins, 17, None, 0, 16, 0, None) == bg.BGCR_ERR_INVALID
    assert sp(ins, 2, outs, 5, 16, 0, None) == bg.BGCR_ERR_INVALID
    assert sp(ins, 2, None, 1, 16, 0, None) == bg.BGCR_ERR_INVALID
    assert sp(ins, 2, outs, 1, 15, 0, None) == bg.BGCR_ERR_INVALID
    assert sp(ins, 2, outs, 1, 16, -1, None) == bg.BGCR_ERR_INVALID
    odd = (P * 1)(P(0x1008))
    assert sp(odd, 1, outs, 1, 16, 0, None) == bg.BGCR_ERR_INVALID
    # nothing to stream: accepted without a launch
    assert sp(ins, 2, outs, 1, 0, 0, None) == bg.BGCR_OK
