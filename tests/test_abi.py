"""The C-ABI library loads and exports every function include/ks.h declares (CPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ks.h")
LIB = os.path.join(ROOT, "paper_1511_07207_amd", "libks.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ks_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_documented_entry_points():
    names = declared_functions()
    for must in ("ks_create", "ks_solve", "ks_free", "ks_workspace_bytes", "ks_strerror",
                 "ks_gemv", "ks_arnoldi"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libks.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libks.so not built")
def test_binding_lists_the_same_symbols():
    from paper_1511_07207_amd._native import EXPORTS

    assert sorted(EXPORTS) == declared_functions()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libks.so not built")
def test_host_only_entry_points_without_gpu():
    # parameter defaults, workspace sizing and argument validation run on the
    # host and need no device
    from paper_1511_07207_amd import _native as N

    L = N.lib()
    p = N.KsParams()
    assert L.ks_params_init(ctypes.byref(p), 1000, N.KS_GMRES) == 0
    assert p.n == 1000 and p.lda == 1000 and p.restart == 30 and p.tol == 1e-10
    sz = ctypes.c_size_t(0)
    assert L.ks_workspace_bytes(ctypes.byref(p), ctypes.byref(sz)) == 0
    full = sz.value
    assert L.ks_workspace_bytes_borrowed(ctypes.byref(p), ctypes.byref(sz)) == 0
    assert full - sz.value >= 1000 * 1000 * 8
    p.restart = 0
    assert L.ks_workspace_bytes(ctypes.byref(p), ctypes.byref(sz)) == N.KS_EINVAL
    p.restart = 30
    p.tol = 0.0
    assert L.ks_workspace_bytes(ctypes.byref(p), ctypes.byref(sz)) == N.KS_EINVAL
    assert L.ks_params_init(ctypes.byref(p), 0, N.KS_CG) == N.KS_EINVAL
    assert L.ks_strerror(0) == b"converged"
    assert L.ks_gemv(0, 0, 0, None, None, None, None) == N.KS_EINVAL
    L.ks_free(None)


@pytest.mark.skipif(not os.path.exists(LIB), reason="libks.so not built")
def test_bicgstab_parameters_on_host():
    # BiCGSTAB keeps six vectors (r, r0, p, v, s, t) and one State, three more
    # than CG above the fused small-n size (4096, where CG keeps six too); it
    # is a one-right-hand-side method, so nrhs > 1 is rejected
    from paper_1511_07207_amd import _native as N

    L = N.lib()
    p = N.KsParams()
    assert L.ks_params_init(ctypes.byref(p), 5000, N.KS_BICGSTAB) == 0
    assert p.method == N.KS_BICGSTAB
    sz, szc = ctypes.c_size_t(0), ctypes.c_size_t(0)
    assert L.ks_workspace_bytes_borrowed(ctypes.byref(p), ctypes.byref(sz)) == 0
    q = N.KsParams()
    assert L.ks_params_init(ctypes.byref(q), 5000, N.KS_CG) == 0
    assert L.ks_workspace_bytes_borrowed(ctypes.byref(q), ctypes.byref(szc)) == 0
    assert sz.value >= szc.value + 3 * 5000 * 8
    p.nrhs = 4
    assert L.ks_workspace_bytes(ctypes.byref(p), ctypes.byref(sz)) == N.KS_EINVAL
    p.nrhs = 1
    p.timing_every = -1                           # a timing sample stride is >= 0
    assert L.ks_workspace_bytes(ctypes.byref(p), ctypes.byref(sz)) == N.KS_EINVAL
    p.timing_every = 0
    p.precision = N.KS_IR_BF16
    assert L.ks_workspace_bytes(ctypes.byref(p), ctypes.byref(sz)) == 0
    assert L.ks_params_init(ctypes.byref(p), 10, 5) == N.KS_EINVAL


@pytest.mark.skipif(not os.path.exists(LIB), reason="libks.so not built")
def test_stationary_parameters_on_host():
    # Jacobi and Gauss-Seidel: binary64 only, one right-hand side, general
    # storage; Gauss-Seidel keeps three more vectors than Jacobi (U x twice,
    # b - U x); the request server takes neither
    from paper_1511_07207_amd import _native as N

    L = N.lib()
    sizes = {}
    for m in (N.KS_JACOBI, N.KS_GAUSS_SEIDEL):
        p = N.KsParams()
        assert L.ks_params_init(ctypes.byref(p), 1000, m) == 0
        assert p.method == m
        sz = ctypes.c_size_t(0)
        assert L.ks_workspace_bytes_borrowed(ctypes.byref(p), ctypes.byref(sz)) == 0
        sizes[m] = sz.value
        for field, bad in (("precision", N.KS_IR_FP32), ("precision", N.KS_IR_BF16),
                           ("nrhs", 2), ("flags", N.KS_FLAG_SYMMETRIC)):
            q = N.KsParams()
            assert L.ks_params_init(ctypes.byref(q), 1000, m) == 0
            setattr(q, field, bad)
            assert L.ks_workspace_bytes(ctypes.byref(q), ctypes.byref(sz)) == N.KS_EINVAL, field
    assert sizes[N.KS_GAUSS_SEIDEL] >= sizes[N.KS_JACOBI] + 3 * 1024 * 8
    assert L.ks_params_init(ctypes.byref(N.KsParams()), 10, 5) == N.KS_EINVAL


@pytest.mark.skipif(not os.path.exists(LIB), reason="libks.so not built")
def test_gmres_ir_lu_parameters_on_host():
    # GMRES-IR with the binary32 LU: GMRES only, one right-hand side,
    # n <= 4096; the workspace holds the binary32 factors (n x round_up(n, 64))
    from paper_1511_07207_amd import _native as N

    L = N.lib()
    p = N.KsParams()
    assert L.ks_params_init(ctypes.byref(p), 1000, N.KS_GMRES) == 0
    p.precision = N.KS_IR_LU32
    sz, sz64 = ctypes.c_size_t(0), ctypes.c_size_t(0)
    assert L.ks_workspace_bytes_borrowed(ctypes.byref(p), ctypes.byref(sz)) == 0
    q = N.KsParams()
    assert L.ks_params_init(ctypes.byref(q), 1000, N.KS_GMRES) == 0
    assert L.ks_workspace_bytes_borrowed(ctypes.byref(q), ctypes.byref(sz64)) == 0
    assert sz.value >= sz64.value + 4 * 1000 * 1024
    for method in (N.KS_CG, N.KS_BICGSTAB, N.KS_JACOBI):
        r = N.KsParams()
        assert L.ks_params_init(ctypes.byref(r), 1000, method) == 0
        r.precision = N.KS_IR_LU32
        assert L.ks_workspace_bytes(ctypes.byref(r), ctypes.byref(sz)) == N.KS_EINVAL
    r = N.KsParams()
    assert L.ks_params_init(ctypes.byref(r), 32769, N.KS_GMRES) == 0
    r.precision = N.KS_IR_LU32
    assert L.ks_workspace_bytes(ctypes.byref(r), ctypes.byref(sz)) == N.KS_EINVAL
    r.n = r.lda = 32768
    assert L.ks_workspace_bytes(ctypes.byref(r), ctypes.byref(sz)) == 0
    # the binary64 A, its binary32 copy holding the factors, and the 16 KiB
    # work area of the factorization beside the pivots
    assert sz.value >= 32768 * 32768 * (8 + 4) + 16384
    info = ctypes.c_int32(0)
    assert L.ks_lu32_factor(32769, 32769, None, 32769, None, None, ctypes.byref(info), None) == N.KS_EINVAL


@pytest.mark.skipif(not os.path.exists(LIB), reason="libks.so not built")
def test_symmetric_flag_and_symv_on_host():
    from paper_1511_07207_amd import _native as N

    L = N.lib()
    sz = ctypes.c_size_t(0)
    assert L.ks_symv_workspace_bytes(16384, ctypes.byref(sz)) == 0
    tiles = 64 * 65 // 2                          # 256 x 256 tiles of the lower triangle
    assert sz.value == tiles * 2 * 256 * 8        # a row part and a column part per tile
    assert L.ks_symv_workspace_bytes(0, ctypes.byref(sz)) == N.KS_EINVAL
    assert L.ks_symv(10, 10, None, None, None, None, 0, None) == N.KS_EINVAL
    assert L.ks_symv_f32(10, 12, None, None, None, None, 0, None) == N.KS_EINVAL
    assert L.ks_symv_f32(-1, 12, None, None, None, None, 0, None) == N.KS_EINVAL
    p = N.KsParams()
    assert L.ks_params_init(ctypes.byref(p), 16384, N.KS_CG) == 0
    base = ctypes.c_size_t(0)
    assert L.ks_workspace_bytes_borrowed(ctypes.byref(p), ctypes.byref(base)) == 0
    p.flags = N.KS_FLAG_SYMMETRIC
    assert L.ks_workspace_bytes_borrowed(ctypes.byref(p), ctypes.byref(sz)) == 0
    # CG also keeps a p'Ap share per tile and two partials per 64-element finishing block
    assert sz.value >= base.value + (tiles * 2 * 256 + tiles + 2 * 16384 // 64) * 8
    p.nrhs = 4
    assert L.ks_workspace_bytes(ctypes.byref(p), ctypes.byref(sz)) == N.KS_EINVAL
    p.nrhs = 1
    p.timing_every = -1                           # a timing sample stride is >= 0
    assert L.ks_workspace_bytes(ctypes.byref(p), ctypes.byref(sz)) == N.KS_EINVAL
    q = N.KsParams()
    assert L.ks_params_init(ctypes.byref(q), 100, N.KS_GMRES) == 0
    q.flags = N.KS_FLAG_SYMMETRIC
    assert L.ks_workspace_bytes(ctypes.byref(q), ctypes.byref(sz)) == N.KS_EINVAL


@pytest.mark.skipif(not os.path.exists(LIB), reason="libks.so not built")
def test_cholesky_refinement_parameters_on_host():
    """KS_IR_CHOL32 is CG with one right-hand side and the general product;
    the factorization entry point validates its arguments before any device
    call."""
    from paper_1511_07207_amd import _native as N

    L = N.lib()
    sz = ctypes.c_size_t(0)
    p = N.KsParams()
    assert L.ks_params_init(ctypes.byref(p), 32768, N.KS_CG) == 0
    p.precision = N.KS_IR_CHOL32
    assert L.ks_workspace_bytes_borrowed(ctypes.byref(p), ctypes.byref(sz)) == 0
    # the binary32 factor (n x round_up(n, 64) floats) dominates
    assert sz.value >= 32768 * 32768 * 4
    for method in (N.KS_GMRES, N.KS_BICGSTAB):
        q = N.KsParams()
        assert L.ks_params_init(ctypes.byref(q), 100, method) == 0
        q.precision = N.KS_IR_CHOL32
        assert L.ks_workspace_bytes(ctypes.byref(q), ctypes.byref(sz)) == N.KS_EINVAL
    p.flags = N.KS_FLAG_SYMMETRIC
    assert L.ks_workspace_bytes(ctypes.byref(p), ctypes.byref(sz)) == N.KS_EINVAL
    p.flags = 0
    p.nrhs = 2
    assert L.ks_workspace_bytes(ctypes.byref(p), ctypes.byref(sz)) == N.KS_EINVAL
    p.nrhs = 1
    p.precision = N.KS_IR_CHOL32 + 1
    assert L.ks_workspace_bytes(ctypes.byref(p), ctypes.byref(sz)) == N.KS_EINVAL
    info = ctypes.c_int32(0)
    assert L.ks_chol32_factor(0, 1, None, 1, None, ctypes.byref(info), None) == N.KS_EINVAL
    assert L.ks_chol32_factor(10, 10, 16, 9, 16, ctypes.byref(info), None) == N.KS_EINVAL  # ldl < n
    assert L.ks_chol32_factor(10, 10, 16, 10, 16, ctypes.byref(info), None) == N.KS_EINVAL  # ldl % 4


@pytest.mark.skipif(not os.path.exists(LIB), reason="libks.so not built")
def test_symv_noalloc_limits_on_host():
    """The fixed-array product refuses an order beyond its array and bad
    arguments before any device call."""
    from paper_1511_07207_amd import _native as N

    L = N.lib()
    assert L.ks_symv_noalloc(32769, 32769, 16, 16, 16, None) == N.KS_ETOOLARGE
    assert L.ks_symv_noalloc(0, 1, 16, 16, 16, None) == N.KS_EINVAL
    assert L.ks_symv_noalloc(100, 99, 16, 16, 16, None) == N.KS_EINVAL
    assert L.ks_symv_noalloc(100, 100, None, 16, 16, None) == N.KS_EINVAL
    assert L.ks_symv_noalloc(100, 101, 16, 16, 16, None) == N.KS_EINVAL  # rows not 16-byte aligned


@pytest.mark.skipif(not os.path.exists(LIB), reason="libks.so not built")
def test_gemm_mr_limits_on_host():
    """The lockstep contraction entry point: its workspace (a zero-padded copy
    of P plus one partial product per split of K: 4 at n = 16384 in either
    precision) and its argument checks, all before any device call."""
    from paper_1511_07207_amd import _native as N

    L = N.lib()
    sz = ctypes.c_size_t(0)
    assert L.ks_gemm_mr_workspace_bytes(16384, 64, N.KS_DT_F64, ctypes.byref(sz)) == 0
    assert sz.value == (1 + 4) * 64 * 16384 * 8
    assert L.ks_gemm_mr_workspace_bytes(16384, 64, N.KS_DT_F32, ctypes.byref(sz)) == 0
    assert sz.value == (1 + 4) * 64 * 16384 * 4
    assert L.ks_gemm_mr_workspace_bytes(777, 5, N.KS_DT_F32, ctypes.byref(sz)) == 0
    assert sz.value == (1 + 1) * 16 * 832 * 4     # s padded to 16, rows to 64; one split
    for s in (0, 65):
        assert L.ks_gemm_mr_workspace_bytes(100, s, N.KS_DT_F64, ctypes.byref(sz)) == N.KS_EINVAL
    assert L.ks_gemm_mr_workspace_bytes(100, 4, N.KS_DT_BF16, ctypes.byref(sz)) == N.KS_EINVAL
    big = 1 << 40
    assert L.ks_gemm_mr(100, 100, N.KS_DT_F64, 16, 0, 16, 100, 16, 16, big, None) == N.KS_EINVAL
    assert L.ks_gemm_mr(100, 100, N.KS_DT_F64, 16, 65, 16, 100, 16, 16, big, None) == N.KS_EINVAL
    assert L.ks_gemm_mr(100, 99, N.KS_DT_F64, 16, 4, 16, 100, 16, 16, big, None) == N.KS_EINVAL
    assert L.ks_gemm_mr(100, 100, N.KS_DT_F64, 16, 4, 16, 99, 16, 16, big, None) == N.KS_EINVAL
    assert L.ks_gemm_mr(100, 102, N.KS_DT_F32, 16, 4, 16, 100, 16, 16, big, None) == N.KS_EINVAL
    assert L.ks_gemm_mr(100, 100, N.KS_DT_F64, 8, 4, 16, 100, 16, 16, big, None) == N.KS_EINVAL
    assert L.ks_gemm_mr(100, 100, N.KS_DT_BF16, 16, 4, 16, 100, 16, 16, big, None) == N.KS_EINVAL
    assert L.ks_gemm_mr(100, 100, N.KS_DT_F64, 16, 4, None, 100, 16, 16, big, None) == N.KS_EINVAL
    assert L.ks_gemm_mr(100, 100, N.KS_DT_F64, 16, 4, 16, 100, 16, 16, 1024, None) == N.KS_ENOMEM
