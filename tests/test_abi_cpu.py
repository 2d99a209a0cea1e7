"""Host-side checks of the C ABI (no GPU needed): the library loads, every
entry point declared in include/rf.h is exported, and invalid arguments are
rejected synchronously before anything touches a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    import paper_2605_09755_amd as rf
    if not os.path.exists(rf.library_path):
        from paper_2605_09755_amd import build
        build.build()
    return rf, rf.lib()


def declared_symbols():
    txt = open(os.path.join(ROOT, "include", "rf.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(rf_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_entry_points():
    syms = declared_symbols()
    for name in ("rf_range_finder", "rf_svd", "rf_lowrank", "rf_nystrom", "rf_workspace_size",
                 "rf_sketch_table", "rf_gaussian", "rf_sketch_apply", "rf_sketch_apply_left",
                 "rf_sketch_apply_left_ws", "rf_status_string"):
        assert name in syms


def test_library_exports_every_declared_symbol():
    rf, L = _lib()
    for name in declared_symbols():
        assert hasattr(L, name), name


def test_status_strings():
    rf, L = _lib()
    assert rf.rf_status_string(0) == "ok"
    assert "invalid" in rf.rf_status_string(1)


FAKE = 0x1000  # never dereferenced: every call below fails validation first


def _mat(rows, cols, ld=None, dtype=0, scales=None, reserved=0):
    import paper_2605_09755_amd as rf
    return rf.RfMatrix(FAKE, scales, rows, cols, cols if ld is None else ld, dtype, reserved)


@pytest.mark.parametrize("k,l,q,s,prec", [
    (0, 10, 1, 2, 0),      # k < 1
    (11, 10, 1, 2, 0),     # k > sketch
    (5, 101, 1, 2, 0),     # sketch > min(m, n)
    (5, 10, -1, 2, 0),     # q < 0
    (5, 10, 1, 0, 0),      # s < 1
    (5, 10, 1, 11, 0),     # s > sketch
    (5, 10, 1, 2, 7),      # bad precision
])
def test_invalid_params_rejected(k, l, q, s, prec):
    rf, L = _lib()
    A = _mat(200, 100)
    p = rf.params(k, l, q, s, 1, prec)
    assert L.rf_workspace_size(0, ctypes.byref(A), ctypes.byref(p)) == 0
    st = L.rf_range_finder(ctypes.byref(A), ctypes.byref(p), FAKE, max(k, 1), FAKE, 1 << 40, None, None)
    assert st == rf.RF_EINVAL


def test_invalid_matrix_rejected():
    rf, L = _lib()
    p = rf.params(5, 10, 1, 2, 1)
    for A in (_mat(200, 100, ld=50), _mat(0, 100), _mat(200, 100, dtype=1), _mat(200, 100, dtype=3),
              _mat(200, 100, reserved=1), _mat(200, 100, dtype=0, scales=FAKE)):
        assert L.rf_workspace_size(1, ctypes.byref(A), ctypes.byref(p)) == 0
        assert L.rf_svd(ctypes.byref(A), ctypes.byref(p), FAKE, 5, FAKE, FAKE, 100, FAKE, 1 << 40, None,
                        None) == rf.RF_EINVAL


def test_workspace_too_small():
    rf, L = _lib()
    A = _mat(200, 100)
    p = rf.params(5, 10, 1, 2, 1)
    need = L.rf_workspace_size(0, ctypes.byref(A), ctypes.byref(p))
    assert need > 0
    assert L.rf_range_finder(ctypes.byref(A), ctypes.byref(p), FAKE, 5, FAKE, need - 1, None, None) == rf.RF_EWORKSPACE
    assert L.rf_range_finder(ctypes.byref(A), ctypes.byref(p), FAKE, 5, None, need, None, None) == rf.RF_EWORKSPACE


def test_nystrom_needs_square_and_small_ld():
    rf, L = _lib()
    p = rf.params(5, 10, 1, 2, 1)
    A = _mat(200, 100)
    assert L.rf_workspace_size(3, ctypes.byref(A), ctypes.byref(p)) == 0
    Asq = _mat(100, 100)
    assert L.rf_workspace_size(3, ctypes.byref(Asq), ctypes.byref(p)) > 0
    st = L.rf_nystrom(ctypes.byref(Asq), ctypes.byref(p), FAKE, 4, FAKE, 5, None, 0, FAKE, 1 << 40, None, None)
    assert st == rf.RF_EINVAL                      # ldc < k


def test_workspace_monotone_in_size():
    rf, L = _lib()
    p = rf.params(20, 40, 2, 8, 1)
    a = L.rf_workspace_size(1, ctypes.byref(_mat(1000, 500)), ctypes.byref(p))
    b = L.rf_workspace_size(1, ctypes.byref(_mat(2000, 500)), ctypes.byref(p))
    assert 0 < a < b


@pytest.mark.parametrize("N", [1, 64, 65, 500, 1000, 2000, 4000])
def test_eig_workspace_covers_the_solver_layout(N):
    """The eigensolver lays out two G buffers and Z (K x K FP64, K = N rounded up
    to a multiple of 64), two slots of p = K / 64 rotation blocks of 64 x 64 FP64,
    a K-int permutation and small flags; the size the library reports must cover
    all of it (a regression check: the block storage was once sized for 32 x 32
    blocks and the solver wrote past the end of its workspace)."""
    rf, L = _lib()
    L.rf_test_eig_ws.restype = ctypes.c_size_t
    L.rf_test_eig_ws.argtypes = [ctypes.c_int64]
    K = max(64, -(-N // 64) * 64)
    p = K // 64
    need = 3 * K * K * 8 + 2 * p * 64 * 64 * 8 + K * 4 + 2 * p * 4 + 4 * 8
    assert L.rf_test_eig_ws(N) >= need + 255   # the entry aligns its workspace to 256 bytes


def test_hooks_reject_bad_args():
    rf, L = _lib()
    assert L.rf_sketch_table(10, 0, 5, 1, 0, 0, FAKE, None) == rf.RF_EINVAL
    assert L.rf_sketch_table(10, 6, 5, 1, 0, 0, FAKE, None) == rf.RF_EINVAL
    assert L.rf_gaussian(-1, 5, 1, 1, 0, FAKE, None) == rf.RF_EINVAL
    assert L.rf_test_gemm(1, 1, 1, FAKE, 4, FAKE, 4, FAKE, 4, 4, 4, 4, 0, None, None) == rf.RF_EINVAL
    assert L.rf_test_eig(FAKE, 5000, 1e-12, FAKE, FAKE, None, FAKE, None) == rf.RF_EUNSUPPORTED
    assert L.rf_test_eig(FAKE, 50, 0.0, FAKE, FAKE, None, FAKE, None) == rf.RF_EINVAL


def test_batched_entry_points_validate_without_gpu():
    """Argument checks of the batched plan run before any HIP call."""
    rf, L = _lib()
    M = rf.RfMatrix(FAKE, None, 100, 50, 50, rf.RF_F32, 0)
    P = rf.params(10, 20, 1, 4, 0, "mixed")
    mats = (rf.RfMatrix * 1)(M)
    prms = (rf.RfParams * 1)(P)
    assert L.rf_svd_batched_ws(0, ctypes.cast(mats, ctypes.c_void_p), ctypes.cast(prms, ctypes.c_void_p)) == 0
    assert L.rf_svd_batched_ws(1, ctypes.cast(mats, ctypes.c_void_p), ctypes.cast(prms, ctypes.c_void_p)) > 0
    h = ctypes.c_void_p()
    # null output arrays
    assert L.rf_svd_batched_plan(1, ctypes.cast(mats, ctypes.c_void_p), ctypes.cast(prms, ctypes.c_void_p),
                                 None, None, None, None, None, None, None, 0, 0, None, ctypes.byref(h)) == rf.RF_EINVAL
    ptrs = (ctypes.c_void_p * 1)(FAKE)
    lds = (ctypes.c_int64 * 1)(1000)
    args = [ctypes.cast(ptrs, ctypes.c_void_p), ctypes.cast(lds, ctypes.c_void_p), ctypes.cast(ptrs, ctypes.c_void_p),
            ctypes.cast(ptrs, ctypes.c_void_p), ctypes.cast(lds, ctypes.c_void_p)]
    # unsupported: 8 nonzeros per column in a batch
    P8 = (rf.RfParams * 1)(rf.params(10, 20, 1, 8, 0, "mixed"))
    assert L.rf_svd_batched_plan(1, ctypes.cast(mats, ctypes.c_void_p), ctypes.cast(P8, ctypes.c_void_p), *args,
                                 None, None, 0, 0, None, ctypes.byref(h)) == rf.RF_EUNSUPPORTED
    # invalid: sketch below k
    Pb = (rf.RfParams * 1)(rf.params(30, 20, 1, 4, 0, "mixed"))
    assert L.rf_svd_batched_plan(1, ctypes.cast(mats, ctypes.c_void_p), ctypes.cast(Pb, ctypes.c_void_p), *args,
                                 None, None, 0, 0, None, ctypes.byref(h)) == rf.RF_EINVAL
    # workspace too small
    assert L.rf_svd_batched_plan(1, ctypes.cast(mats, ctypes.c_void_p), ctypes.cast(prms, ctypes.c_void_p), *args,
                                 None, FAKE, 16, 0, None, ctypes.byref(h)) == rf.RF_EWORKSPACE
    L.rf_svd_batched_destroy(None)


def test_gemm_rules_validate():
    rf, L = _lib()
    big = 1 << 62
    ok = [(0, 128, 4, big, big, big), (2, 256, 0, 4096, 4096, big)]
    rf.set_gemm_rules(ok)
    for bad in [(0, 256, 1, big, big, big),      # 256 tiles are BF16 only
                (2, 64, 1, big, big, big),       # no such tile
                (2, 128, 17, big, big, big),     # split above 16
                (1, 128, 1, big, big, big)]:     # dtype
        with pytest.raises(rf.RFError) as e:
            rf.set_gemm_rules([bad])
        assert e.value.status == rf.RF_EINVAL
    with pytest.raises(rf.RFError):
        rf.set_gemm_rules([ok[0]] * 257)
    rf.set_gemm_rules([])
