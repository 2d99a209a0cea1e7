"""Thin Python binding of librf.so, the MI355X (gfx950) sketch-powered range finder.

Every function here only marshals arguments (torch tensors on the GPU ->
device pointers, sizes, the current HIP stream) and calls the C ABI declared in
include/rf.h; every step of the computation runs in the library's HIP kernels.
There is no CPU fallback: if librf.so is missing or cannot be loaded, the
functions raise.

Method: Chenakkod & Derezinski, "Accelerating Power Method with Fast Sketching
for Stronger Low-Rank Approximation" (arXiv 2605.09755) -- Algorithm 1
(range_finder), the randomised SVD finisher of Section 2 (svd), Algorithm 2
(lowrank) and Algorithm 3 (nystrom).
"""
import ctypes
import os
import struct

import torch

__all__ = [
    "RF_F32", "RF_BF16", "RF_FP8E4M3_B128", "RF_PREC_FP32", "RF_PREC_MIXED",
    "RF_OP_RANGE_FINDER", "RF_OP_SVD", "RF_OP_LOWRANK", "RF_OP_NYSTROM",
    "lib", "library_path", "rf_status_string", "rf_workspace_size", "rf_sketch_table", "rf_gaussian",
    "rf_sketch_apply", "rf_sketch_apply_left", "rf_range_finder", "rf_svd", "rf_lowrank", "rf_nystrom", "RFError",
    "BatchPlan", "rf_svd_batched", "set_gemm_rules", "load_tuning", "rf_range_finder_ex", "RF_FLAG_CLASSICAL",
    "rf_quantize_bf16", "rf_quantize_fp8_b128", "rf_sketch_apply_noalloc",
    "Csr", "rf_range_finder_csr", "rf_svd_csr", "rf_sketch_apply_csr",
]

RF_OK, RF_EINVAL, RF_EWORKSPACE, RF_EUNSUPPORTED, RF_EHIP = 0, 1, 2, 3, 4
RF_F32, RF_F64, RF_BF16, RF_FP8E4M3_B128 = 0, 1, 2, 3
RF_PREC_FP32, RF_PREC_MIXED = 0, 1
RF_OP_RANGE_FINDER, RF_OP_SVD, RF_OP_LOWRANK, RF_OP_NYSTROM = 0, 1, 2, 3
RF_FLAG_ORTH_ERR = 1
RF_FLAG_CLASSICAL = 2
# sketch family of Algorithm 1's S (Lemma 3.2), bits 2-3 of the flags
RF_SKETCH = {"sparse": 0, "rademacher": 1 << 2, "gaussian": 2 << 2, "srht": 3 << 2}

_HERE = os.path.dirname(os.path.abspath(__file__))
library_path = os.path.join(_HERE, "librf.so")


class RfMatrix(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("block_scales", ctypes.c_void_p), ("rows", ctypes.c_int64),
                ("cols", ctypes.c_int64), ("ld", ctypes.c_int64), ("dtype", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class RfParams(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("sketch", ctypes.c_int32), ("q", ctypes.c_int32),
                ("nnz_per_col", ctypes.c_int32), ("seed", ctypes.c_uint64), ("precision", ctypes.c_int32),
                ("flags", ctypes.c_uint32)]


class RfCsr(ctypes.Structure):
    _fields_ = [("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p), ("values", ctypes.c_void_p),
                ("rows", ctypes.c_int64), ("cols", ctypes.c_int64), ("nnz", ctypes.c_int64)]


INFO_BYTES = 24  # int32 x 4 + double


class RFError(RuntimeError):
    def __init__(self, fn, status):
        super().__init__("%s failed: %s (%d)" % (fn, _status_name(status), status))
        self.status = status


_lib = None


def lib():
    """Load librf.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(library_path):
            raise RuntimeError("librf.so not found at %s: build it with "
                               "`python -m paper_2605_09755_amd.build` (no CPU fallback exists)" % library_path)
        L = ctypes.CDLL(library_path)
        vp, i64, i32, u32, u64, sz = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32,
                                      ctypes.c_uint64, ctypes.c_size_t)
        M, P = ctypes.POINTER(RfMatrix), ctypes.POINTER(RfParams)
        L.rf_status_string.restype = ctypes.c_char_p
        L.rf_status_string.argtypes = [i32]
        L.rf_workspace_size.restype = sz
        L.rf_workspace_size.argtypes = [ctypes.c_int, M, P]
        L.rf_sketch_table.restype = i32
        L.rf_sketch_table.argtypes = [i64, i32, i32, u64, u32, u32, vp, vp]
        L.rf_gaussian.restype = i32
        L.rf_gaussian.argtypes = [i64, i64, u64, u32, u32, vp, vp]
        L.rf_sketch_apply_ws.restype = sz
        L.rf_sketch_apply_ws.argtypes = [M, P]
        L.rf_sketch_apply.restype = i32
        L.rf_sketch_apply.argtypes = [M, P, vp, i64, vp, sz, vp]
        L.rf_sketch_apply_noalloc.restype = i32
        L.rf_sketch_apply_noalloc.argtypes = [M, P, vp, i64, vp]
        L.rf_sketch_apply_left_ws.restype = sz
        L.rf_sketch_apply_left_ws.argtypes = [M, P]
        L.rf_sketch_apply_left.restype = i32
        L.rf_sketch_apply_left.argtypes = [M, P, vp, i64, vp, sz, vp]
        L.rf_range_finder.restype = i32
        L.rf_range_finder.argtypes = [M, P, vp, i64, vp, sz, vp, vp]
        L.rf_range_finder_ex.restype = i32
        L.rf_range_finder_ex.argtypes = [M, vp, vp, P, vp, i64, vp, sz, vp, vp]
        L.rf_svd.restype = i32
        L.rf_svd.argtypes = [M, P, vp, i64, vp, vp, i64, vp, sz, vp, vp]
        L.rf_lowrank.restype = i32
        L.rf_lowrank.argtypes = [M, P, vp, i64, vp, i64, vp, sz, vp, vp]
        L.rf_nystrom.restype = i32
        L.rf_nystrom.argtypes = [M, P, vp, i64, vp, i64, vp, i64, vp, sz, vp, vp]
        L.rf_set_gemm_rules.restype = i32
        L.rf_set_gemm_rules.argtypes = [vp, i32]
        L.rf_svd_batched_ws.restype = sz
        L.rf_svd_batched_ws.argtypes = [i32, vp, vp]
        L.rf_svd_batched_plan.restype = i32
        L.rf_svd_batched_plan.argtypes = [i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, sz, i32, vp,
                                          ctypes.POINTER(ctypes.c_void_p)]
        L.rf_svd_batched_run.restype = i32
        L.rf_svd_batched_run.argtypes = [vp, vp]
        L.rf_svd_batched_destroy.restype = None
        L.rf_svd_batched_destroy.argtypes = [vp]
        C = ctypes.POINTER(RfCsr)
        L.rf_workspace_size_csr.restype = sz
        L.rf_workspace_size_csr.argtypes = [ctypes.c_int, C, P]
        L.rf_range_finder_csr.restype = i32
        L.rf_range_finder_csr.argtypes = [C, P, vp, i64, vp, sz, vp, vp]
        L.rf_svd_csr.restype = i32
        L.rf_svd_csr.argtypes = [C, P, vp, i64, vp, vp, i64, vp, sz, vp, vp]
        L.rf_sketch_apply_csr.restype = i32
        L.rf_sketch_apply_csr.argtypes = [C, P, vp, i64, vp, sz, vp]
        L.rf_quantize_bf16.restype = i32
        L.rf_quantize_bf16.argtypes = [vp, i64, i64, i64, vp, i64, vp]
        L.rf_quantize_fp8_b128.restype = i32
        L.rf_quantize_fp8_b128.argtypes = [vp, i64, i64, i64, vp, i64, vp, vp]
        L.rf_test_gemm_ws.restype = sz
        L.rf_test_gemm_ws.argtypes = [i64, i64, i64]
        L.rf_test_gemm.restype = i32
        L.rf_test_gemm.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, i64, vp, i64, vp, i64, i64, i64,
                                   i64, ctypes.c_int, vp, vp]
        L.rf_test_gemm_fp8a.restype = i32
        L.rf_test_gemm_fp8a.argtypes = [vp, i64, vp, vp, i64, ctypes.c_int, vp, i64, i64, i64, i64, vp]
        L.rf_test_qf8_bytes.restype = sz
        L.rf_test_qf8_bytes.argtypes = [i64, i64, ctypes.c_int]
        L.rf_test_quant_q_fp8.restype = i32
        L.rf_test_quant_q_fp8.argtypes = [vp, i64, i64, i64, vp, vp, vp]
        L.rf_test_gemm_fp8_ws.restype = sz
        L.rf_test_gemm_fp8_ws.argtypes = [i64, i64, i64]
        L.rf_test_gemm_fp8.restype = i32
        L.rf_test_gemm_fp8.argtypes = [vp, i64, vp, vp, vp, vp, i64, i64, i64, i64, vp, sz, vp]
        L.rf_test_gram_ws.restype = sz
        L.rf_test_gram_ws.argtypes = [i64, i64, i64]
        L.rf_test_gram.restype = i32
        L.rf_test_gram.argtypes = [vp, vp, i64, i64, i64, ctypes.c_int, vp, vp, vp]
        L.rf_test_chol_ws.restype = sz
        L.rf_test_chol_ws.argtypes = [i64]
        L.rf_test_cholqr_factor.restype = i32
        L.rf_test_cholqr_factor.argtypes = [vp, i64, vp, vp, vp, vp]
        L.rf_test_eig_ws.restype = sz
        L.rf_test_eig_ws.argtypes = [i64]
        L.rf_test_eig.restype = i32
        L.rf_test_eig.argtypes = [vp, i64, ctypes.c_double, vp, vp, vp, vp, vp]
        _lib = L
        if os.path.exists(tuning_path):
            load_tuning(tuning_path)
    return _lib


class RfGemmRule(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int32), ("tile", ctypes.c_int32), ("split", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("max_m", ctypes.c_int64), ("max_n", ctypes.c_int64),
                ("max_k", ctypes.c_int64)]


tuning_path = os.path.join(_HERE, "tuning.json")


def set_gemm_rules(rules):
    """Install a GEMM tuning table: rules = [(dtype, tile, split, max_m, max_n, max_k), ...]
    (dtype 0 FP32 / 2 BF16); [] restores the built-in heuristics."""
    arr = (RfGemmRule * max(len(rules), 1))(*[RfGemmRule(int(d), int(t), int(sp), 0, int(a), int(b), int(c))
                                              for d, t, sp, a, b, c in rules])
    _check("rf_set_gemm_rules", lib().rf_set_gemm_rules(ctypes.cast(arr, ctypes.c_void_p), len(rules)))


def load_tuning(path):
    """Install the rule table written by paper_2605_09755_amd.autotune."""
    import json
    with open(path) as f:
        doc = json.load(f)
    set_gemm_rules([(r["dtype"], r["tile"], r["split"], r["max_m"], r["max_n"], r["max_k"]) for r in doc["rules"]])
    return doc


def _status_name(s):
    return {0: "ok", 1: "invalid argument", 2: "workspace too small", 3: "unsupported", 4: "HIP launch error"}.get(
        s, "unknown")


def rf_status_string(s):
    return lib().rf_status_string(int(s)).decode()


def _check(fn, st):
    if st != RF_OK:
        raise RFError(fn, st)


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def matrix(A, scales=None):
    """rf_matrix descriptor for a 2-D row-major device tensor (float32, bfloat16,
    or uint8 holding OCP e4m3 bytes together with 128x128 block `scales`).
    Every shape, dtype and device the kernels index by is checked here, before
    any launch: the library trusts these pointers."""
    if A.dim() != 2 or A.stride(1) != 1:
        raise ValueError("A must be a 2-D tensor with unit column stride")
    if A.device.type != "cuda":
        raise ValueError("A must be a device tensor (got %s)" % A.device)
    if A.dtype == torch.float32:
        dt = RF_F32
    elif A.dtype == torch.bfloat16:
        dt = RF_BF16
    elif A.dtype in (torch.uint8, getattr(torch, "float8_e4m3fn", torch.uint8)):
        dt = RF_FP8E4M3_B128
        if scales is None:
            raise ValueError("FP8 storage needs block scales")
        want = ((A.shape[0] + 127) // 128, (A.shape[1] + 127) // 128)
        if tuple(scales.shape) != want or scales.dtype != torch.float32 or not scales.is_contiguous() \
                or scales.device != A.device:
            raise ValueError("block scales must be a contiguous float32 tensor of shape %s on %s (got %s %s on %s)"
                             % (want, A.device, tuple(scales.shape), scales.dtype, scales.device))
    else:
        raise ValueError("unsupported dtype %s" % A.dtype)
    if dt != RF_FP8E4M3_B128 and scales is not None:
        raise ValueError("block scales are only taken with FP8 storage")
    return RfMatrix(A.data_ptr(), scales.data_ptr() if scales is not None else None, A.shape[0], A.shape[1],
                    max(A.stride(0), A.shape[1]), dt, 0)


def _check_out(name, t, shape, dtype, device):
    if (t is None or tuple(t.shape) != tuple(shape) or t.dtype != dtype or t.device != device
            or not t.is_contiguous()):
        raise ValueError("%s must be a contiguous %s tensor of shape %s on %s" % (name, dtype, tuple(shape), device))


def _check_ws(workspace, need, device):
    ws, nws = workspace
    if ws.dtype != torch.uint8 or ws.device != device or not ws.is_contiguous() or ws.numel() < nws or nws < need:
        raise ValueError("workspace must be a contiguous uint8 device tensor of at least %d bytes on %s" % (need, device))
    return ws, nws


def params(k, sketch, q=0, nnz_per_col=8, seed=0, precision=RF_PREC_FP32, flags=0):
    if isinstance(precision, str):
        precision = {"fp32": RF_PREC_FP32, "mixed": RF_PREC_MIXED}[precision]
    return RfParams(int(k), int(sketch), int(q), int(nnz_per_col), int(seed) & 0xFFFFFFFFFFFFFFFF, int(precision),
                    int(flags))


def rf_workspace_size(op, A, p, scales=None):
    return int(lib().rf_workspace_size(int(op), ctypes.byref(matrix(A, scales)), ctypes.byref(p)))


def _workspace(op, A, p, scales, given=None):
    n = rf_workspace_size(op, A, p, scales)
    if n == 0:
        raise RFError("rf_workspace_size", RF_EINVAL)
    if given is not None:
        return _check_ws(given, n, A.device)
    return torch.empty(n, dtype=torch.uint8, device=A.device), n


def _info(buf):
    raw = bytes(buf.cpu().numpy().tobytes())
    status, rank, retries, nonf, orth = struct.unpack("<iiiid", raw)
    return {"status": status, "rank_found": rank, "chol_retries": retries, "nonfinite": nonf, "orth_err": orth}


def rf_sketch_table(n, s, r1, seed, stream_id=0, b=0, device="cuda"):
    out = torch.empty((n, s), dtype=torch.int32, device=device)
    _check("rf_sketch_table", lib().rf_sketch_table(n, s, r1, seed, stream_id, b, _ptr(out), _stream(out.device)))
    return out


def rf_gaussian(rows, cols, seed, stream_id=1, b=0, device="cuda"):
    out = torch.empty((rows, cols), dtype=torch.float32, device=device)
    _check("rf_gaussian", lib().rf_gaussian(rows, cols, seed, stream_id, b, _ptr(out), _stream(out.device)))
    return out


def rf_sketch_apply(A, sketch, nnz_per_col, seed, scales=None, family="sparse", precision="fp32"):
    """A S (m x sketch) for the sketch family of Algorithm 1's S (the parity hook)."""
    p = params(1, sketch, 0, nnz_per_col, seed, precision, RF_SKETCH[family])
    nws = int(lib().rf_sketch_apply_ws(ctypes.byref(matrix(A, scales)), ctypes.byref(p)))
    if nws == 0:
        raise RFError("rf_sketch_apply_ws", RF_EINVAL)
    ws = torch.empty(nws, dtype=torch.uint8, device=A.device)
    out = torch.empty((A.shape[0], sketch), dtype=torch.float32, device=A.device)
    _check("rf_sketch_apply", lib().rf_sketch_apply(ctypes.byref(matrix(A, scales)), ctypes.byref(p), _ptr(out),
                                                    sketch, _ptr(ws), nws, _stream(A.device)))
    return out


def rf_sketch_apply_noalloc(A, sketch, nnz_per_col, seed, scales=None, out=None):
    """A S as rf_sketch_apply computes it, through the library's allocation-free
    entry point (no workspace; calls on one GPU must not overlap)."""
    p = params(1, sketch, 0, nnz_per_col, seed)
    if out is None:
        out = torch.empty((A.shape[0], sketch), dtype=torch.float32, device=A.device)
    else:
        _check_out("out", out, (A.shape[0], sketch), torch.float32, A.device)
    _check("rf_sketch_apply_noalloc", lib().rf_sketch_apply_noalloc(ctypes.byref(matrix(A, scales)), ctypes.byref(p),
                                                                    _ptr(out), sketch, _stream(A.device)))
    return out


def rf_sketch_apply_left(A, sketch, nnz_per_col, seed, scales=None):
    """S2^T A (sketch x n) with the stream-2 sketch of rf_lowrank."""
    p = params(1, sketch, 0, nnz_per_col, seed)
    nws = int(lib().rf_sketch_apply_left_ws(ctypes.byref(matrix(A, scales)), ctypes.byref(p)))
    if nws == 0:
        raise RFError("rf_sketch_apply_left_ws", RF_EINVAL)
    ws = torch.empty(nws, dtype=torch.uint8, device=A.device)
    out = torch.empty((sketch, A.shape[1]), dtype=torch.float32, device=A.device)
    _check("rf_sketch_apply_left", lib().rf_sketch_apply_left(ctypes.byref(matrix(A, scales)), ctypes.byref(p),
                                                              _ptr(out), A.shape[1], _ptr(ws), nws,
                                                              _stream(A.device)))
    return out


def _flags(orth_err=False, classical=False, family="sparse"):
    return (RF_FLAG_ORTH_ERR if orth_err else 0) | (RF_FLAG_CLASSICAL if classical else 0) | RF_SKETCH[family]


def rf_range_finder(A, k, sketch, q=0, nnz_per_col=8, seed=0, precision="fp32", scales=None, orth_err=False,
                    workspace=None, classical=False, family="sparse"):
    """Algorithm 1.  classical=True runs S = I (Omega n x k): the baseline of Section 2.
    family: "sparse" (Lemma 3.2 item 2), "rademacher" / "gaussian" (item 1), "srht" (item 3)."""
    p = params(k, sketch, q, nnz_per_col, seed, precision, _flags(orth_err, classical, family))
    ws, nws = _workspace(RF_OP_RANGE_FINDER, A, p, scales, workspace)
    Q = torch.empty((A.shape[0], k), dtype=torch.float32, device=A.device)
    info = torch.zeros(INFO_BYTES, dtype=torch.uint8, device=A.device)
    _check("rf_range_finder", lib().rf_range_finder(ctypes.byref(matrix(A, scales)), ctypes.byref(p), _ptr(Q), k,
                                                    _ptr(ws), nws, _ptr(info), _stream(A.device)))
    return Q, info


def rf_range_finder_ex(A, k, sketch, S_table=None, Omega=None, q=0, nnz_per_col=8, seed=0, precision="fp32",
                       scales=None, orth_err=False, classical=False, workspace=None, family="sparse"):
    """Algorithm 1 with a caller-given sketch table (int32 n x s, the layout of
    rf_sketch_table) and/or Omega (float32 rows x k; rows = sketch, or n when
    classical).  None draws that input from the seed."""
    p = params(k, sketch, q, nnz_per_col, seed, precision, _flags(orth_err, classical, family))
    ws, nws = _workspace(RF_OP_RANGE_FINDER, A, p, scales, workspace)
    n = A.shape[1]
    if S_table is not None:
        _check_out("S_table", S_table, (n, nnz_per_col), torch.int32, A.device)
    if Omega is not None:
        _check_out("Omega", Omega, (n if classical else sketch, k), torch.float32, A.device)
    Q = torch.empty((A.shape[0], k), dtype=torch.float32, device=A.device)
    info = torch.zeros(INFO_BYTES, dtype=torch.uint8, device=A.device)
    _check("rf_range_finder_ex", lib().rf_range_finder_ex(ctypes.byref(matrix(A, scales)), _ptr(S_table),
                                                          _ptr(Omega), ctypes.byref(p), _ptr(Q), k, _ptr(ws), nws,
                                                          _ptr(info), _stream(A.device)))
    return Q, info


def rf_svd(A, k, sketch, q=0, nnz_per_col=8, seed=0, precision="fp32", scales=None, orth_err=False,
           workspace=None, out=None, classical=False, family="sparse"):
    p = params(k, sketch, q, nnz_per_col, seed, precision, _flags(orth_err, classical, family))
    ws, nws = _workspace(RF_OP_SVD, A, p, scales, workspace)
    m, n = A.shape
    if out is None:
        U = torch.empty((m, k), dtype=torch.float32, device=A.device)
        sig = torch.empty(k, dtype=torch.float64, device=A.device)
        Vt = torch.empty((k, n), dtype=torch.float32, device=A.device)
        info = torch.zeros(INFO_BYTES, dtype=torch.uint8, device=A.device)
    else:
        U, sig, Vt, info = out
        _check_out("U", U, (m, k), torch.float32, A.device)
        _check_out("sigma", sig, (k,), torch.float64, A.device)
        _check_out("Vt", Vt, (k, n), torch.float32, A.device)
        _check_out("info", info, (INFO_BYTES,), torch.uint8, A.device)
    _check("rf_svd", lib().rf_svd(ctypes.byref(matrix(A, scales)), ctypes.byref(p), _ptr(U), k, _ptr(sig), _ptr(Vt),
                                  n, _ptr(ws), nws, _ptr(info), _stream(A.device)))
    return U, sig, Vt, info


def rf_lowrank(A, k, sketch, q=0, nnz_per_col=8, seed=0, precision="fp32", scales=None, workspace=None,
               classical=False, family="sparse"):
    """Algorithm 2; classical=True runs it with S1 = I (S2 still has `sketch` rows)."""
    p = params(k, sketch, q, nnz_per_col, seed, precision, _flags(False, classical, family))
    ws, nws = _workspace(RF_OP_LOWRANK, A, p, scales, workspace)
    m, n = A.shape
    Y = torch.empty((m, k), dtype=torch.float32, device=A.device)
    X = torch.empty((k, n), dtype=torch.float32, device=A.device)
    info = torch.zeros(INFO_BYTES, dtype=torch.uint8, device=A.device)
    _check("rf_lowrank", lib().rf_lowrank(ctypes.byref(matrix(A, scales)), ctypes.byref(p), _ptr(Y), k, _ptr(X), n,
                                          _ptr(ws), nws, _ptr(info), _stream(A.device)))
    return Y, X, info


def rf_nystrom(A, k, sketch, q=0, nnz_per_col=8, seed=0, precision="fp32", scales=None, want_F=True,
               workspace=None):
    p = params(k, sketch, q, nnz_per_col, seed, precision)
    ws, nws = _workspace(RF_OP_NYSTROM, A, p, scales, workspace)
    n = A.shape[0]
    C = torch.empty((n, k), dtype=torch.float32, device=A.device)
    W = torch.empty((k, k), dtype=torch.float64, device=A.device)
    F = torch.empty((n, k), dtype=torch.float32, device=A.device) if want_F else None
    info = torch.zeros(INFO_BYTES, dtype=torch.uint8, device=A.device)
    _check("rf_nystrom", lib().rf_nystrom(ctypes.byref(matrix(A, scales)), ctypes.byref(p), _ptr(C), k, _ptr(W), k,
                                          _ptr(F), k, _ptr(ws), nws, _ptr(info), _stream(A.device)))
    return C, W, F, info


class Csr:
    """A sparse m x n matrix in CSR form on the device: row_ptr (int64, m + 1),
    col_idx (int32, nnz), values (float32, nnz)."""

    def __init__(self, row_ptr, col_idx, values, shape):
        m, n = int(shape[0]), int(shape[1])
        dev = values.device
        if row_ptr.dtype != torch.int64 or row_ptr.numel() != m + 1 or not row_ptr.is_contiguous():
            raise ValueError("row_ptr must be a contiguous int64 tensor of m + 1 entries")
        if col_idx.dtype != torch.int32 or values.dtype != torch.float32 or col_idx.numel() != values.numel():
            raise ValueError("col_idx (int32) and values (float32) must have nnz entries each")
        if not (col_idx.is_contiguous() and values.is_contiguous()) or dev.type != "cuda" or \
                row_ptr.device != dev or col_idx.device != dev:
            raise ValueError("CSR arrays must be contiguous device tensors on one device")
        self.row_ptr, self.col_idx, self.values, self.shape, self.device = row_ptr, col_idx, values, (m, n), dev
        self.nnz = values.numel()

    @classmethod
    def from_scipy(cls, S, device="cuda"):
        S = S.tocsr()
        S.sort_indices()
        return cls(torch.from_numpy(S.indptr.astype("int64")).to(device),
                   torch.from_numpy(S.indices.astype("int32")).to(device),
                   torch.from_numpy(S.data.astype("float32")).to(device), S.shape)

    def desc(self):
        return RfCsr(self.row_ptr.data_ptr(), self.col_idx.data_ptr(), self.values.data_ptr(), self.shape[0],
                     self.shape[1], self.nnz)


def _csr_ws(op, A, p):
    n = int(lib().rf_workspace_size_csr(int(op), ctypes.byref(A.desc()), ctypes.byref(p)))
    if n == 0:
        raise RFError("rf_workspace_size_csr", RF_EINVAL)
    return torch.empty(n, dtype=torch.uint8, device=A.device), n


def rf_range_finder_csr(A, k, sketch, q=0, nnz_per_col=8, seed=0, precision="fp32", orth_err=False):
    """Algorithm 1 on a sparse A (Csr)."""
    p = params(k, sketch, q, nnz_per_col, seed, precision, _flags(orth_err))
    ws, nws = _csr_ws(RF_OP_RANGE_FINDER, A, p)
    Q = torch.empty((A.shape[0], k), dtype=torch.float32, device=A.device)
    info = torch.zeros(INFO_BYTES, dtype=torch.uint8, device=A.device)
    _check("rf_range_finder_csr", lib().rf_range_finder_csr(ctypes.byref(A.desc()), ctypes.byref(p), _ptr(Q), k,
                                                            _ptr(ws), nws, _ptr(info), _stream(A.device)))
    return Q, info


def rf_svd_csr(A, k, sketch, q=0, nnz_per_col=8, seed=0, precision="fp32", orth_err=False):
    """Randomised SVD on top of Algorithm 1 for a sparse A (Csr)."""
    p = params(k, sketch, q, nnz_per_col, seed, precision, _flags(orth_err))
    ws, nws = _csr_ws(RF_OP_SVD, A, p)
    m, n = A.shape
    U = torch.empty((m, k), dtype=torch.float32, device=A.device)
    sig = torch.empty(k, dtype=torch.float64, device=A.device)
    Vt = torch.empty((k, n), dtype=torch.float32, device=A.device)
    info = torch.zeros(INFO_BYTES, dtype=torch.uint8, device=A.device)
    _check("rf_svd_csr", lib().rf_svd_csr(ctypes.byref(A.desc()), ctypes.byref(p), _ptr(U), k, _ptr(sig), _ptr(Vt),
                                          n, _ptr(ws), nws, _ptr(info), _stream(A.device)))
    return U, sig, Vt, info


def rf_sketch_apply_csr(A, sketch, nnz_per_col, seed):
    """A S for a sparse A (Csr), the sketch of rf_sketch_apply."""
    p = params(1, sketch, 0, nnz_per_col, seed)
    nws = 4 * A.shape[1] * nnz_per_col + 1024
    ws = torch.empty(nws, dtype=torch.uint8, device=A.device)
    out = torch.empty((A.shape[0], sketch), dtype=torch.float32, device=A.device)
    _check("rf_sketch_apply_csr", lib().rf_sketch_apply_csr(ctypes.byref(A.desc()), ctypes.byref(p), _ptr(out),
                                                            sketch, _ptr(ws), nws, _stream(A.device)))
    return out


def _check_f32_2d(name, A):
    if A.dim() != 2 or A.stride(1) != 1 or A.dtype != torch.float32 or A.device.type != "cuda":
        raise ValueError("%s must be a 2-D float32 device tensor with unit column stride" % name)


def rf_quantize_bf16(A):
    """A (FP32, device) rounded to BF16, nearest-even (the library's kernel)."""
    _check_f32_2d("A", A)
    out = torch.empty(A.shape, dtype=torch.bfloat16, device=A.device)
    _check("rf_quantize_bf16", lib().rf_quantize_bf16(_ptr(A), A.shape[0], A.shape[1], A.stride(0), _ptr(out),
                                                      A.shape[1], _stream(A.device)))
    return out


def rf_quantize_fp8_b128(A):
    """A (FP32, device) -> (uint8 OCP e4m3 codes, FP32 128 x 128 block scales)."""
    _check_f32_2d("A", A)
    m, n = A.shape
    codes = torch.empty((m, n), dtype=torch.uint8, device=A.device)
    scales = torch.empty(((m + 127) // 128, (n + 127) // 128), dtype=torch.float32, device=A.device)
    _check("rf_quantize_fp8_b128", lib().rf_quantize_fp8_b128(_ptr(A), m, n, A.stride(0), _ptr(codes), n,
                                                              _ptr(scales), _stream(A.device)))
    return codes, scales


class BatchPlan:
    """A planned batched randomised SVD over a list of FP32 device matrices
    (rf_svd_batched_plan).  Holds the workspace and the outputs; run() enqueues
    one batched factorisation on the current stream (a hipGraph launch when
    use_graph), results in .U, .sigma, .Vt (lists) and .info (count x 24 bytes)."""

    def __init__(self, As, ks, sketches, q=2, nnz_per_col=4, seeds=0, precision="mixed", use_graph=True):
        count = len(As)
        if isinstance(seeds, int):
            seeds = [seeds] * count
        dev = As[0].device
        mats = (RfMatrix * count)(*[matrix(A) for A in As])
        prms = (RfParams * count)(*[params(k, l, q, nnz_per_col, sd, precision) for k, l, sd in zip(ks, sketches, seeds)])
        self.As = list(As)
        self.U = [torch.empty((A.shape[0], k), dtype=torch.float32, device=dev) for A, k in zip(As, ks)]
        self.sigma = [torch.empty(k, dtype=torch.float64, device=dev) for k in ks]
        self.Vt = [torch.empty((k, A.shape[1]), dtype=torch.float32, device=dev) for A, k in zip(As, ks)]
        self.info = torch.zeros((count, INFO_BYTES), dtype=torch.uint8, device=dev)
        nws = int(lib().rf_svd_batched_ws(count, ctypes.cast(mats, ctypes.c_void_p), ctypes.cast(prms, ctypes.c_void_p)))
        self.ws = torch.empty(max(nws, 1), dtype=torch.uint8, device=dev)
        Up = (ctypes.c_void_p * count)(*[_ptr(t) for t in self.U])
        ldu = (ctypes.c_int64 * count)(*[t.stride(0) for t in self.U])
        Sp = (ctypes.c_void_p * count)(*[_ptr(t) for t in self.sigma])
        Vp = (ctypes.c_void_p * count)(*[_ptr(t) for t in self.Vt])
        ldv = (ctypes.c_int64 * count)(*[t.stride(0) for t in self.Vt])
        h = ctypes.c_void_p()
        _check("rf_svd_batched_plan", lib().rf_svd_batched_plan(
            count, ctypes.cast(mats, ctypes.c_void_p), ctypes.cast(prms, ctypes.c_void_p),
            ctypes.cast(Up, ctypes.c_void_p), ctypes.cast(ldu, ctypes.c_void_p), ctypes.cast(Sp, ctypes.c_void_p),
            ctypes.cast(Vp, ctypes.c_void_p), ctypes.cast(ldv, ctypes.c_void_p), _ptr(self.info),
            _ptr(self.ws) if nws else ctypes.c_void_p(0), nws,
            1 if use_graph else 0, _stream(dev), ctypes.byref(h)))
        self._h = h
        self.device = dev

    def run(self):
        _check("rf_svd_batched_run", lib().rf_svd_batched_run(self._h, _stream(self.device)))
        return self

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().rf_svd_batched_destroy(h)
            self._h = None


def rf_svd_batched(As, ks, sketches, q=2, nnz_per_col=4, seeds=0, precision="mixed", use_graph=False):
    """One batched randomised SVD (plan + run); returns the BatchPlan with the outputs."""
    return BatchPlan(As, ks, sketches, q, nnz_per_col, seeds, precision, use_graph).run()


# ---- kernel-level parity hooks -------------------------------------------------------
def rf_test_gemm(A, B, M, N, K, a_kc, b_kc, b_upper=False, split=True):
    """C = op(A) op(B) (FP32 out) with the library's MFMA GEMM.  A, B: float32 or
    bfloat16 device tensors in the layouts described in include/rf.h."""
    if A.dtype == torch.float32 and B.dtype == torch.bfloat16:
        dtype = 4                      # A rounded to BF16 as it is loaded
    elif A.dtype == torch.float32:
        dtype = 0
    else:
        dtype = 2
    lda = A.stride(0)
    ldb = B.stride(0)
    C = torch.empty((M, N), dtype=torch.float32, device=A.device)
    ws = torch.empty(int(lib().rf_test_gemm_ws(M, N, K)), dtype=torch.uint8, device=A.device) if split else None
    _check("rf_test_gemm", lib().rf_test_gemm(dtype, int(a_kc), int(b_kc), _ptr(A), lda, _ptr(B), ldb, _ptr(C), N, M,
                                              N, K, int(b_upper), _ptr(ws), _stream(A.device)))
    return C


def rf_test_gemm_fp8a(A8, scales, B, M, N, K, b_kc):
    """C = op(A) op(B): A8 (K x M uint8 e4m3 codes, 128 x 128 block scales), B bfloat16."""
    C = torch.empty((M, N), dtype=torch.float32, device=A8.device)
    _check("rf_test_gemm_fp8a", lib().rf_test_gemm_fp8a(_ptr(A8), A8.stride(0), _ptr(scales), _ptr(B), B.stride(0),
                                                        int(b_kc), _ptr(C), N, M, N, K, _stream(A8.device)))
    return C


def rf_test_quant_q_fp8(Q):
    """FP8 operand form of Q (m x k FP32): (codes, scales) uint8 device buffers in
    the layout of include/rf.h (rf_test_quant_q_fp8)."""
    m, k = Q.shape
    if Q.dtype != torch.float32 or Q.stride(1) != 1:
        raise ValueError("Q must be float32 with unit column stride")
    codes = torch.empty(int(lib().rf_test_qf8_bytes(m, k, 0)), dtype=torch.uint8, device=Q.device)
    scales = torch.empty(int(lib().rf_test_qf8_bytes(m, k, 1)), dtype=torch.uint8, device=Q.device)
    _check("rf_test_quant_q_fp8", lib().rf_test_quant_q_fp8(_ptr(Q), m, k, Q.stride(0), _ptr(codes), _ptr(scales),
                                                            _stream(Q.device)))
    return codes, scales


def rf_test_gemm_fp8(A8, scales, Q, M, N, K, qform=None, split=True):
    """C = op(A) Q on FP8 MFMA: A8 (K x M uint8 e4m3 codes, 128 x 128 block scales),
    Q (K x N FP32) taken to its FP8 operand form first (or qform = (codes, scales)
    from rf_test_quant_q_fp8(Q) to skip that step)."""
    if A8.dtype != torch.uint8 or A8.stride(1) != 1 or A8.shape != (K, M):
        raise ValueError("A8 must be K x M uint8 with unit column stride")
    if scales.shape != ((K + 127) // 128, (M + 127) // 128) or scales.dtype != torch.float32 \
            or not scales.is_contiguous():
        raise ValueError("scales must be contiguous float32 ceil(K/128) x ceil(M/128)")
    if qform is None:
        if Q.shape != (K, N):
            raise ValueError("Q must be K x N")
        qform = rf_test_quant_q_fp8(Q)
    qc, qs = qform
    if qc.numel() < int(lib().rf_test_qf8_bytes(K, N, 0)) or qs.numel() < int(lib().rf_test_qf8_bytes(K, N, 1)):
        raise ValueError("Q operand form too small for K x N")
    C = torch.empty((M, N), dtype=torch.float32, device=A8.device)
    nws = int(lib().rf_test_gemm_fp8_ws(M, N, K)) if split else 0
    ws = torch.empty(nws, dtype=torch.uint8, device=A8.device) if split else None
    _check("rf_test_gemm_fp8", lib().rf_test_gemm_fp8(_ptr(A8), A8.stride(0), _ptr(scales), _ptr(qc), _ptr(qs),
                                                      _ptr(C), N, M, N, K, _ptr(ws), nws, _stream(A8.device)))
    return C


def rf_test_gram(X, Y=None, sym=False, split=True):
    Y = X if Y is None else Y
    K, M = X.shape
    N = Y.shape[1]
    C = torch.zeros((M, N), dtype=torch.float64, device=X.device)
    ws = torch.empty(int(lib().rf_test_gram_ws(K, M, N)), dtype=torch.uint8, device=X.device) if split else None
    _check("rf_test_gram", lib().rf_test_gram(_ptr(X), _ptr(Y), K, M, N, int(sym), _ptr(C), _ptr(ws),
                                              _stream(X.device)))
    return C


def rf_test_cholqr_factor(G):
    N = G.shape[0]
    G = G.clone().contiguous()
    Rinv = torch.zeros_like(G)
    counters = torch.zeros(16, dtype=torch.int32, device=G.device)
    ws = torch.empty(int(lib().rf_test_chol_ws(N)), dtype=torch.uint8, device=G.device)
    _check("rf_test_cholqr_factor", lib().rf_test_cholqr_factor(_ptr(G), N, _ptr(Rinv), _ptr(counters), _ptr(ws),
                                                                _stream(G.device)))
    return G, Rinv, counters


def rf_test_eig(G, trace=False, tol=1e-12):
    N = G.shape[0]
    G = G.contiguous()
    lam = torch.empty(N, dtype=torch.float64, device=G.device)
    V = torch.empty((N, N), dtype=torch.float64, device=G.device)
    tr = torch.zeros(32, dtype=torch.float64, device=G.device) if trace else None
    ws = torch.empty(int(lib().rf_test_eig_ws(N)), dtype=torch.uint8, device=G.device)
    _check("rf_test_eig", lib().rf_test_eig(_ptr(G), N, float(tol), _ptr(lam), _ptr(V), _ptr(tr), _ptr(ws),
                                            _stream(G.device)))
    return (lam, V, tr) if trace else (lam, V)


def info_dict(info):
    """Decode an rf_info device buffer (synchronises)."""
    return _info(info)
