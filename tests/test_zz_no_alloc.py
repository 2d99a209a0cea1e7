"""rf_sketch_apply_noalloc (the allocation-free entry point) against
rf_sketch_apply on the same inputs, through the C ABI: two calls in a row, the
second on a smaller input, then a request beyond the library's fixed scratch."""
import ctypes

import numpy as np
import pytest
import torch

import paper_2605_09755_amd as rf

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _call_noalloc(A, sketch, s, seed, out):
    p = rf.params(1, sketch, 0, s, seed)
    return rf.lib().rf_sketch_apply_noalloc(ctypes.byref(rf.matrix(A)), ctypes.byref(p), ctypes.c_void_p(out.data_ptr()),
                                            out.stride(0), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))


def _rand(m, n, seed):
    g = torch.Generator(device=DEV)
    g.manual_seed(seed)
    return torch.randn((m, n), generator=g, device=DEV)


def test_noalloc_matches_workspace_entry_point_twice():
    print("no-alloc: call 1 (3000 x 16384, sketch 2000, s 8), call 2 (500 x 3000, sketch 300, s 4)", flush=True)
    A1 = _rand(3000, 16384, 1)
    out1 = torch.full((3000, 2000), float("nan"), device=DEV)
    assert _call_noalloc(A1, 2000, 8, 42, out1) == rf.RF_OK
    ref1 = rf.rf_sketch_apply(A1, 2000, 8, 42)
    A2 = _rand(500, 3000, 2)
    out2 = torch.full((500, 300), float("nan"), device=DEV)
    assert _call_noalloc(A2, 300, 4, 7, out2) == rf.RF_OK
    ref2 = rf.rf_sketch_apply(A2, 300, 4, 7)
    torch.cuda.synchronize()
    # same kernels on the same inputs; the fixed-point passes are deterministic
    assert torch.equal(out1, ref1)
    assert torch.equal(out2, ref2)


def test_noalloc_generic_and_countsketch_paths():
    """s = 1 and s = 3 go through kernels whose float sums depend on atomic
    order: compared with the workspace entry point within FP32 rounding."""
    for (m, n, sk_, s) in [(300, 2000, 500, 1), (200, 1500, 90, 3)]:
        A = _rand(m, n, 3 + s)
        out = torch.empty((m, sk_), device=DEV)
        assert _call_noalloc(A, sk_, s, 5, out) == rf.RF_OK
        ref = rf.rf_sketch_apply(A, sk_, s, 5)
        torch.cuda.synchronize()
        tol = (n * s / sk_ + 8) * 4 * 2.0 ** -24 * (A.abs().max().item() * n * s / sk_)
        assert float((out - ref).abs().max()) <= tol


def test_noalloc_rejects_beyond_scratch():
    A = torch.zeros((4, 300000), device=DEV)
    out = torch.full((4, 16), 7.0, device=DEV)
    assert _call_noalloc(A, 16, 8, 0, out) == rf.RF_EUNSUPPORTED
    torch.cuda.synchronize()
    assert torch.all(out == 7.0)
