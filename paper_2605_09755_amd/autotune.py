"""Autotuner for the dense products: times every tile / split-K choice of the
library's MFMA GEMMs on the shapes the power method runs (the tall-skinny
products of Algorithm 1 and the Q^T A product of the randomised SVD) and writes
the fastest per shape bucket as a rule table (JSON) that rf_set_gemm_rules reads.

    python -m paper_2605_09755_amd.autotune [--out PATH] [--quick]

The BF16 rules also serve FP32-stored A rounded to BF16 on load; for the Q^T A
shapes, whose A is FP32 in the mixed form, the BF16 candidates are timed with
FP32 A (the other shapes' BF16 operands are BF16).
A rule covers the bucket obtained by rounding the tuned shape up to powers of
two; rules are ordered from the smallest bucket up, so the first match (the
library's rule) is the tightest bucket that contains a product.  The binding
loads paper_2605_09755_amd/tuning.json, when present, the first time the
library is opened.
"""
import argparse
import json
import os
import time

import torch

from . import lib, rf_test_gemm, set_gemm_rules

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_OUT = os.path.join(HERE, "tuning.json")

# (name, M, N, K, a_kc, b_kc): products of the workloads -- Q^T A as A^T Q, the
# power products At^T Q (TN over m) and At Z (NN over the sketch size), Y R^{-1}
SHAPES = [
    ("qta_65k_16k_k1000", 16384, 1000, 65536, 0, 0),
    ("qta_65k_32k_k2000", 32768, 2000, 65536, 0, 0),
    ("atq_65k_l2000_k1000", 2000, 1000, 65536, 0, 0),
    ("atq_65k_l4000_k2000", 4000, 2000, 65536, 0, 0),
    ("atz_65k_l2000_k1000", 65536, 1000, 2000, 1, 0),
    ("yr_65k_k1000", 65536, 1000, 1000, 1, 0),
    ("qta_8k_4k_k256", 4096, 256, 8192, 0, 0),
    ("atq_8k_l512_k256", 512, 256, 8192, 0, 0),
]
QUICK = [("tiny_tn", 1024, 256, 4096, 0, 0), ("tiny_nn", 4096, 256, 512, 1, 0)]

MAXI = (1 << 62)


def _pow2_up(x):
    p = 1
    while p < x:
        p <<= 1
    return p


def _operands(M, N, K, a_kc, b_kc, dtype, dev, a_dtype=None):
    g = torch.Generator(device=dev)
    g.manual_seed(M * 31 + N * 7 + K)
    A = torch.randn((M, K) if a_kc else (K, M), generator=g, device=dev).to(a_dtype or dtype)
    B = torch.randn((N, K) if b_kc else (K, N), generator=g, device=dev).to(dtype)
    return A, B


def _time(fn, reps):
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def candidates(dtype_code):
    tiles = (128, 256) if dtype_code == 2 else (128,)
    return [(t, s) for t in tiles for s in (1, 2, 4, 8, 16)]


def tune(shapes, reps=10, dev="cuda:0", log=print):
    lib()
    rules = []
    for dtype, code in ((torch.float32, 0), (torch.bfloat16, 2)):
        for name, M, N, K, a_kc, b_kc in shapes:
            a_dtype = torch.float32 if (code == 2 and name.startswith("qta_")) else None
            A, B = _operands(M, N, K, a_kc, b_kc, dtype, dev, a_dtype)
            res = {}
            for tile, split in candidates(code):
                set_gemm_rules([(code, tile, split, MAXI, MAXI, MAXI)])
                res["%d/%d" % (tile, split)] = _time(lambda: rf_test_gemm(A, B, M, N, K, a_kc, b_kc), reps)
            set_gemm_rules([])
            best = min(res, key=res.get)
            tile, split = (int(x) for x in best.split("/"))
            flops = 2.0 * M * N * K
            log("%-22s %s: best tile %d split %2d  %.3f ms (%.1f TFLOP/s)" % (
                name, "bf16" if code else "fp32", tile, split, res[best], flops / res[best] / 1e9))
            rules.append({"dtype": code, "tile": tile, "split": split, "max_m": _pow2_up(M), "max_n": _pow2_up(N),
                          "max_k": _pow2_up(K), "shape": [M, N, K], "layout": [a_kc, b_kc], "ms": res[best],
                          "candidates_ms": res})
            del A, B
    rules.sort(key=lambda r: (r["dtype"], r["max_m"] * r["max_n"] * r["max_k"]))
    return rules


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_OUT)
    ap.add_argument("--quick", action="store_true", help="two small shapes only")
    ap.add_argument("--reps", type=int, default=10)
    args = ap.parse_args()
    t0 = time.time()
    rules = tune(QUICK if args.quick else SHAPES, args.reps)
    doc = {"device": torch.cuda.get_device_name(0), "tuned_in_s": time.time() - t0, "rules": rules}
    with open(args.out, "w") as f:
        json.dump(doc, f, indent=1)
    print("wrote %d rules to %s" % (len(rules), args.out))


if __name__ == "__main__":
    main()
