"""Sweep of the compiled GEMM tile shapes and K splits on the GPU.

Times ``spca_gemm_nt_f32_shape`` for every (shape, splits) on the products
of the AM iteration at the given sizes, with HIP events on the launch
stream, and reports TFLOP/s next to the library's own choice
(``spca_gemm_nt_f32_plan``, FP32 model).  --dtype bf16 sweeps the BF16
kernels on the same shapes.  Its output is what the efficiency table of the
tile-shape model in gemm_f32.hip is calibrated from.

    python -m paper_1212_4137_amd.tune_gemm [--products 1024x10000x1000,...]
"""
import argparse
import json
import sys

SHAPES = ["128x128", "128x160", "128x96", "128x64", "64x128", "32x128", "64x256", "256x128",
          "256x256"]


def time_launch(fn, reps, warmup=3):
    import torch

    for _ in range(warmup):
        fn()
    st = torch.cuda.current_stream()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(st)
    for _ in range(reps):
        fn()
    b.record(st)
    b.synchronize()
    return a.elapsed_time(b) / reps


def sweep(M, N, K, max_splits, reps, dtype="fp32"):
    import torch

    import paper_1212_4137_amd as spca

    g = torch.Generator(device="cuda").manual_seed(M * 7 + N * 3 + K)
    ldk = (K + 7) // 8 * 8
    P = torch.randn((M, ldk), device="cuda", generator=g)[:, :K]
    Q = torch.randn((N, ldk), device="cuda", generator=g)[:, :K]
    if dtype == "bf16":
        P, Q = P.bfloat16(), Q.bfloat16()
    flops = 2.0 * M * N * K
    chosen = spca.gemm_plan(M, N, K, max_splits)
    rows = []
    for shape in range(len(SHAPES)):
        sp = 1
        while sp <= max_splits:
            if sp > 1 and (K + 31) // 32 // sp < 8:
                break
            ms = time_launch(lambda: spca.gemm_nt_shape(P, Q, shape, sp), reps)
            rows.append({"shape": SHAPES[shape], "splits": sp, "ms": round(ms, 4),
                         "tflops": round(flops / ms / 1e9, 2),
                         "chosen": (shape, sp) == chosen})
            sp *= 2
    rows.sort(key=lambda r: r["ms"])
    return {"M": M, "N": N, "K": K, "dtype": dtype, "chosen": {"shape": SHAPES[chosen[0]],
                                                "splits": chosen[1]},
            "results": rows}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--products", default="1024x10000x1000:1,1024x1000x10000:16")
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--dtype", default="fp32", choices=["fp32", "bf16"])
    args = ap.parse_args()
    out = []
    for item in args.products.split(","):
        dims, _, ms = item.partition(":")
        M, N, K = (int(v) for v in dims.split("x"))
        res = sweep(M, N, K, int(ms or 1), args.reps, args.dtype)
        out.append(res)
        print(json.dumps(res), flush=True)
    return out


if __name__ == "__main__":
    sys.exit(0 if main() else 1)
