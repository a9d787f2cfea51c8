"""Autotuner of the FP64 GEMM kernel choice (vector ALU vs matrix cores).

Times both kernels (t2s2_debug_gemm) for every shape bucket the solver's
dispatcher distinguishes -- M, N, K in buckets of ceil(log2) from 16 to 8192,
unbatched and batched -- on the current GPU, and writes
csrc/gemm_tune.h with the faster kernel per bucket.  Rebuild afterwards.

Usage:  python -m paper_2506_04732_amd.autotune [--out PATH] [--reps R]
"""
from __future__ import annotations

import argparse
import ctypes as C
import datetime
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
NB = 10
MAX_WORK = 2 ** 31      # M N K batch beyond this is not timed (filled from the large measured shapes)


def _time(lib, torch, variant, M, N, K, batch, reps, bufs):
    A, B, Cc = bufs
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)

    def call():
        rc = lib.t2s2_debug_gemm(variant, 0, 0, M, N, K, batch, 1.0, C.c_void_p(A.data_ptr()), K, M * K,
                                 C.c_void_p(B.data_ptr()), N, K * N, 0.0, C.c_void_p(Cc.data_ptr()), N, M * N, stream)
        if rc != 0:
            raise RuntimeError(lib.t2s2_last_error().decode())

    for _ in range(2):
        call()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        call()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps * 1e3  # us


def tune(reps=10, log=True):
    import torch
    from ._lib import lib
    L = lib()
    size = lambda b: 2 ** (b + 4)
    table = [[[[-1] * NB for _ in range(NB)] for _ in range(NB)] for _ in range(2)]
    meas = []
    for batched in (0, 1):
        batch = 64 if batched else 1
        for bm in range(NB):
            for bn in range(NB):
                for bk in range(NB):
                    M, N, K = size(bm), size(bn), size(bk)
                    if M * N * K * batch > MAX_WORK:
                        continue
                    A = torch.randn(batch * M * K, dtype=torch.float64, device="cuda")
                    B = torch.randn(batch * K * N, dtype=torch.float64, device="cuda")
                    Cc = torch.zeros(batch * M * N, dtype=torch.float64, device="cuda")
                    t0 = _time(L, torch, 0, M, N, K, batch, reps, (A, B, Cc))
                    t1 = _time(L, torch, 1, M, N, K, batch, reps, (A, B, Cc))
                    table[batched][bm][bn][bk] = 1 if t1 < t0 else 0
                    meas.append({"batched": batched, "M": M, "N": N, "K": K, "simt_us": t0, "mfma_us": t1})
            if log:
                print(f"autotune: batched={batched} M bucket {bm} done", file=sys.stderr, flush=True)
    # untimed (largest) shapes take the choice of the largest timed ones
    big = [m for m in meas if m["M"] * m["N"] * m["K"] * (64 if m["batched"] else 1) >= MAX_WORK // 8]
    fill = 1 if sum(m["mfma_us"] < m["simt_us"] for m in big) * 2 >= len(big) else 0
    for t in table:
        for a in t:
            for b in a:
                for k in range(NB):
                    if b[k] < 0:
                        b[k] = fill
    return table, meas


def write_header(table, path, source):
    rows = []
    for t in table:
        rows.append("{" + ",\n  ".join("{" + ", ".join("{" + ", ".join(str(v) for v in row) + "}" for row in a) + "}"
                                     for a in t) + "}")
    body = ",\n ".join(rows)
    with open(path, "w") as fh:
        fh.write(f"""// Kernel choice of the FP64 GEMM per shape bucket: 0 the vector-ALU kernel,
// 1 the matrix-core (MFMA) kernel.  Written by paper_2506_04732_amd/autotune.py
// from timings on the target GPU ({source}).
// Buckets: b(x) = clamp(ceil(log2 x) - 4, 0, 9) for M, N, K; batched = batch > 1.
#pragma once
namespace t2s2 {{
constexpr int kGemmTuneB = {NB};
constexpr const char* kGemmTuneSource = "{source}";
constexpr unsigned char kGemmTune[2][kGemmTuneB][kGemmTuneB][kGemmTuneB] = {{
 {body}}};
}}  // namespace t2s2
""")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(HERE, "csrc", "gemm_tune.h"))
    ap.add_argument("--json", default=None, help="also write the timings here")
    ap.add_argument("--reps", type=int, default=10)
    args = ap.parse_args()
    import torch
    table, meas = tune(args.reps)
    name = torch.cuda.get_device_name(0)
    source = f"{name}, {datetime.date.today().isoformat()}, {len(meas)} shapes timed"
    write_header(table, args.out, source)
    if args.json:
        with open(args.json, "w") as fh:
            json.dump({"source": source, "measurements": meas}, fh)
    print(f"wrote {args.out}: {source}", flush=True)


if __name__ == "__main__":
    main()
