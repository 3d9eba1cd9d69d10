"""Benchmark of the KRP sketch / randomized STHOSVD hot path on one MI355X.

A step is one mixed-precision randomized STHOSVD with Khatri-Rao products
(Algorithm 8 plus the fp64 truncation of the core) of a 512 x 512 x 512 fp32
low-multilinear-rank tensor (rank 32, ell = 40 per mode, 1e-3 noise): for
every mode the KRP sketch of the current core, its fp64 CholeskyQR2 and the
TTM, all in one captured HIP graph.  The tensor is resident in HBM before
timing starts.

Printed JSON line (one, on stdout):
  value        algorithmic bytes of the step / step time (GB/s)
  roofline     the single-mode KRP sketch of X (the dominant launch) timed
               with HIP events on its stream, against 8 TB/s
  cpu_baseline the fp64 oracle on the host cores on a sample of the step
  plus the fp64 GPU form of the same STHOSVD, the Tucker errors of both and
  the sketch GB/s of every mode.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "KRP-sketch tensor GB/s (% HBM peak); STHOSVD time mixed vs FP64 at equal error"
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--prec", default="bf16x3", choices=["fp32", "bf16x3", "bf16"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true", help="skip the fp64 GPU form")
    ap.add_argument("--dims", default="512,512,512")
    ap.add_argument("--rank", type=int, default=32)
    ap.add_argument("--oversample", type=int, default=8)
    return ap.parse_args()


def sthosvd_bytes(dims, ells, elem):
    """Algorithmic HBM bytes of one STHOSVD sweep (natural order, no truncation).

    Per mode: the sketch reads the current core once and writes Y (n_i x ell_i);
    the TTM reads the current core and writes the next one."""
    cur = list(dims)
    total = 0
    for i, l in enumerate(ells):
        size = math.prod(cur)
        total += size * elem + cur[i] * l * elem       # sketch
        nxt = size // cur[i] * l
        total += size * elem + nxt * elem               # TTM
        cur[i] = l
    return total


def time_calls(fn, steps, warmup, stream):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for a, b in ev:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    ms = [a.elapsed_time(b) for a, b in ev]
    return sum(ms) / len(ms), wall * 1e3


def cpu_baseline(x_np, ranks, p, sample_modes=1):
    """The fp64 oracle (explicit KRPs and unfoldings) on the host cores.

    Sample: the first `sample_modes` mode steps of Algorithm 8 (sketch, QR,
    TTM) on the full tensor; the rate is algorithmic bytes of those steps per
    second, in the same unit as the GPU value."""
    import numpy as np
    from oracle import rng as orng
    from oracle import tucker as ot
    from oracle.linalg import qr_pos
    from oracle.tensor import mttkrp, ttm

    g = np.asarray(x_np, dtype=np.float64)
    dims = list(g.shape)
    ells = [r + p for r in ranks]
    nbytes = 0
    t0 = time.perf_counter()
    for i in range(sample_modes):
        f = ot.sketch_factors(2507, 0, i, g.shape, ells[i], i)
        y = mttkrp(g, f, i)
        q = qr_pos(y)[0]
        size = g.size
        g = ttm(g, q.T, i)
        nbytes += size * 4 + dims[i] * ells[i] * 4 + size * 4 + g.size * 4
    dt = time.perf_counter() - t0
    threads = os.environ.get("OPENBLAS_NUM_THREADS") or os.environ.get("OMP_NUM_THREADS")
    cores = int(threads) if threads else (os.cpu_count() or 1)
    return dict(value=nbytes / dt / 1e9, unit="GB/s", cores=cores, kind="oracle",
                sample=f"Algorithm 8 mode-{sample_modes} prefix (explicit-KRP sketch, LAPACK QR, "
                       f"unfolding TTM) of the full {'x'.join(map(str, dims))} tensor in fp64: "
                       f"{nbytes / 1e9:.2f} GB algorithmic in {dt:.2f} s")


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; multi-GPU sharding is "
                                   "described in DESIGN.md but not built", "n_gpus": args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2507_23207_amd as krp
    from synth import WORKLOADS, low_rank_tensor_torch

    torch.cuda.set_device(0)
    dims = [int(v) for v in args.dims.split(",")]
    ranks = [args.rank] * len(dims)
    p = args.oversample
    ells = [r + p for r in ranks]
    w = WORKLOADS["sthosvd_512x3_fp32"]
    x = low_rank_tensor_torch(dims, ranks, decay=w["decay"], noise=w["noise"], seed=w["seed"],
                              dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()

    # --- the step: mixed-precision STHOSVD with truncation -------------------
    def step():
        return krp.sthosvd(x, ranks, p, prec=args.prec, truncate=True)

    step_ms, step_wall_ms = time_calls(step, args.steps, args.warmup, stream)
    core, qs, err_mixed = krp.sthosvd(x, ranks, p, prec=args.prec, truncate=True, rel_err=True)
    step_bytes = sthosvd_bytes(dims, ells, 4)

    # --- dominant launch: KRP sketch of X for each mode ----------------------
    sketch = {}
    for m in range(len(dims)):
        fn = lambda m=m: krp.sketch(x, [m], [ells[m]], prec=args.prec)
        ms, _ = time_calls(fn, max(5, args.steps), 2, stream)
        b = x.numel() * 4 + dims[m] * ells[m] * 4
        sketch[m] = dict(ms=ms, gbps=b / ms / 1e6, bytes=b)

    # --- fp64 GPU form of the same STHOSVD ------------------------------------
    fp64 = None
    if not args.no_fp64:
        x64 = x.to(torch.float64)  # converted once, outside the timed region
        def step64():
            return krp.sthosvd(x64, ranks, p, prec="fp64", truncate=True)
        ms64, _ = time_calls(step64, max(3, args.steps // 2), 2, stream)
        _, _, err64 = krp.sthosvd(x64, ranks, p, prec="fp64", truncate=True, rel_err=True)
        fp64 = dict(ms=ms64, tucker_rel_err=err64, speedup_mixed=ms64 / step_ms,
                    err_ratio=err_mixed / err64)
        del x64

    cpu = None
    if not args.no_cpu_baseline:
        x_np = x.permute(*reversed(range(len(dims)))).contiguous().cpu().numpy()
        x_np = np.ascontiguousarray(x_np).transpose(*reversed(range(len(dims))))
        cpu = cpu_baseline(x_np, ranks, p, sample_modes=1)

    dom = sketch[0]
    out = {
        "metric": METRIC,
        "value": step_bytes / step_ms / 1e6,
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.prec,
        "data": "synthetic",
        "config": {"workload": "randomized STHOSVD with KRPs (Algorithm 8) + fp64 core truncation, "
                               f"{'x'.join(map(str, dims))} fp32 tensor, multilinear rank {args.rank}, "
                               f"ell {ells[0]}, core decay {w['decay']}, noise {w['noise']}",
                   "dims": dims, "rank": args.rank, "ell": ells[0], "prec": args.prec,
                   "storage": "f32", "truncate": True, "algorithmic_bytes_per_step": step_bytes},
        "roofline": {"bound": "hbm", "achieved": dom["gbps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": dom["gbps"] / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "krp_sketch of mode 1 of X (MTTKRP kernel + its reduction)",
                     "bytes_per_launch": dom["bytes"], "ms_per_launch": dom["ms"]},
        "cpu_baseline": cpu,
        "sketch_gbps_by_mode": [sketch[m]["gbps"] for m in range(len(dims))],
        "sketch_ms_by_mode": [sketch[m]["ms"] for m in range(len(dims))],
        "step_wall_ms": step_wall_ms,
        "tucker_rel_err_mixed": err_mixed,
        "fp64_form": fp64,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
