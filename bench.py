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
COPY_ELEMS = 128 * 1024 * 1024  # fp32 elements of the counter-calibration copy (512 MiB)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sketch_mode1_512x3_bf16x3_traffic.txt")
# every source the sketch kernel is compiled from (the measured traffic is void once one changes)
SKETCH_SRC = tuple(os.path.join(ROOT, "paper_2507_23207_amd", "csrc", f)
                   for f in ("sketch.hip", "philox.h", "device_common.h", "kernels.h"))


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
    ap.add_argument("--pmc-probe", action="store_true",
                    help="only run a 512 MiB copy and the dominant sketch launch (for counter runs)")
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
    """Wall-clock ms per call (synchronised on both sides, the step contract)."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps * 1e3


def gpu_ms(fn, reps, stream):
    """GPU time per call from HIP events on `stream`.

    A spin kernel keeps the GPU busy while the calls are enqueued, so the
    interval between the two events holds only the calls' own kernels."""
    import torch
    fn()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    torch.cuda._sleep(int(2.0e7))
    a.record(stream)
    for _ in range(reps):
        fn()
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def source_hash(paths):
    import hashlib
    h = hashlib.sha256()
    for path in paths:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(prec):
    """HBM bytes per launch of the dominant sketch from the committed counter
    runs, or None when they are missing or were taken on other kernel source."""
    try:
        kv = {}
        with open(TRAFFIC_FILE) as f:
            for line in f:
                if "=" in line and not line.startswith("#"):
                    k, v = line.strip().split("=", 1)
                    kv[k.strip()] = v.strip()
        if kv.get("sketch_source_sha256_16") != source_hash(SKETCH_SRC) or kv.get("prec") != prec:
            return None
        return float(kv["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def cpu_baseline(x_np, ranks, p, min_seconds=10.0):
    """The fp64 oracle (explicit KRPs, unfoldings, LAPACK) on the host cores.

    Sample: complete steps (Algorithm 8 on the full tensor, then the core
    truncation) repeated until `min_seconds` have elapsed; the rate is the
    step's algorithmic bytes per second, in the unit of the GPU value."""
    import numpy as np
    from oracle import tucker as ot

    x = np.asarray(x_np, dtype=np.float64)
    dims = list(x.shape)
    ells = [r + p for r in ranks]
    step_bytes = sthosvd_bytes(dims, ells, 4)
    reps = 0
    t0 = time.perf_counter()
    while True:
        g, qs = ot.rsthosvd_krp(x, ranks, p)
        ot.truncate(g, qs, ranks)
        reps += 1
        dt = time.perf_counter() - t0
        if dt >= min_seconds:
            break
    threads = os.environ.get("OPENBLAS_NUM_THREADS") or os.environ.get("OMP_NUM_THREADS")
    cores = int(threads) if threads else (os.cpu_count() or 1)
    return dict(value=step_bytes * reps / dt / 1e9, unit="GB/s", cores=cores, kind="oracle",
                sample=f"{reps} full step(s) (Algorithm 8 with explicit KRPs and unfoldings, then the "
                       f"core truncation) on the {'x'.join(map(str, dims))} tensor in fp64, "
                       f"{dt:.1f} s", s_per_step=dt / reps)


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

    if args.pmc_probe:
        # Three plain copies of 512 MiB (the counter calibration) and three
        # launches of the dominant sketch, nothing else; run under
        # rocprofv3 --pmc FETCH_SIZE (then WRITE_SIZE).
        src = torch.empty(COPY_ELEMS, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        for _ in range(3):
            krp.sketch(x, [0], [ells[0]], prec=args.prec, graph=False)
        torch.cuda.synchronize()
        print("pmc probe done", flush=True)
        return

    # --- the step: mixed-precision STHOSVD with truncation -------------------
    def step():
        return krp.sthosvd(x, ranks, p, prec=args.prec, truncate=True)

    step_ms = time_calls(step, args.steps, args.warmup, stream)
    step_gpu_ms = gpu_ms(step, args.steps, stream)
    core, qs, err_mixed = krp.sthosvd(x, ranks, p, prec=args.prec, truncate=True, rel_err=True)
    step_bytes = sthosvd_bytes(dims, ells, 4)

    # --- dominant launch: KRP sketch of X for each mode ----------------------
    sketch = {}
    for m in range(len(dims)):
        fn = lambda m=m: krp.sketch(x, [m], [ells[m]], prec=args.prec)
        ms = gpu_ms(fn, max(10, args.steps), stream)
        b = x.numel() * 4 + dims[m] * ells[m] * 4
        sketch[m] = dict(ms=ms, gbps=b / ms / 1e6, bytes=b)

    # --- fp64 GPU form of the same STHOSVD ------------------------------------
    fp64 = None
    if not args.no_fp64:
        x64 = x.to(torch.float64)  # converted once, outside the timed region
        def step64():
            return krp.sthosvd(x64, ranks, p, prec="fp64", truncate=True)
        ms64 = time_calls(step64, max(3, args.steps // 2), 2, stream)
        gms64 = gpu_ms(step64, max(3, args.steps // 2), stream)
        _, _, err64 = krp.sthosvd(x64, ranks, p, prec="fp64", truncate=True, rel_err=True)
        fp64 = dict(ms=ms64, gpu_ms=gms64, tucker_rel_err=err64, speedup_mixed=ms64 / step_ms,
                    speedup_mixed_gpu=gms64 / step_gpu_ms,
                    err_ratio=err_mixed / err64)
        del x64

    cpu = None
    if not args.no_cpu_baseline:
        x_np = x.permute(*reversed(range(len(dims)))).contiguous().cpu().numpy()
        x_np = np.ascontiguousarray(x_np).transpose(*reversed(range(len(dims))))
        cpu = cpu_baseline(x_np, ranks, p)

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
                     "frac": dom["gbps"] / HBM_PEAK_GBS, "traffic": measured_traffic(args.prec),
                     "kernel": "krp_sketch of mode 1 of X (MTTKRP kernel + its reduction)",
                     "bytes_per_launch": dom["bytes"], "ms_per_launch": dom["ms"]},
        "cpu_baseline": cpu,
        "sketch_gbps_by_mode": [sketch[m]["gbps"] for m in range(len(dims))],
        "sketch_ms_by_mode": [sketch[m]["ms"] for m in range(len(dims))],
        "step_gpu_ms": step_gpu_ms,
        "tucker_rel_err_mixed": err_mixed,
        "fp64_form": fp64,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
