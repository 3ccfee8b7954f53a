"""Profiling driver: a few TTVc sweeps on a synthetic workload, plus a plain
device copy of known size that calibrates hardware byte counters.

  python -m paper_2403_01778_amd.profile_ttvc --dims 800,800,800 --reps 5 --copy-mb 1024

Run it under rocprofv3 (kernel trace / stats, or one counter pass at a time).
"""
from __future__ import annotations

import argparse
import sys

import torch

from . import hoscf, synth


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--dims", default="800,800,800")
    ap.add_argument("--dtype", default="f32", choices=["f32", "f64", "bf16", "fp8"])
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--copy-mb", type=int, default=1024, help="size of the calibration copy (0 = none)")
    args = ap.parse_args(argv)
    dims = tuple(int(v) for v in args.dims.split(","))
    T, _ = synth.large_planted(dims, seed=args.seed)
    x0 = torch.from_numpy(synth.init_factors(dims, args.seed))
    Td = torch.from_numpy(T).cuda()
    del T
    scale = 1.0
    if args.dtype == "f64":
        Td = Td.double()
    elif args.dtype in ("bf16", "fp8"):
        Tq, sc = hoscf.quantize(Td, args.dtype)
        scale = float(sc.item())
        Td = Tq
    if args.copy_mb > 0:
        n = args.copy_mb * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        print(f"copy: {n * 4} bytes read, {n * 4} bytes written", flush=True)
    ms = hoscf.profile_sweep(Td, x0, reps=args.reps, scale=scale)
    print(f"dims={dims} dtype={args.dtype} sweep_ms={ms[0]:.4f} ttvc_kernels_ms={ms[1]:.4f} level1_ms={ms[2]:.4f} "
          f"bytes={ms[3]} level1_GBps={ms[3] / ms[2] / 1e6:.1f}", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
