"""Profiling driver for the post-sweep kernel: runs solves capped at 1, 2, 4
iterations and prints the phase timings the kernel records in its
SolveState (device clock at 100 MHz): the epilogue, and per Lanczos step the
J products, the two reorthogonalisation passes, the next Krylov vector with
the convergence check (which overlaps the barrier's arrival half) and the
barrier's remaining wait, plus the final normalisation.

  python -m paper_2403_01778_amd.profile_eigen --dims 800,800,800
"""
from __future__ import annotations

import argparse
import sys

import numpy as np
import torch

from . import hoscf, synth

# SolveState: 6 doubles, 8 int32, 2 uint32, 1 uint64, then uint64 trace[32];
# it is the first object carved from the solve workspace.
TRACE_OFFSET = 6 * 8 + 8 * 4 + 2 * 4 + 8


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--dims", default="800,800,800")
    ap.add_argument("--seed", type=int, default=2)
    args = ap.parse_args(argv)
    dims = tuple(int(v) for v in args.dims.split(","))
    T, _ = synth.large_planted(dims, seed=args.seed)
    x0 = torch.from_numpy(synth.init_factors(dims, args.seed)).cuda()
    Td = torch.from_numpy(T).cuda()
    del T
    desc = hoscf.describe(Td)
    for it in (1, 2, 4):
        opts = hoscf.options("hoscf", tol=1e-6, max_iter=it)
        ws = torch.zeros(hoscf.workspace_size(hoscf.OP_SOLVE, desc, opts), dtype=torch.uint8, device="cuda")
        hoscf.solve_raw(Td, x0, opts, workspace=ws, raise_on_error=False)
        torch.cuda.synchronize()
        tr = ws[:TRACE_OFFSET + 256].cpu().numpy()[TRACE_OFFSET:TRACE_OFFSET + 256].view(np.uint64).astype(np.int64)
        t = tr[16:32]
        if t[0] == 0 or t[9] == 0:
            print(f"dims={dims} iteration {it}: converged before an eigen-step", flush=True)
            continue
        m = int(t[9])
        us = lambda a, b: (t[b] - t[a]) * 0.01  # noqa: E731
        s = [v * 0.01 for v in t[10:15]]
        print(f"dims={dims} eigen-step {it}: lanczos_steps={m} total_us={us(0, 8):.1f} epilogue_us={us(0, 3):.1f} "
              f"per_step_us: J_product={s[0] / max(m - 1, 1):.1f} pass1={s[1] / m:.1f} pass2={s[2] / m:.1f} "
              f"new_vector_and_check={s[3] / m:.1f} barrier_wait={s[4] / m:.1f} final_us={us(7, 8):.1f}", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
