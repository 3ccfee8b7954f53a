#!/usr/bin/env python3
"""Benchmark of the HOSCF hot path on one MI355X.

Workload (one "step" = one full solve through every step of the path: TTVc
sweeps, FP64 eigen-steps, normalisation and signs, the stopping test, the final
sign fix): order-3 800 x 800 x 800 FP32 tensor (2.048 GB), N(0,1) noise plus a
planted rank-one term with lambda = 3 sqrt(prod I)/sqrt(max I) = 2400 and unit
Gaussian factors, seeded (seed 2); seeded Gaussian unit initial factors; plain
HOSCF (exact inner eigen-steps), tol 1e-6.  The input is resident in HBM
before the timed region.

Printed: one JSON line.
  value         whole-job TTVc throughput: bytes of T streamed by all sweeps of
                the timed solves / their wall time (eigen-steps and host round
                trips count against it).
  chosen_vs_plain  the same workload under the solver variants (inexact inner
                solves, iHOSCF), each with its sigma error against the FP64
                oracle; "chosen" is the fastest with error <= 1e-6.
  roofline      the level-1 TTVc kernel alone, timed with HIP events on its own
                stream, against 8 TB/s; traffic = HBM bytes per launch from the
                rocprofv3 counter passes (null once the kernel source differs
                from the one they were taken on).
  extras        the precision form (64^5, FP32 vs BF16 / FP8 storage), the
                batched form (4096 tensors, rank 8, one launch) and the backward
                pass (256^3 items).
  cpu_baseline  the FP64 oracle on the host cores over a bounded sample.
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

HBM_PEAK_GBPS = 8000.0

# HBM traffic of the level-1 TTVc kernel on this workload, from two
# rocprofv3 counter passes (FETCH_SIZE x 2.000 and WRITE_SIZE x 1.000, the
# factors a 1 GiB device copy reads on the same counters); summary in
# profiles/ttvc3_kernel_800cubed_f32_pmc.md.  Valid only for the kernel source
# the counters were taken on.
TRAFFIC = {"kernel_source_sha256": "108314f6f7477369b623a9916a3bafb0aff87d6c40eb5cf46b38f75067bb4a6c",
           "read_bytes": 2_007_698.1 * 1024, "write_bytes": 55_060.9 * 1024}


def measured_traffic():
    import hashlib
    src = os.path.join(ROOT, "paper_2403_01778_amd", "csrc", "ttvc.hip")
    with open(src, "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != TRAFFIC["kernel_source_sha256"]:
            return None
    return round(TRAFFIC["read_bytes"] + TRAFFIC["write_bytes"])
METRIC = "TTVc HBM GB/s (% peak); HOSCF solves/s, chosen vs plain at σ rel err≤1e-6"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the precision, batched and backward legs")
    ap.add_argument("--profile-reps", type=int, default=20)
    return ap.parse_args()


def cpu_baseline(T, x0):
    """The oracle as it stands: a bounded sample of HOSCF iterations (FP64
    sweep = three separate contraction chains over T in FP64 slabs, then a
    dense LAPACK eigen-step), timed on the host cores."""
    import numpy as np

    import oracle
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    xs = oracle.normalize_blocks(x0, T.shape)
    iters = 8  # about 10 s of host work
    t0 = time.perf_counter()
    for _ in range(iters):
        sw = oracle.sweep(T, xs)
        J = oracle.j_matrix(sw.blocks, T.shape)
        _, y = oracle.top_magnitude_eigpair(J)
        xs = oracle.canonical_signs(oracle.normalize_blocks(y, T.shape))
    dt = time.perf_counter() - t0
    return {"value": round(iters * T.nbytes / dt / 1e9, 4), "unit": "GB/s", "cores": int(cores), "kind": "oracle",
            "sample": f"{iters} oracle HOSCF iterations (FP64 sweep + dense eigh) on the 800^3 FP32 workload, "
                      f"{dt:.1f} s; {cores} BLAS threads"}


def _timed(fn, reps):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = None
    for _ in range(reps):
        out = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps, out


def leg_precision(hoscf, synth, reps=2):
    """Order-5 64^5 rank-5 CP + 1% noise: plain FP32 HOSCF against the
    two-phase precision form (BF16 / FP8-E4M3 sweeps, then FP32 refinement),
    sigma error against the FP64 oracle's T(u) on the FP32 tensor, and the
    level-1 TTVc bandwidth per storage format."""
    import numpy as np
    import torch

    import oracle
    dims = (64,) * 5
    T32, _, _ = synth.cp_plus_noise(dims, 5, 0.01, seed=4)
    x0 = torch.from_numpy(synth.init_factors(dims, 1004))
    Td = torch.from_numpy(T32).cuda()
    out = {"workload": "order-5 64^5 rank-5 N(0,1) CP + 1% noise, seed 4, tol 1e-6, tol_lp 1e-3"}
    opts = hoscf.options(algo="hoscf", tol=1e-6, max_iter=300, tol_lp=1e-3)
    hoscf.solve_raw(Td, x0, opts)
    dt, (sig32, x32, inf32) = _timed(lambda: hoscf.solve_raw(Td, x0, opts), reps)
    xs = oracle.split(x32.cpu().numpy(), dims)
    s_ref = oracle.objective(T32, xs)
    r = hoscf.profile_sweep(Td, x32, reps=5)
    out["f32"] = {"solves_per_s": round(1 / dt, 3), "sweeps": inf32.sweeps, "status": inf32.status,
                  "sigma": sig32, "sigma_rel_err_vs_oracle": abs(sig32 - s_ref) / abs(s_ref),
                  "ttvc_GBps": round(r[3] / r[2] / 1e6, 1)}
    for fmt in ("bf16", "fp8"):
        Tq, sc = hoscf.quantize(Td, fmt)
        scale = float(sc.item())
        run = lambda: hoscf.solve_raw(Tq, x0, opts, scale=scale, data_f32=Td)  # noqa: E731
        run()
        dt_q, (sig, x, inf) = _timed(run, reps)
        xs = oracle.split(x.cpu().numpy(), dims)
        s_o = oracle.objective(T32, xs)
        ang = max(oracle.angle(a, b) for a, b in zip(xs, oracle.split(x32.cpu().numpy(), dims)))
        rq = hoscf.profile_sweep(Tq, x, reps=5, scale=scale)
        out[fmt] = {"solves_per_s": round(1 / dt_q, 3), "speedup_vs_f32": round(dt / dt_q, 3),
                    "sweeps": inf.sweeps, "lp_sweeps": inf.lp_sweeps, "status": inf.status, "sigma": sig,
                    "sigma_rel_err_vs_oracle": abs(sig - s_o) / abs(s_o),
                    "sigma_rel_diff_vs_f32": abs(sig - sig32) / abs(sig32), "max_angle_vs_f32": ang,
                    "ttvc_GBps": round(rq[3] / rq[2] / 1e6, 1)}
        del Tq
    del Td
    torch.cuda.empty_cache()
    return out


def leg_batched(hoscf, synth, reps=1):
    """4096 order-3 FP32 tensors (dims uniform in {8..96}, planted rank-one,
    lambda ~ U[1, 20]), greedy rank-8 deflation, one persistent launch."""
    import numpy as np
    import torch
    tensors, _, _ = synth.batched_planted(4096, 5)
    host = np.concatenate([t.ravel() for t in tensors])
    buf = torch.from_numpy(host).cuda()
    views, off = [], 0
    for t in tensors:
        views.append(buf[off:off + t.size].view(*t.shape))
        off += t.size
    plan = hoscf.BatchPlan(views, R=8, tol=1e-6, max_iter=500)
    x0 = np.empty(plan.total)
    for b, dims in enumerate(plan.dims):
        for r in range(plan.R):
            o = plan.offsets[b] + r * plan.D[b]
            x0[o:o + plan.D[b]] = synth.init_factors(dims, 5 * 100003 + b * 17 + r)  # as in the tests
    x0 = torch.from_numpy(x0).cuda()
    terms = len(tensors) * plan.R
    out = {"workload": "4096 x order-3 FP32, dims U{8..96}, N(0,1) + U[1,20] planted, rank 8, tol 1e-6",
           "bytes": int(host.nbytes)}
    plans = {"plain": plan,
             "inexact_inner": hoscf.BatchPlan(views, R=8, tol=1e-6, max_iter=500, inner_rel=1e-3),
             "ihoscf": hoscf.BatchPlan(views, R=8, tol=1e-6, max_iter=500, algo="ihoscf"),
             "ihoscf_inexact": hoscf.BatchPlan(views, R=8, tol=1e-6, max_iter=500, algo="ihoscf", inner_rel=1e-3)}
    for name, p in plans.items():
        outs = p.outputs()
        if name == "plain":
            p.run(x0, outs)  # warm-up (the same kernel serves both plans)
        dt, _ = _timed(lambda: p.run(x0, outs), reps)
        st = outs[2].cpu().numpy()
        it = outs[3].cpu().numpy()
        out[name] = {"launch_s": round(dt, 4), "rank_one_solves_per_s": round(terms / dt, 1),
                     "tensors_per_s": round(len(tensors) / dt, 1), "ok_terms": int((st == 0).sum()),
                     "not_converged_terms": int((st == 1).sum()), "mean_iters": round(float(it.mean()), 1)}
    return out


def leg_backward(hoscf, synth, items=4):
    """Items of the 64 x 256^3 differentiation workload (planted rank-2,
    lambdas 768 and 512): solve, then dL/dT for L = sigma + w'x (one sweep,
    the projected adjoint solve, one 67 MB write)."""
    import numpy as np
    import torch
    dims = (256, 256, 256)
    t_solve = t_bwd = 0.0
    steps = []
    for i in range(items):
        T, _ = synth.planted_cp(dims, [768.0, 512.0], 6000 + i)
        Td = torch.from_numpy(T).cuda()
        x0 = torch.from_numpy(synth.init_factors(dims, 7000 + i))
        w = torch.from_numpy(np.concatenate(synth.loss_weights(dims, 6000 + i))).cuda()
        opts = hoscf.options(algo="hoscf", tol=1e-6, max_iter=300)
        hoscf.solve_raw(Td, x0, opts)
        dt_s, (sig, x, _) = _timed(lambda: hoscf.solve_raw(Td, x0, opts), 1)
        for _ in range(2):  # warm-up: first-call allocations and cache state
            hoscf.backward(Td, x, sig, 1.0, w)
        dt_b, (g, mu, info) = _timed(lambda: hoscf.backward(Td, x, sig, 1.0, w, return_info=True), 5)
        t_solve += dt_s
        t_bwd += dt_b
        steps.append(info[0])
        del Td, g
    torch.cuda.empty_cache()
    n = float(np.prod(dims))
    return {"workload": f"{items} items of 64 x 256^3 FP32 planted rank-2 (768, 512), L = sigma + w'x",
            "solve_ms": round(t_solve / items * 1e3, 3), "backward_ms": round(t_bwd / items * 1e3, 3),
            "backward_GBps": round(items * n * 8 / t_bwd / 1e9, 1),
            "adjoint_lanczos_steps": steps}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build runs the path on a single MI355X "
              "(the multi-GPU sharding is a design note, not built). Use --gpus 1.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2403_01778_amd import hoscf, synth

    dev = torch.device("cuda:0")
    dims = (800, 800, 800)
    t_gen = time.perf_counter()
    T, fac = synth.large_planted(dims, seed=2)
    x0 = synth.init_factors(dims, 2)
    print(f"[bench] generated {dims} FP32 in {time.perf_counter() - t_gen:.1f}s", file=sys.stderr, flush=True)
    Td = torch.from_numpy(T).to(dev)
    x0d = torch.from_numpy(x0).to(dev)
    # plain: HOSCF with exact inner eigen-steps (Algorithm 1); the other
    # variants are timed on the same input for the chosen-vs-plain report
    variants = {"hoscf": hoscf.options(algo="hoscf", tol=1e-6, max_iter=200),
                "hoscf_inexact": hoscf.options(algo="hoscf", tol=1e-6, max_iter=200, inner_rel=1e-3),
                "ihoscf": hoscf.options(algo="ihoscf", tol=1e-6, max_iter=200),
                "ihoscf_inexact": hoscf.options(algo="ihoscf", tol=1e-6, max_iter=200, inner_rel=1e-3)}
    desc = hoscf.describe(Td)
    ws = torch.empty(hoscf.workspace_size(hoscf.OP_SOLVE, desc, variants["hoscf"]), dtype=torch.uint8, device=dev)

    def run(name, n):
        sweeps, last = 0, None
        for _ in range(n):
            sig, x, info = hoscf.solve_raw(Td, x0d, variants[name], workspace=ws)
            if info.status != 0:
                raise RuntimeError(f"{name} solve did not converge: {info}")
            sweeps += info.sweeps
            last = (sig, x, info)
        return sweeps, last

    def timed(name, n, warm):
        run(name, warm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sw, last = run(name, n)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, sw, last

    dt, sweeps, (sig, x, info) = timed("hoscf", args.steps, args.warmup)
    print(f"[bench] hoscf: {args.steps} solves in {dt:.3f}s, iters={info.iters} sweeps/solve={info.sweeps} "
          f"lanczos={info.lanczos_steps}", file=sys.stderr, flush=True)
    others = {name: timed(name, args.steps, 1) for name in ("hoscf_inexact", "ihoscf", "ihoscf_inexact")}

    # level-1 TTVc kernel, HIP events on the launching stream
    ms_sweep, ms_k1, ms_root, nbytes = hoscf.profile_sweep(Td, x, reps=args.profile_reps)
    achieved = nbytes / (ms_root * 1e-3) / 1e9

    # accuracy against FP64 evaluation by the oracle on the stored values
    import oracle
    xs = oracle.split(x.cpu().numpy(), dims)
    sig_ref = oracle.objective(T, xs)
    rel = abs(sig - sig_ref) / abs(sig_ref)
    report = {}
    for name, (dt_v, sw_v, (sig_v, x_v, info_v)) in others.items():
        xs_v = oracle.split(x_v.cpu().numpy(), dims)
        rel_v = abs(sig_v - oracle.objective(T, xs_v)) / abs(sig_ref)
        report[name] = {"solves_per_s": round(args.steps / dt_v, 3), "speedup_vs_plain": round(dt / dt_v, 3),
                        "sigma_rel_err": rel_v, "sweeps_per_solve": info_v.sweeps,
                        "lanczos_steps_per_solve": info_v.lanczos_steps,
                        "ttvc_GBps_whole_job": round(sw_v * nbytes / dt_v / 1e9, 1)}
    ok = {k: v for k, v in report.items() if v["sigma_rel_err"] <= 1e-6}
    chosen = max(ok, key=lambda k: ok[k]["solves_per_s"]) if ok else None
    value = sweeps * nbytes / dt / 1e9
    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded N(0,1) + planted rank-one, generated on the host)",
        "config": {"workload": "order-3 800x800x800 FP32 (2.048 GB), N(0,1) + 2400*a o b o c, plain HOSCF tol 1e-6",
                   "dims": list(dims), "seed": 2, "algo": "hoscf", "tol": 1e-6},
        "solves_per_s": round(args.steps / dt, 3),
        "sweeps_per_solve": info.sweeps,
        "iters_per_solve": info.iters,
        "sigma": sig,
        "sigma_rel_err_vs_oracle_fp64": rel,
        "lanczos_steps_per_solve": info.lanczos_steps,
        "chosen_vs_plain": {"plain": "hoscf (exact inner eigen-steps), fp32 storage",
                            "plain_solves_per_s": round(args.steps / dt, 3),
                            "chosen": chosen,
                            "ratio": ok[chosen]["speedup_vs_plain"] if chosen else None,
                            "variants": report},
        "ttvc_sweep_ms": round(ms_sweep, 4),
        "ttvc_kernels_ms": round(ms_k1, 4),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": measured_traffic(),
                     "kernel": "level-1 TTVc launch over T (ttvc3_split_kernel for this shape)", "bytes_per_launch": nbytes,
                     "launch_ms": round(ms_root, 5)},
    }
    if not args.no_extras:
        del Td
        torch.cuda.empty_cache()
        extras = {}
        for name, fn in (("precision_form", leg_precision), ("batched_form", leg_batched),
                         ("differentiation_form", leg_backward)):
            t_leg = time.perf_counter()
            try:
                extras[name] = fn(hoscf, synth)
            except Exception as e:  # a failing extra never hides the main line
                extras[name] = {"error": f"{type(e).__name__}: {e}"}
            print(f"[bench] {name} leg: {time.perf_counter() - t_leg:.1f}s", file=sys.stderr, flush=True)
        out["extras"] = extras
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(T, x0)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
