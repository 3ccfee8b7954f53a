"""GPU parity of the precision form: the quantiser (bit-exact against the
oracle's encoders), TTVc sweeps that read BF16 / FP8-E4M3 storage, and the
two-phase solve (low-precision sweeps, then FP32 refinement sweeps).

Bars: codes and scales are compared bit for bit.  A sweep over low-precision
storage is compared with the oracle run on the dequantised values (the very
numbers the GPU reads), entrywise within 1e-5 of the |T|,|u| contraction
(FP32 accumulation).  The two-phase solve must reach the FP32 problem's KKT
point: sigma within 1e-6 and factors within 1e-5 rad of the oracle run on the
FP32 tensor from the same start.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import quant
from paper_2403_01778_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _bf16_cases(rng, n):
    x = (rng.standard_normal(n) * np.exp2(rng.integers(-30, 30, n))).astype(np.float32)
    bits = x.view(np.uint32)
    # exact ties (low half 0x8000), odd and even high halves
    bits[: n // 8] = (bits[: n // 8] & 0xffff0000) | 0x8000
    x[n // 8: n // 8 + 8] = np.array([0.0, -0.0, 1e-40, -1e-40, 3.0e38, -3.0e38, 1.0, -1.0], np.float32)
    return x


def test_quantize_bf16_bit_exact(lib):
    rng = np.random.default_rng(5)
    x = _bf16_cases(rng, 1_000_003)
    q, sc = lib.quantize(torch.from_numpy(x).to(DEV), "bf16")
    got = q.view(torch.int16).cpu().numpy().view(np.uint16)
    want = quant.bf16_bits(x)
    assert np.array_equal(got, want), int(np.sum(got != want))
    assert float(sc.item()) == 1.0


@pytest.mark.parametrize("with_max", [True, False])
def test_quantize_fp8_bit_exact(lib, with_max):
    """Scale = amax/448 in binary32; codes by RNE with saturation.  With
    with_max the tensor holds 448 so the scale is 1 and exact E4M3 midpoints
    (normal and subnormal) test the tie rule."""
    rng = np.random.default_rng(6)
    n = 777_777
    x = (rng.standard_normal(n) * 40).astype(np.float32)
    if with_max:
        x[0] = 448.0
        x[1] = -300.0
        mids = [1.0625, 1.1875, -2.125, 0.5 * (2.0 ** -9), 1.5 * (2.0 ** -9), 2.0 ** -7 + 2.0 ** -10, 464.0 - 1.0]
        x[2:2 + len(mids)] = np.array(mids, np.float32)
        x[20:40] = np.float32(2.0 ** -12) * np.arange(20, dtype=np.float32)
    q, sc = lib.quantize(torch.from_numpy(x).to(DEV), "fp8")
    s_gpu = np.float32(sc.item())
    want, s_ref = quant.quantize_fp8(x)
    assert s_gpu.view(np.uint32) == np.float32(s_ref).view(np.uint32)
    got = q.view(torch.uint8).cpu().numpy()
    assert np.array_equal(got, want), int(np.sum(got != want))


def _lowprec_case(lib, dims, fmt, seed):
    rng = np.random.default_rng(seed)
    T32 = (rng.standard_normal(dims) * 3).astype(np.float32)
    Tq, sc = lib.quantize(torch.from_numpy(T32).to(DEV), fmt)
    scale = float(sc.item())
    if fmt == "bf16":
        Tdeq = quant.bf16_value(quant.bf16_bits(T32)).astype(np.float64).reshape(dims)
    else:
        codes = Tq.view(torch.uint8).cpu().numpy().reshape(dims)
        Tdeq = quant.dequantize_fp8(codes, np.float32(scale))
    return T32, Tq, scale, Tdeq


@pytest.mark.parametrize("fmt", ["bf16", "fp8"])
@pytest.mark.parametrize("dims", [(37, 29, 64), (37, 29, 23), (9, 10, 11, 16), (6, 7, 5, 4, 32), (40, 48),
                                  (10, 20, 576), (6, 10, 1152), (6, 10, 1088)])  # split sweeps
def test_ttvc_lowprec_parity(lib, fmt, dims):
    print(f"[ttvc-lp] fmt={fmt} dims={dims}", flush=True)
    _, Tq, scale, Tdeq = _lowprec_case(lib, dims, fmt, 100 + sum(dims))
    x = synth.init_factors(dims, 7)
    r = lib.ttvc(Tq, torch.from_numpy(x), scale=scale)
    xs = oracle.normalize_blocks(x, dims)
    ref = oracle.sweep(Tdeq, xs)
    absb = oracle.blocks(np.abs(Tdeq), [np.abs(v) for v in xs])
    for k, (key, A_ref) in enumerate(ref.blocks.items()):
        A = r.blocks[k].double().cpu().numpy()
        err = np.abs(A - A_ref)
        assert np.all(err <= 1e-5 * absb[key] + 1e-300), (key, float(np.max(err / (absb[key] + 1e-300))))
    g_ref = oracle.stack(oracle.mode_vectors(Tdeq, xs))
    g_abs = oracle.stack(oracle.mode_vectors(np.abs(Tdeq), [np.abs(v) for v in xs]))
    assert np.all(np.abs(r.g.cpu().numpy() - g_ref) <= 1e-5 * g_abs + 1e-300)
    sig_abs = oracle.objective(np.abs(Tdeq), [np.abs(v) for v in xs])
    assert abs(r.sigma - ref.sigma) <= 1e-5 * sig_abs


def _two_phase(lib, T32, fmt, x0, algo, tol=1e-6, max_iter=300):
    Td = torch.from_numpy(T32).to(DEV)
    Tq, sc = lib.quantize(Td, fmt)
    opts = lib.options(algo=algo, tol=tol, max_iter=max_iter, tol_lp=1e-3)
    sig, x, info = lib.solve_raw(Tq, torch.from_numpy(x0), opts, scale=float(sc.item()), data_f32=Td,
                                 raise_on_error=False)
    return sig, x.cpu().numpy(), info


@pytest.mark.parametrize("fmt", ["bf16", "fp8"])
@pytest.mark.parametrize("algo", ["hoscf", "ihoscf"])
def test_two_phase_solve_matches_fp32_oracle(lib, fmt, algo):
    """Order-5 rank-5 CP + 1% noise (the 64^5 workload's recipe at 20^5):
    low-precision sweeps, then FP32 refinement, land on the FP32 problem's
    KKT point reached by the oracle from the same start."""
    dims = (20, 20, 20, 20, 20)
    T32, _, _ = synth.cp_plus_noise(dims, 5, 0.01, seed=4)
    x0 = synth.init_factors(dims, 1004)
    ref = oracle.hoscf(T32.astype(np.float64), x0, algo="hoscf", tol=1e-12, max_iter=2000)
    assert ref.status == oracle.OK
    sig, x, info = _two_phase(lib, T32, fmt, x0, algo)
    print(f"[two-phase] fmt={fmt} algo={algo} sigma={sig!r} ref={ref.sigma!r} status={info.status} "
          f"iters={info.iters} sweeps={info.sweeps} lp_sweeps={info.lp_sweeps}", flush=True)
    assert info.status == 0
    assert info.lp_sweeps >= 1 and info.sweeps > info.lp_sweeps
    assert sig == pytest.approx(ref.sigma, rel=1e-6)
    for n, (a, b) in enumerate(zip(oracle.split(x, dims), ref.xs)):
        assert oracle.angle(a, b) <= 1e-5, n


@pytest.mark.parametrize("fmt", ["bf16", "fp8"])
def test_c3_full_size_two_phase(lib, fmt):
    """64^5 rank-5 CP + 1% noise (4.3 GB FP32): the two-phase solve and the
    plain FP32 solve from the same start agree (sigma 1e-6, angle 1e-5), and
    the point is a KKT point of the FP32 problem by the oracle's own
    contractions."""
    dims = (64,) * 5
    T32, _, _ = synth.cp_plus_noise(dims, 5, 0.01, seed=4)
    x0 = synth.init_factors(dims, 1004)
    Td = torch.from_numpy(T32).to(DEV)
    sig32, x32, info32 = lib.solve_raw(Td, torch.from_numpy(x0), lib.options(algo="hoscf", tol=1e-6, max_iter=300),
                                       raise_on_error=False)
    sig, x, info = _two_phase(lib, T32, fmt, x0, "hoscf")
    print(f"[c3] fmt={fmt} sigma={sig!r} fp32={sig32!r} status={info.status}/{info32.status} "
          f"sweeps={info.sweeps} lp={info.lp_sweeps} fp32 sweeps={info32.sweeps}", flush=True)
    assert info.status == 0 and info32.status == 0
    assert sig == pytest.approx(sig32, rel=1e-6)
    xs = oracle.split(x, dims)
    for a, b in zip(xs, oracle.split(x32.cpu().numpy(), dims)):
        assert oracle.angle(a, b) <= 1e-5
    g = oracle.mode_vectors(T32, xs)
    s_ref = float(xs[0] @ g[0])
    assert sig == pytest.approx(s_ref, rel=1e-6)
    for n in range(5):
        assert np.linalg.norm(g[n] - s_ref * xs[n]) <= 1e-5 * s_ref
