"""Benchmark of the SYK hot path on one MI355X.

Workload (default): N = 52 Majoranas (dim 2^26, 270,725 couplings, 15,276
flip masks), couplings seed 0, typical state seed 1.  One step = one Lanczos
time step of the OTOC propagation (m = 12 applications of H, two-pass
Gram-Schmidt with FP64 inner products, FP64 tridiagonal exponential, basis
combination) of one complex128 state by dt = 0.25.

Printed: one JSON line with the OTOC time-steps/s (value); the apply_H figures
in "apply_H": the rocprofv3-measured HBM bytes of one call over its
HIP-event-timed duration against 8 TB/s (when the counters were taken on the
current kernel source), and beside it the effective rate of the method's byte
model (one gather per flip mask), which LDS staging lets exceed the HBM peak;
the same duration against the FP64 vector-ALU roof in "roofline"; the
complex64 leg with its state error against complex128 after the same steps;
the F(t) window of the N = 52 OTOC (beta J = 10, m = 12) in both precisions
with |dF|; the disorder-averaging block as an OTOC window at N = 40; the
gradient cost ratio; N = 60; and the CPU checker timed on bounded samples.

One apply_H call is the unit of work of the roofline: the apply kernel over
the masks of the natural row layout, the same kernel over the masks of the
bit-rotated layout, and the two transposes between the layouts.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Vector-ALU roofs of MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x
# 2.4 GHz = 78.6 TFLOP/s in FP64; the published FP32 figure, 157.3 TFLOP/s,
# counts packed FP32 FMAs (two per lane per instruction).  The library compiles
# without packed FP32, and non-packed FP32 FMAs issue at the FP64 rate (an FMA
# throughput probe on the MI355X: 76.5 TFLOP/s), so the complex64 figures are
# given against both.
FP64_VECTOR_PEAK_TFLOPS = 78.6
FP32_VECTOR_PEAK_TFLOPS = 157.3
FP32_NONPACKED_PEAK_TFLOPS = 78.6
# Arithmetic per (row, flip mask) pair of the grouped product: one complex
# multiply-accumulate, coefficient x gathered amplitude = 4 real FMA = 8 flops.
FLOPS_PER_PAIR = 8
METRIC = "apply_H GB/s (% HBM peak) and OTOC time-steps/s at N=52; grad/fwd cost ratio"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    with open(os.path.join(ROOT, "paper_2002_05725_amd", "csrc", "apply_h.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def traffic_from_profile(workload_key: str):
    """HBM bytes per apply from a committed rocprofv3 counter summary, if it was
    taken on the current kernel source; else None."""
    p = os.path.join(ROOT, "profiles", "apply_h_traffic.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        d = json.load(f)
    e = d.get(workload_key)
    if not e or e.get("kernel_sha") != kernel_source_hash():
        return None
    return e.get("bytes_per_apply")


def run_steps(api, T, psi, n, m, dt, after=None, done=0):
    """n time steps; after(k) is called once step k (counted from 1 over every
    call, `done` steps before this one) has finished."""
    for i in range(n):
        api.krylov_expmv(T, psi, -1j, dt, m=m, dt=dt)
        if after:
            after(done + i + 1)


def timed_leg(api, torch, T, psi, steps, warmup, m, dt, after=None):
    run_steps(api, T, psi, warmup, m, dt, after, 0)
    torch.cuda.synchronize()
    api.timing_reset()
    api.timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run_steps(api, T, psi, steps, m, dt, after, warmup)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    api.timing_enable(False)
    n_apply, apply_ms = api.timing_read()
    api.timing_reset()
    return t1 - t0, n_apply, apply_ms


def otoc_window(api, torch, T, x, times, beta, m, dt, tau, real=None):
    """F(t) of the regularized OTOC (i, j = 0, 1) on an output window; returns
    (F [nt, nvec], F_im, wall seconds, Lanczos time steps taken per column,
    summed apply_H milliseconds)."""
    torch.cuda.synchronize()
    api.timing_reset()
    api.timing_enable(True)
    t0 = time.perf_counter()
    F, Fi, _ = api.otoc(T, 0, 1, beta, times, x, m=m, dt=dt, tau_step=tau, real_of_col=real)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    api.timing_enable(False)
    n, ms = api.timing_read()
    api.timing_reset()
    return F, Fi, wall, n / m, ms


def beta10_window_leg(api, torch, T, psi_host, dev, N):
    """The N = 52 OTOC (beta J = 10, Lanczos m = 12, real step 0.25, imaginary
    step 0.625) on its first output window, t in {0, 0.5}, in complex128 and in
    complex64 (FP64 inner products) from the same typical state."""
    times, beta, m, dt, tau = [0.0, 0.5], 10.0, 12, 0.25, 0.625
    out = {"N": N, "beta": beta, "m": m, "dt": dt, "tau_step": tau, "times": times}
    res = {}
    for name, dtp in (("c128", torch.complex128), ("c64", torch.complex64)):
        torch.cuda.empty_cache()
        x = torch.from_numpy(psi_host).to(dev).to(dtp)
        log(f"[bench] N={N} F(t) window {name}")
        F, Fi, wall, steps, ms = otoc_window(api, torch, T, x, times, beta, m, dt, tau)
        del x
        res[name] = F[:, 0]
        out[name] = {"F": F[:, 0].tolist(), "F_im": Fi[:, 0].tolist(), "wall_s": wall, "time_steps": steps,
                     "otoc_time_steps_per_s": steps / wall, "apply_ms": ms / (steps * m)}
    dF = float(abs(res["c64"] - res["c128"]).max())
    out["max_abs_dF_c64_vs_c128"] = dF
    out["within_2e-5"] = dF <= 2e-5
    return out


def batched_leg(api, inputs, torch, np, dev, N, m, dt):
    """Disorder-averaging workload: 32 realisations x 2 typical states at N as
    one 64-column block, the regularized OTOC at beta J = 5 on the output
    window t in {0, 0.5} (Lanczos m, real step dt, imaginary step 0.625): the
    complex64 block (FP64 inner products), the complex128 block, and one
    column alone in complex128 (the plain path), all on the same GPU.  The
    apply runs in its automatic shape: the complex64 block with the two
    columns of each realisation in one workgroup, complex128 one column per
    workgroup."""
    R = 32
    times, beta, tau = [0.0, 0.5], 5.0, 0.625
    Js = np.stack([inputs.couplings(N, inputs.batch_coupling_seed(N, r)) for r in range(R)])
    T = api.Terms(N, Js)
    real = np.repeat(np.arange(R), 2)
    host = np.stack([inputs.typical_state(N, inputs.batch_state_seed(N, r, s)) for r in range(R) for s in range(2)])
    out = {"N": N, "columns": 64, "realisations": R, "m": m, "dt": dt, "tau_step": tau, "beta": beta,
           "times": times, "apply_columns_per_workgroup": {"block_c64": 2, "block_c128": 1, "single_c128": 1}}
    flops_apply = FLOPS_PER_PAIR * T.n_masks * T.dim
    F = {}
    for name, dtp, x_host, rc, cols in (("block_c64", torch.complex64, host, real, 64),
                                        ("block_c128", torch.complex128, host, real, 64),
                                        ("single_c128", torch.complex128, host[0], None, 1)):
        torch.cuda.empty_cache()
        x = torch.from_numpy(x_host).to(dev).to(dtp)
        log(f"[bench] batched {name}")
        Fw, _, wall, steps, ms = otoc_window(api, torch, T, x, times, beta, m, dt, tau, real=rc)
        del x
        F[name] = Fw
        per_apply_s = ms / (steps * m) / 1e3
        rec = {"wall_s": wall, "time_steps_per_column": steps, "vector_steps_per_s": cols * steps / wall,
               "apply_ms": per_apply_s * 1e3, "apply_TFLOPs": cols * flops_apply / per_apply_s / 1e12}
        roof = FP32_VECTOR_PEAK_TFLOPS if dtp == torch.complex64 else FP64_VECTOR_PEAK_TFLOPS
        rec["apply_frac_vector_peak"] = rec["apply_TFLOPs"] / roof
        if dtp == torch.complex64:
            rec["apply_frac_fp32_nonpacked_issue"] = rec["apply_TFLOPs"] / FP32_NONPACKED_PEAK_TFLOPS
        rec["share_outside_apply"] = 1.0 - ms / 1e3 / wall
        out[name] = rec
    out["max_abs_dF_c64_vs_c128"] = float(abs(F["block_c64"] - F["block_c128"]).max())
    out["max_abs_dF_block_vs_single_c128"] = float(abs(F["block_c128"][:, 0] - F["single_c128"][:, 0]).max())
    out["speedup_per_vector_c64_block_vs_single_c128"] = (out["block_c64"]["vector_steps_per_s"] /
                                                          out["single_c128"]["vector_steps_per_s"])
    out["speedup_per_vector_c128_block_vs_single_c128"] = (out["block_c128"]["vector_steps_per_s"] /
                                                           out["single_c128"]["vector_steps_per_s"])
    T.close()
    return out


def n60_leg(api, inputs, torch, dev):
    """Largest single-GPU size: N=60 (dim 2^30, 487,635 couplings, 16 GiB per
    complex128 state): one apply_H in each precision and one Lanczos step of two
    iterations (complex128), on a seeded random state drawn on the device."""
    N = 60
    T = api.Terms(N, inputs.couplings(N, 0))
    out = {"N": N, "dim": T.dim, "n_masks": T.n_masks}
    g = torch.Generator(device=dev).manual_seed(1)
    x = torch.randn(T.dim, dtype=torch.complex128, device=dev, generator=g)
    x /= torch.linalg.vector_norm(x)
    y = torch.empty_like(x)

    def timed(fn):
        torch.cuda.synchronize()
        api.timing_reset()
        api.timing_enable(True)
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        api.timing_enable(False)
        n, ms = api.timing_read()
        api.timing_reset()
        return wall, n, ms

    api.apply_H(T, x, y)   # first call: launch tables and the diagonal of H
    _, n, ms = timed(lambda: api.apply_H(T, x, y))
    out["apply_c128_ms"] = ms / n
    wall, _, _ = timed(lambda: api.krylov_expmv(T, x, -1j, 0.01, m=2, dt=0.01))
    out["lanczos_m2_c128_s"] = wall
    del y
    x64 = x.to(torch.complex64)
    del x
    torch.cuda.empty_cache()
    y64 = torch.empty_like(x64)
    api.apply_H(T, x64, y64)
    _, n, ms = timed(lambda: api.apply_H(T, x64, y64))
    out["apply_c64_ms"] = ms / n
    del x64, y64
    T.close()
    torch.cuda.empty_cache()
    return out


def grad_leg(api, inputs, torch, dev, N, t_star, degree, dt, beta):
    """Cost of dF/dJ for every coupling against the Chebyshev forward alone."""
    J = inputs.couplings(N, 0)
    T = api.Terms(N, J)
    psi = torch.from_numpy(inputs.typical_state(N, 1)).to(dev)
    lo, hi = api.spectrum_bounds(T, psi, 60)
    o = api.cheb_opts(degree=degree, dt=dt, tau_steps=1, checkpoint_every=10, e_halfwidth=1.1 * max(abs(lo), abs(hi)))
    api.cheb_otoc(T, 0, 1, beta, t_star, psi, o)            # warmup
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    F = api.cheb_otoc(T, 0, 1, beta, t_star, psi, o)
    torch.cuda.synchronize()
    tf = time.perf_counter() - t0
    t0 = time.perf_counter()
    F2, g = api.grad_couplings(T, 0, 1, beta, t_star, psi, o)
    torch.cuda.synchronize()
    tg = time.perf_counter() - t0
    T.close()
    return {"N": N, "t_star": t_star, "degree": degree, "dt": dt, "beta": beta, "n_couplings": int(g.size),
            "forward_s": tf, "grad_s": tg, "grad_fwd_ratio": tg / tf, "F": F, "F_from_grad_call": F2}


def cpu_rows_seconds(N, J, psi_host, rows):
    """Seconds the CPU checker takes for rows [0, rows) of H psi (all its threads)."""
    from oracle import native
    t0 = time.perf_counter()
    native.apply_range(N, J, psi_host, 0, rows)
    return time.perf_counter() - t0


_ONE_CORE = """
import json, sys, time
sys.path.insert(0, {root!r})
from oracle import native
from paper_2002_05725_amd import inputs
N, rows = {N}, {rows}
J = inputs.couplings(N, 0)
psi = inputs.typical_state(N, 1)
native.apply_range(N, J, psi, 0, 64)
t0 = time.perf_counter()
native.apply_range(N, J, psi, 0, rows)
print(json.dumps({{"seconds": time.perf_counter() - t0, "threads": native.num_threads()}}))
"""


def cpu_one_core(N, rows):
    """The same sample on one core (OpenMP limited to one thread in a child process)."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", _ONE_CORE.format(root=ROOT, N=N, rows=rows)], env=env,
                       capture_output=True, text=True, timeout=600)
    if r.returncode != 0:
        return None
    return json.loads(r.stdout.strip().splitlines()[-1])


def cpu_baseline(N, J, psi_host, m, target_s):
    """The CPU checker's term-by-term apply on a contiguous block of rows,
    scaled to one full apply, times m applications per time step; also on one
    core."""
    from oracle import native
    D = psi_host.size
    t0 = time.perf_counter()
    native.apply_range(N, J, psi_host, 0, 4096)         # calibration
    rate = 4096 / max(time.perf_counter() - t0, 1e-6)
    rows = int(min(D, max(256, rate * target_s)))
    t = cpu_rows_seconds(N, J, psi_host, rows)
    t_apply = t / rows * D
    out = {
        "value": 1.0 / (m * t_apply),
        "unit": "time-steps/s",
        "cores": native.num_threads(),
        "kind": "oracle",
        "sample": (f"term-by-term H|psi> on rows [0, {rows}) of the N={N} apply ({t:.1f} s), "
                   f"scaled by dim/rows to {t_apply:.1f} s per apply (extrapolated), times m={m} applies per "
                   "step; Gram-Schmidt and combination not counted"),
    }
    rows1 = max(64, rows // max(1, native.num_threads()))
    one = cpu_one_core(N, rows1)
    if one:
        t1 = one["seconds"] / rows1 * D
        out["one_core"] = {"value": 1.0 / (m * t1), "cores": one["threads"], "apply_s_extrapolated": t1,
                           "sample": f"rows [0, {rows1}) on one thread ({one['seconds']:.1f} s)"}
    return out


def cpu_full_applies(api, inputs, torch, dev):
    """Whole applies beside the GPU at sizes the checker finishes: N = 32 in
    full on all cores; N = 44 on a block of 2^14 rows, extrapolated."""
    from oracle import native
    out = []
    for N, rows in ((32, None), (44, 1 << 14)):
        J = inputs.couplings(N, 0)
        psi = inputs.typical_state(N, 1)
        D = psi.size
        T = api.Terms(N, J)
        x = torch.from_numpy(psi).to(dev)
        y = torch.empty_like(x)
        api.apply_H(T, x, y)
        torch.cuda.synchronize()
        api.timing_reset()
        api.timing_enable(True)
        for _ in range(5):
            api.apply_H(T, x, y)
        torch.cuda.synchronize()
        api.timing_enable(False)
        n, ms = api.timing_read()
        api.timing_reset()
        T.close()
        n_rows = D if rows is None else rows
        t = cpu_rows_seconds(N, J, psi, n_rows)
        rec = {"N": N, "gpu_apply_ms": ms / n, "cpu_cores": native.num_threads(),
               "cpu_apply_s": t * D / n_rows, "cpu_rows_timed": n_rows,
               "extrapolated": rows is not None}
        rec["gpu_speedup"] = rec["cpu_apply_s"] / (rec["gpu_apply_ms"] / 1e3)
        out.append(rec)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--N", type=int, default=52)
    ap.add_argument("--m", type=int, default=12)
    ap.add_argument("--dt", type=float, default=0.25)
    ap.add_argument("--c64-steps", type=int, default=2,
                    help="timed complex64 steps after one warmup step; the complex64 state is compared with the "
                         "complex128 state after the same number of steps")
    ap.add_argument("--no-window", action="store_true",
                    help="skip the F(t) window of the OTOC at N in both precisions")
    ap.add_argument("--sector-steps", type=int, default=1,
                    help="time steps of the parity-sector leg (complex128, half-size state; 0: skip)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch-N", type=int, default=40, help="size of the batched leg (0: skip)")
    ap.add_argument("--grad-N", type=int, default=44, help="size of the gradient leg (0: skip)")
    ap.add_argument("--grad-t", type=float, default=0.5,
                    help="t* of the gradient leg (a multiple of dt = 0.1; the cost ratio barely depends on it)")
    ap.add_argument("--no-n60", action="store_true", help="skip the N=60 leg (dim 2^30)")
    ap.add_argument("--profile-apply", type=int, default=0,
                    help="only run this many apply_H calls and one 1 GiB device copy "
                         "(for hardware-counter runs), then exit")
    ap.add_argument("--profile-dtype", choices=("c128", "c64"), default="c128",
                    help="state precision of the --profile-apply calls")
    ap.add_argument("--profile-block", type=int, default=0,
                    help="only run this many apply_H calls on the batched leg's 64-column block (--batch-N, "
                         "--profile-dtype) with one column per workgroup, then as many with two columns of "
                         "one realisation per workgroup (2048-row tiles), and exit (for kernel-trace runs)")
    ap.add_argument("--profile-bins", type=int, default=0,
                    help="only run this many derivative-bin calls (32 pairs of seeded random states at the "
                         "gradient leg's N) and exit (for kernel-trace and counter runs)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the sharded design is described, not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2002_05725_amd import api, inputs

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    dev = torch.device("cuda:0")
    if args.profile_block > 0:
        Nk, R = args.batch_N, 32
        Tk = api.Terms(Nk, np.stack([inputs.couplings(Nk, inputs.batch_coupling_seed(Nk, r)) for r in range(R)]))
        real = np.repeat(np.arange(R), 2)
        dtp = torch.complex128 if args.profile_dtype == "c128" else torch.complex64
        x = torch.from_numpy(np.stack([inputs.typical_state(Nk, inputs.batch_state_seed(Nk, r, s))
                                       for r in range(R) for s in range(2)])).to(dev).to(dtp)
        out = torch.empty_like(x)
        for nc in (1, 2):
            api.set_apply_tuning(Tk, 11, 1, nc)
            for k in range(args.profile_block):
                api.apply_H(Tk, x, out, real_of_col=real)
                torch.cuda.synchronize()
                log(f"[bench] block apply, {nc} column(s) per workgroup: {k + 1}/{args.profile_block} done")
        print(json.dumps({"profile_block": args.profile_block, "dtype": args.profile_dtype, "N": Nk,
                          "columns": 64, "realisations": R}), flush=True)
        return
    if args.profile_bins > 0:
        Nb = args.grad_N
        Tb = api.Terms(Nb, inputs.couplings(Nb, 0))
        gen = torch.Generator(device=dev).manual_seed(3)
        vs = [torch.randn(Tb.dim, dtype=torch.complex128, device=dev, generator=gen) for _ in range(64)]
        pairs = [(vs[2 * p], vs[2 * p + 1], 1.0) for p in range(32)]
        for k in range(args.profile_bins):
            api.coupling_overlaps(Tb, pairs)
            torch.cuda.synchronize()
            log(f"[bench] bins call {k + 1}/{args.profile_bins} done")
        print(json.dumps({"profile_bins": args.profile_bins, "N": Nb, "pairs": 32}), flush=True)
        return
    N, m, dt = args.N, args.m, args.dt
    log(f"[bench] N={N}: drawing couplings and state")
    J = inputs.couplings(N, 0)
    psi_host = inputs.typical_state(N, 1)
    D = psi_host.size
    T = api.Terms(N, J)
    log(f"[bench] dim={D} terms={T.n_terms} masks={T.n_masks}")

    psi = torch.from_numpy(psi_host).to(dev)
    if args.profile_apply > 0:
        x = psi if args.profile_dtype == "c128" else psi.to(torch.complex64)
        out = torch.empty_like(x)
        for k in range(args.profile_apply):
            api.apply_H(T, x, out)
            torch.cuda.synchronize()
            log(f"[bench] apply {k + 1}/{args.profile_apply} done")
        a = torch.empty(1 << 27, dtype=torch.float64, device=dev)   # 1 GiB
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"profile_apply": args.profile_apply, "dtype": args.profile_dtype, "N": N,
                          "copy_bytes": 1 << 30}), flush=True)
        return
    log(f"[bench] complex128: {args.warmup} warmup + {args.steps} timed steps (m={m}, dt={dt})")
    # the complex128 state after as many steps as the complex64 leg takes, for
    # its error (one device copy; inside the timed region only when the warmup
    # is shorter than the complex64 leg)
    n_cmp = 1 + args.c64_steps if args.c64_steps > 0 else 0
    snap = {}

    def keep_state(k):
        if k == n_cmp:
            snap["psi"] = psi.clone()

    wall, n_apply, apply_ms = timed_leg(api, torch, T, psi, args.steps, args.warmup, m, dt, after=keep_state)
    norm = float(torch.linalg.vector_norm(psi))
    if not math.isfinite(norm) or abs(norm - 1) > 1e-9:
        raise SystemExit(f"unitarity check failed: |psi| = {norm}")
    ms_step = wall / args.steps * 1e3
    avg_apply_s = apply_ms / n_apply / 1e3
    alg_bytes = (T.n_masks + 1) * D * 16
    effective = alg_bytes / avg_apply_s / 1e9
    alu_tflops = FLOPS_PER_PAIR * T.n_masks * D / avg_apply_s / 1e12
    log(f"[bench] c128: {ms_step:.0f} ms/step, apply {avg_apply_s * 1e3:.1f} ms")

    c64 = None
    if args.c64_steps > 0:
        torch.cuda.empty_cache()
        p64 = torch.from_numpy(psi_host).to(dev).to(torch.complex64)
        log(f"[bench] complex64: 1 warmup + {args.c64_steps} timed steps")
        w64, n64, ms64 = timed_leg(api, torch, T, p64, args.c64_steps, 1, m, dt)
        a64 = ms64 / n64 / 1e3
        c64 = {
            "otoc_time_steps_per_s": args.c64_steps / w64,
            "ms_per_step": w64 / args.c64_steps * 1e3,
            "apply_ms": a64 * 1e3,
            "apply_alg_GBps": (T.n_masks + 1) * D * 8 / a64 / 1e9,
        }
        c64["apply_pct_hbm_peak"] = 100 * c64["apply_alg_GBps"] / HBM_PEAK_GBS
        c64["apply_TFLOPs"] = FLOPS_PER_PAIR * T.n_masks * D / a64 / 1e12
        c64["apply_frac_fp32_vector_peak"] = c64["apply_TFLOPs"] / FP32_VECTOR_PEAK_TFLOPS
        c64["apply_frac_fp32_nonpacked_issue"] = c64["apply_TFLOPs"] / FP32_NONPACKED_PEAK_TFLOPS
        # precision of the complex64 form: the same state propagated by the same
        # number of steps in both precisions
        if "psi" in snap:
            ref = snap.pop("psi")
            diff = torch.linalg.vector_norm(p64.to(torch.complex128) - ref).item()
            c64["rel_state_error_vs_c128"] = diff / torch.linalg.vector_norm(ref).item()
            c64["steps_compared"] = n_cmp
            del ref
        del p64
        log(f"[bench] c64: {c64['ms_per_step']:.0f} ms/step, apply {a64 * 1e3:.1f} ms")

    del psi
    snap.clear()
    window = None
    if not args.no_window:
        window = beta10_window_leg(api, torch, T, psi_host, dev, N)
        log(f"[bench] window: |dF| c64 vs c128 = {window['max_abs_dF_c64_vs_c128']:.2e}")
    sector = None
    if args.sector_steps > 0:
        torch.cuda.empty_cache()
        u_host = inputs.typical_sector_state(N, 0, 1)
        u = torch.from_numpy(u_host).to(dev)
        del u_host
        log(f"[bench] parity sector 0: 1 warmup + {args.sector_steps} timed steps")
        api.krylov_expmv(T, u, -1j, dt, m=m, dt=dt, sector=0)
        torch.cuda.synchronize()
        api.timing_reset()
        api.timing_enable(True)
        t0 = time.perf_counter()
        for _ in range(args.sector_steps):
            api.krylov_expmv(T, u, -1j, dt, m=m, dt=dt, sector=0)
        torch.cuda.synchronize()
        ws = time.perf_counter() - t0
        api.timing_enable(False)
        ns, mss = api.timing_read()
        api.timing_reset()
        sector = {"sector": 0, "dim": D // 2, "otoc_time_steps_per_s": args.sector_steps / ws,
                  "ms_per_step": ws / args.sector_steps * 1e3, "apply_ms": mss / ns}
        del u
        log(f"[bench] sector: {sector['ms_per_step']:.0f} ms/step, apply {sector['apply_ms']:.1f} ms")

    batched = None
    if args.batch_N > 0:
        torch.cuda.empty_cache()
        log(f"[bench] batched leg: N={args.batch_N}, 32 realisations x 2 states")
        batched = batched_leg(api, inputs, torch, np, dev, args.batch_N, 16, 0.5)
        log(f"[bench] batched: |dF| c64 vs c128 {batched['max_abs_dF_c64_vs_c128']:.2e}")
    grad = None
    if args.grad_N > 0:
        torch.cuda.empty_cache()
        log(f"[bench] gradient leg: N={args.grad_N}")
        grad = grad_leg(api, inputs, torch, dev, args.grad_N, args.grad_t, 32, 0.1, 5.0)
        log(f"[bench] grad/fwd = {grad['grad_fwd_ratio']:.2f}")

    n60 = None
    if not args.no_n60:
        torch.cuda.empty_cache()
        log("[bench] N=60 leg: one apply_H per precision, one m=2 Lanczos step")
        try:
            n60 = n60_leg(api, inputs, torch, dev)
            log(f"[bench] N=60: apply {n60['apply_c128_ms']:.0f} ms (c128), {n60['apply_c64_ms']:.0f} ms (c64)")
        except (RuntimeError, MemoryError) as e:   # reported, not fatal to the headline
            n60 = {"error": str(e)[:300]}
            log(f"[bench] N=60 leg failed: {e}")

    traffic = traffic_from_profile(f"N{N}_c128")
    hbm_gbs = traffic / avg_apply_s / 1e9 if traffic else None
    out = {
        "metric": METRIC,
        "value": args.steps / wall,
        "unit": "time-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128",
        "data": "synthetic",
        "config": {
            "workload": f"OTOC Lanczos time step at N={N} (dim 2^{N // 2}, {T.n_terms} couplings), "
                        f"m={m}, dt={dt}, complex128 state, FP64 inner products",
            "N": N, "dim": D, "n_terms": T.n_terms, "n_masks": T.n_masks, "m": m, "dt": dt,
            "couplings_seed": 0, "state_seed": 1,
        },
        "apply_H": {
            "ms": avg_apply_s * 1e3,
            "launches_timed": n_apply,
            "hbm_GBps_measured": hbm_gbs,
            "hbm_pct_peak_measured": 100 * hbm_gbs / HBM_PEAK_GBS if hbm_gbs else None,
            "hbm_bytes_measured": traffic,
            "effective_GBps_byte_model": effective,
            "effective_pct_hbm_peak_byte_model": 100 * effective / HBM_PEAK_GBS,
            "byte_model": "(n_masks + 1) * dim * 16 B: one HBM gather per flip mask; LDS staging reuses each "
                          "source tile across the masks of a chunk, so this effective rate is not a bandwidth",
            "binding_roof": "FP64 vector ALU (see roofline)",
        },
        "roofline": {
            "bound": "alu",
            "achieved": alu_tflops,
            "peak": FP64_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": alu_tflops / FP64_VECTOR_PEAK_TFLOPS,
            "traffic": traffic,
            "flops_model": f"{FLOPS_PER_PAIR} flops (one complex FMA) per (row, flip mask) pair, n_masks * dim "
                           "pairs per apply_H call",
            "unit_of_work": "one apply_H call (k_apply natural layout + k_apply rotated layout + 2 transposes), "
                            "HIP events on the call's stream",
            "traffic_unit": "bytes per apply_H call (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
        },
        "complex64": c64,
        "otoc_window": window,
        "parity_sector": sector,
        "batched": batched,
        "gradient": grad,
        "grad_fwd_ratio": grad["grad_fwd_ratio"] if grad else None,
        "n60": n60,
    }
    T.close()
    if not args.no_cpu_baseline:
        log("[bench] CPU checker baseline")
        out["cpu_baseline"] = cpu_baseline(N, J, psi_host, m, args.cpu_seconds)
        log("[bench] CPU checker full applies")
        out["cpu_baseline"]["full_applies"] = cpu_full_applies(api, inputs, torch, dev)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
