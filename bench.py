#!/usr/bin/env python3
"""Benchmark of the reduced implicit-Euler Newton iteration on one MI355X.

Workload (one "step" = one implicit-Euler time step = weight net + 4 full
Newton iterations, each: decoder jets, output layer, cubature, mass terms,
sums, complex-step backpropagation, assemble + FP64 LU + update):
  10,000-vertex bar (20 x 20 x 25 grid, 43,320 tets), r = n_q = 15, ELU
  decoder [15, 64, 128, 256, 512 x 5, 256, 30000], 500 cubature tets with
  weights from a 15 -> 64 -> 64 -> 500 softplus weight net, FP32, single
  instance.  Inputs are seeded synthetic data already resident in HBM.

Prints ONE JSON line.  `value` = Newton iterations per second of that single
FP32 instance; `variants` adds the BF16 form and batched forms (instances
sharing the decoder advanced by one launch sequence), `roofline` the dominant
kernel measured live with HIP events, `cpu_baseline` the FP64 oracle timed on
a bounded sample on this host's cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "reduced Newton iters/s at n=10k,r=15 (batched vs plain, BF16 vs FP32); p99 step ms"
ITERS = 4
HBM_PEAK_GBS = 8000.0
FP32_MFMA_PEAK_TFLOPS = 157.3
BF16_MFMA_PEAK_TFLOPS = 2500.0
FRAME_BUDGET_MS = 1000.0 / 60.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def phase_roofline(p, inst, phase: str, us: float, prec: str):
    """Algorithmic bytes / flops of one launch of a phase's kernel.

    dec_out  (k_fwd_out): reads W_L [N x K] once, the folded activations
             [Cf x K], bias and mask [N]; writes the DOF records [N x Cf];
             2 N K Cf flops with Cf = 2 n_q + 2.
    bwd_out  (k_bwd_out): reads W_L [N x K] and the seed [N]; writes one
             K-vector partial per 128 rows; 2 N K flops.
    """
    N = p.N
    K = p.weights[-1].shape[1]
    nq = p.n_q
    cf = 2 * nq + 2
    sw = 2 if prec == "bf16" else 4
    if phase == "dec_out":
        byts = N * K * sw + cf * K * 4 + 2 * N * 4 + N * cf * 4
        flops = 2.0 * N * K * cf
    elif phase == "bwd_out":
        nblk = (N + 127) // 128
        byts = N * K * sw + N * 4 + nblk * K * 8
        flops = 2.0 * N * K
    else:
        return None
    ai = flops / byts
    ridge = (BF16_MFMA_PEAK_TFLOPS if prec == "bf16" else FP32_MFMA_PEAK_TFLOPS) * 1e12 / (HBM_PEAK_GBS * 1e9)
    if ai < ridge:
        ach = byts / (us * 1e-6) / 1e9
        return dict(bound="hbm", achieved=round(ach, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(ach / HBM_PEAK_GBS, 4), traffic=None, kernel=phase, us_per_launch=round(us, 3),
                    algorithmic_bytes_per_launch=int(byts), algorithmic_flops_per_launch=int(flops))
    peak = BF16_MFMA_PEAK_TFLOPS if prec == "bf16" else FP32_MFMA_PEAK_TFLOPS
    ach = flops / (us * 1e-6) / 1e12
    return dict(bound="mfma", achieved=round(ach, 3), peak=peak, unit="TFLOP/s", frac=round(ach / peak, 4),
                traffic=None, kernel=phase, us_per_launch=round(us, 3),
                algorithmic_bytes_per_launch=int(byts), algorithmic_flops_per_launch=int(flops))


def run_steps(nmr, ctx, insts, steps: int, warmup: int):
    import torch
    if warmup:
        st, _ = nmr.step_many(ctx, insts, warmup, ITERS, timings=False)
        assert all(s == 0 for s in st), st
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, ms = nmr.step_many(ctx, insts, steps, ITERS, timings=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    assert all(s == 0 for s in st), st
    return t1 - t0, np.asarray(ms)


def cpu_baseline(p, seconds: float):
    """The FP64 oracle, untuned, on this host's cores: Newton iterations of the
    same problem from its initial state until about `seconds` have passed."""
    from threadpoolctl import threadpool_info
    from oracle.newton import Instance as OracleInstance
    oi = OracleInstance(p)
    st = oi.initial_state()
    n = 0
    t0 = time.perf_counter()
    while True:
        st, _ = oi.step(st, ITERS)
        n += ITERS
        if time.perf_counter() - t0 > seconds:
            break
    dt = time.perf_counter() - t0
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    return dict(value=round(n / dt, 4), unit="Newton iters/s", cores=int(threads), kind="oracle",
                sample=f"first {n // ITERS} implicit-Euler steps x {ITERS} Newton iterations of the same "
                       f"10k-vertex problem (FP64 numpy/BLAS oracle), {dt:.1f} s")


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--batch", type=int, nargs="*", default=[16])
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the path has no multi-GPU form (instances would shard "
              "across GPUs with no exchange); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2102_11026_amd import nmr, synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    nmr.lib()
    log("generating the 10k-vertex problem")
    p = synth.config_single_10k()
    ctx = nmr.Context(0)
    inst = nmr.Instance(ctx, p, "fp32")
    log("timing the plain FP32 instance")
    secs, ms = run_steps(nmr, ctx, [inst], args.steps, args.warmup)
    value = ITERS * args.steps / secs
    out = dict(metric=METRIC, value=round(value, 2), unit="Newton iters/s", n_gpus=1, steps=args.steps,
               warmup=args.warmup, ms_per_step=round(1000.0 * secs / args.steps, 4), higher_is_better=True,
               scaling="weak", vs_baseline=None, dtype="f32", data="synthetic",
               config=dict(workload="bar10k_r15: 20x20x25-vertex bar (10,000 vertices, 43,320 tets), "
                                    "r = n_q = 15, ELU decoder [15,64,128,256,512x5,256,30000], 500 cubature "
                                    "tets weighted by a softplus weight net, 4 Newton iterations per step, "
                                    "one instance",
                           n_vertices=p.n, r=p.R, newton_iters_per_step=ITERS, precision="fp32",
                           instances=1),
               p50_step_ms=round(float(np.percentile(ms, 50)), 4),
               p99_step_ms=round(float(np.percentile(ms, 99)), 4),
               frame_budget_ms=round(FRAME_BUDGET_MS, 2),
               frames_per_s=round(args.steps / secs, 2))
    # per-phase device time (HIP events on the library's stream)
    phases = {}
    for k, name in enumerate(nmr.PHASES):
        phases[name] = round(inst.time_phase(k, reps=50), 3)
    out["phase_us"] = phases
    cand = {k: v for k, v in phases.items() if k in ("dec_out", "bwd_out")}
    dom = max(cand, key=cand.get)
    out["roofline"] = phase_roofline(p, inst, dom, phases[dom], "fp32")
    log("phases (us):", phases)

    if not args.no_variants:
        var = {}
        ib = nmr.Instance(ctx, p, "bf16")
        s_b, ms_b = run_steps(nmr, ctx, [ib], max(args.steps // 2, 10), 3)
        nb = max(args.steps // 2, 10)
        var["plain_bf16"] = dict(newton_iters_per_s=round(ITERS * nb / s_b, 2),
                                 p99_step_ms=round(float(np.percentile(ms_b, 99)), 4))
        bphase = {name: round(ib.time_phase(k, reps=50), 3) for k, name in enumerate(nmr.PHASES)}
        var["plain_bf16"]["phase_us"] = bphase
        ib.close()
        for prec in ("fp32", "bf16"):
            dec = nmr.Decoder(ctx, p.weights, p.biases, p.act, prec)
            for B in args.batch:
                insts = []
                for k in range(B):
                    r0 = np.zeros(p.R)
                    r0[p.n_p:] = 0.1 * synth.normal(f"q0/{k}", p.n_q)
                    insts.append(nmr.Instance(ctx, p.replace(r0=r0), prec, shared=dec))
                nsteps = max(args.steps // 5, 5)
                s_m, ms_m = run_steps(nmr, ctx, insts, nsteps, 2)
                var[f"batched_{prec}_B{B}"] = dict(
                    newton_iters_per_s=round(ITERS * nsteps * B / s_m, 2),
                    p50_step_ms=round(float(np.percentile(ms_m, 50)), 4),
                    p99_step_ms=round(float(np.percentile(ms_m, 99)), 4))
                for x in insts:
                    x.close()
            dec.close()
        out["variants"] = var
        log("variants:", var)
    inst.close()
    ctx.close()
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on the host")
        out["cpu_baseline"] = cpu_baseline(p, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
