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
PHASE_KERNEL = dict(dec_hidden="k_fwd_hidden", dec_out="k_fwd_out", bwd_out="k_bwd_out", bwd_hidden="k_bwd_hidden")
# Bytes per launch that reach the memory side of L2 on the FP32 10k-vertex
# bar, from two rocprofv3 --pmc runs (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0, the
# factors a plain 512 MiB device copy gives), averaged over one pass of the
# phase; see profiles/k_fwd_hidden_bar10k_fp32_pmc.md.  They hold only for the
# kernel sources they were taken on: with any other sources traffic is null.
MEASURED_TRAFFIC = dict(k_fwd_hidden=1634304, k_bwd_hidden=972676, k_fwd_out=6220032, k_bwd_out=5776384)
MEASURED_TRAFFIC_SOURCES = "74f3584eaa7a3f1b"
KERNEL_SOURCES = ("paper_2102_11026_amd/csrc/decoder.hip", "paper_2102_11026_amd/csrc/nmr_internal.h")


def kernel_sources_digest() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cubature_dofs(p) -> int:
    """DOFs of the cubature tets: the rows the Gram-folded path decodes."""
    v = np.unique(np.asarray(p.tets)[np.asarray(p.cub_ids)].ravel())
    return 3 * v.size


def phase_work(p, phase: str, prec: str, gram: bool):
    """(algorithmic bytes, algorithmic flops, launches) of one pass of a phase.

    Widths are the decoder's own (unpadded); C = 4 + 4 n_q jet channels
    forward, 1 + n_q channels backward, Cf = 2 + 2 n_q folded channels.
    dec_hidden (k_fwd_hidden, one launch per hidden layer): reads W_l, b_l and
        the input jets [C x m_in], writes the output jets [C x m_out] (the
        folded channels [Cf x m_out] after the last hidden layer) and the
        pre-activation jets [(1 + n_q) x m_out]; 2 m_out m_in C flops.
    bwd_hidden (k_bwd_hidden, one launch per hidden layer): reads W_l, the
        seed [(1 + n_q) x m_out] and the pre-activations, writes the seed of
        the layer below [(1 + n_q) x m_in]; 2 m_out m_in (1 + n_q) flops.
    dec_out (k_fwd_out): reads the rows of W_L that are decoded (all N, or
        the cubature DOFs on the Gram-folded path), the folded activations
        [Cf x K], bias and mask of those rows, writes their records [rows x
        Cf]; 2 rows K Cf flops.
    bwd_out (k_bwd_out): reads the same rows of W_L and their seeds, writes
        one K-vector partial per 128 rows for each of the 1 + n_q channels;
        2 rows K (1 + n_q) flops.
    """
    nq = p.n_q
    sw = 2 if prec == "bf16" else 4
    Ws = p.weights
    L = len(Ws)
    C, Cb, Cf = 4 + 4 * nq, 1 + nq, 2 + 2 * nq
    if phase == "dec_hidden":
        byts = flops = 0.0
        for l in range(L - 1):
            mo, mi = Ws[l].shape
            cout = Cf if l == L - 2 else C
            byts += mo * mi * sw + mo * 4 + C * mi * 4 + cout * mo * 4 + Cb * mo * 4
            flops += 2.0 * mo * mi * C
        return byts, flops, L - 1
    if phase == "bwd_hidden":
        byts = flops = 0.0
        for l in range(L - 1):
            mo, mi = Ws[l].shape
            byts += mo * mi * sw + 2 * Cb * mo * 4 + Cb * mi * 4
            flops += 2.0 * mo * mi * Cb
        return byts, flops, L - 1
    K = Ws[-1].shape[1]
    rows = cubature_dofs(p) if gram else p.N
    if phase == "dec_out":
        return rows * K * sw + Cf * K * 4 + 2 * rows * 4 + rows * Cf * 4, 2.0 * rows * K * Cf, 1
    if phase == "bwd_out":
        nblk = (rows + 127) // 128
        return rows * K * sw + rows * 4 + nblk * K * Cb * 4, 2.0 * rows * K * Cb, 1
    return None


def phase_roofline(p, phase: str, us: float, prec: str, gram: bool):
    """Roofline of one launch of a phase's kernel, `us` being the phase's
    device time (all its launches).  The bound follows the arithmetic
    intensity against the ridge point of the MFMA peak of the phase's dtype."""
    w = phase_work(p, phase, prec, gram)
    if w is None:
        return None
    byts, flops, launches = w
    byts /= launches
    flops /= launches
    us_l = us / launches
    peak_tf = BF16_MFMA_PEAK_TFLOPS if prec == "bf16" else FP32_MFMA_PEAK_TFLOPS
    ridge = peak_tf * 1e12 / (HBM_PEAK_GBS * 1e9)
    traffic = None
    if prec == "fp32" and gram and kernel_sources_digest() == MEASURED_TRAFFIC_SOURCES:
        traffic = MEASURED_TRAFFIC.get(PHASE_KERNEL[phase])
    common = dict(traffic=traffic, traffic_unit="bytes per launch", kernel=PHASE_KERNEL[phase], phase=phase,
                  launches_per_pass=launches,
                  us_per_launch=round(us_l, 3), algorithmic_bytes_per_launch=int(byts),
                  algorithmic_flops_per_launch=int(flops), arithmetic_intensity=round(flops / byts, 2),
                  ridge=round(ridge, 2))
    if flops / byts < ridge:
        ach = byts / (us_l * 1e-6) / 1e9
        return dict(bound="hbm", achieved=round(ach, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(ach / HBM_PEAK_GBS, 4), **common)
    ach = flops / (us_l * 1e-6) / 1e12
    return dict(bound="mfma", achieved=round(ach, 3), peak=peak_tf, unit="TFLOP/s", frac=round(ach / peak_tf, 4),
                **common)


def tile_report(nmr, ctx, p):
    """The autotuned tiles of the batched forward jet layers, each with its
    algorithmic MFMA rate (2 w_out w_in (4 + 4 n_q) flops per instance, true
    widths) against the peak of its precision."""
    w = [p.weights[0].shape[1]] + [W.shape[0] for W in p.weights]
    pad = lambda x: -(-x // 32) * 32
    cols = 4 + 4 * p.n_q
    out = []
    for e in ctx.tiling_table():
        if not e["forward"]:
            continue
        layers = [l for l in range(len(w) - 2) if pad(w[l]) == e["m_in"] and pad(w[l + 1]) == e["m_out"]]
        if not layers:
            continue
        l = layers[0]
        flops = 2.0 * w[l] * w[l + 1] * cols * e["n_inst"]
        peak = BF16_MFMA_PEAK_TFLOPS if e["prec"] == nmr.PREC["bf16"] else FP32_MFMA_PEAK_TFLOPS
        tf = flops / (e["us"] * 1e-6) / 1e12
        out.append(dict(prec={v: k for k, v in nmr.PREC.items()}[e["prec"]], instances=e["n_inst"],
                        layer=f"{w[l]}->{w[l + 1]}", ib=e["ib"], mr=e["mr"], jet_groups=e["jet_groups"], us_per_launch=round(e["us"], 2),
                        tflops=round(tf, 2), frac_of_mfma_peak=round(tf / peak, 4)))
    return out


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


def cpu_baseline(p, seconds: float, threads: int = 0):
    """The FP64 oracle, untuned, on this host's cores: Newton iterations of the
    same problem from its initial state until about `seconds` have passed
    (threads > 0: with the BLAS pools limited to that many threads)."""
    from threadpoolctl import threadpool_info, threadpool_limits
    from oracle.newton import Instance as OracleInstance
    oi = OracleInstance(p)
    st = oi.initial_state()
    n = 0
    with threadpool_limits(limits=threads if threads > 0 else None):
        used = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
        t0 = time.perf_counter()
        while True:
            st, _ = oi.step(st, ITERS)
            n += ITERS
            if time.perf_counter() - t0 > seconds:
                break
        dt = time.perf_counter() - t0
    return dict(value=round(n / dt, 4), unit="Newton iters/s", cores=int(used), kind="oracle",
                sample=f"first {n // ITERS} implicit-Euler steps x {ITERS} Newton iterations of the same "
                       f"10k-vertex problem (FP64 numpy/BLAS oracle), {dt:.1f} s")


def rel(a, b) -> float:
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


GOLDEN = os.path.join(ROOT, "tests", "golden", "bar10k_trajectory_fp64.npz")


def training_report(nmr, ctx, n_poses: int, cpu: bool = True):
    """Neural cubature training (Sec. 5) on the 10,000-vertex bar: training
    data of n_poses poses (FP32 decoder derivatives, FP64 element forces), then
    alternations of 15 epochs per net (FP64).  The dominant kernel is the
    selection net's element backward pass; its algorithmic bytes per launch
    are the element forces F (P m R doubles), the stored logits (P m), the
    element adjoints it writes (P m 8) and the vertex features it gathers
    (P n 8)."""
    import torch
    from paper_2102_11026_amd import synth
    t = synth.config_cubature_bar10k(n_poses)
    inst = nmr.Instance(ctx, t.prob, "fp32")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tr = nmr.Trainer(inst, t.poses, t.wnet_weights, t.wnet_biases, t.scale, t.theta, t.n_c0, t.K, t.epochs)
    create_s = time.perf_counter() - t0
    lw0, ls0, _, _ = tr.run(1)
    lw, ls, added, ms = tr.run(2)
    alt_ms = ms / 2
    ph = {k: tr.time_phase(k, 3) for k in nmr.TRAIN_PHASES}
    P, m, n, R = n_poses, int(t.prob.tets.shape[0]), t.prob.n, t.prob.R
    bwd_bytes = 8.0 * P * (m * R + m + 8 * m + 8 * n)
    achieved = bwd_bytes / (ph["s_elem_bwd"] * 1e-6) / 1e9
    C, _, _, _ = tr.get()
    out = dict(poses=P, tets=m, R=R, epochs_per_net=t.epochs, K=t.K, cubature_elements=len(C),
               training_data_s=round(create_s, 3), training_data_gb=round(8.0 * P * m * R / 1e9, 3),
               alternation_ms=round(alt_ms, 2), pose_epochs_per_s=round(P * 2 * t.epochs / (alt_ms / 1e3), 1),
               s_epoch_ms=round(ph["s_epoch"] / 1e3, 3), w_epoch_ms=round(ph["w_epoch"] / 1e3, 3),
               s_elem_fwd_ms=round(ph["s_elem_fwd"] / 1e3, 3), s_elem_bwd_ms=round(ph["s_elem_bwd"] / 1e3, 3),
               loss_w_first_last=[round(float(lw0[0][0]), 5), round(float(lw[-1][-1]), 5)],
               loss_s_first_last=[round(float(ls0[0][0]), 5), round(float(ls[-1][-1]), 5)],
               paper_scale_projection_s=round(alt_ms / 1e3 * (20000 / P) * 24, 1),
               roofline=dict(kernel="k_sbwd_elem", bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS,
                             unit="GB/s", frac=round(achieved / HBM_PEAK_GBS, 4), algorithmic_bytes=int(bwd_bytes)))
    tr.close()
    inst.close()
    if cpu:
        out["cpu_baseline"] = training_cpu_baseline(t)
    return out


def training_cpu_baseline(t, n_poses: int = 2):
    """The FP64 oracle of neural cubature training, untuned, on this host's
    cores: the training data of the first n_poses poses, then one epoch of each
    net's loss and gradient over them (C = the first n_c0 elements of a
    uniform stride, the selection net over every other element)."""
    from threadpoolctl import threadpool_info
    from oracle import cubature_train as ct
    from oracle.newton import Instance as OracleInstance
    oi = OracleInstance(t.prob)
    used = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    t0 = time.perf_counter()
    data = [ct.element_forces(oi, r) for r in t.poses[:n_poses]]
    t1 = time.perf_counter()
    m = int(t.prob.tets.shape[0])
    C0 = list(range(0, m, m // t.n_c0))[:t.n_c0]
    ct.loss_W(t.wnet_weights, t.wnet_biases, t.scale, C0, [(r, F, f) for r, (F, f, _) in zip(t.poses, data)])
    t2 = time.perf_counter()
    A = ct.mesh_graph(t.prob.tets, t.prob.n)
    inC = np.zeros(m, bool)
    inC[C0] = True
    t3 = time.perf_counter()
    ct.loss_S(t.theta, A, t.prob.tets, np.flatnonzero(~inC), [(u, F, f) for (F, f, u) in data])
    t4 = time.perf_counter()
    per_pose_epochs = (t2 - t1 + t4 - t3) / n_poses   # one W and one S epoch of one pose
    return dict(value=round(2.0 / per_pose_epochs, 3), unit="pose-epochs/s", cores=int(used), kind="oracle",
                training_data_s_per_pose=round((t1 - t0) / n_poses, 3),
                sample=f"training data of {n_poses} poses of the 10k-vertex bar, then one weight-net and one "
                       f"selection-net epoch over them (FP64 numpy/BLAS oracle, dense graph), "
                       f"{t4 - t0:.1f} s")


def precision_report(nmr, ctx, p):
    """FP32 and BF16 forms against the FP64 oracle.

    Trajectory: 100 steps x 4 Newton iterations against the stored oracle
    trajectory (tests/golden/make_bar10k_trajectory.py, written by the oracle
    alone).  The bar comes to rest within a few steps, so errors are
    normalised by the trajectory's largest magnitude: max_t |r - r_or| /
    max_t |r_or| (every step), and |u - u_or| / max_t |u_or| for u after
    steps 1, 10 and 100 and for the frames steps 2 and 11 emit (those of
    steps 1 and 10).
    Newton system: J (Frobenius) at the initial state, and phi (relative to
    |phi| at the start of the step, evaluated at the same iterate) and A at
    a perturbed initial state, the oracle evaluated live."""
    import torch
    from oracle.newton import Instance as OracleInstance
    g = np.load(GOLDEN)
    oi = OracleInstance(p)
    rng = np.random.default_rng(7)
    r1 = p.r0 + rng.normal(size=p.R) * 0.005
    w0 = oi.cubature_weights(p.r0)
    sys_o = oi.system(r1, p.r0, p.rdot0, w0)
    phi0 = np.linalg.norm(oi.system(p.r0, p.r0, p.rdot0, w0)["phi"])
    zeros = np.zeros(p.n_q)
    dec_o = oi.decode(p.r0[p.n_p:], zeros, zeros)
    steps = g["rbar"].shape[0] - 1
    rmax = float(np.linalg.norm(g["rbar"], axis=1).max())
    umax = float(g["u_norm"].max())
    ustep = {int(t): g["u"][k] for k, t in enumerate(g["u_steps"])}
    rep = dict(steps=steps, newton_iters_per_step=ITERS, source="tests/golden/bar10k_trajectory_fp64.npz",
               r_norm_max=rmax, r_norm_last=float(np.linalg.norm(g["rbar"][-1])), u_norm_max=umax)
    for prec in ("fp32", "bf16"):
        x = nmr.Instance(ctx, p, prec)
        try:
            A, phi = x.newton_system(r1)
            J = x.decoder_jacobian_hessian(p.r0[p.n_p:], zeros, zeros)["J"].cpu().numpy()
            r_err, u_err, f_err, status = 0.0, {}, {}, 0
            for t in range(1, steps + 1):
                st, _ = nmr.step_many(ctx, [x], 1, ITERS)
                status = status or st[0]
                if t - 1 in ustep and t - 1 > 0:
                    f_err[t - 1] = float(np.linalg.norm(x.get_frame() - ustep[t - 1]) / umax)
                if t in ustep:
                    r, _, u = x.get_state(with_u=True)
                    u_err[t] = float(np.linalg.norm(u - ustep[t]) / umax)
                else:
                    r, _ = x.get_state()
                r_err = max(r_err, float(np.linalg.norm(r - g["rbar"][t]) / rmax))
            torch.cuda.synchronize()
        finally:
            x.close()
        rep[prec] = dict(status=int(status), r_err_max_over_steps=r_err,
                         u_err_at_step={str(k): v for k, v in u_err.items()},
                         frame_err_at_step={str(k): v for k, v in f_err.items()},
                         J_rel=rel(J, dec_o["J"]),
                         phi_rel_to_phi0=float(np.linalg.norm(phi.cpu().numpy() - sys_o["phi"]) / phi0),
                         A_rel=rel(A.cpu().numpy(), sys_o["A"]))
    return rep


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--batch", type=int, nargs="*", default=[4, 16, 64, 128])
    ap.add_argument("--tiling", choices=["rule", "autotune"], default="rule",
                    help="tile choice of the batched hidden layers in --profile-batch mode")
    ap.add_argument("--precision", choices=["fp32", "bf16"], default="fp32",
                    help="decoder precision in --profile-batch mode")
    ap.add_argument("--serve-seconds", type=float, default=2.0, help="arrival window of the served form (0: skip)")
    ap.add_argument("--serve-slots", type=int, default=64)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run 5 plain device copies of MIB MiB (the reference kernel that scales "
                         "hardware byte counters) and exit")
    ap.add_argument("--profile-batch", type=int, default=0, metavar="B",
                    help="only step B instances of the 10k-vertex problem sharing one decoder (for a "
                         "profiler) and exit")
    ap.add_argument("--profile-coupled", type=int, default=0, metavar="RODS",
                    help="only step the coupled scene with RODS rods tied to the 21^3 core (for a profiler) "
                         "and exit")
    ap.add_argument("--profile-pools", type=int, default=0, metavar="SLOTS",
                    help="only tick full slot pools of the three serving classes, SLOTS each (for a "
                         "profiler), and exit")
    ap.add_argument("--train-poses", type=int, default=1024, help="poses of the cubature-training variant (0: skip)")
    ap.add_argument("--profile-training", type=int, default=0, metavar="P",
                    help="only build the training data of P poses of the 10,000-vertex bar and run one "
                         "alternation (for a profiler), and exit")
    args = ap.parse_args()
    if args.profile_training:
        from paper_2102_11026_amd import nmr, synth
        t = synth.config_cubature_bar10k(args.profile_training)
        ctx = nmr.Context(0)
        inst = nmr.Instance(ctx, t.prob, "fp32")
        tr = nmr.Trainer(inst, t.poses, t.wnet_weights, t.wnet_biases, t.scale, t.theta, t.n_c0, t.K, t.epochs)
        lw, ls, added, ms = tr.run(1)
        print(json.dumps(dict(poses=args.profile_training, alternation_ms=round(ms, 2),
                              loss_w=[float(lw[0][0]), float(lw[0][-1])], loss_s=[float(ls[0][0]), float(ls[0][-1])])))
        tr.close()
        inst.close()
        ctx.close()
        return
    if args.profile_coupled:
        from paper_2102_11026_amd import nmr, synth
        scene = synth.config_puffer(args.profile_coupled)
        ctx = nmr.Context(0)
        core = nmr.Instance(ctx, scene.core, args.precision)
        dec = nmr.Decoder(ctx, scene.rods[0].weights, scene.rods[0].biases, scene.rods[0].act, args.precision)
        rods = [nmr.Instance(ctx, q, args.precision, shared=dec) for q in scene.rods]
        cs = nmr.Coupled(ctx, core, rods, scene.ties, scene.kappa)
        cs.step(args.warmup, scene.newton_iters)
        st, ms = cs.step(args.steps, scene.newton_iters, timings=True)
        print(json.dumps(dict(rods=len(rods), precision=args.precision, steps=args.steps, status=sorted(set(st)),
                              p50_step_ms=round(float(np.median(ms)), 4))))
        cs.close()
        for x in [core] + rods:
            x.close()
        dec.close()
        ctx.close()
        return
    if args.profile_pools:
        from paper_2102_11026_amd import nmr, synth
        ctx = nmr.Context(0)
        probs = {"A": synth.config_serve_a(), "B": synth.config_serve_b(), "C": synth.config_serve_c()}
        pools, keep = {}, []
        for name, q in probs.items():
            dec = nmr.Decoder(ctx, q.weights, q.biases, q.act, args.precision)
            pool = nmr.Pool(ctx, args.profile_pools)
            for k in range(args.profile_pools):
                r0 = np.zeros(q.R)
                r0[q.n_p:] = 0.1 * synth.normal(f"serve/q0/{1000 + k}", q.n_q)
                x = nmr.Instance(ctx, q.replace(r0=r0), args.precision, shared=dec)
                pool.attach(x)
                keep.append(x)
            pools[name] = pool
            keep.append(dec)
        for _ in range(args.warmup):
            for pool in pools.values():
                pool.step(ITERS)
        ticks = {k: [] for k in pools}
        for _ in range(args.steps):
            for name, pool in pools.items():
                ticks[name].append(pool.step(ITERS, timing=True)[1])
        print(json.dumps(dict(slots=args.profile_pools, precision=args.precision,
                              median_pool_step_ms={k: round(float(np.median(v)), 3) for k, v in ticks.items()})))
        for pool in pools.values():
            pool.close()
        for x in keep:
            x.close()
        ctx.close()
        return
    if args.profile_batch:
        import torch
        from paper_2102_11026_amd import nmr, synth
        p = synth.config_single_10k()
        ctx = nmr.Context(0)
        ctx.set_tiling(args.tiling)
        dec = nmr.Decoder(ctx, p.weights, p.biases, p.act, args.precision)
        insts = []
        for k in range(args.profile_batch):
            r0 = np.zeros(p.R)
            r0[p.n_p:] = 0.1 * synth.normal(f"q0/{k}", p.n_q)
            insts.append(nmr.Instance(ctx, p.replace(r0=r0), args.precision, shared=dec))
        secs, ms = run_steps(nmr, ctx, insts, args.steps, args.warmup)
        print(json.dumps(dict(instances=args.profile_batch, precision=args.precision, steps=args.steps,
                              newton_iters_per_s=round(ITERS * args.steps * args.profile_batch / secs, 1))))
        for x in insts:
            x.close()
        dec.close()
        ctx.close()
        return
    if args.copy_calibration:
        import torch
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps(dict(copy_calibration_bytes_per_copy=2 * n * 4, read_bytes=n * 4, write_bytes=n * 4)))
        return
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
               frames_per_s=round(args.steps / secs, 2),
               frame_output="each timed step writes the full-space displacement u (30,000 DOFs) of the frame it "
                            "starts from into the instance's frame buffer, inside the same graph launch")
    # per-phase device time (HIP events on the library's stream)
    phases = {}
    for k, name in enumerate(nmr.PHASES):
        phases[name] = round(inst.time_phase(k, reps=50), 3)
    out["phase_us"] = phases
    gram = inst.gram
    cand = {k: v for k, v in phases.items() if k in PHASE_KERNEL}
    dom = max(cand, key=cand.get)
    out["roofline"] = phase_roofline(p, dom, phases[dom], "fp32", gram)
    out["roofline"]["timing"] = ("HIP events on the library's stream around 50 replays of the phase's launches "
                                 "(nmr_time_phase), divided by the launches per pass")
    out["phase_rooflines"] = {k: phase_roofline(p, k, phases[k], "fp32", gram) for k in PHASE_KERNEL}
    out["newton_path"] = "gram-folded" if gram else "direct"
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
        # the direct Newton path: every one of the 30,000 output rows decoded in every iteration
        idr = nmr.Instance(ctx, p, "fp32", path="direct")
        nd = max(args.steps // 2, 10)
        s_d, ms_d = run_steps(nmr, ctx, [idr], nd, 3)
        dphase = {name: round(idr.time_phase(k, reps=50), 3) for k, name in enumerate(nmr.PHASES)}
        var["plain_fp32_direct_path"] = dict(newton_iters_per_s=round(ITERS * nd / s_d, 2),
                                             p99_step_ms=round(float(np.percentile(ms_d, 99)), 4),
                                             phase_us=dphase,
                                             dec_out_roofline=phase_roofline(p, "dec_out", dphase["dec_out"],
                                                                             "fp32", False),
                                             bwd_out_roofline=phase_roofline(p, "bwd_out", dphase["bwd_out"],
                                                                             "fp32", False))
        idr.close()
        log("direct path:", var["plain_fp32_direct_path"])
        for prec in ("fp32", "bf16"):
            dec = nmr.Decoder(ctx, p.weights, p.biases, p.act, prec)
            for B in args.batch:
                insts = []
                for k in range(B):
                    r0 = np.zeros(p.R)
                    r0[p.n_p:] = 0.1 * synth.normal(f"q0/{k}", p.n_q)
                    insts.append(nmr.Instance(ctx, p.replace(r0=r0), prec, shared=dec))
                nsteps = max(args.steps // 5, 5)
                rec = {}
                for tiling in ("rule", "autotune"):
                    ctx.set_tiling(tiling)
                    s_m, ms_m = run_steps(nmr, ctx, insts, nsteps, 2)
                    rec[tiling] = dict(newton_iters_per_s=round(ITERS * nsteps * B / s_m, 2),
                                       p50_step_ms=round(float(np.percentile(ms_m, 50)), 4),
                                       p99_step_ms=round(float(np.percentile(ms_m, 99)), 4))
                ctx.set_tiling("rule")
                var[f"batched_{prec}_B{B}"] = dict(rec["rule"], tiling="rule", autotuned=rec["autotune"])
                log(f"batched {prec} B={B}:", var[f"batched_{prec}_B{B}"])
                for x in insts:
                    x.close()
            dec.close()
        var["decoder_gemm_tiles"] = tile_report(nmr, ctx, p)
        # batched ragged rods: 320 rods sharing one decoder, one launch sequence
        rods = synth.config_rods(320)
        for prec in ("fp32", "bf16"):
            dec = nmr.Decoder(ctx, rods[0].weights, rods[0].biases, rods[0].act, prec)
            insts = [nmr.Instance(ctx, q, prec, shared=dec) for q in rods]
            t0 = time.perf_counter()
            st, ms_r = nmr.step_many(ctx, insts, 2, 3, timings=True)
            torch.cuda.synchronize()
            st, ms_r = nmr.step_many(ctx, insts, 20, 3, timings=True)
            torch.cuda.synchronize()
            sec = float(np.sum(ms_r)) / 1000.0
            assert all(s == 0 for s in st), st
            var[f"rods320_{prec}"] = dict(rod_newton_iters_per_s=round(320 * 3 * 20 / sec, 1),
                                          p99_step_ms=round(float(np.percentile(ms_r, 99)), 4),
                                          steps=20, newton_iters_per_step=3)
            for x in insts:
                x.close()
            dec.close()
        # coupled multi-domain scene: 320 rods tied to a 9,261-vertex reduced core (one coupled system)
        scene = synth.config_puffer(320)
        for prec in ("fp32", "bf16"):
            core = nmr.Instance(ctx, scene.core, prec)
            dec = nmr.Decoder(ctx, scene.rods[0].weights, scene.rods[0].biases, scene.rods[0].act, prec)
            rods = [nmr.Instance(ctx, q, prec, shared=dec) for q in scene.rods]
            cs = nmr.Coupled(ctx, core, rods, scene.ties, scene.kappa)
            st, _ = cs.step(2, scene.newton_iters, timings=True)
            st, ms_c = cs.step(20, scene.newton_iters, timings=True)
            assert all(x == 0 for x in st), st
            sec = float(np.sum(ms_c)) / 1000.0
            nd = len(rods) + 1
            var[f"coupled_puffer_{prec}"] = dict(
                domains=nd, rods=len(rods), core_vertices=scene.core.n, rod_vertices=int(sum(q.n for q in scene.rods)),
                domain_newton_iters_per_s=round(nd * scene.newton_iters * 20 / sec, 1),
                coupled_steps_per_s=round(20 / sec, 2), p50_step_ms=round(float(np.percentile(ms_c, 50)), 4),
                p99_step_ms=round(float(np.percentile(ms_c, 99)), 4), steps=20,
                newton_iters_per_step=scene.newton_iters)
            log(f"coupled puffer {prec}:", var[f"coupled_puffer_{prec}"])
            cs.close()
            for x in [core] + rods:
                x.close()
            dec.close()
        if args.serve_seconds > 0:
            from paper_2102_11026_amd import serve
            probs = {"A": synth.config_serve_a(), "B": synth.config_serve_b(), "C": synth.config_serve_c()}
            for prec in ("fp32", "bf16"):
                sctx = nmr.Context(0, budget_bytes=200 * (1 << 30))
                classes = [serve.RequestClass(k, v, capacity=args.serve_slots) for k, v in probs.items()]
                srv = serve.Server(sctx, classes, prec, n_iters=ITERS)
                reqs = serve.poisson_arrivals(200.0, args.serve_seconds, list(probs), 120, probs)
                stats = srv.run(reqs, max_seconds=args.serve_seconds + 60.0, log=log)
                srv.close()
                sctx.close()
                stats.update(rate_req_s=200.0, horizon_s=args.serve_seconds, steps_per_request=120,
                             budget_gb=200, slots_per_class=args.serve_slots)
                var[f"served_{prec}"] = stats
                log(f"served {prec}:", stats)
        # NEXT row: neural cubature training (Sec. 5)
        if args.train_poses > 0:
            var["cubature_training_bar10k"] = training_report(nmr, ctx, args.train_poses,
                                                              cpu=not args.no_cpu_baseline)
            log("cubature training:", var["cubature_training_bar10k"])
        # NEXT row: the fictitious force and consistency in dt (FP64, through the C ABI)
        from paper_2102_11026_amd import experiments
        var["experiment_fictitious_force"] = experiments.consistency_in_dt(nmr, ctx, "fp64")
        var["experiment_fd_vs_csfd"] = experiments.fd_vs_csfd(nmr, ctx)
        out["variants"] = var
        log("variants:", var)
    inst.close()
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on the host")
        out["cpu_baseline"] = cpu_baseline(p, args.cpu_seconds)
        out["cpu_baseline_1thread"] = cpu_baseline(p, args.cpu_seconds, threads=1)
        log("precision forms against the oracle")
        out["precision_vs_oracle"] = precision_report(nmr, ctx, p)
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
