"""GPU results of the batched and served configurations against the FP64
oracle (through the C ABI): a request of a served class stepped inside a
busy slot pool, 128 instances of the 10k-vertex bar sharing one decoder
under the default launch shapes (tall tiles, the wide output-layer kernel
with paired instances), the decoder at the hidden widths of the largest
served class, and the 10k-vertex trajectory over 100 steps against the
stored oracle trajectory (tests/golden/make_bar10k_trajectory.py).

States and displacements that pass close to zero (a bar coming to rest) are
compared element-wise against the largest magnitude along the oracle's
trajectory; every other quantity with `close` (element-wise and Frobenius).
"""
import os

import numpy as np
import pytest

from oracle.newton import Instance as OInst
from paper_2102_11026_amd import synth
from parity import close, close_scaled, rel

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "bar10k_trajectory_fp64.npz")
TOL = {"fp32": 1e-4, "bf16": 3e-2}


@pytest.fixture(scope="module")
def nmr():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2102_11026_amd import nmr as m
    m.lib()
    return m


@pytest.fixture(scope="module")
def ctx(nmr):
    c = nmr.Context(0)
    yield c
    c.close()


def oracle_run(p, steps, iters):
    """Oracle states after each step, and max_t |r(t)|, max_t |u(t)|."""
    oi = OInst(p)
    st = oi.initial_state()
    traj = [st]
    for _ in range(steps):
        st, _ = oi.step(st, iters)
        traj.append(st)
    rmax = max(float(np.abs(s.rbar).max()) for s in traj)
    return oi, traj, rmax


# ---------------------------------------------------------------------------
# served class: one request inside a busy pool
# ---------------------------------------------------------------------------
SERVE_STEPS = 6


@pytest.fixture(scope="module")
def served_oracle():
    """Served class A (2,000-vertex bar, r = 5, full quadrature) with the
    request seed of serve.poisson_arrivals for request 3, stepped by the
    oracle."""
    p = synth.config_serve_a()
    r0 = np.zeros(p.R)
    r0[p.n_p:] = 0.1 * synth.normal("serve/q0/3", p.n_q)
    p = p.replace(r0=r0)
    oi, traj, rmax = oracle_run(p, SERVE_STEPS, p.newton_iters)
    u = [oi.displacement(s.rbar) for s in traj]
    return p, traj, rmax, u, max(float(np.abs(x).max()) for x in u)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_served_request_in_a_busy_pool_against_oracle(nmr, ctx, served_oracle, prec):
    p, traj, rmax, u_or, umax = served_oracle
    tol = TOL[prec]
    dec = nmr.Decoder(ctx, p.weights, p.biases, p.act, prec)
    pool = nmr.Pool(ctx, 8)
    others = []
    for k in range(4):
        r0 = np.zeros(p.R)
        r0[p.n_p:] = 0.1 * synth.normal(f"serve/q0/{10 + k}", p.n_q)
        others.append(nmr.Instance(ctx, p.replace(r0=r0), prec, shared=dec))
    me = nmr.Instance(ctx, p, prec, shared=dec)
    try:
        slots = [pool.attach(x) for x in others[:3]]
        pool.step(p.newton_iters)                        # the pool is busy before the request joins
        s_me = pool.attach(me)
        for t in range(1, SERVE_STEPS + 1):
            if t == 3:                                   # members leave and join around it
                pool.detach(slots[1])
                pool.attach(others[3])
            st, _ = pool.step(p.newton_iters, status=True)
            assert st[s_me] == 0, st
            r, rd = me.get_state()
            e = close_scaled(r, traj[t].rbar, tol, rmax, (prec, "r", t))
            print(prec, "step", t, "max |r - r_oracle| / max_t |r| =", f"{e:.2e}")
        r, rd, u = me.get_state(with_u=True)
        close_scaled(u, u_or[-1], tol, umax, (prec, "u"))
    finally:
        pool.close()
        for x in others + [me]:
            x.close()
        dec.close()


# ---------------------------------------------------------------------------
# 128 instances of the 10k-vertex bar sharing one decoder (default rule)
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def bar10k_two_starts():
    """The 10k-vertex bar from two seeded initial states, one oracle step each."""
    base = synth.config_single_10k()
    out = []
    for k in range(2):
        r0 = np.zeros(base.R)
        r0[base.n_p:] = 0.1 * synth.normal(f"q0/{k}", base.n_q)
        p = base.replace(r0=r0)
        oi, traj, rmax = oracle_run(p, 1, base.newton_iters)
        out.append((p, oi, traj[1], rmax))
    return out


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_128_shared_decoder_instances_against_oracle(nmr, ctx, bar10k_two_starts, prec):
    """128 instances (two initial states, alternating) in one step_many under
    the default launch rule: at this count the hidden layers take four-row
    tall tiles with four instances per block and the output layer the wide
    kernel with two instances per block.  After one step every instance
    matches the oracle of its initial state, and every frame (u of the start
    state, decoded for all 128 instances by one GEMM) the oracle's."""
    tol = TOL[prec]
    base = bar10k_two_starts[0][0]
    ctx.set_tiling("rule")
    dec = nmr.Decoder(ctx, base.weights, base.biases, base.act, prec)
    insts = [nmr.Instance(ctx, bar10k_two_starts[k % 2][0], prec, shared=dec) for k in range(128)]
    try:
        st, _ = nmr.step_many(ctx, insts, 1, base.newton_iters)
        assert st == [0] * 128
        worst = 0.0
        for k, x in enumerate(insts):
            p, oi, s1, rmax = bar10k_two_starts[k % 2]
            r, rd = x.get_state()
            worst = max(worst, close_scaled(r, s1.rbar, tol, rmax, (prec, k)))
        print(prec, "128 instances, worst max |r - r_oracle| / max |r|:", f"{worst:.2e}")
        # the frames of the step (its start state), all 128 from one batched GEMM
        u0 = [bar10k_two_starts[k][1].displacement(bar10k_two_starts[k][0].r0) for k in (0, 1)]
        for k, x in enumerate(insts):
            close(x.get_frame(), u0[k % 2], tol, (prec, "frame", k))
        for k in (0, 1):                                  # the displacement of one instance per start
            p, oi, s1, rmax = bar10k_two_starts[k]
            _, _, u = insts[k].get_state(with_u=True)
            close(u, oi.displacement(s1.rbar), tol, (prec, "u", k))
    finally:
        for x in insts:
            x.close()
        dec.close()


# ---------------------------------------------------------------------------
# decoder at the hidden widths of served class C (1024 wide, n_q = 30)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_class_c_hidden_widths_decoder_against_oracle(nmr, ctx, prec):
    """decoder_jacobian_hessian with the hidden layers of served class C
    (30 -> 64 -> 128 -> 256 -> 512 -> 1024 x 5 -> 512 -> 256) and a small output
    head on a 3 x 3 x 4 bar, against the oracle."""
    widths = list(synth.SERVE_C_WIDTHS[:-1]) + [108]
    p = synth.tiny_problem(grid=(3, 3, 4), widths=widths, act="elu", name="clsC", q_std=0.1)
    rng = np.random.default_rng(11)
    q = p.r0 + rng.normal(size=p.n_q) * 0.01
    dq = rng.normal(size=p.n_q) * 0.01
    qdot = rng.normal(size=p.n_q) * 0.3
    a = rng.normal(size=p.N)
    inst = nmr.Instance(ctx, p, prec)
    try:
        got = inst.decoder_jacobian_hessian(q, dq, qdot, a)
    finally:
        inst.close()
    oi = OInst(p)
    ref = oi.decode(q, dq, qdot)
    JTa, B = oi.left(q, a)
    tol = dict(fp32=dict(u=1e-5, J=1e-4, dJ=1e-3, Hdd=1e-3, B=1e-3, JTa=1e-4),
               bf16=dict(u=3e-2, J=3e-2, dJ=1e-1, Hdd=1e-1, B=1e-1, JTa=3e-2))[prec]
    pairs = dict(u=(got["u"], ref["m"]), J=(got["J"], ref["J"]), dJ=(got["dJ"], ref["dJ"]),
                 Hdd=(got["Hdd"], ref["Hdd"]), B=(got["B"], B), JTa=(got["JTa"], JTa))
    print(prec, {k: f"{rel(*v):.1e}" for k, v in pairs.items()})
    for k, (g, o) in pairs.items():
        close(g, o, tol[k], (prec, k))


# ---------------------------------------------------------------------------
# the 10k-vertex trajectory over 100 steps against the stored oracle run
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("prec,tol", [("fp32", 1e-3), ("bf16", 5e-2)])
def test_bar10k_100_steps_against_stored_oracle_trajectory(nmr, ctx, prec, tol):
    """100 steps x 4 Newton iterations of the 10k-vertex bar.  The state after
    every step, u after steps 1, 10 and 100, and the frames that steps 2 and
    11 emit (those of steps 1 and 10), are compared element-wise
    against the stored FP64 oracle trajectory, relative to the largest
    magnitude along it (the bar comes to rest under gravity within a few
    steps, where relative errors of a near-zero state say nothing)."""
    g = np.load(GOLDEN)
    p = synth.config_single_10k()
    rmax = float(np.abs(g["rbar"]).max())
    umax = float(g["u_norm"].max())
    inst = nmr.Instance(ctx, p, prec)
    try:
        worst_r, u_err = 0.0, {}
        for t in range(1, 101):
            st, _ = nmr.step_many(ctx, [inst], 1, 4)
            assert st == [0]
            r, _ = inst.get_state()
            worst_r = max(worst_r, close_scaled(r, g["rbar"][t], tol, rmax, (prec, "r", t)))
            if t - 1 in (1, 10):                         # the frame the step started from
                ref = g["u"][list(g["u_steps"]).index(t - 1)]
                close_scaled(inst.get_frame(), ref, tol, float(np.abs(g["u"]).max()), (prec, "frame", t - 1))
            if t in g["u_steps"]:
                _, _, u = inst.get_state(with_u=True)
                ref = g["u"][list(g["u_steps"]).index(t)]
                u_err[t] = float(np.linalg.norm(u - ref) / umax)
                assert u_err[t] < tol, (prec, t, u_err[t])
                close_scaled(u, ref, tol, float(np.abs(g["u"]).max()), (prec, "u", t))
        print(prec, f"worst max|r - r_oracle| / max|r| = {worst_r:.2e}", "||u - u_oracle|| / max_t ||u|| =",
              {k: f"{v:.2e}" for k, v in u_err.items()})
    finally:
        inst.close()
