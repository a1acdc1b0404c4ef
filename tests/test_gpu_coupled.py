"""Coupled multi-domain step on the GPU (nmr_coupled_*, through the C ABI)
against the FP64 oracle's stacked coupled step (oracle/coupled.py): a core
with rods tied to its faces, every member's state after each step, the
frames the steps emit, the decoupled limit, and the freeze of the whole set
when one member fails.

States are compared element-wise relative to the largest magnitude of that
member's coordinates along the oracle's trajectory (`close_scaled`)."""
import numpy as np
import pytest

from oracle.coupled import Coupled as OCoupled
from paper_2102_11026_amd import synth
from parity import close, close_scaled

pytestmark = pytest.mark.gpu


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


def build(nmr, ctx, scene, prec, kappa=None):
    """GPU members (rods sharing one decoder) and the coupled set."""
    core = nmr.Instance(ctx, scene.core, prec)
    r0 = scene.rods[0]
    dec = nmr.Decoder(ctx, r0.weights, r0.biases, r0.act, prec)
    rods = [nmr.Instance(ctx, p, prec, shared=dec) for p in scene.rods]
    cs = nmr.Coupled(ctx, core, rods, scene.ties, scene.kappa if kappa is None else kappa)
    return cs, core, rods, dec


def close_all(cs, core, rods, dec):
    cs.close()
    for x in [core] + rods:
        x.close()
    dec.close()


def oracle_traj(scene, steps, kappa=None):
    oc = OCoupled(scene.core, scene.rods, scene.ties, scene.kappa if kappa is None else kappa)
    sts = oc.initial_state()
    traj, norms = [sts], []
    for _ in range(steps):
        sts, n = oc.step(sts, scene.newton_iters)
        traj.append(sts)
        norms.append(n)
    return oc, traj, norms


@pytest.fixture(scope="module")
def tiny():
    s = synth.config_coupled_tiny(2)
    return s, oracle_traj(s, s.steps)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-9), ("fp32", 1e-3)])
def test_coupled_tiny_against_oracle(nmr, ctx, tiny, prec, tol):
    s, (oc, traj, norms) = tiny
    nd = 1 + len(s.rods)
    rmax = [max(float(np.abs(t[d].rbar).max()) for t in traj) for d in range(nd)]
    umax = [max(float(np.abs(oc.insts[d].displacement(t[d].rbar)).max()) for t in traj) for d in range(nd)]
    cs, core, rods, dec = build(nmr, ctx, s, prec)
    members = [core] + rods
    try:
        for t in range(1, s.steps + 1):
            st, _ = cs.step(1, s.newton_iters)
            assert st == [0] * nd, st
            for d, x in enumerate(members):
                r, rd = x.get_state()
                close_scaled(r, traj[t][d].rbar, tol, rmax[d], (prec, "r", t, d))
                # the frame the step started from
                close_scaled(x.get_frame(), oc.insts[d].displacement(traj[t - 1][d].rbar), tol, umax[d],
                             (prec, "frame", t, d))
        if prec == "fp64":
            rd = [x.get_state()[1] for x in members]
            for d in range(nd):
                close(rd[d], traj[-1][d].rdot_bar, 1e-7, ("rdot", d))
    finally:
        close_all(cs, core, rods, dec)


def test_coupled_zero_kappa_equals_separate_steps(nmr, ctx):
    """kappa = 0: the coupled set steps each member exactly as step_many does
    on its own (different elimination orders: rounding-level agreement)."""
    s = synth.config_coupled_tiny(2)
    s.core = s.core.replace(r0=np.zeros(s.core.R))
    s.rods = [p.replace(r0=np.zeros(p.R)) for p in s.rods]
    cs, core, rods, dec = build(nmr, ctx, s, "fp64", kappa=0.0)
    sep = [nmr.Instance(ctx, p, "fp64") for p in [s.core] + s.rods]
    try:
        st, _ = cs.step(2, 3)
        assert st == [0] * 3
        for x in sep:
            st, _ = nmr.step_many(ctx, [x], 2, 3)
            assert st == [0]
        for a, b in zip([core] + rods, sep):
            ra, _ = a.get_state()
            rb, _ = b.get_state()
            close(ra, rb, 1e-10, "r")
    finally:
        close_all(cs, core, rods, dec)
        for x in sep:
            x.close()


def test_a_failing_member_freezes_the_set(nmr, ctx):
    """A rod started far outside its subspace's valid range inverts a tet: the
    whole set keeps its previous state and every member reports the failure."""
    s = synth.config_coupled_tiny(2)
    cs, core, rods, dec = build(nmr, ctx, s, "fp64")
    try:
        st, _ = cs.step(1, 3)
        assert st == [0] * 3
        before = [x.get_state() for x in [core] + rods]
        r, rd = rods[1].get_state()
        bad = r.copy()
        bad[:rods[1].n_p] += 5.0          # 5 m of rigid-body-like motion of the rod's linear modes
        bad[rods[1].n_p:] += 40.0         # and a wildly deformed latent state
        rods[1].set_state(bad, rd)
        before[2] = (bad, rd)
        st, _ = cs.step(1, 3)
        assert all(x != 0 for x in st), st
        for x, (r0, rd0) in zip([core] + rods, before):
            r1, rd1 = x.get_state()
            np.testing.assert_array_equal(r1, r0)
            np.testing.assert_array_equal(rd1, rd0)
    finally:
        close_all(cs, core, rods, dec)


def test_member_cannot_be_destroyed_while_coupled(nmr, ctx):
    s = synth.config_coupled_tiny(1)
    cs, core, rods, dec = build(nmr, ctx, s, "fp32")
    try:
        assert nmr.lib().nmr_instance_destroy(rods[0].h) == -1
    finally:
        close_all(cs, core, rods, dec)


def test_coupled_puffer_subset_against_oracle_fp32(nmr, ctx):
    """A 9 x 9 x 9 core (n_p = 10, n_q = 6) with 8 rods of 20 or 30 vertex
    layers (n_p = 10, n_q = 5, the shared rod decoder), FP32, two steps of
    three Newton iterations against the oracle."""
    s = synth.coupled_scene("puffer_sub", (9, 9, 9), 8, (20, 30), core_np=10, core_widths=[6, 32, 64, 128, 2187],
                            rod_np=10, rod_widths=synth.ROD_WIDTHS, steps=2, newton_iters=3)
    oc, traj, norms = oracle_traj(s, 2)
    nd = 1 + len(s.rods)
    rmax = [max(float(np.abs(t[d].rbar).max()) for t in traj) for d in range(nd)]
    cs, core, rods, dec = build(nmr, ctx, s, "fp32")
    try:
        for t in (1, 2):
            st, _ = cs.step(1, 3)
            assert st == [0] * nd, st
            for d, x in enumerate([core] + rods):
                r, _ = x.get_state()
                close_scaled(r, traj[t][d].rbar, 1e-3, rmax[d], ("r", t, d))
    finally:
        close_all(cs, core, rods, dec)
