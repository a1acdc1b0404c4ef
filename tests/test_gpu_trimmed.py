"""GPU tests of the trimmed formulation (fictitious force dropped, as in
latent space dynamics) against the oracle's trimmed formulation, and the
consistency-in-dt experiment that separates it from the paper's."""
import numpy as np
import pytest

from oracle.newton import Instance as OInst
from paper_2102_11026_amd import synth
from parity import close, rel

pytestmark = pytest.mark.gpu

TOL = {"fp64": dict(u=1e-12, J=1e-11, dJ=1e-10, B=1e-10, JTa=1e-11, A=1e-10, phi=1e-10),
       "fp32": dict(u=1e-5, J=1e-4, dJ=1e-3, B=1e-3, JTa=1e-4, A=1e-4, phi=1e-4)}



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


def trimmed_problems():
    return {
        "tiny_elu_np": synth.tiny_problem(grid=(3, 3, 5), widths=(4, 24, 40, 135), act="elu", n_p=3, name="t1",
                                          q_std=0.3, out_scale=0.1).replace(formulation="trimmed"),
        "lsd": synth.lsd_problem().replace(formulation="trimmed"),
    }


PROBS = trimmed_problems()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", list(PROBS))
def test_trimmed_decoder_and_system(nmr, ctx, name, prec):
    p = PROBS[name]
    rng = np.random.default_rng(11)
    rdot = rng.normal(size=p.R) * 0.3
    inst = nmr.Instance(ctx, p.replace(rdot0=rdot), prec)
    try:
        oi = OInst(p)
        t = TOL[prec]
        q = p.r0[p.n_p:] + rng.normal(size=p.n_q) * 0.05
        dq = rng.normal(size=p.n_q) * 0.02
        qdot = rng.normal(size=p.n_q) * 0.5
        a = rng.normal(size=p.N)
        got = inst.decoder_jacobian_hessian(q, dq, qdot, a)
        ref = oi.decode(q, dq, qdot)
        JTa, B = oi.left(q, a)
        close(got["J"].cpu(), ref["J"], t["J"], "J")
        close(got["dJ"].cpu(), ref["dJ"], t["dJ"], "dJ")
        assert np.abs(got["Hdd"].cpu().numpy()).max() == 0.0
        close(got["JTa"].cpu(), JTa, t["JTa"], "JTa")
        close(got["B"].cpu(), B, t["B"], "B")
        r = p.r0 + rng.normal(size=p.R) * 0.01
        A, phi = inst.newton_system(r)
        sysd = oi.system(r, p.r0, rdot, oi.cubature_weights(p.r0))
        close(phi.cpu().numpy(), sysd["phi"], t["phi"], "phi")
        close(A.cpu().numpy(), sysd["A"], t["A"], "A")
    finally:
        inst.close()


def test_trimmed_trajectory_fp64(nmr, ctx):
    p = PROBS["lsd"]
    inst = nmr.Instance(ctx, p, "fp64")
    try:
        oi = OInst(p)
        st = oi.initial_state()
        for s in range(6):
            inst.step(p.newton_iters, resid=False)
            st, _ = oi.step(st, p.newton_iters)
            close(inst.get_state()[0], st.rbar, 1e-9, s)
    finally:
        inst.close()


def test_trimmed_gram_path_equals_direct_path(nmr, ctx):
    p = PROBS["lsd"]
    rng = np.random.default_rng(12)
    r = p.r0 + rng.normal(size=p.R) * 0.01
    out = []
    for path in ("auto", "direct"):
        inst = nmr.Instance(ctx, p, "fp64", path=path)
        try:
            assert inst.gram == (path == "auto")
            A, phi = inst.newton_system(r)
            out.append((A.cpu().numpy(), phi.cpu().numpy()))
        finally:
            inst.close()
    close(out[0][0], out[1][0], 1e-11, "A")
    close(out[0][1], out[1][1], 1e-11, "phi")


def test_fictitious_force_is_needed_for_consistency_in_dt(nmr, ctx):
    """The paper's formulation converges to the fine-step reference as dt
    halves; the trimmed one stops improving (fast motion, converged solves)."""
    from paper_2102_11026_amd import experiments
    rep = experiments.consistency_in_dt(nmr, ctx, "fp64", T=0.25, levels=5, ref_level=7)
    print(rep)
    full = [row["full"] for row in rep["levels"]]
    trim = [row["trimmed"] for row in rep["levels"]]
    assert all(e is not None for e in full + trim)
    # first order: each halving of dt cuts the error by at least 1.6x
    for a, b in zip(full[1:], full[2:]):
        assert b < a / 1.6
    # the trimmed error levels off well above the paper's at the finest step
    assert trim[-1] > 2.0 * full[-1]
    assert trim[-1] > 0.6 * trim[-2]
