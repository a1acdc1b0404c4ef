"""GPU tests of the central-difference derivative mode against the oracle's
central differences, and the complex-step vs central-difference experiment."""
import numpy as np
import pytest

from oracle.newton import Instance as OInst
from paper_2102_11026_amd import synth
from parity import close, rel

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


FD_PROBS = {
    "bar192": synth.config_plain_fp64(),
    "tiny_elu_np": synth.tiny_problem(grid=(3, 3, 5), widths=(4, 24, 40, 135), act="elu", n_p=3, name="t1",
                                      q_std=0.3, out_scale=0.1),
}


@pytest.mark.parametrize("formulation", ["full", "trimmed"])
@pytest.mark.parametrize("name", list(FD_PROBS))
def test_fd_mode_matches_oracle_fd(nmr, ctx, name, formulation):
    """FP64, h = 1e-2: rounding enters the third-order stencil amplified by
    1 / h^3 = 1e6, so the bound is 1e-6 rather than the 1e-10 of complex steps."""
    h = 1e-2
    p = FD_PROBS[name].replace(fd_h=h, formulation=formulation)
    rng = np.random.default_rng(31)
    rdot = rng.normal(size=p.R) * 0.3
    inst = nmr.Instance(ctx, p.replace(rdot0=rdot), "fp64")
    try:
        oi = OInst(p)
        assert oi.fd_h == h
        q = p.r0[p.n_p:] + rng.normal(size=p.n_q) * 0.05
        dq, qd = rng.normal(size=p.n_q) * 0.02, rng.normal(size=p.n_q) * 0.5
        a = rng.normal(size=p.N)
        got = inst.decoder_jacobian_hessian(q, dq, qd, a)
        ref = oi.decode(q, dq, qd)
        JTa, B = oi.left(q, a)
        for k, kk in (("u", "m"), ("J", "J"), ("dJ", "dJ")):
            close(got[k].cpu(), ref[kk], 1e-6, k)
        if formulation == "full":
            close(got["Hdd"].cpu(), ref["Hdd"], 1e-6, "Hdd")
        close(got["JTa"].cpu(), JTa, 1e-10, "JTa")
        close(got["B"].cpu(), B, 1e-6, "B")
        r = p.r0 + rng.normal(size=p.R) * 0.01
        A, phi = inst.newton_system(r)
        sysd = oi.system(r, p.r0, rdot, oi.cubature_weights(p.r0))
        close(phi.cpu().numpy(), sysd["phi"], 1e-6, "phi")
        close(A.cpu().numpy(), sysd["A"], 1e-6, "A")
    finally:
        inst.close()


def test_fd_mode_rejects_wide_latent_spaces(nmr, ctx):
    p = synth.config_single_10k().replace(fd_h=1e-3)  # n_q = 15: 213 stencil columns
    with pytest.raises(nmr.NmrError):
        nmr.Instance(ctx, p, "fp32")


def test_central_differences_fail_where_complex_steps_do_not(nmr, ctx):
    """The comparison of Sec. 6 on the GPU path (fast motion): in FP32 the
    central-difference dJ is wrong by more than half at every step the paper
    tried, and no FP32 run converges (Newton stalls, the run fails, or it
    leaves the complex-step trajectory); in FP64, h = 1e-3 still works."""
    from paper_2102_11026_amd import experiments
    rep = experiments.fd_vs_csfd(nmr, ctx)
    print(rep)
    runs = {(r["precision"], r["h"]): r for r in rep["runs"]}
    for h in (1e-3, 1e-5, 1e-7, 1e-9):
        r32 = runs[("fp32", h)]
        assert r32["dJ_rel_err"] > 0.5, r32
        failed = r32["status"] != "ok" or (r32["worst_newton_ratio"] or 0) > 1e-2 or r32["max_r_rel_dev"] > 1e-2
        assert failed, r32
    r64 = runs[("fp64", 1e-3)]
    assert r64["status"] == "ok" and r64["dJ_rel_err"] < 1e-3 and r64["max_r_rel_dev"] < 1e-4, r64
    assert runs[("fp64", 1e-9)]["dJ_rel_err"] > 0.5
