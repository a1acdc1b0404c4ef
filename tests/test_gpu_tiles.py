"""GPU tests of the tile configurations of batched hidden-layer launches:
every forced configuration (instances per block x 16-row tiles per wave)
against the oracle and against the rule, the autotuner, and argument checks
(all through the C ABI)."""
import numpy as np
import pytest

from oracle.newton import Instance as OInst
from paper_2102_11026_amd import synth
from parity import close, rel

pytestmark = pytest.mark.gpu

CONFIGS = [(1, 1), (2, 1), (4, 1), (4, 2), (4, 4)]



@pytest.fixture(scope="module")
def nmr():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2102_11026_amd import nmr as m
    m.lib()
    return m


def family(n_q, n_inst, name, q_scale=0.6):
    """n_inst instances sharing one decoder whose hidden widths (64, 128, 64)
    admit every tall tile; each starts from its own latent state."""
    base = synth.tiny_problem(grid=(3, 3, 6), widths=(n_q, 64, 128, 64, 162), act="tanh", name=name,
                              q_std=0.3, out_scale=0.1)
    probs = []
    for k in range(n_inst):
        r0 = np.zeros(base.R)
        r0[base.n_p:] = (q_scale / np.sqrt(n_q)) * synth.normal(f"{name}/q0/{k}", base.n_q)
        probs.append(base.replace(r0=r0))
    return base, probs


def run(nmr, ctx, base, probs, prec, steps, iters, tiling, full=False):
    ctx.set_tiling(*tiling)
    dec = nmr.Decoder(ctx, base.weights, base.biases, base.act, prec)
    insts = [nmr.Instance(ctx, q, prec, shared=dec) for q in probs]
    try:
        st, _ = nmr.step_many(ctx, insts, steps, iters)
        assert st == [0] * len(insts)
        if full:
            return [x.get_state(with_u=True) for x in insts]
        return [x.get_state()[0] for x in insts]
    finally:
        for x in insts:
            x.close()
        dec.close()
        ctx.set_tiling("rule")


def oracle_states(probs, steps, iters):
    out = []
    for q in probs:
        oi = OInst(q)
        s = oi.initial_state()
        for _ in range(steps):
            s, _ = oi.step(s, iters)
        out.append(s.rbar)
    return out


@pytest.mark.parametrize("n_q,q_scale", [(15, 0.6), (4, 0.6), (30, 0.3)])
def test_forced_tiles_fp32_match_oracle(nmr, n_q, q_scale):
    """Six instances (a ragged last block of four slots), every configuration
    forced: each instance against the FP64 oracle, and every configuration
    against the one-instance-per-block tiles.  n_q = 30 gives 128 jet
    columns, where only the two-row tall tile is eligible forward."""
    base, probs = family(n_q, 6, f"tiles{n_q}", q_scale)
    ref = oracle_states(probs, 3, 3)
    ctx = nmr.Context(0)
    try:
        got = {cfg: run(nmr, ctx, base, probs, "fp32", 3, 3, ("force",) + cfg) for cfg in CONFIGS}
    finally:
        ctx.close()
    for cfg, rs in got.items():
        print(cfg, ["%.1e" % rel(r, o) for r, o in zip(rs, ref)])
    # the FP32 bar against the oracle; between configurations, which round
    # the K sums differently, the same bar
    for cfg, rs in got.items():
        for k, (r, o) in enumerate(zip(rs, ref)):
            close(r, o, 1e-4, (cfg, k, rel(r, o)))
            close(r, got[(1, 1)][k], 1e-4, (cfg, k))


def test_forced_tiles_bf16_match_oracle(nmr):
    base, probs = family(15, 5, "tilesbf")
    ref = oracle_states(probs, 2, 3)
    ctx = nmr.Context(0)
    try:
        for cfg in [(1, 1), (4, 1), (4, 2), (4, 4)]:
            rs = run(nmr, ctx, base, probs, "bf16", 2, 3, ("force",) + cfg)
            for k, (r, o) in enumerate(zip(rs, ref)):
                close(r, o, 3e-2, (cfg, k, rel(r, o)))
    finally:
        ctx.close()


@pytest.mark.parametrize("n_q,prec,form", [(4, "fp32", "full"), (15, "fp32", "trimmed"), (15, "bf16", "full"),
                                           (30, "fp32", "full")])
def test_jet_groups_are_bitwise_the_whole_tile(nmr, n_q, prec, form):
    """One and three instances: under the rule the forward jet layers split
    their columns into groups of three perturbations (a ragged last group for
    n_q = 4), forced (1, 1) keeps whole tiles.  Up to 64 jet columns (n_q <=
    15) both split K over eight waves, so every column is the same sum and
    the states (r, rdot, u) agree bitwise.  Whole tiles of 128 columns (n_q =
    30) split K over four waves: there the bar between the two is the one
    between tile configurations.  The FP32 rule run is also held to the
    oracle."""
    base, probs = family(n_q, 3, f"jg{n_q}", 0.3 if n_q == 30 else 0.6)
    base = base.replace(formulation=form)
    probs = [q.replace(formulation=form) for q in probs]
    ctx = nmr.Context(0)
    try:
        for n in (1, 3):
            grouped = run(nmr, ctx, base, probs[:n], prec, 2, 3, ("rule",), full=True)
            whole = run(nmr, ctx, base, probs[:n], prec, 2, 3, ("force", 1, 1), full=True)
            for k in range(n):
                for a, b in zip(grouped[k], whole[k]):
                    if n_q <= 15:
                        np.testing.assert_array_equal(a, b)
                    else:
                        close(a, b, 1e-4, 'a')
        if prec == "fp32":
            for (r, _, _), o in zip(grouped, oracle_states(probs, 2, 3)):
                close(r, o, 1e-4, 'r')
    finally:
        ctx.close()


def test_tall_tiles_at_headline_shape(nmr):
    """Eight 10k-vertex instances (K = 512 layers, 64 jet columns): the tall
    tiles against the rule after one step.  With a tanh decoder of the same
    shape and weights, to 1e-4.  With the headline's ELU, to 1e-2: ELU's
    second and third derivatives jump at 0 (e^x on the left, 0 on the
    right), and along these steps pre-activations come within 3e-9 to 1e-6
    of 0 (oracle iterates), below the rounding of an FP32 512-term sum.
    Two summation orders may then take a neuron's Hessian terms from
    different sides, and with them the Newton matrix of the fixed number of
    iterations (one of the eight moves by 2.5e-3 when the tall tiles split K
    over two waves)."""
    elu = synth.config_single_10k()
    assert elu.act == "elu"
    for p, tol in ((elu.replace(act="tanh"), 1e-4), (elu, 1e-2)):
        probs = []
        for k in range(8):
            r0 = p.r0 + 0.02 * synth.normal(f"tiles10k/q0/{k}", p.R)
            probs.append(p.replace(r0=r0))
        ctx = nmr.Context(0)
        try:
            rule = run(nmr, ctx, p, probs, "fp32", 1, p.newton_iters, ("rule",))
            for cfg in [(4, 2), (4, 4)]:
                rs = run(nmr, ctx, p, probs, "fp32", 1, p.newton_iters, ("force",) + cfg)
                for k in range(8):
                    close(rs[k], rule[k], tol, (p.act, cfg, k, rel(rs[k], rule[k])))
        finally:
            ctx.close()


def test_autotune_records_eligible_choices(nmr):
    base, probs = family(15, 8, "tilestune")
    ref = oracle_states(probs, 2, 3)
    ctx = nmr.Context(0)
    try:
        ctx.set_tiling("autotune")
        dec = nmr.Decoder(ctx, base.weights, base.biases, base.act, "fp32")
        insts = [nmr.Instance(ctx, q, "fp32", shared=dec) for q in probs]
        try:
            st, _ = nmr.step_many(ctx, insts, 2, 3)
            assert st == [0] * 8
            for x, o in zip(insts, ref):
                close(x.get_state()[0], o, 1e-4, 'x.get_state()[0]')
        finally:
            for x in insts:
                x.close()
            dec.close()
        table = ctx.tiling_table()
        # forward: 3 hidden layers; backward: 3 (each with more than one candidate)
        print(table)
        assert sum(e["forward"] for e in table) == 3 and len(table) == 6, table
        for e in table:
            assert e["n_inst"] == 8 and e["us"] > 0
            assert (e["ib"], e["mr"]) in CONFIGS
            if e["jet_groups"]:
                assert e["forward"] and e["ib"] == 1 and e["mr"] == 1
            if e["mr"] > 1:
                rows = e["m_out"] if e["forward"] else e["m_in"]
                assert e["ib"] == 4 and rows % (16 * e["mr"]) == 0
                assert e["cols"] <= ((128 if e["mr"] == 2 else 64) if e["forward"] else 32)
    finally:
        ctx.close()


def test_tiling_arguments_are_checked(nmr):
    ctx = nmr.Context(0)
    try:
        with pytest.raises(nmr.NmrError) as e:
            nmr._check(nmr.lib().nmr_set_tiling(ctx.h, 7, 1, 1))
        assert nmr.STATUS[e.value.code] == "arg"
        with pytest.raises(nmr.NmrError):
            ctx.set_tiling("force", 3, 1)
        with pytest.raises(nmr.NmrError):
            ctx.set_tiling("force", 4, 8)
        ctx.set_tiling("force", 4, 4)
        ctx.set_tiling("rule")
        assert ctx.tiling_table() == []
    finally:
        ctx.close()
