"""GPU tests of the launch shapes that only large batches take: the wide
output-layer kernel (folded activations staged once per block; the same bits
as the split kernel) and merged cubature blocks (a different FP64 summation
order: equal to rounding).  All through the C ABI."""
import numpy as np
import pytest

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


def batch_vs_alone(nmr, ctx, probs, prec, steps, iters, path="auto"):
    dec = nmr.Decoder(ctx, probs[0].weights, probs[0].biases, probs[0].act, prec)
    together = [nmr.Instance(ctx, q, prec, shared=dec, path=path) for q in probs]
    try:
        st, _ = nmr.step_many(ctx, together, steps, iters)
        assert st == [0] * len(probs)
        got = [x.get_state(with_u=True) for x in together]
    finally:
        for x in together:
            x.close()
    alone = []
    for q in probs:
        x = nmr.Instance(ctx, q, prec, shared=dec, path=path)
        try:
            st, _ = nmr.step_many(ctx, [x], steps, iters)
            assert st == [0]
            alone.append(x.get_state(with_u=True))
        finally:
            x.close()
    dec.close()
    return got, alone


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_wide_output_layer_is_bitwise_the_split_one(nmr, ctx, prec):
    """Eleven 10k-vertex instances on the direct path (30,000 decoded rows
    each, the same for all): the output layer runs the wide kernel with two
    instances per block (the last block holds one).  The hidden layers are
    forced to one-instance tiles, so everything else runs as alone."""
    p = synth.config_single_10k()
    probs = [p.replace(r0=p.r0 + 0.02 * synth.normal(f"wide/q0/{k}", p.R)) for k in range(11)]
    ctx.set_tiling("force", 1, 1)
    try:
        got, alone = batch_vs_alone(nmr, ctx, probs, prec, 1, p.newton_iters, path="direct")
    finally:
        ctx.set_tiling("rule")
    for (r, rd, u), (ra, rda, ua) in zip(got, alone):
        np.testing.assert_array_equal(r, ra)
        np.testing.assert_array_equal(rd, rda)
        np.testing.assert_array_equal(u, ua)


def test_wide_output_layer_rows_per_instance(nmr, ctx):
    """48 10k-vertex instances on the Gram path.  With one cubature set the
    output layer pairs instances (shared weight rows); with two alternating
    sets it must not, and every instance still decodes its own rows.  All
    three batches take the same launch shapes otherwise, and the paired and
    single kernels give the same bits, so each instance of the mixed batch
    equals the same instance of the one-set batch bitwise."""
    p = synth.config_single_10k()
    other = np.sort(synth.permutation("wide/cub2", len(p.tets))[:p.cub_ids.size]).astype(np.int32)
    assert not np.array_equal(other, p.cub_ids)

    def batch(sets):
        probs = []
        for k, use_other in enumerate(sets):
            q = p.replace(r0=p.r0 + 0.02 * synth.normal(f"wide48/q0/{k}", p.R))
            probs.append(q.replace(cub_ids=other) if use_other else q)
        dec = nmr.Decoder(ctx, p.weights, p.biases, p.act, "fp32")
        insts = [nmr.Instance(ctx, q, "fp32", shared=dec) for q in probs]
        try:
            st, _ = nmr.step_many(ctx, insts, 1, p.newton_iters)
            assert st == [0] * len(insts)
            return [x.get_state(with_u=True) for x in insts]
        finally:
            for x in insts:
                x.close()
            dec.close()

    first, second = batch([False] * 48), batch([True] * 48)
    mixed = batch([k % 2 == 1 for k in range(48)])
    for k in range(48):
        ref = second[k] if k % 2 else first[k]
        for a, b in zip(mixed[k], ref):
            np.testing.assert_array_equal(a, b)
    # the two sets decode different rows: the states differ
    assert rel(first[1][2], second[1][2]) > 1e-3


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_merged_cubature_blocks_match_alone(nmr, ctx, prec, tol):
    """Twenty instances: the cubature pass merges four blocks of tets into
    one and the sums read a quarter of the partials."""
    base = synth.tiny_problem(grid=(3, 3, 6), widths=(4, 32, 48, 162), act="tanh", name="merge", q_std=0.3,
                              out_scale=0.1)
    probs = []
    for k in range(20):
        r0 = np.zeros(base.R)
        r0[base.n_p:] = 0.2 * synth.normal(f"merge/q0/{k}", base.n_q)
        probs.append(base.replace(r0=r0))
    got, alone = batch_vs_alone(nmr, ctx, probs, prec, 4, 3)
    for k, ((r, rd, u), (ra, rda, ua)) in enumerate(zip(got, alone)):
        close(r, ra, tol, ("r", k))
        close(rd, rda, tol, ("rdot", k))
        close(u, ua, tol, ("u", k))


def test_large_pool_matches_alone(nmr, ctx):
    """A request in a 32-slot pool (merged cubature blocks) against the same
    request alone, to FP32 rounding."""
    base = synth.tiny_problem(grid=(3, 3, 6), widths=(4, 32, 48, 162), act="elu", name="bigpool", q_std=0.3,
                              out_scale=0.1, n_cub=20)
    probs = []
    for k in range(20):
        r0 = np.zeros(base.R)
        r0[base.n_p:] = 0.1 * synth.normal(f"bigpool/q0/{k}", base.n_q)
        probs.append(base.replace(r0=r0))
    dec = nmr.Decoder(ctx, base.weights, base.biases, base.act, "fp32")
    pool = nmr.Pool(ctx, 32)
    insts = [nmr.Instance(ctx, q, "fp32", shared=dec) for q in probs]
    ref = nmr.Instance(ctx, probs[0], "fp32", shared=dec)
    try:
        for x in insts:
            pool.attach(x)
        for _ in range(5):
            st, _ = pool.step(3, status=True)
            assert all(v == 0 for v in st)
        st, _ = nmr.step_many(ctx, [ref], 5, 3)
        assert st == [0]
        close(insts[0].get_state()[0], ref.get_state()[0], 1e-5, 'insts[0].get_state()[0]')
    finally:
        pool.close()
        for x in insts + [ref]:
            x.close()
        dec.close()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("n_p,n_q", [(3, 4), (3, 12), (11, 12)])
def test_packed_cubature_is_bitwise_the_four_wave_form(nmr, ctx, prec, n_p, n_q):
    """Four instances of 1,375 tets each (R = 7, 15 and 23, direct path): the
    batched launch has 1,376 blocks of tets and takes the packed form for
    R <= 16 (one wave of four 16-lane groups, one FP64 accumulator set per
    virtual wave; R = 23 stays four-wave), each instance alone the four-wave
    form; the same merge factor (one), so the same bits."""
    base = synth.tiny_problem(grid=(6, 6, 12), widths=(n_q, 16, 32, 1296), act="tanh", n_p=n_p,
                              name=f"pack{n_p}_{n_q}", q_std=0.3, out_scale=0.1)
    assert base.tets.shape[0] == 1375 and base.R == n_p + n_q
    probs = []
    for k in range(4):
        r0 = np.zeros(base.R)
        r0[base.n_p:] = 0.2 * synth.normal(f"pack/q0/{k}", base.n_q)
        probs.append(base.replace(r0=r0))
    got, alone = batch_vs_alone(nmr, ctx, probs, prec, 2, 3)
    for (r, rd, u), (ra, rda, ua) in zip(got, alone):
        np.testing.assert_array_equal(r, ra)
        np.testing.assert_array_equal(rd, rda)
        np.testing.assert_array_equal(u, ua)


@pytest.mark.parametrize("prec,tiles,tol", [("fp32", None, 1e-4), ("bf16", None, 3e-2), ("bf16", (4, 4), 3e-2)])
def test_paired_output_layer_in_a_pool_with_a_stale_slot(nmr, ctx, prec, tiles, tol):
    """A 64-slot pool of 10k-vertex instances (Gram path, 5,710 decoded rows)
    runs the output layer two instances per block, rows from the pool's own
    copy, and its 512-wide hidden layers in tall tiles (BF16: staged through
    LDS; tiles=(4, 4) forces four 16-row blocks).  Slot 0's instance is
    destroyed after attaching, so the pair (0, 1) has a stale first entry and
    61 slots were never filled (null pointers): no kernel may follow an empty
    slot's pointers, slot 1's request must be bitwise the one of a pool whose
    slot 0 stays live, and match the request alone (to the precision's
    rounding: the pool's tiles and merged cubature blocks sum in other
    orders)."""
    p = synth.config_single_10k()
    probs = [p.replace(r0=p.r0 + 0.01 * synth.normal(f"pairpool/q0/{k}", p.R)) for k in range(3)]
    dec = nmr.Decoder(ctx, p.weights, p.biases, p.act, prec)
    if tiles:
        ctx.set_tiling("force", *tiles)

    def run(stale):
        pool = nmr.Pool(ctx, 64)
        insts = [nmr.Instance(ctx, q, prec, shared=dec) for q in probs]
        try:
            slots = [pool.attach(x) for x in insts]
            assert slots == [0, 1, 2]
            if stale:
                insts[0].close()             # detached and freed: slot 0 keeps a stale entry
            for _ in range(2):
                st, _ = pool.step(p.newton_iters, status=True)
                assert st[1] == 0 and st[2] == 0
            return [insts[k].get_state(with_u=True) for k in (1, 2)]
        finally:
            pool.close()
            for x in insts[(1 if stale else 0):]:
                x.close()

    try:
        live, stale = run(False), run(True)
    finally:
        ctx.set_tiling("rule")
    for a, b in zip(live, stale):
        for x, y in zip(a, b):
            np.testing.assert_array_equal(x, y)
    ref = nmr.Instance(ctx, probs[1], prec, shared=dec)
    try:
        st, _ = nmr.step_many(ctx, [ref], 2, p.newton_iters)
        assert st == [0]
        ra, rda, ua = ref.get_state(with_u=True)
        close(stale[0][0], ra, tol, "r")
        close(stale[0][2], ua, tol, "u")
    finally:
        ref.close()
        dec.close()
