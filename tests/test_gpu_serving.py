"""GPU tests of the batched rods and the served form (slot pools, request loop)."""
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


def test_rods_batched_against_oracle(nmr, ctx):
    """Eight uneven rods (shared decoder, own U, prefix rows of the shared
    head) advanced together, each compared with the oracle."""
    dec_w = synth.rod_decoder()
    rods = [synth.rod_problem(i, 320, dec_w) for i in (0, 1, 2, 3, 40, 41, 200, 319)]
    dec = nmr.Decoder(ctx, dec_w[0], dec_w[1], "tanh", "fp64")
    insts = [nmr.Instance(ctx, p, "fp64", shared=dec) for p in rods]
    try:
        st, ms = nmr.step_many(ctx, insts, 2, 3)
        assert st == [0] * len(rods)
        for x, p in zip(insts, rods):
            oi = OInst(p)
            s = oi.initial_state()
            for _ in range(2):
                s, _ = oi.step(s, 3)
            close(x.get_state()[0], s.rbar, 1e-9, p.name)
    finally:
        for x in insts:
            x.close()
        dec.close()


def small_class(k):
    p = synth.tiny_problem(grid=(3, 3, 6), widths=(4, 32, 48, 162), act="elu", name="srv", q_std=0.3,
                           out_scale=0.1, n_cub=20)
    r0 = np.zeros(p.R)
    r0[p.n_p:] = 0.1 * synth.normal(f"srv/q0/{k}", p.n_q)  # at 0.3 request 0 inverts in the oracle
    return p.replace(r0=r0)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_pool_alone_vs_mix(nmr, ctx, prec):
    """A request stepped alone and the same request joining a busy pool mid-way
    (others attaching and leaving around it) end bitwise equal."""
    probs = [small_class(k) for k in range(5)]
    dec = nmr.Decoder(ctx, probs[0].weights, probs[0].biases, probs[0].act, prec)
    alone_pool, mix_pool = nmr.Pool(ctx, 1), nmr.Pool(ctx, 8)
    insts = [nmr.Instance(ctx, p, prec, shared=dec) for p in probs]
    ref = nmr.Instance(ctx, probs[0], prec, shared=dec)
    try:
        alone_pool.attach(ref)
        for _ in range(6):
            alone_pool.step(3)
        slots = [mix_pool.attach(x) for x in insts[1:4]]
        for _ in range(2):
            mix_pool.step(3)
        s0 = mix_pool.attach(insts[0])
        mix_pool.step(3)
        mix_pool.detach(slots[1])
        s4 = mix_pool.attach(insts[4])
        for _ in range(5):
            st, ms = mix_pool.step(3, status=True)
        assert all(v == 0 for v in st)
        np.testing.assert_array_equal(insts[0].get_state()[0], ref.get_state()[0])
        np.testing.assert_array_equal(insts[0].get_state()[1], ref.get_state()[1])
        mix_pool.detach(s0)
        mix_pool.detach(s4)
    finally:
        alone_pool.close()
        mix_pool.close()
        for x in insts + [ref]:
            x.close()
        dec.close()


def test_serve_loop_drains_and_matches_alone(nmr, ctx):
    from paper_2102_11026_amd import serve
    pa = small_class(0)
    pb = synth.tiny_problem(grid=(3, 3, 4), widths=(3, 32, 108), act="tanh", name="srvb", q_std=0.2,
                            out_scale=0.1)
    classes = [serve.RequestClass("a", pa, capacity=6), serve.RequestClass("b", pb, capacity=6)]
    srv = serve.Server(ctx, classes, "fp32", n_iters=3, keep_results=True)
    try:
        reqs = serve.poisson_arrivals(200.0, 0.15, ["a", "b"], 8, {"a": pa, "b": pb})
        stats = srv.run(reqs, max_seconds=60.0)
        assert stats["completed"] == len(reqs) > 5
        assert stats["p99_step_ms"] >= stats["p50_step_ms"] > 0
        # two completed requests re-run alone
        for req in reqs[:2]:
            p = (pa if req.cls == "a" else pb).replace(r0=req.r0)
            x = nmr.Instance(ctx, p, "fp32", shared=srv.classes[req.cls].decoder)
            st, _ = nmr.step_many(ctx, [x], 8, 3)
            np.testing.assert_array_equal(x.get_state()[0], srv.results[req.rid][0])
            x.close()
    finally:
        srv.close()


def test_pool_rejects_other_classes(nmr, ctx):
    """Instances whose Newton path, decoded cubature DOFs, formulation or
    derivative scheme differ from the pool's first member are refused, even
    with the same sizes and decoder (the pool's graph is captured from the
    first member)."""
    p = small_class(0)
    dec = nmr.Decoder(ctx, p.weights, p.biases, p.act, "fp32")
    pool = nmr.Pool(ctx, 4)
    other_ids = np.sort(synth.permutation("srv/other-cub", p.tets.shape[0])[: p.cub_ids.size]).astype(np.int32)
    variants = {
        "direct path": (p, "direct"),
        "other cubature tets": (p.replace(cub_ids=other_ids), "auto"),
        "trimmed": (p.replace(formulation="trimmed"), "auto"),
    }
    first = nmr.Instance(ctx, p, "fp32", shared=dec)
    made = [first]
    try:
        pool.attach(first)
        with pytest.raises(nmr.NmrError) as e:
            pool.attach(first)                       # already attached
        assert nmr.STATUS[e.value.code] == "arg"
        for name, (q, path) in variants.items():
            x = nmr.Instance(ctx, q, "fp32", shared=dec, path=path)
            made.append(x)
            with pytest.raises(nmr.NmrError) as e:
                pool.attach(x)
            assert nmr.STATUS[e.value.code] == "arg", name
        same = nmr.Instance(ctx, small_class(1), "fp32", shared=dec)
        made.append(same)
        pool.attach(same)                            # same class, other initial state: accepted
    finally:
        pool.close()
        for x in made:
            x.close()
        dec.close()


def test_destroying_an_attached_instance_detaches_it(nmr, ctx):
    """nmr_instance_destroy of a pool member frees its slot first, so the
    pool's next step never reaches the freed buffers; the remaining member
    continues as if stepped alone."""
    probs = [small_class(k) for k in range(2)]
    dec = nmr.Decoder(ctx, probs[0].weights, probs[0].biases, probs[0].act, "fp32")
    pool = nmr.Pool(ctx, 4)
    a, b = (nmr.Instance(ctx, q, "fp32", shared=dec) for q in probs)
    ref = nmr.Instance(ctx, probs[0], "fp32", shared=dec)
    try:
        sa = pool.attach(a)
        sb = pool.attach(b)
        pool.step(3)
        b.close()                                    # destroyed while attached
        st, _ = pool.step(3, status=True)
        assert st[sb] == 0 and st[sa] == 0
        c = nmr.Instance(ctx, probs[1], "fp32", shared=dec)
        s2 = pool.attach(c)
        assert s2 == sb                              # the freed slot is reused
        pool.detach(s2)
        c.close()
        st, _ = nmr.step_many(ctx, [ref], 2, 3)
        assert st == [0]
        # a (two pool steps) against the same request stepped alone twice
        close(a.get_state()[0], ref.get_state()[0], 1e-5, "r")
    finally:
        pool.close()
        for x in (a, ref):
            x.close()
        dec.close()
