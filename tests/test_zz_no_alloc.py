"""cubature_force_stiffness_noalloc (working memory in the library's static
device array, no allocation per call) against cubature_force_stiffness on
the same inputs, through the C ABI: two calls in a row, the second with a
smaller cubature set and reduced size, in FP32 and FP64.  Both run the same
kernels in the same order, so the results must be the same bits.  A
cubature set whose working memory exceeds the 16 MiB array is refused with
NMR_ERR_ARG before any device work.
"""
import numpy as np
import pytest

from paper_2102_11026_amd import synth

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


def inputs(p, seed):
    rng = np.random.default_rng(seed)
    u = rng.normal(size=p.N) * 0.004 * np.repeat(1 - p.pinned, 3)
    Jt = rng.normal(size=(p.N, p.R)) * 0.1
    w = rng.uniform(0.5, 2.0, size=p.cub_ids.size)
    return u, Jt, w


def compare(nmr, ctx, p, prec, seed):
    inst = nmr.Instance(ctx, p, prec)
    try:
        u, Jt, w = inputs(p, seed)
        got = inst.cubature_force_stiffness(u, Jt, w, noalloc=True)
        ref = inst.cubature_force_stiffness(u, Jt, w)
        for k in ("f_int", "fr", "Kr"):
            g, r = got[k].cpu().numpy(), ref[k].cpu().numpy()
            assert g.shape == r.shape, k
            assert np.array_equal(g, r), (p.name, prec, k, float(np.abs(g - r).max()))
        # the instance's own weights (w = NULL) as well
        got = inst.cubature_force_stiffness(u, Jt, None, want_fint=False, noalloc=True)
        ref = inst.cubature_force_stiffness(u, Jt, None, want_fint=False)
        assert np.array_equal(got["Kr"].cpu().numpy(), ref["Kr"].cpu().numpy())
        assert np.array_equal(got["fr"].cpu().numpy(), ref["fr"].cpu().numpy())
    finally:
        inst.close()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_noalloc_equals_allocating_call_twice_second_smaller(nmr, ctx, prec):
    big = synth.config_single_10k()                              # |C| = 500, R = 15, N = 30,000
    small = synth.tiny_problem(grid=(2, 2, 4), widths=(2, 4, 4, 48), name="noalloc_small")  # 15 tets, R = 2
    assert small.cub_ids.size < big.cub_ids.size and small.R < big.R and small.N < big.N
    compare(nmr, ctx, big, prec, seed=3)
    compare(nmr, ctx, small, prec, seed=4)


def test_noalloc_refuses_a_cubature_set_beyond_the_static_array(nmr, ctx):
    p = synth.config_single_10k()
    m = p.tets.shape[0]                                          # 43,320 tets: 20.8 MB of partials at R = 15
    p = p.replace(cub_ids=np.arange(m, dtype=np.int32), cub_w=np.ones(m), wnet_weights=None, wnet_biases=None,
                  wnet_scale=1.0)
    inst = nmr.Instance(ctx, p, "fp32")
    try:
        u, Jt, w = inputs(p, 5)
        with pytest.raises(nmr.NmrError) as e:
            inst.cubature_force_stiffness(u, Jt, w, noalloc=True)
        assert e.value.code == -1 and "static scratch" in str(e.value)
        # the allocating call still takes it
        out = inst.cubature_force_stiffness(u, Jt, w, want_fint=False)
        assert np.isfinite(out["Kr"].cpu().numpy()).all()
    finally:
        inst.close()
