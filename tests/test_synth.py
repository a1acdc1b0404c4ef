"""The seeded input generator: published SplitMix64 outputs, determinism, shapes."""
import numpy as np
import pytest

from paper_2102_11026_amd import synth


def test_splitmix64_known_answers():
    """SplitMix64 from state 0: the first two outputs of the published generator."""
    ctr = np.array([1, 2], dtype=np.uint64)
    with np.errstate(over="ignore"):
        out = synth._mix(ctr * synth._GAMMA)
    assert [int(x) for x in out] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4]


def test_streams_are_deterministic_and_independent():
    a = synth.normal("dec/0", 1000)
    b = synth.normal("dec/0", 1000)
    c = synth.normal("dec/1", 1000)
    np.testing.assert_array_equal(a, b)
    assert abs(np.corrcoef(a, c)[0, 1]) < 0.1
    assert abs(a.mean()) < 0.1 and abs(a.std() - 1) < 0.1
    u = synth.uniform("x", 10000)
    assert u.min() > 0 and u.max() <= 1


def test_headline_config_shapes():
    p = synth.config_single_10k()
    assert p.n == 10000 and p.N == 30000 and p.tets.shape == (43320, 4)
    assert [W.shape for W in p.weights][0] == (64, 15) and p.weights[-1].shape == (30000, 256)
    assert sum(W.size for W in p.weights) == 9032640
    assert p.cub_ids.size == 500 and np.unique(p.cub_ids).size == 500
    assert p.pinned.sum() == 400
    assert p.steps == 100 and p.newton_iters == 4


def test_plain_config_shapes():
    p = synth.config_plain_fp64()
    assert p.N == 576 and p.tets.shape == (495, 4) and p.R == 3 and p.pinned.sum() == 16
    assert [W.shape for W in p.weights] == [(32, 3), (64, 32), (128, 64), (576, 128)]
