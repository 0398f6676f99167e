"""The rule by which FP32 parity tests explain a site that differs from the
oracle (tests/gpu_util.explainable): a decision within 1e-4 of its
threshold in half-sweep h of an nsw-sweep pass may come out the other way,
and its effect reaches at most 2 nsw - 1 - h sites further by the end of
the pass.  Host logic only."""
import numpy as np
import pytest

from tests.gpu_util import chain_margins, explainable, mismatches


def _margins(shape, near=()):
    m = {k: np.full(shape, np.inf) for k in ("accept", "or_edge", "wrap")}
    for (y, x), key in near:
        m[key][y, x] = 1e-6
    return m


def _ball(shape, y0, x0, r):
    yy, xx = np.mgrid[0:shape[0], 0:shape[1]]
    return (np.abs(yy - y0) + np.abs(xx - x0)) <= r


def test_first_half_sweep_reaches_the_rest_of_the_pass():
    shape = (11, 11)
    # colour-0 site (4, 4) in sweep 0 of two: three later half-sweeps
    expl = explainable([_margins(shape, [((4, 4), "accept")]), _margins(shape)])
    assert np.array_equal(expl, _ball(shape, 4, 4, 3))


def test_last_half_sweep_explains_only_its_site():
    shape = (9, 9)
    # colour-1 site (4, 5) in the last sweep of two
    expl = explainable([_margins(shape), _margins(shape, [((4, 5), "wrap")])])
    assert np.array_equal(expl, _ball(shape, 4, 5, 0))


def test_one_sweep_colour0_reaches_its_colour1_neighbours():
    shape = (6, 7)
    expl = explainable([_margins(shape, [((2, 2), "or_edge")])])
    assert np.array_equal(expl, _ball(shape, 2, 2, 1))
    # at the frame's corner the ball is cut, not wrapped
    expl = explainable([_margins(shape, [((0, 0), "accept")])])
    assert np.array_equal(expl, _ball(shape, 0, 0, 1))


def test_origin_sets_the_colour():
    shape = (9, 9)
    # (4, 4) of a frame whose (0, 0) is grid site (0, 1) has colour 1
    expl = explainable([_margins(shape, [((4, 4), "accept")])], origin=(0, 1))
    assert np.array_equal(expl, _ball(shape, 4, 4, 0))


def test_far_margins_explain_nothing():
    shape = (5, 5)
    m = _margins(shape)
    m["accept"][2, 2] = 2e-4  # beyond the 1e-4 threshold
    assert not explainable([m]).any()
    assert explainable([m], thr=1e-3)[2, 2]


def test_mismatches_counts_gap_sites_only():
    ref = np.zeros((4, 4))
    got = ref.copy()
    got[0, 0] = got[1, 1] = got[2, 3] = 0.01
    known = np.zeros((4, 4), dtype=np.uint8)
    known[2, 3] = 1  # a sample site: never counted
    expl = np.zeros((4, 4), dtype=bool)
    expl[1, 1] = True
    n_bad, n_expl, unexpl = mismatches(got, ref, expl, known, 1e-3)
    assert (n_bad, n_expl) == (2, 1)
    assert unexpl.tolist() == [[0, 0]]


def test_chain_margins_and_shape_check():
    m = {k: np.full((3, 4, 5), np.inf) for k in ("accept", "or_edge", "wrap")}
    m["accept"][1, 2, 3] = 0.0
    one = chain_margins(m, 1)
    assert one["accept"].shape == (4, 5) and one["accept"][2, 3] == 0.0
    with pytest.raises(AssertionError):
        explainable([m])
