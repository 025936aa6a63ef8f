"""Host-side parts of the hypothesis tests: the library's chi-square tail
and the data / coefficient selection of the Hausman-McFadden refit."""
import math

import numpy as np
import pytest
import scipy.stats

import synth


@pytest.fixture(scope="module")
def mnl():
    import paper_1404_3177_amd as m
    m._lib.load()
    return m


@pytest.mark.parametrize("x,df", [(0.5, 1), (3.84, 1), (10.0, 3), (100.0, 50),
                                  (1e-3, 7), (50.0, 2), (400.0, 300),
                                  (2.0, 0.5), (1e4, 9000)])
def test_chi2_sf_against_scipy(mnl, x, df):
    assert mnl.chi2_sf(x, df) == pytest.approx(scipy.stats.chi2.sf(x, df),
                                               rel=1e-12, abs=1e-300)


def test_chi2_sf_closed_forms_and_edges(mnl):
    for x in (0.1, 1.0, 7.5, 60.0):
        assert mnl.chi2_sf(x, 2) == pytest.approx(math.exp(-x / 2), rel=1e-13)
        assert mnl.chi2_sf(x, 1) == pytest.approx(math.erfc(math.sqrt(x / 2)),
                                                  rel=1e-12)
    assert mnl.chi2_sf(0.0, 4) == 1.0
    assert math.isnan(mnl.chi2_sf(1.0, 0.0))


def test_lrtest_in_the_library(mnl):
    # the statistic 2 (l_full - l_restricted) and its chi-square tail come
    # from mnl_lrtest; df <= 0 is an argument error
    from paper_1404_3177_amd import hypothesis as hyp
    s, df, p = hyp.lrtest(-1000.25, -1003.5, 2)
    assert s == 6.5 and df == 2
    assert p == pytest.approx(math.exp(-3.25), rel=1e-13)
    with pytest.raises(mnl.MnlError):
        mnl.lr_stat(-1.0, -2.0, 0)


def test_common_coefficients_layout():
    from paper_1404_3177_amd.hypothesis import common_coefficients
    # K = 4, p = 2, g = 1, a = 1: beta_1..3 at 0..5, gamma_0..3 at 6..9,
    # alpha at 10; the model on alternatives (0, 2, 3)
    assert common_coefficients(4, 2, 1, 1, [0, 2, 3]) == \
        [2, 3, 4, 5, 6, 8, 9, 10]
    assert common_coefficients(3, 1, 0, 0, [0, 1, 2]) == [0, 1]


def test_subset_problem_selects_rows_and_alternatives(mnl):
    import torch
    from paper_1404_3177_amd.hypothesis import subset_problem
    pr = synth.make_problem(200, 5, 3, 2, 1, seed=5, weights="uniform")
    t = lambda x, dt: torch.from_numpy(np.ascontiguousarray(x)).to(dt)
    prob = mnl.Problem(t(pr.X, torch.float64), t(pr.Y, torch.float64),
                       t(pr.Z, torch.float64), t(pr.choice, torch.int32),
                       t(pr.w, torch.float64))
    alts = [0, 3, 1]
    sub = subset_problem(prob, alts)
    m = np.isin(pr.choice, alts)
    lut = {0: 0, 3: 1, 1: 2}
    X, Y, Z, c, w = sub._refs
    assert np.array_equal(X.numpy(), pr.X[m])
    assert np.array_equal(Y.numpy(), pr.Y[m][:, alts])
    assert np.array_equal(Z.numpy(), pr.Z[m][:, alts])
    assert np.array_equal(c.numpy(), [lut[k] for k in pr.choice[m]])
    assert np.array_equal(w.numpy(), pr.w[m])
    with pytest.raises(ValueError):
        subset_problem(prob, [1, 2])
