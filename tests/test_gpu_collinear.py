"""Parity of the GPU collinearity check (linDepTol, App. B) and column
selection with the oracle."""
import numpy as np
import pytest

import synth
from oracle import mnl_ref as R
from tests.gpu_util import device_problem

pytestmark = pytest.mark.gpu
GTOL = 1e-8


@pytest.fixture(scope="module")
def ctx():
    import paper_1404_3177_amd as mnl
    return mnl.Context(0)


def _dependent_problem(seed):
    """Data with exact and near dependencies of every kind."""
    pr = synth.make_problem(2000, 5, 6, 3, 3, seed=seed, weights="uniform")
    rng = np.random.default_rng(seed)
    pr.X[:, 3] = 2.0 * pr.X[:, 1] - pr.X[:, 2]            # exact
    pr.X[:, 5] = pr.X[:, 4] + 1e-9 * rng.normal(size=pr.N)  # below tol
    pr.X[:, 2] += 0.0
    pr.Z[:, 2, 2] = pr.Z[:, 2, 0] - 3.0 * pr.Z[:, 2, 1]   # one alternative
    pr.Y[:, :, 2] = pr.Y[:, :, 0] + 1e-3 * rng.normal(size=(pr.N, 5))  # kept
    return pr


@pytest.mark.parametrize("case", ["random", "dependent", "zero", "app_b",
                                  "wide"])
def test_masks_match_oracle(ctx, case):
    if case == "random":
        pr = synth.make_problem(3000, 7, 5, 2, 2, seed=31)
    elif case == "wide":
        # fewer observations than columns: X keeps at most N columns
        pr = synth.make_problem(12, 3, 20, 1, 1, seed=39)
    elif case == "dependent":
        pr = _dependent_problem(32)
    elif case == "zero":
        pr = synth.make_problem(500, 4, 4, 2, 2, seed=33)
        pr.X[:, 2] = 0.0
        pr.Z[:, :, 1] = 0.0
    else:
        pr = synth.make_problem(500, 4, 2, 2, 1, seed=18)
        pr.Y = np.ascontiguousarray(np.repeat(pr.Y[:, :1, :], 4, axis=1))
    ref = R.collinearity_mask(pr.X, pr.Y, pr.Z)
    got = ctx.collinear(device_problem(pr))
    for r, g_ in zip(ref, got):
        np.testing.assert_array_equal(g_, r, err_msg=case)


def test_dependent_masks_as_constructed(ctx):
    kx, ky, kz = ctx.collinear(device_problem(_dependent_problem(32)))
    np.testing.assert_array_equal(kx, [1, 1, 1, 0, 1, 0])
    np.testing.assert_array_equal(ky, [1, 1, 1])
    np.testing.assert_array_equal(kz, [1, 1, 0])


def test_select_columns_exact(ctx):
    pr = _dependent_problem(34)
    dp = device_problem(pr)
    kx, ky, kz = ctx.collinear(dp)
    dq = ctx.select_columns(dp, kx, ky, kz)
    X, Y, Z, c, w = dq._refs
    assert np.array_equal(X.cpu().numpy(), pr.X[:, kx])
    assert np.array_equal(Y.cpu().numpy(), pr.Y[:, :, ky])
    assert np.array_equal(Z.cpu().numpy(), pr.Z[:, :, kz])


def test_singular_model_fits_after_dropping(ctx):
    # App. B: generic data constant over alternatives make H singular; the
    # reduced problem fits and matches the oracle's fit of the same data
    pr = synth.make_problem(3000, 5, 3, 2, 1, seed=35, weights="uniform")
    pr.Y = np.ascontiguousarray(np.repeat(pr.Y[:, :1, :], 5, axis=1))
    pr.X[:, 2] = 0.5 * pr.X[:, 1] + 2.0 * pr.X[:, 0]
    dp = device_problem(pr)
    _, info = ctx.fit(dp, gtol=GTOL, ftol=0.0)
    assert info["stop_reason"] == R.STOP_NOT_PD
    kx, ky, kz = ctx.collinear(dp)
    dq = ctx.select_columns(dp, kx, ky, kz)
    theta, info = ctx.fit(dq, gtol=GTOL, ftol=0.0)
    assert info["stop_reason"] == R.STOP_GTOL
    ref = R.fit(pr.X[:, kx], pr.Y[:, :, ky], pr.Z[:, :, kz], pr.choice, pr.w,
                opts=R.FitOptions(gtol=GTOL, ftol=0.0))
    th = theta.cpu().numpy()
    assert np.linalg.norm(th - ref.theta) <= 1e-8 * np.linalg.norm(ref.theta)


def test_config_data_full_rank(ctx):
    pr = synth.make_config("c2")
    kx, ky, kz = ctx.collinear(device_problem(pr))
    assert kx.all() and ky.all() and kz.all()


@pytest.mark.parametrize("case", ["many_alternatives", "library_route"])
def test_masks_match_oracle_other_routes(ctx, case):
    rng = np.random.default_rng(36)
    if case == "many_alternatives":
        # 129 alternatives: long staged rows in the one-pass Gram kernel
        pr = synth.make_problem(1500, 129, 3, 2, 2, seed=37)
        pr.Z[:, 100, 1] = 2.0 * pr.Z[:, 100, 0]
        pr.Y[:, :, 1] = pr.Y[:, :, 0] + 0.5      # Ytil_1 = Ytil_0
    else:
        # 5,050 X^T X entries: the library GEMM route (Ytil formed first)
        pr = synth.make_problem(3000, 4, 100, 2, 1, seed=38)
        pr.X[:, 70] = pr.X[:, 3] - pr.X[:, 50]
        pr.X[:, 99] = 0.0
        pr.Y[:, :, 1] = 3.0 * pr.Y[:, :, 0] + rng.normal(size=(3000, 1))
    ref = R.collinearity_mask(pr.X, pr.Y, pr.Z)
    got = ctx.collinear(device_problem(pr))
    for r, g_ in zip(ref, got):
        np.testing.assert_array_equal(g_, r, err_msg=case)
    if case == "many_alternatives":
        np.testing.assert_array_equal(got[1], [1, 0])
        np.testing.assert_array_equal(got[2], [1, 0])
    else:
        assert got[0].sum() == 98 and not got[0][70] and not got[0][99]
