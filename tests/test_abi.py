"""C-ABI library checks that need no GPU: it builds, loads, exports every
function include/mnl.h declares, and its host-only functions behave."""
import ctypes
import os
import re
import subprocess

import pytest

from tests.conftest import ROOT, read_golden

HEADER = os.path.join(ROOT, "include", "mnl.h")
LIB = os.path.join(ROOT, "paper_1404_3177_amd", "libmnl.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mnl_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1404_3177_amd import build
        build.build()
    from paper_1404_3177_amd import _lib
    return _lib.load(LIB)


def test_header_declares_the_four_calls_and_helpers():
    fns = declared_functions()
    for f in ("mnl_fit", "mnl_loglik_grad", "mnl_hessian", "mnl_newton_step",
              "mnl_create", "mnl_destroy", "mnl_num_params"):
        assert f in fns


def test_library_exports_every_declared_symbol(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", LIB],
                         capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (mnl_[a-z_0-9]+)$", out, flags=re.M))
    missing = [f for f in declared_functions() if f not in exported]
    assert not missing, missing
    for f in declared_functions():
        assert hasattr(lib, f)


def test_binding_names_match_header():
    from paper_1404_3177_amd import _lib
    assert sorted(_lib.EXPORTS) == declared_functions()


def test_num_params(lib):
    for K, p, g, a, n_p, *_ in read_golden("num_params.txt"):
        assert lib.mnl_num_params(int(K), int(p), int(g), int(a)) == int(n_p)
    assert lib.mnl_num_params(1, 3, 0, 0) == -1
    assert lib.mnl_num_params(3, -1, 0, 0) == -1


def test_default_opts_are_mnlogit_defaults(lib):
    from paper_1404_3177_amd import _lib
    o = _lib.MnlFitOpts()
    lib.mnl_default_opts(ctypes.byref(o))
    assert (o.maxiter, o.ftol, o.gtol) == (50, 1e-6, 1e-6)
    assert o.prec == 0 and o.ls_max == 30 and o.ls_tol_ulps == 64.0


def test_strerror_and_version(lib):
    assert lib.mnl_version().decode().count(".") == 1
    assert lib.mnl_strerror(0) == b"ok"
    assert b"Hessian" in lib.mnl_strerror(-3)
    assert lib.mnl_strerror(-99) == b"unknown error"


def test_null_context_is_rejected(lib):
    # argument errors are caught before any device call
    assert lib.mnl_create(None, 0, 0) == -1
    assert lib.mnl_loglik_grad(None, None, None, None, None, None, None) == -1
    assert lib.mnl_fit(None, None, None, None, None, None, None) == -1
    assert lib.mnl_workspace_bytes(None) == 0
    lib.mnl_destroy(None)
    # the calls that widen the fit: methods, preprocessing, tests
    assert lib.mnl_hessian(None, None, None, 0, None, None) == -1
    assert lib.mnl_newton_step(None, None, None, None, None, None) == -1
    assert lib.mnl_hessvec(None, None, None, None, None, None) == -1
    assert lib.mnl_predict(None, None, None, None, None) == -1
    assert lib.mnl_stderr(None, None, None, None, None, None, None) == -1
    assert lib.mnl_covariance(None, None, None, None, 0, None, None) == -1
    assert lib.mnl_quadform(None, None, None, None, None, 1, 0, None,
                            None) == -1
    assert lib.mnl_collinear(None, None, 1e-6, None, None, None, None) == -1
    assert lib.mnl_select_columns(None, None, None, None, None, None, None,
                                  None, None) == -1


def test_default_method_is_exact_newton(lib):
    from paper_1404_3177_amd import _lib
    o = _lib.MnlFitOpts()
    lib.mnl_default_opts(ctypes.byref(o))
    assert o.method == 0 and o.cg_maxiter == 250 and o.validate == 0
    # graph-captured steps for small fits only (MNL_GRAPH_AUTO)
    assert o.graph == -1


def test_struct_layouts_match_header():
    # sizes of the ABI structs as laid out by the C compiler
    from paper_1404_3177_amd import _lib
    names = ["mnl_problem", "mnl_fit_opts", "mnl_fit_info",
             "mnl_server_opts", "mnl_server_result", "mnl_server_stats"]
    fmt = " ".join(["%zu"] * len(names))
    args = ", ".join(f"sizeof({n})" for n in names)
    src = f'#include "{HEADER}"\n#include <stdio.h>\nint main(void){{' \
          f'printf("{fmt}\\n", {args}); return 0;}}'
    exe = os.path.join("/tmp", "mnl_sizes")
    subprocess.run(["gcc", "-x", "c", "-", "-o", exe], input=src, text=True,
                   check=True)
    sizes = [int(x) for x in subprocess.run([exe], capture_output=True,
                                            text=True).stdout.split()]
    assert sizes == [ctypes.sizeof(_lib.MnlProblem),
                     ctypes.sizeof(_lib.MnlFitOpts),
                     ctypes.sizeof(_lib.MnlFitInfo),
                     ctypes.sizeof(_lib.MnlServerOpts),
                     ctypes.sizeof(_lib.MnlServerResult),
                     ctypes.sizeof(_lib.MnlServerStats)]


def test_server_null_arguments_are_rejected(lib):
    assert lib.mnl_server_create(None, None) == -1
    assert lib.mnl_server_submit(None, None, None, None, None, 0.0, None) == -1
    assert lib.mnl_server_wait(None, None, 0, 0.0, None) == -1
    assert lib.mnl_server_get_stats(None, None) == -1
    lib.mnl_server_destroy(None)
    t0 = lib.mnl_server_now_ms()
    assert lib.mnl_server_now_ms() >= t0


def test_batch_entry_points_without_a_device(lib):
    from paper_1404_3177_amd import _lib
    assert lib.mnl_fit_batch(None, 0, None, None, None, None, None,
                             None) == -1
    assert lib.mnl_batch_eligible(None, None) == 0
    shape = _lib.MnlProblem(N=2000, K=10, p=6, g=1, a=0)
    assert lib.mnl_batch_eligible(ctypes.byref(shape), None) == 1
    o = _lib.MnlFitOpts()
    lib.mnl_default_opts(ctypes.byref(o))
    o.maxiter = -1   # invalid options are never eligible
    assert lib.mnl_batch_eligible(ctypes.byref(shape), ctypes.byref(o)) == 0


def _footprint(N, K, p, g, a, prec="fp64", weights=False):
    import paper_1404_3177_amd as mnl
    return mnl.fit_footprint(N, K, p, g, a, prec, weights)


def test_fit_footprint_covers_data_and_grows_with_the_shape(lib):
    # host-only: the footprint comes from the kernels' plans, no device
    N, K, p, g, a = 100_000, 50, 21, 5, 5
    n_p = (K - 1) * p + K * a + g
    f = _footprint(N, K, p, g, a)
    data = 8 * N * (p + K * g + K * a) + 4 * N
    # data, two FP64 probability arrays and the Hessian at least
    assert f >= data + 2 * 8 * N * K + 8 * n_p * n_p
    assert _footprint(2 * N, K, p, g, a) > f
    # the observation split count of the Hessian follows the device's fill,
    # so the footprint is not monotone in K; it still covers data and P
    n_p1 = K * p + (K + 1) * a + g
    assert _footprint(N, K + 1, p, g, a) >= \
        8 * N * (p + (K + 1) * (g + a)) + 2 * 8 * N * (K + 1) + 8 * n_p1 * n_p1
    assert _footprint(N, K, p, g, a, weights=True) >= f + 8 * N
    # mixed precision adds the FP32 copies of P (and keeps FP64 room)
    assert _footprint(N, K, p, g, a, "bf16") > f
    assert _footprint(N, 1, p, g, a) == -1
    assert _footprint(0, K, p, g, a) == -1
    assert lib.mnl_fit_footprint(None, 0) == -1


def test_plans_of_every_kernel_path_build_on_the_host(lib):
    # shapes on both sides of the Hessian kernels' switches (the x rows of
    # the per-alternative sums in their own kernel for p <= 64 and
    # K (a + g) <= 512; outer-panel factorisation; no alternative-varying
    # data): each plan is built on the host by the footprint query
    shapes = [(1000, 5, 3, 2, 1), (1000, 5, 70, 2, 1), (1000, 200, 3, 2, 1),
              (400_000, 100, 51, 5, 0), (100_000, 50, 21, 5, 5),
              (1000, 3, 0, 2, 2), (500, 40, 20, 0, 16), (2000, 8, 64, 3, 3),
              (2000, 8, 65, 3, 3), (50_000, 500, 11, 0, 0)]
    for sh in shapes:
        for prec in ("fp64", "fp32", "bf16"):
            assert _footprint(*sh, prec) > 0, (sh, prec)
