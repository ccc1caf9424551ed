"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every entry point include/cggm.h declares, and rejects bad arguments before
touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "cggm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cggm_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    import paper_1509_04681_amd as m
    if not os.path.exists(m.LIB_PATH):
        from paper_1509_04681_amd import build
        build.build()
    return m.load()


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("cggm_solve", "cggm_objective", "cggm_gradient", "cggm_result_info",
                     "cggm_result_copy", "cggm_result_free", "cggm_status_string",
                     "cggm_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings(lib):
    import paper_1509_04681_amd as m
    for code in (0, 1, 2, -1, -2, -3, -4, -5, -6):
        assert m.cggm_status_string(code) != "unknown status"
    assert m.cggm_status_string(42) == "unknown status"


def test_argument_errors_without_device(lib):
    import paper_1509_04681_amd as m
    r = ctypes.c_void_p()
    fake = ctypes.c_void_p(64)          # never dereferenced: validation fails first
    assert lib.cggm_solve(None, fake, 4, 3, 2, 0, 0.1, 0.1, 0.01, None, ctypes.byref(r), None) \
        == m.CGGM_EINVAL
    assert lib.cggm_solve(fake, fake, 0, 3, 2, 0, 0.1, 0.1, 0.01, None, ctypes.byref(r), None) \
        == m.CGGM_EINVAL
    assert lib.cggm_solve(fake, fake, 4, 3, 2, 0, -0.1, 0.1, 0.01, None, ctypes.byref(r), None) \
        == m.CGGM_EINVAL
    assert lib.cggm_solve(fake, fake, 4, 3, 2, 0, 0.1, float("nan"), 0.01, None, ctypes.byref(r),
                          None) == m.CGGM_EINVAL
    assert lib.cggm_solve(fake, fake, 4, 3, 2, 0, 0.1, 0.1, -1.0, None, ctypes.byref(r), None) \
        == m.CGGM_EINVAL
    assert b"tol" in lib.cggm_last_error()
    assert lib.cggm_solve(fake, fake, 4, 3, 2, 2, 0.1, 0.1, 0.01, None, ctypes.byref(r),
                          None) == m.CGGM_EINVAL            # dtype neither F64 nor F32
    assert b"dtype" in lib.cggm_last_error()
    f = ctypes.c_double()
    assert lib.cggm_objective(fake, fake, 4, 3, 2, 5, fake, fake, 0.1, 0.1, ctypes.byref(f),
                              None) == m.CGGM_EINVAL
    assert lib.cggm_objective_noalloc(fake, fake, 4, 3, 2, -1, fake, fake, 0.1, 0.1,
                                      ctypes.byref(f), None) == m.CGGM_EINVAL
    opt = m.Options()
    lib.cggm_default_options(ctypes.byref(opt))
    opt.ls_beta = 1.5
    assert lib.cggm_solve(fake, fake, 4, 3, 2, 0, 0.1, 0.1, 0.01, ctypes.byref(opt),
                          ctypes.byref(r), None) == m.CGGM_EINVAL
    lib.cggm_default_options(ctypes.byref(opt))
    opt.tile = 65
    assert lib.cggm_solve(fake, fake, 4, 3, 2, 0, 0.1, 0.1, 0.01, ctypes.byref(opt),
                          ctypes.byref(r), None) == m.CGGM_EINVAL
    lib.cggm_default_options(ctypes.byref(opt))
    opt.precision = 2
    assert lib.cggm_solve(fake, fake, 4, 3, 2, 0, 0.1, 0.1, 0.01, ctypes.byref(opt),
                          ctypes.byref(r), None) == m.CGGM_EINVAL
    lib.cggm_default_options(ctypes.byref(opt))
    opt.lambda_passes = -1
    assert lib.cggm_solve(fake, fake, 4, 3, 2, 0, 0.1, 0.1, 0.01, ctypes.byref(opt),
                          ctypes.byref(r), None) == m.CGGM_EINVAL
    lib.cggm_default_options(ctypes.byref(opt))
    opt.mixed_min_q = -1
    assert lib.cggm_solve(fake, fake, 4, 3, 2, 0, 0.1, 0.1, 0.01, ctypes.byref(opt),
                          ctypes.byref(r), None) == m.CGGM_EINVAL


def test_workspace_budget_is_checked_before_allocation(lib):
    import paper_1509_04681_amd as m
    need = m.cggm_solve_workspace_bytes(50, 40, 30)
    assert need > 8 * (30 * 30 * 11 + 40 * 30 * 5 + 40 * 40)
    opt = m.Options()
    lib.cggm_default_options(ctypes.byref(opt))
    opt.workspace_budget = need - 1
    r = ctypes.c_void_p()
    fake = ctypes.c_void_p(64)
    assert lib.cggm_solve(fake, fake, 50, 40, 30, 0, 0.1, 0.1, 0.01, ctypes.byref(opt),
                          ctypes.byref(r), None) == m.CGGM_ENOMEM
    # footprint at the 20000 x 20000 workload fits one 288 GB device
    assert m.cggm_solve_workspace_bytes(1000, 20000, 20000) < 100e9


def test_default_options(lib):
    import paper_1509_04681_amd as m
    opt = m.Options()
    lib.cggm_default_options(ctypes.byref(opt))
    assert (opt.max_iter, opt.max_ls, opt.ls_beta, opt.ls_sigma, opt.stall_iters) == \
        (500, 30, 0.5, 1e-3, 3)
    assert opt.sweep == m.CGGM_SWEEP_TILED
    assert opt.lambda_passes == 0            # auto: 4 when n >= q / 4, else 6
    assert opt.precision == m.CGGM_PRECISION_FP64
    assert opt.mixed_min_q == 4096
    assert (opt.theta_passes, opt.split_level, opt.split_adapt) == (1, 0, 1)
    assert m.cggm_status_string(m.CGGM_STALLED).startswith("stopped at the rounding floor")


def test_path_and_workspace_arguments_without_device(lib):
    import paper_1509_04681_amd as m
    fake = ctypes.c_void_p(64)
    lam = (ctypes.c_double * 3)(0.3, 0.2, 0.1)
    bad = (ctypes.c_double * 3)(0.3, -0.2, 0.1)
    out = (ctypes.c_void_p * 3)()
    dp = ctypes.POINTER(ctypes.c_double)
    L = ctypes.cast(lam, dp)
    assert lib.cggm_solve_path(fake, fake, 4, 3, 2, 0, 0, L, L, 0.01, None, out, None) \
        == m.CGGM_EINVAL
    assert lib.cggm_solve_path(fake, fake, 4, 3, 2, 0, 3, None, L, 0.01, None, out, None) \
        == m.CGGM_EINVAL
    assert lib.cggm_solve_path(fake, fake, 4, 3, 2, 0, 3, L, ctypes.cast(bad, dp), 0.01, None, out,
                               None) == m.CGGM_EINVAL
    assert lib.cggm_solve_path(fake, fake, 4, 3, 2, 0, 3, L, L, 0.01, None, None, None) \
        == m.CGGM_EINVAL
    # footprints: the mixed mode adds the BF16 planes; invalid options give 0
    fp64 = m.cggm_workspace_bytes(300, 200, 100)
    assert fp64 == m.cggm_solve_workspace_bytes(300, 200, 100)
    # the mixed mode's buffers (BF16 pieces, FP32 sweep copies) only from q = 4096 on
    opt = m.Options()
    lib.cggm_default_options(ctypes.byref(opt))
    opt.precision = m.CGGM_PRECISION_MIXED
    small = lib.cggm_workspace_bytes(300, 200, 100, ctypes.byref(opt))
    assert small == fp64
    opt.mixed_min_q = 0
    forced = lib.cggm_workspace_bytes(300, 200, 100, ctypes.byref(opt))
    assert forced - small >= 4 * (4 * 100 * 100 + 200 * 200 + 200 * 100)
    for field, value in (("lambda_passes", -1), ("theta_passes", 0), ("split_level", -1),
                         ("split_level", 7)):
        opt = m.Options()
        lib.cggm_default_options(ctypes.byref(opt))
        setattr(opt, field, value)
        assert lib.cggm_workspace_bytes(300, 200, 100, ctypes.byref(opt)) == 0, (field, value)
    assert lib.cggm_workspace_bytes(0, 200, 100, None) == 0


def test_blockwise_footprint(lib):
    """The block-wise mode holds a slab of Sxx columns (the budget, whole row
    tiles of 64 p doubles, at least one) in place of the p x p matrix."""
    import paper_1509_04681_amd as m
    n, p, q = 1000, 20000, 4000
    dense = m.cggm_workspace_bytes(n, p, q)
    block = m.cggm_workspace_bytes(n, p, q, blockwise=True, sxx_cache_bytes=1 << 30)
    slab = (1 << 30) // (64 * p * 8) * 64 * p * 8
    assert dense - block == 8 * p * p - slab
    tiny = m.cggm_workspace_bytes(n, p, q, blockwise=True, sxx_cache_bytes=1)
    assert dense - tiny == 8 * p * p - 64 * p * 8
    # the block-wise configuration's size: p = 200000, q = 40000 -- Sxx alone
    # would be 320 GB; the dense p x q arrays (Theta, V, the gradient, Sxy and
    # the guard's copy of Theta, 64 GB each) still exceed one device
    big_dense = m.cggm_workspace_bytes(n, 200000, 40000)
    big_block = m.cggm_workspace_bytes(n, 200000, 40000, blockwise=True)
    assert big_dense - big_block == 8 * 200000 ** 2 - (2 << 30) // (64 * 200000 * 8) * 64 * 200000 * 8
    assert big_block > 288e9


def test_server_arguments_without_device(lib):
    import paper_1509_04681_amd as m
    h = ctypes.c_void_p()
    assert lib.cggm_server_create(0, 1 << 20, 4, ctypes.byref(h)) == m.CGGM_EINVAL
    assert lib.cggm_server_create(65, 1 << 20, 4, ctypes.byref(h)) == m.CGGM_EINVAL
    assert lib.cggm_server_create(2, 100, 4, ctypes.byref(h)) == m.CGGM_EINVAL
    assert lib.cggm_server_create(2, 1 << 20, -1, ctypes.byref(h)) == m.CGGM_EINVAL
    assert lib.cggm_server_create(2, 1 << 20, 4, None) == m.CGGM_EINVAL
    t = ctypes.c_int64()
    req = m.Request()
    assert lib.cggm_server_submit(None, ctypes.byref(req), ctypes.byref(t)) == m.CGGM_EINVAL
    assert lib.cggm_server_wait(None, 1, None, None, None) == m.CGGM_EINVAL
    st = m.ServerStats()
    assert lib.cggm_server_stats_get(None, ctypes.byref(st)) == m.CGGM_EINVAL
    lib.cggm_server_destroy(None)


def test_sigma_columns_arguments_without_device(lib):
    import numpy as np
    import paper_1509_04681_amd as m
    fake = ctypes.c_void_p(64)          # never dereferenced: validation fails first
    cols = np.array([0, 3], dtype=np.int32)
    cp = cols.ctypes.data_as(ctypes.c_void_p)
    it, res = ctypes.c_int(7), ctypes.c_double(7.0)

    def call(q, c, k, tol, max_iter, ptr=fake):
        return lib.cggm_sigma_columns(ptr, fake, fake, q, c, k, tol, max_iter, fake,
                                      ctypes.byref(it), ctypes.byref(res), None)

    assert call(0, cp, 2, 1e-10, 100) == m.CGGM_EINVAL          # q >= 1
    assert call(4, cp, -1, 1e-10, 100) == m.CGGM_EINVAL         # k >= 0
    assert call(4, cp, 2, 1e-10, 0) == m.CGGM_EINVAL            # max_iter >= 1
    assert call(4, cp, 2, -1.0, 100) == m.CGGM_EINVAL           # tol >= 0
    assert call(4, cp, 2, float("nan"), 100) == m.CGGM_EINVAL
    assert call(4, cp, 2, float("inf"), 100) == m.CGGM_EINVAL
    assert call(3, cp, 2, 1e-10, 100) == m.CGGM_EINVAL          # column 3 outside [0, 3)
    assert "column index 3" in m.load().cggm_last_error().decode()
    assert call(4, cp, 2, 1e-10, 100, ptr=None) == m.CGGM_EINVAL
    # no columns: nothing to do, outputs zeroed, no device access
    assert call(4, None, 0, 1e-10, 100) == m.CGGM_OK
    assert it.value == 0 and res.value == 0.0


def test_remaining_entry_points_reject_bad_arguments_without_device(lib):
    """The gradient, the Newton-direction probe, the tile tuner and the result
    accessors validate their arguments before any device work."""
    import paper_1509_04681_amd as m
    fake = ctypes.c_void_p(64)          # never dereferenced: validation fails first
    assert lib.cggm_gradient(None, fake, 4, 3, 2, 0, fake, fake, fake, fake, None) \
        == m.CGGM_EINVAL
    assert lib.cggm_gradient(fake, fake, 4, 3, 2, 0, fake, fake, None, fake, None) \
        == m.CGGM_EINVAL
    assert lib.cggm_gradient(fake, fake, 0, 3, 2, 0, fake, fake, fake, fake, None) \
        == m.CGGM_EINVAL
    assert lib.cggm_gradient(fake, fake, 4, 3, 2, 7, fake, fake, fake, fake, None) \
        == m.CGGM_EINVAL
    assert lib.cggm_lambda_direction(fake, fake, 4, 3, 2, 0, None, fake, 0.1, 0.1, None,
                                     fake, None, None, None) == m.CGGM_EINVAL
    assert lib.cggm_lambda_direction(fake, fake, 4, 3, 2, 0, fake, fake, -0.1, 0.1, None,
                                     fake, None, None, None) == m.CGGM_EINVAL
    assert lib.cggm_lambda_direction(fake, fake, 4, -3, 2, 0, fake, fake, 0.1, 0.1, None,
                                     fake, None, None, None) == m.CGGM_EINVAL
    tile = ctypes.c_int()
    assert lib.cggm_autotune_tile(100, 50, 50, None, 4, None, None, None) == m.CGGM_EINVAL
    assert lib.cggm_autotune_tile(100, 50, 50, None, 0, ctypes.byref(tile), None, None) \
        == m.CGGM_EINVAL
    assert lib.cggm_autotune_tile(0, 50, 50, None, 4, ctypes.byref(tile), None, None) \
        == m.CGGM_EINVAL
    nL, nT, it, f = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int(), ctypes.c_double()
    st = ctypes.c_int()
    assert lib.cggm_result_info(None, ctypes.byref(nL), ctypes.byref(nT), ctypes.byref(it),
                                ctypes.byref(f), ctypes.byref(st)) == m.CGGM_EINVAL
    assert lib.cggm_result_dense(None, fake, fake, 0) == m.CGGM_EINVAL
    lib.cggm_result_free(None)            # a no-op
