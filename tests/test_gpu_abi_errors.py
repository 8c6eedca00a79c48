"""Input validation of the C ABI: every setter, option and solve argument
check returns its status code, leaves a readable message, and leaves the
context as it was (a valid solve afterwards gives the same result).  No
kernel runs for a rejected call."""
import ctypes

import numpy as np
import pytest

from paper_1903_00548_amd import _lib
from paper_1903_00548_amd import workloads as W

pytestmark = pytest.mark.gpu

ETA = 1e-6


@pytest.fixture(scope="module")
def ready():
    dev = W.small_random_device(3, 4, 6, uniform=False, same_leads=False, pot_mode=W.POT_LINEAR_FE)
    ctx = _lib.context_for(dev, 0)
    E = np.linspace(-1.0, 1.0, 5)
    T0, L0, _, _ = ctx.solve(E, ETA)
    return dev, ctx, E, T0, L0


def _status(fn, *args):
    with pytest.raises(_lib.QtxError) as ei:
        fn(*args)
    return ei.value.status


def _unchanged(ctx, E, T0, L0):
    T, L, _, st = ctx.solve(E, ETA)
    assert st == _lib.OK and np.array_equal(T, T0) and np.array_equal(L, L0)


def test_lead_validation(gpu_lib, ready):
    dev, ctx, E, T0, L0 = ready
    ld = dev.lead_L
    m = ld.m
    assert _status(ctx.set_lead, 2, ld.H00, ld.H01, ld.S00, ld.S01) == _lib.EINVAL          # bad side
    assert _status(ctx.set_lead, _lib.LEFT, ld.H00, ld.H01, ld.S00, ld.S01, np.nan) == _lib.EINVAL
    bad = ld.S00.copy()
    bad[0, 1] += 0.5                                                                        # S00 not Hermitian
    assert _status(ctx.set_lead, _lib.LEFT, ld.H00, ld.H01, bad, ld.S01) == _lib.EINVAL
    big = np.eye(m + 1, dtype=complex)                                                     # m differs
    assert _status(ctx.set_lead, _lib.RIGHT, big, big, big, big) == _lib.EINVAL
    null = ctx.lib.qtx_set_lead(ctx.h, _lib.LEFT, m, None, None, None, None, 0.0)
    assert null == _lib.EINVAL and b"NULL" in ctx.lib.qtx_last_error(ctx.h)
    for mm in (0, 129):
        assert ctx.lib.qtx_set_lead(ctx.h, _lib.LEFT, mm, None, None, None, None, 0.0) == _lib.EINVAL
    _unchanged(ctx, E, T0, L0)


def test_device_and_potential_validation(gpu_lib, ready):
    dev, ctx, E, T0, L0 = ready
    N, m = dev.N, dev.m
    Hd = dev.Hd.copy()
    Hd[1, 0, 2] += 1.0                                                                     # on-site block not Hermitian
    assert _status(ctx.set_device, N, m, Hd, dev.Hu, dev.Sd, dev.Su) == _lib.EINVAL
    assert ctx.lib.qtx_set_device(ctx.h, 0, m, None, None, None, None) == _lib.EINVAL      # N < 1
    assert ctx.lib.qtx_set_device(ctx.h, N, m + 1, None, None, None, None) == _lib.EINVAL  # m differs
    hd = np.ascontiguousarray(dev.Hd)
    assert ctx.lib.qtx_set_device(ctx.h, N, m, hd.ctypes.data_as(ctypes.c_void_p), None, None,
                                  None) == _lib.EINVAL                                     # some blocks only
    V = np.zeros(N)
    V[1] = np.inf
    assert _status(ctx.set_potential, V, W.POT_DIAG) == _lib.EINVAL
    assert _status(ctx.set_potential, np.zeros(N), 7) == _lib.EINVAL
    assert ctx.lib.qtx_set_potential(ctx.h, None, W.POT_DIAG) == _lib.EINVAL
    _unchanged(ctx, E, T0, L0)


def test_solve_argument_validation(gpu_lib, ready):
    dev, ctx, E, T0, L0 = ready
    assert _status(ctx.solve, np.array([0.1, np.nan]), ETA) == _lib.EINVAL
    assert _status(ctx.solve, E, -1e-3) == _lib.EINVAL
    assert _status(ctx.solve, E, ETA, 5) == _lib.EINVAL
    T = np.empty(len(E))
    Ep = E.ctypes.data_as(ctypes.c_void_p)
    assert ctx.lib.qtx_solve(ctx.h, Ep, -1, ETA, 0, T.ctypes.data_as(ctypes.c_void_p), None, None) == _lib.EINVAL
    assert ctx.lib.qtx_solve(ctx.h, Ep, len(E), ETA, 0, None, None, None) == _lib.EINVAL
    assert ctx.lib.qtx_solve(ctx.h, None, len(E), ETA, 0, T.ctypes.data_as(ctypes.c_void_p), None,
                             None) == _lib.EINVAL
    assert ctx.lib.qtx_solve(ctx.h, None, 0, ETA, 0, None, None, None) == _lib.OK           # empty grid
    _unchanged(ctx, E, T0, L0)


@pytest.mark.parametrize("name,bad,good", [
    ("decimation_tol", [0.0, 1.0, -1e-3, np.nan], 1e-14),
    ("decimation_max_iters", [0, 1001, 2.5], 60),
    ("decimation_refine_cond", [-1.0, np.nan], 1e4),
    ("refine_tol", [0.0, 1.0], 1e-12),
    ("refine_max_steps", [-1, 21, 1.5], 3),
    ("refine_weight_tol", [-0.1, 1.1], 1e-8),
    ("workgroups_per_cu", [0, 5, 1.5], 2),
    ("sigma_cache_bytes", [-1.0, 2e13], 16.0 * (1 << 30)),
    ("use_graph", [2, 0.5], 1),
    ("density_matrix_bytes", [-1.0, 2e13], 64.0 * (1 << 30)),
    ("sweep_workspace_bytes", [0.0, -1.0, 2e13, np.nan], 160.0 * (1 << 30)),
    ("self_energy_method", [2, -1], 0),
    ("mode_tol", [0.0, 0.5], 1e-8),
    ("energies_per_launch", [0, 2 ** 21, 3.5], 4096),
])
def test_option_validation(gpu_lib, ready, name, bad, good):
    dev, ctx, E, T0, L0 = ready
    for v in bad:
        assert _status(ctx.set_option, name, v) == _lib.EINVAL, (name, v)
    ctx.set_option(name, good)                       # the default is accepted
    _unchanged(ctx, E, T0, L0)


def test_unknown_option_and_null_name(gpu_lib, ready):
    dev, ctx, E, T0, L0 = ready
    assert _status(ctx.set_option, "no_such_option", 1.0) == _lib.EINVAL
    assert b"unknown option" in ctx.lib.qtx_last_error(ctx.h)
    assert ctx.lib.qtx_set_option(ctx.h, None, 1.0) == _lib.EINVAL


def test_null_context(gpu_lib):
    lib = _lib.load()
    assert lib.qtx_solve(None, None, 0, ETA, 0, None, None, None) == _lib.EINVAL
    assert lib.qtx_set_option(None, b"use_graph", 1.0) == _lib.EINVAL
    assert lib.qtx_density_matrix(None, None, None, None, 0, ETA, None, None, None, None, None) == _lib.EINVAL
    assert lib.qtx_last_error(None) == b"null context"
    lib.qtx_destroy(None)
