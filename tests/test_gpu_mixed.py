"""GPU parity of the mixed-precision path (QTX_MIXED) against the FP64 oracle
and against the FP64 GPU path.

The bulk of the sweep runs in single precision; the heavy columns of the
broadening factors are refined against an FP64 residual and the energies
whose refinement does not converge are re-solved in FP64.

Tolerances: |dT| <= 1e-8 absolute per energy; slab densities
|dn| <= 1e-8 * max(1, max_i |n_i|) per energy and contact (single-energy
densities reach 10^3 near resonances; the charge, summed over energies,
is held to 1e-8 absolute against the oracle in test_gpu_charge.py).
"""
import numpy as np
import pytest

import oracle
from paper_1903_00548_amd import _lib
from paper_1903_00548_amd import workloads as W

import small_cases

pytestmark = pytest.mark.gpu

TOL_T = 1e-8
TOL_N = 1e-8


def _errors(T, L, Tref, Lref):
    dT = np.abs(T - Tref)
    scale = np.maximum(1.0, np.abs(Lref).max(axis=2))
    dn = np.abs(L - Lref).max(axis=2) / scale
    return dT.max(), dn.max()


def _check(T, L, Tref, Lref, label="", tolT=TOL_T, tolN=TOL_N):
    assert np.all(np.isfinite(T)) and np.all(np.isfinite(L)), label
    dT, dn = _errors(T, L, Tref, Lref)
    print(f"{label}: max|dT| = {dT:.3e}, max rel|dn| = {dn:.3e}")
    assert dT <= tolT, f"{label} max|dT|={dT:.3e}"
    assert dn <= tolN, f"{label} max rel|dn|={dn:.3e}"


def test_mixed_cfg0(gpu_lib):
    wl = W.config0()
    ctx = _lib.context_for(wl.device, 0)
    T, L, info, st = ctx.solve(wl.E, wl.eta, _lib.MIXED)
    assert st == _lib.OK
    Tref, Lref = oracle.solve_device(wl.device, wl.E, wl.eta)
    _check(T, L, Tref, Lref, "cfg0 mixed")
    assert np.all(info["refine_steps"] <= 3)
    assert np.all((info["resid"] <= 3e-11) | (info["fell_back_fp64"] == 1))


@pytest.mark.parametrize("case", small_cases.CASES, ids=lambda c: f"seed{c[0]}-N{c[1]}-m{c[2]}")
def test_mixed_small_devices(gpu_lib, case):
    dev = small_cases.device(*case)
    E = small_cases.energies()
    ctx = _lib.context_for(dev, 0)
    T, L, info, st = ctx.solve(E, small_cases.ETA, _lib.MIXED)
    Tref, Lref = small_cases.reference(*case)
    _check(T, L, Tref, Lref, label=f"seed{case[0]} mixed")


def test_mixed_cfg1_full_size(gpu_lib, cfg1_oracle):
    """Headline workload, 2048 energies in one call: every energy against the
    FP64 GPU path (held to 1e-10 of the oracle by the FP64 parity tests),
    64 sampled energies against the oracle directly."""
    wl, idx, Tref, Lref = cfg1_oracle
    dev = wl.device
    ctx = _lib.context_for(dev, 0)
    T64, L64, _, _ = ctx.solve(wl.E, wl.eta, _lib.FP64)
    T, L, info, st = ctx.solve(wl.E, wl.eta, _lib.MIXED)
    assert st == _lib.OK
    _check(T, L, T64, L64, "cfg1 mixed vs fp64 (all 2048)", tolT=TOL_T - 1e-10, tolN=TOL_N)
    _check(T[idx], L[idx], Tref, Lref, "cfg1 mixed vs oracle (64 sampled)")
    steps = info["refine_steps"]
    print("refinement steps histogram:", np.bincount(steps, minlength=4).tolist(),
          "fallbacks:", int(info["fell_back_fp64"].sum()))
    assert steps.max() <= 3


def test_mixed_cfg2_full_size(gpu_lib, cfg2_oracle):
    """N = 400, m = 128, all 4096 energies (3840 uniform, 256 within 1 meV of
    a band edge) in one mixed call, as the benchmark runs it: every energy
    within 1e-8 of the FP64 path, the 16 sampled energies against the
    oracle."""
    wl, idx, n_uni, Tref, Lref = cfg2_oracle
    ctx = _lib.context_for(wl.device, 0)
    T64, L64, _, _ = ctx.solve(wl.E, wl.eta, _lib.FP64)
    T, L, info, st = ctx.solve(wl.E, wl.eta, _lib.MIXED)
    assert st == _lib.OK
    _check(T[:n_uni], L[:n_uni], T64[:n_uni], L64[:n_uni], "cfg2 mixed vs fp64 (3840 uniform)",
           tolT=TOL_T - 1e-10)
    _check(T[n_uni:], L[n_uni:], T64[n_uni:], L64[n_uni:], "cfg2 mixed vs fp64 (256 band edge)",
           tolT=TOL_T - 1e-10)
    _check(T[idx], L[idx], Tref, Lref, "cfg2 mixed vs oracle (16 sampled)")
    assert info["refine_steps"].max() <= 3


def test_mixed_forced_fallback_is_the_fp64_result(gpu_lib):
    """No correction allowed and an unreachable tolerance: every energy is
    re-solved by the FP64 sweep, whose result must be bitwise the FP64
    path's, with the fallback recorded and no flag left set."""
    wl = W.config0()
    ctx = _lib.context_for(wl.device, 0)
    T64, L64, _, _ = ctx.solve(wl.E, wl.eta, _lib.FP64)
    ctx.set_option("refine_max_steps", 0)
    ctx.set_option("refine_tol", 1e-300)
    T, L, info, st = ctx.solve(wl.E, wl.eta, _lib.MIXED)
    assert st == _lib.OK
    assert np.array_equal(T, T64) and np.array_equal(L, L64)
    assert np.all(info["fell_back_fp64"] == 1)
    assert np.all(info["flags"] == 0)
    assert np.all(info["refine_steps"] == 0)


def test_mixed_refine_every_column(gpu_lib):
    """refine_weight_tol = 0 refines every column of both injections: the
    densities then carry no single-precision error either."""
    wl = W.config0()
    ctx = _lib.context_for(wl.device, 0)
    ctx.set_option("refine_weight_tol", 0.0)
    T, L, info, st = ctx.solve(wl.E, wl.eta, _lib.MIXED)
    Tref, Lref = oracle.solve_device(wl.device, wl.E, wl.eta)
    _check(T, L, Tref, Lref, "cfg0 mixed, all columns refined", tolT=1e-9, tolN=1e-9)


def test_set_option_validation(gpu_lib):
    ctx = _lib.Context(0)
    for name, bad in (("refine_tol", 0.0), ("refine_tol", 2.0), ("refine_max_steps", 1.5),
                      ("refine_max_steps", -1), ("refine_weight_tol", -0.1), ("workgroups_per_cu", 5),
                      ("energies_per_launch", 0), ("decimation_max_iters", 0), ("no_such_option", 1.0)):
        with pytest.raises(_lib.QtxError) as ei:
            ctx.set_option(name, bad)
        assert ei.value.status == _lib.EINVAL, name
    for name, ok in (("refine_tol", 1e-10), ("refine_max_steps", 2), ("refine_weight_tol", 0.0),
                     ("workgroups_per_cu", 1), ("energies_per_launch", 100), ("decimation_tol", 1e-13),
                     ("decimation_max_iters", 80)):
        ctx.set_option(name, ok)


def test_mixed_chunked_launches_match_single_launch(gpu_lib):
    """Energies split over several launches (and one workgroup per CU) give
    the same results as one launch."""
    wl = W.config0()
    ctx = _lib.context_for(wl.device, 0)
    T1, L1, _, _ = ctx.solve(wl.E, wl.eta, _lib.MIXED)
    ctx.set_option("energies_per_launch", 7)
    ctx.set_option("workgroups_per_cu", 1)
    T2, L2, _, _ = ctx.solve(wl.E, wl.eta, _lib.MIXED)
    assert np.array_equal(T1, T2) and np.array_equal(L1, L2)


def test_mixed_band_edge_energies_m128(gpu_lib):
    """Mixed path at N = 400, m = 128 on 64 energies within 1 meV of the lead
    band edges (the hardest-conditioned set): every energy within 1e-8 of
    the FP64 path, two of them against the oracle."""
    import os
    edges = np.loadtxt(os.path.join(os.path.dirname(__file__), "golden", "cfg2_band_edge_energies.txt"))
    wl = W.config2()
    dev = wl.device
    E = edges[::4]
    ctx = _lib.context_for(dev, 0)
    T64, L64, _, _ = ctx.solve(E, wl.eta, _lib.FP64)
    T, L, info, st = ctx.solve(E, wl.eta, _lib.MIXED)
    assert st == _lib.OK
    _check(T, L, T64, L64, "band-edge mixed vs fp64", tolT=TOL_T - 1e-10)
    Tref, Lref = oracle.solve_device(dev, E[[3, 40]], wl.eta)
    _check(T[[3, 40]], L[[3, 40]], Tref, Lref, "band-edge mixed vs oracle")
