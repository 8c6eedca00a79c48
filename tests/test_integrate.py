"""Adaptive Simpson driver (host logic) pinned by closed forms, and the
oracle's reference integrals checked against the same closed forms."""
import numpy as np
import pytest

from oracle import integrals as oint
from paper_1903_00548_amd import integrate as I


def _counting(f):
    calls = []

    def F(E):
        calls.append(np.array(E))
        return f(E)
    return F, calls


def test_cubic_is_exact_and_batched():
    F, calls = _counting(lambda E: np.stack([1 + E - 3 * E ** 2 + 0.5 * E ** 3, E ** 2], axis=1))
    r = I.adaptive_simpson(F, -1.0, 2.0, 1e-12, n0=4)
    exact = np.array([3.0 + 1.5 - 9.0 + 0.5 * (16 - 1) / 4, 3.0])
    assert np.abs(r.value - exact).max() < 1e-13
    assert r.converged and r.rounds == 1 and len(calls) == 1          # one batched evaluation
    allE = np.concatenate(calls)
    assert len(np.unique(allE)) == len(allE)                            # no abscissa evaluated twice


def test_sqrt_singularity_refines_near_the_edge():
    F, calls = _counting(lambda E: np.sqrt(np.maximum(E, 0.0))[:, None] + 1.0 / np.sqrt(E + 1e-3)[:, None])
    exact = 2.0 / 3.0 + 2 * (np.sqrt(1 + 1e-3) - np.sqrt(1e-3))
    r = I.adaptive_simpson(F, 0.0, 1.0, 1e-9)
    assert abs(r.value[0] - exact) < 1e-8
    assert r.converged and r.rounds == len(calls) > 1
    # later rounds only bring new points, concentrated at the singular end
    assert np.median(calls[-1]) < 0.05
    allE = np.concatenate(calls)
    assert len(np.unique(allE)) == len(allE)


def test_lorentzian_peak_and_error_estimate():
    g, x0 = 1e-3, 0.3171
    F = lambda E: (g / np.pi / ((E - x0) ** 2 + g * g))[:, None]
    exact = (np.arctan((1 - x0) / g) - np.arctan((-1 - x0) / g)) / np.pi
    for tol in (1e-6, 1e-9):
        r = I.adaptive_simpson(F, -1.0, 1.0, tol)
        assert abs(r.value[0] - exact) < 10 * tol
        assert r.error_estimate < tol


def test_fermi_integrals_closed_form():
    mu, kT, A, B = 0.137, 0.0259, -1.0, 1.0
    # antiderivative of f: E - kT ln(1 + exp((E - mu)/kT))
    prim = lambda E: E - kT * np.logaddexp(0.0, (E - mu) / kT)
    r = I.adaptive_simpson(lambda E: I.fermi(E - mu, kT)[:, None], A, B, 1e-11)
    assert abs(r.value[0] - (prim(B) - prim(A))) < 1e-10
    r = I.adaptive_simpson(lambda E: I.minus_dfermi(E - mu, kT)[:, None], A, B, 1e-11)
    assert abs(r.value[0] - (I.fermi(A - mu, kT) - I.fermi(B - mu, kT))) < 1e-10
    x = np.linspace(-30, 30, 101) * kT
    assert np.allclose(I.fermi(x, kT) + I.fermi(-x, kT), 1.0, atol=1e-15)
    assert np.allclose(I.fermi(x, kT), oint.fermi(x, 0.0, kT), atol=1e-15)
    assert np.allclose(I.minus_dfermi(x, kT), oint.minus_dfermi(x, 0.0, kT), rtol=1e-12, atol=1e-300)


def test_integrand_assembly():
    """density / jacobian / current integrands from a fake solver."""
    N = 3
    def solve(E):
        T = 0.5 + 0.1 * E
        L = np.stack([np.outer(1 + E, np.arange(1, N + 1)), np.outer(2 - E, np.ones(N))], axis=1)
        return T, L
    E = np.array([-0.2, 0.0, 0.4])
    muL, muR, kT = 0.1, -0.1, 0.05
    fL, fR = I.fermi(E - muL, kT), I.fermi(E - muR, kT)
    T, L = solve(E)
    d = I.integrand("density", solve, muL, muR, kT)(E)
    assert np.allclose(d, fL[:, None] * L[:, 0] + fR[:, None] * L[:, 1])
    c = I.integrand("current", solve, muL, muR, kT)(E)
    assert np.allclose(c[:, 0], T * (fL - fR))
    with pytest.raises(ValueError):
        I.integrand("charge", solve, muL, muR, kT)


def test_oracle_simpson_weights():
    w = oint.simpson_weights(0.0, 2.0, 8)
    E = np.linspace(0.0, 2.0, 9)
    assert abs(w @ E ** 3 - 4.0) < 1e-14 and abs(w.sum() - 2.0) < 1e-14
    with pytest.raises(ValueError):
        oint.simpson_weights(0.0, 1.0, 3)


def test_unconverged_is_reported():
    r = I.adaptive_simpson(lambda E: (1.0 / np.sqrt(np.abs(E - 0.123456) + 1e-14))[:, None], 0.0, 1.0, 1e-14,
                           max_rounds=3)
    assert not r.converged and np.isfinite(r.value).all()


def test_weights_reproduce_the_value():
    """The returned quadrature weights give the integral of every component,
    accepted panels (Boole weights) and unconverged ones alike."""
    F = lambda E: np.stack([np.sqrt(np.abs(E - 0.3)), np.cos(3 * E), E ** 3], axis=1)
    for rounds in (40, 2):
        r = I.adaptive_simpson(F, -1.0, 2.0, 1e-9, n0=8, max_rounds=rounds)
        assert r.weights.shape == r.energies.shape
        direct = r.weights @ F(r.energies)
        assert np.allclose(direct, r.value, rtol=1e-13, atol=1e-15), (direct, r.value)
    assert abs(r.weights.sum() - 3.0) < 1e-12           # the constant 1 integrates exactly


@pytest.mark.parametrize("fill", [64, 512])
def test_taking_levels_ahead_keeps_the_result_and_cuts_calls(fill):
    """fill > 0 evaluates further levels of the failing panels in the same
    call: the accepted panels, the value and the weights of every abscissa
    used are those of the plain driver, no call exceeds fill new abscissae
    unless the plain driver's calls do, and there are fewer calls."""
    g, x0 = 1e-3, 0.3171

    def f(E):
        return np.stack([g / np.pi / ((E - x0) ** 2 + g * g), np.sqrt(np.abs(E + 0.8))], axis=1)

    F0, calls0 = _counting(f)
    F1, calls1 = _counting(f)
    r0 = I.adaptive_simpson(F0, -1.0, 1.0, 1e-9)
    r1 = I.adaptive_simpson(F1, -1.0, 1.0, 1e-9, fill=fill)
    assert r0.converged and r1.converged
    assert np.array_equal(r0.value, r1.value)
    assert len(calls1) < len(calls0)
    used = r1.weights != 0
    assert np.array_equal(r1.energies[used], r0.energies[r0.weights != 0])
    assert np.array_equal(r1.weights[used], r0.weights[r0.weights != 0])
    assert set(r0.energies) <= set(r1.energies)
    assert max(len(c) for c in calls1) <= max(fill, max(len(c) for c in calls0))
    allE = np.concatenate(calls1)
    assert len(np.unique(allE)) == len(allE)
