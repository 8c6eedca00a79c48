"""Energy integration over the transport solve (Sec. "Density", eq.
density_3d; Sec. "Transmission and Ballistic Current", eq. current; the
charge Jacobian of eq. density_jacobian).

The integrals run over energies whose integrand is one solve each, with
singular features (band edges of the contacts) at places not known in
advance, so they are taken by adaptive Simpson quadrature.  The driver is
batched: every round collects the new abscissae of all panels that fail
their error test and evaluates them in ONE solver call (one launch sequence
on the GPU), instead of recursing panel by panel.

Panel [a, b] with midpoint m and quarter points l, r: S1 = Simpson on
(a, m, b), S2 = Simpson on (a, l, m) + (m, r, b); the panel is accepted
when max|S2 - S1| / 15 <= tol (b - a) / (B - A) (the absolute tolerance
spread over the interval [A, B]) and contributes the Richardson value
S2 + (S2 - S1) / 15; otherwise it is split at m.  That value is linear in
the samples, (b - a)/90 (7, 32, 12, 32, 7) on (a, l, m, r, b), so the
driver also returns one quadrature weight per abscissa: the integral is
sum_k w_k F(E_k).  Sec. "Density" keeps exactly these energies and weights
of the node-density integration to build the density matrix in one more
pass (density_matrix below).

Quantities (n^L_i, n^R_i: slab densities of states per injecting contact,
T: transmission; f: Fermi function):
  density   n_i = int dE [f(E - muL) n^L_i(E) + f(E - muR) n^R_i(E)]
  jacobian  dn_i/dmu = int dE [-f'(E - muL) n^L_i(E) - f'(E - muR) n^R_i(E)]
            (the derivative of the density with respect to a rigid shift
            of both electrochemical potentials; eq. density_jacobian writes
            it with df/dE, whose sign is opposite)
  current   J = int dE T(E) [f(E - muL) - f(E - muR)]  (eV);
            I = (2 e^2 / h) J  with spin degeneracy 2.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, Dict, Optional

import numpy as np

TWO_E2_OVER_H = 7.748091729e-5      # A per eV of J (2 e^2 / h in siemens)


def fermi(x, kT):
    """1 / (1 + exp(x / kT)), evaluated without overflow."""
    return 0.5 * (1.0 - np.tanh(0.5 * np.asarray(x, dtype=float) / kT))


def minus_dfermi(x, kT):
    """-df/dx = 1 / (4 kT cosh^2(x / 2kT))."""
    c = np.cosh(np.minimum(np.abs(0.5 * np.asarray(x, dtype=float) / kT), 350.0))
    return 1.0 / (4.0 * kT * c * c)


@dataclasses.dataclass
class Result:
    value: np.ndarray                 # integral of every integrand component
    error_estimate: float             # sum of the accepted panels' |S2 - S1| / 15 (max norm)
    converged: bool
    evaluations: int                  # distinct abscissae evaluated
    rounds: int                       # solver calls
    energies: np.ndarray              # all abscissae, sorted
    weights: np.ndarray               # quadrature weight of each abscissa (value = weights @ F(energies))


def adaptive_simpson(F: Callable[[np.ndarray], np.ndarray], A: float, B: float, tol: float,
                     n0: int = 16, max_rounds: int = 40, min_width: float = 1e-10, fill: int = 0,
                     max_ahead: int = 6) -> Result:
    """Integrate the vector function F over [A, B] to absolute tolerance tol
    (max norm over components).  F takes a 1-D array of energies and returns
    an array of shape (len(E), K).

    fill > 0: a round whose new abscissae number fewer than fill also takes
    the abscissae of up to max_ahead further levels of its failing panels'
    halves (as many whole levels as keep the call within fill).  A GPU call
    costs about the same for any count up to one energy per resident
    workgroup, so late rounds, which carry few energies, get their next
    levels for free and the number of calls drops.  Panels accepted before
    those levels are needed leave the extra abscissae unused (weight 0);
    the accepted panels, the value and the weights of the used abscissae
    are those of fill = 0."""
    if not (B > A) or not (tol > 0):
        raise ValueError("need B > A and tol > 0")
    vals: Dict[float, np.ndarray] = {}
    rounds = 0

    def evaluate(points):
        nonlocal rounds
        new = sorted(p for p in points if p not in vals)
        if not new:
            return
        out = np.asarray(F(np.array(new)), dtype=float)
        if out.ndim == 1:
            out = out[:, None]
        for e, v in zip(new, out):
            vals[e] = v
        rounds += 1

    edges = np.linspace(A, B, n0 + 1)
    pending = [(float(edges[k]), float(edges[k + 1])) for k in range(n0)]
    total = None
    err_total = 0.0
    wts: Dict[float, float] = {}

    def add_weights(points, factors, h):
        for p, f in zip(points, factors):
            wts[p] = wts.get(p, 0.0) + h * f
    def panel_points(panels):
        out = set()
        for a, b in panels:
            m = 0.5 * (a + b)
            out.update((a, 0.5 * (a + m), m, 0.5 * (m + b), b))
        return out

    while pending and rounds < max_rounds:
        pts = panel_points(pending)
        if fill > 0:
            n_new = sum(1 for p in pts if p not in vals)
            level = pending
            for _ in range(max_ahead):
                level = [h for a, b in level for h in ((a, 0.5 * (a + b)), (0.5 * (a + b), b))]
                more = {p for p in panel_points(level) if p not in vals and p not in pts}
                if n_new == 0 or n_new + len(more) > fill:
                    break
                pts |= more
                n_new += len(more)
        evaluate(pts)
        nxt = []
        for a, b in pending:
            m = 0.5 * (a + b)
            l, r = 0.5 * (a + m), 0.5 * (m + b)
            fa, fl, fm, fr, fb = vals[a], vals[l], vals[m], vals[r], vals[b]
            s1 = (b - a) / 6.0 * (fa + 4.0 * fm + fb)
            s2 = (m - a) / 6.0 * (fa + 4.0 * fl + fm) + (b - m) / 6.0 * (fm + 4.0 * fr + fb)
            err = float(np.max(np.abs(s2 - s1))) / 15.0
            if err <= tol * (b - a) / (B - A) or (b - a) < min_width:
                v = s2 + (s2 - s1) / 15.0
                total = v if total is None else total + v
                err_total += err
                add_weights((a, l, m, r, b), (7.0, 32.0, 12.0, 32.0, 7.0), (b - a) / 90.0)
            else:
                nxt.extend(((a, m), (m, b)))
        pending = nxt
    converged = not pending
    for a, b in pending:                      # out of rounds: take what is known
        m = 0.5 * (a + b)
        l, r = 0.5 * (a + m), 0.5 * (m + b)
        if all(p in vals for p in (a, l, m, r, b)):
            s2 = (m - a) / 6.0 * (vals[a] + 4.0 * vals[l] + vals[m]) + (b - m) / 6.0 * (vals[m] + 4.0 * vals[r] + vals[b])
            add_weights((a, l, m, r, b), (1.0, 4.0, 2.0, 4.0, 1.0), (b - a) / 12.0)
        else:
            s2 = (b - a) / 6.0 * (vals[a] + 4.0 * vals[m] + vals[b])
            add_weights((a, m, b), (1.0, 4.0, 1.0), (b - a) / 6.0)
        total = s2 if total is None else total + s2
    energies = np.array(sorted(vals))
    return Result(value=np.asarray(total), error_estimate=err_total, converged=converged,
                  evaluations=len(vals), rounds=rounds, energies=energies,
                  weights=np.array([wts.get(e, 0.0) for e in energies]))


def integrand(quantity: str, solve: Callable, muL: float, muR: float, kT: float):
    """Integrand of one quantity from a solver E -> (T, ldos[nE, 2, N])."""
    if quantity not in ("density", "jacobian", "current"):
        raise ValueError(f"unknown quantity {quantity!r}")

    def F(E):
        T, L = solve(E)
        if quantity == "current":
            return (T * (fermi(E - muL, kT) - fermi(E - muR, kT)))[:, None]
        w = fermi if quantity == "density" else minus_dfermi
        return w(E - muL, kT)[:, None] * L[:, 0, :] + w(E - muR, kT)[:, None] * L[:, 1, :]
    return F


def integrate(solve: Callable, quantity: str, A: float, B: float, muL: float, muR: float, kT: float,
              tol: float, n0: int = 16, max_rounds: int = 40, fill: int = 0) -> Result:
    """Adaptive integral of a quantity over [A, B] (see the module docstring)
    with the transport solve as integrand; fill as in adaptive_simpson (one
    energy per resident workgroup, e.g. 512 at m <= 64, keeps late calls
    full)."""
    return adaptive_simpson(integrand(quantity, solve, muL, muR, kT), A, B, tol, n0=n0, max_rounds=max_rounds,
                            fill=fill)


def density_matrix(ctx, result: Result, muL: float, muR: float, kT: float, eta: float):
    """Nearest-neighbour density-matrix blocks rho_ii (N, m, m) and
    rho_{i,i+1} (N-1, m, m) over the energies and quadrature weights of an
    adaptive integration (eq. density_matrices: weight times occupation of
    each contact, one pass of the HIP library's density-matrix solve).  For
    the result of a "density" integration, the trace of rho_ii equals its
    value up to rounding."""
    used = np.asarray(result.weights) != 0.0         # abscissae taken ahead but not needed carry weight 0
    E = np.asarray(result.energies, dtype=np.float64)[used]
    q = np.asarray(result.weights, dtype=np.float64)[used]
    rd, ro, _, _, _, _ = ctx.density_matrix(E, q * fermi(E - muL, kT), q * fermi(E - muR, kT), eta)
    return rd, ro


def qtx_solver(ctx, eta: float, precision: int = 0):
    """E -> (T, ldos) through the HIP library (one batched call per round)."""
    def solve(E):
        T, L, _, _ = ctx.solve(np.ascontiguousarray(E, dtype=np.float64), eta, precision, want_ldos=True)
        return T, L
    return solve
