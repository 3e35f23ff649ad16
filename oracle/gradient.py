"""Reference derivatives of observables of the discrete model.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The objective is a derived observable of the phase field after n steps of the oracle
(volume, centroid offset, deformation D; see ``derived_observables``) started from
``Model.init(phi0, u0)``.  Its derivatives with respect to the surface tension sigma,
the mobility M and the initial field phi0 (along a direction d) are taken two ways:

* complex step: Im O(theta + i h) / h with h = 1e-30 runs the oracle itself in complex
  arithmetic.  Every operation of the step is analytic except the clip of phi to
  [0, 1], which acts on the real part (a derivative of 1 inside the interval, 0
  outside), so for h this small the result is the exact derivative of the discrete
  map, free of cancellation;
* central differences (O(theta + e) - O(theta - e)) / 2e, an independent check with
  truncation error O(e^2) and rounding error O(eps / e).

Reading for long runs: away from the interface psi saturates (phi clipped, or within
rounding of 0 or 1), |grad psi| falls to rounding level, and the exact derivative of
the unit normal n = grad psi / |grad psi| has a gain of order lambda / |grad psi| per
step.  The exact derivative of the discrete map is then dominated by rounding-driven
bulk terms that grow without bound (values of 1e67 after 200 steps of a 128x64 shear
case) and disagree with every finite difference.  The reference derivatives here
therefore hold n fixed where |grad psi| < tau (tau = 0.3 by default; psi is a signed
distance with |grad psi| = 1 across the interface, and results change by less than
1e-8 relative for tau in [0.01, 0.5]); tau = 0 gives the exact derivative.
The values of the forward run are untouched.

sigma enters through beta = 12 sigma / W and kappa = 3 sigma W / 2 (the chemical
potential, Eq. 2), M through the default rates of g, 1 / tau_g = 1 / (1/2 + M / c_s^2)
(Eq. 34).  phi0 directions should stay inside (0, 1) and off the clipped bulk (for
example d = r 4 phi0 (1 - phi0)): where phi0 rounds to 0 or 1 the map has a kink, and
next to it psi (Eq. 37) has slope W / (4 xi) ~ 1e10, so that finite differences leave
the linear range long before they leave rounding noise.
"""
from __future__ import annotations

import numpy as np

from .model import Model, derived_observables, observables_from_phi

DERIVED = ("volume", "centroid_x", "centroid_y", "centroid_z", "D")
NORMAL_TAU = 0.3


def derived_after(p, phi0, u0, nsteps, sigma=None, mobility=None, dphi0=None, dtype=np.float64, tau=0.0):
    """(labels, 5) array of (volume, centroid offset x, y, z, D) after nsteps steps."""
    m = Model(p, dtype=dtype, sigma=sigma, mobility=mobility, normal_tau=tau)
    phi = np.asarray(phi0, dtype=dtype)
    if dphi0 is not None:
        phi = phi + dphi0
    m.init(phi, u0)
    m.step(nsteps)
    d = derived_observables(observables_from_phi(p, m.phi()))
    return np.column_stack([d["volume"], d["centroid"][:, 0], d["centroid"][:, 1], d["centroid"][:, 2],
                            d["D"]])


def complex_step(p, phi0, u0, nsteps, wrt, direction=None, h=1e-30, tau=NORMAL_TAU):
    """Derivative of the derived observables with respect to ``wrt`` in
    {"sigma", "mobility", "phi0"} (phi0: along ``direction``), with the unit normal
    held fixed where |grad psi| < tau (tau = 0: the exact derivative)."""
    c = np.complex128
    if wrt == "sigma":
        v = derived_after(p, phi0, u0, nsteps, sigma=p.sigma + 1j * h, dtype=c, tau=tau)
    elif wrt == "mobility":
        v = derived_after(p, phi0, u0, nsteps, mobility=p.mobility + 1j * h, dtype=c, tau=tau)
    elif wrt == "phi0":
        v = derived_after(p, phi0, u0, nsteps, dphi0=1j * h * np.asarray(direction), dtype=c, tau=tau)
    else:
        raise ValueError(wrt)
    return np.imag(v) / h


def central_difference(p, phi0, u0, nsteps, wrt, eps, direction=None):
    """Central difference of the derived observables with step eps (absolute)."""
    def at(e):
        if wrt == "sigma":
            return derived_after(p, phi0, u0, nsteps, sigma=p.sigma + e)
        if wrt == "mobility":
            return derived_after(p, phi0, u0, nsteps, mobility=p.mobility + e)
        if wrt == "phi0":
            return derived_after(p, phi0, u0, nsteps, dphi0=e * np.asarray(direction))
        raise ValueError(wrt)
    return (at(eps) - at(-eps)) / (2.0 * eps)
