"""Pins of the oracle's reference derivatives (oracle/gradient.py): complex step against
central differences (independent arithmetic), and the exact values conservation fixes:
the total of phi does not depend on sigma or M, and its derivative along a change d of
phi0 is sum(d) (g = g_eq(phi0) sums to phi0, and every step keeps sum_x phi)."""
import numpy as np
import pytest

import workloads as W
from oracle import gradient as G


def _shear():
    p, phi0, u0 = W.shear_droplet(nx=64, ny=32, R=8.0)
    return p, phi0, u0, 120


def _drops():
    p, phi0, u0 = W.two_droplets(scale=1)
    p = p.replace(nx=64, ny=48, label_centres=[(20.0, 24.0, 0.0), (46.0, 22.0, 0.0)])
    phi0 = W.drops_phi(p, [(20.0, 24.0, 0.0, 10.0), (46.0, 22.0, 0.0, 5.0)])
    return p, phi0, None, 60


def _sessile():
    """A drop on the bottom wall of a 64 x 32 channel whose walls move -+0.01 and wet at
    contact angles acos(0.5) (bottom) and acos(-0.3) (top): the interface meets the wall,
    so the wetting ghosts enter the map."""
    p = W.CaseParams(nx=64, ny=32, wall_y=True, wall_u_bottom=(-0.01, 0.0, 0.0), wall_u_top=(0.01, 0.0, 0.0),
                     wall_cos_bottom=0.5, wall_cos_top=-0.3, rho_light=0.5, sigma=0.01, nu=0.1,
                     label_centres=[(32.37, 2.0, 0.0)])
    x = np.arange(p.nx)[None, None, :]
    y = np.arange(p.ny)[None, :, None]
    d = 10.0 - np.sqrt((x - 32.37) ** 2 + (y + 0.5 - 1.13) ** 2)
    return p, 0.5 * (1.0 + np.tanh(2.0 * d / p.W)) * np.ones((1, p.ny, p.nx)), None, 80


def _visc():
    """The 66 x 24 walled shear drop with unequal viscosities (ratio 3.75, density ratio
    1/0.3): the stress rates of f depend on phi (Eq. 27)."""
    p, _, u0 = W.shear_droplet(nx=66, ny=24, R=7.0, U=0.02, Ca=0.2, Re=0.5)
    p = p.replace(rho_light=0.3, nu=0.15, nu_light=0.04, label_centres=[(32.31, 11.17, 0.0)])
    return p, W.drops_phi(p, [(32.31, 11.17, 0.0, 7.0)]), u0, 80


def _direction(phi0, seed=1):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal(phi0.shape) * 4.0 * phi0 * (1.0 - phi0)


@pytest.mark.parametrize("wrt", ["sigma", "mobility"])
def test_complex_step_matches_central_difference_parameters(wrt):
    p, phi0, u0, n = _shear()
    cs = G.complex_step(p, phi0, u0, n, wrt)
    eps = 1e-5 * (p.sigma if wrt == "sigma" else p.mobility)
    fd = G.central_difference(p, phi0, u0, n, wrt, eps)
    # deformation D: a non-trivial derivative; relative agreement to the FD error
    assert abs(cs[0, 4]) > 1e-3
    assert abs(fd[0, 4] - cs[0, 4]) <= 1e-6 * abs(cs[0, 4])


def test_complex_step_matches_central_difference_phi0():
    p, phi0, u0, n = _shear()
    d = _direction(phi0)
    cs = G.complex_step(p, phi0, u0, n, "phi0", direction=d)
    fd = G.central_difference(p, phi0, u0, n, "phi0", 1e-4, direction=d)
    for k in (0, 1, 2, 4):                 # volume, centroid x, y, D
        assert abs(cs[0, k]) > 1e-4
        assert abs(fd[0, k] - cs[0, k]) <= 1e-6 * abs(cs[0, k]), (k, fd[0, k], cs[0, k])


def test_complex_step_matches_central_difference_unequal_viscosities():
    """tau_f(phi) = 1/2 + 3 mu(phi) / rho(phi) is rational in phi, so the complex step stays
    exact: against central differences, for sigma, M and a phi0 direction (tau = 0)."""
    p, phi0, u0, n = _visc()
    d = _direction(phi0)
    for wrt, eps in (("sigma", 1e-6 * p.sigma), ("mobility", 1e-5 * p.mobility), ("phi0", 1e-6)):
        cs = G.complex_step(p, phi0, u0, n, wrt, direction=d, tau=0.0)
        fd = G.central_difference(p, phi0, u0, n, wrt, eps, direction=d)
        for k in (1, 2, 4):                # centroid x, y, D
            if abs(cs[0, k]) < 1e-4:       # a derivative the symmetry of the set-up keeps small
                continue
            assert abs(fd[0, k] - cs[0, k]) <= 1e-6 * abs(cs[0, k]), (wrt, k, fd[0, k], cs[0, k])


def test_complex_step_matches_central_difference_wetting_walls():
    """The wetting ghost is a polynomial of the edge phi, so the complex step stays exact:
    against central differences on the sessile drop, for sigma, M and a phi0 direction
    (the exact derivative, tau = 0, which the differences approximate).  This map is more
    curved than the shear case's, so the differences take smaller steps (their error
    falls as the step squared, to 1e-8 relative at these steps)."""
    p, phi0, u0, n = _sessile()
    d = _direction(phi0)
    for wrt, eps in (("sigma", 1e-6 * p.sigma), ("mobility", 1e-5 * p.mobility), ("phi0", 1e-6)):
        cs = G.complex_step(p, phi0, u0, n, wrt, direction=d, tau=0.0)
        fd = G.central_difference(p, phi0, u0, n, wrt, eps, direction=d)
        for k in (1, 2, 4):                # centroid x, y, D
            assert abs(cs[0, k]) > 1e-4, (wrt, k)
            assert abs(fd[0, k] - cs[0, k]) <= 1e-6 * abs(cs[0, k]), (wrt, k, fd[0, k], cs[0, k])


@pytest.mark.parametrize("case", [_shear, _drops, _sessile, _visc])
def test_total_phi_gradients_fixed_by_conservation(case):
    p, phi0, u0, n = case()
    total = lambda v: v[:, 0].sum()
    V = total(G.derived_after(p, phi0, u0, n))
    for wrt in ("sigma", "mobility"):
        assert abs(total(G.complex_step(p, phi0, u0, n, wrt))) <= 1e-11 * V
    d = _direction(phi0, seed=3)
    dv = total(G.complex_step(p, phi0, u0, n, "phi0", direction=d))
    assert abs(dv - d.sum()) <= 1e-12 * np.abs(d).sum()
    # a direction with mass in the bulk of both phases too
    d2 = np.cos(np.arange(phi0.size).reshape(phi0.shape) * 0.37)
    dv2 = total(G.complex_step(p, phi0, u0, n, "phi0", direction=d2))
    assert abs(dv2 - d2.sum()) <= 1e-11 * np.abs(d2).sum()


def test_normal_cut_restores_agreement_with_differences():
    """On a 128x64 shear case over 200 steps the exact derivative (tau = 0) is dominated by
    rounding-driven bulk terms of the unit normal and misses the finite difference by
    ~5e-3; holding n fixed where |grad psi| < tau brings it to the difference's own
    accuracy, the same for every tau in [0.01, 0.5]."""
    p, phi0, u0 = W.shear_droplet(nx=128, ny=64, R=16.0)
    n = 200
    fd = G.central_difference(p, phi0, u0, n, "sigma", 1e-5 * p.sigma)[0, 4]
    fd6 = G.central_difference(p, phi0, u0, n, "sigma", 1e-6 * p.sigma)[0, 4]
    assert abs(fd - fd6) < 1e-5 * abs(fd)
    exact = G.complex_step(p, phi0, u0, n, "sigma", tau=0.0)[0, 4]
    cut = G.complex_step(p, phi0, u0, n, "sigma")[0, 4]
    cut2 = G.complex_step(p, phi0, u0, n, "sigma", tau=0.05)[0, 4]
    assert abs(exact - fd) > 1e-3 * abs(fd)
    assert abs(cut - fd) < 3e-6 * abs(fd)
    assert abs(cut2 - cut) < 1e-7 * abs(cut)
