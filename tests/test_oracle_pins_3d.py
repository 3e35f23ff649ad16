"""Pins of the oracle's D3Q19 step against what the mathematics fixes.

The paper treats two-dimensional flows; the three-dimensional workload uses the same
generic equations (Eqs. 21-23, 28-29, 31-33, 35, 37, 39-40, all written through the
weights w_i and velocities c_i) on the D3Q19 lattice.  These tests check the oracle's
3D step against things other than itself:

- the stencils of Eqs. 39-40: exact on quadratic polynomials, and their Fourier symbols
  written out by hand for the D3Q19 neighbourhood;
- a dense brute force (tests/bruteforce.py: Dense3D) that builds the relaxation
  operator as projectors onto the polynomial subspaces the rates belong to, streaming
  as a permutation matrix, and visits nodes in a loop;
- invariants: the total of phi on a periodic box, mirror symmetries of a centred drop;
- textbook limits: a shear wave decays at nu k^2 with nu = c_s^2 (tau_f - 1/2)
  (Eq. 27) for every independent component of the traceless stress, a phase-field
  mode diffuses at lambda M k^2 and is carried at the flow velocity;
- Laplace's law for a sphere (pressure jump 2 sigma / R) in the classical limit.

A mistake planted in the oracle's choice of 3D relaxation rows is caught: see
test_planted_rate_row_mistakes_are_caught.
"""
import numpy as np
import pytest

import workloads as W
from oracle import D3Q19, Model
from oracle import lattice as oracle_lattice
from tests.bruteforce import Dense3D


def _case(nx, ny, nz, **kw):
    base = dict(nx=nx, ny=ny, nz=nz, lattice="D3Q19")
    base.update(kw)
    return W.CaseParams(**base)


# --------------------------------------------------------------------------- stencils (Eqs. 39, 40)
def test_d3q19_stencils_exact_on_quadratics():
    n = 8
    m = Model(_case(n, n, n))
    z, y, x = np.meshgrid(*(np.arange(n, dtype=float),) * 3, indexing="ij")
    a, b, c, d, e, f, g1, g2, g3 = 0.3, -0.7, 1.1, 0.25, -0.4, 0.6, 0.9, -1.3, 0.45
    chi = a * x * x + b * y * y + c * z * z + d * x * y + e * y * z + f * x * z + g1 * x + g2 * y + g3 * z
    gr = m.grad(chi)
    lap = m.lap(chi)
    s = (slice(1, n - 1),) * 3
    assert np.allclose(gr[0][s], (2 * a * x + d * y + f * z + g1)[s], atol=1e-12)
    assert np.allclose(gr[1][s], (2 * b * y + d * x + e * z + g2)[s], atol=1e-12)
    assert np.allclose(gr[2][s], (2 * c * z + e * y + f * x + g3)[s], atol=1e-12)
    assert np.allclose(lap[s], 2 * (a + b + c), atol=1e-12)


def test_d3q19_stencil_fourier_symbols():
    # Axis neighbours (w = 1/18) and the twelve face diagonals (w = 1/36) of Eq. 39 give
    # d/dx -> (i/3) sin kx (1 + cos ky + cos kz); Eq. 40 gives
    # lap -> (2/3) sum_a (cos k_a - 1) + (2/3) sum_{a<b} (cos k_a cos k_b - 1).
    n = 8
    m = Model(_case(n, n, n))
    z, y, x = np.meshgrid(*(np.arange(n),) * 3, indexing="ij")
    for kk in ((1, 0, 0), (2, 3, 1), (3, 1, 5), (0, 2, 7)):
        K = [2 * np.pi * v / n for v in kk]
        chi = np.exp(1j * (K[0] * x + K[1] * y + K[2] * z))
        gr = m.grad(chi)
        lap = m.lap(chi)
        cs = [np.cos(v) for v in K]
        for d in range(3):
            o = [cs[e] for e in range(3) if e != d]
            sym = 1j / 3 * np.sin(K[d]) * (1 + o[0] + o[1])
            assert np.allclose(gr[d], sym * chi, atol=1e-13), (kk, d)
        sl = 2 / 3 * sum(v - 1 for v in cs) + 2 / 3 * sum(cs[a] * cs[b] - 1 for a in range(3) for b in range(a + 1, 3))
        assert np.allclose(lap, sl * chi, atol=1e-13), kk


# --------------------------------------------------------------------------- brute force
def test_d3q19_oracle_equals_dense_bruteforce():
    nx, ny, nz = 3, 3, 4
    p = _case(nx, ny, nz, W=2.0, sigma=0.02, mobility=0.07, nu=0.13, rho_heavy=1.0, rho_light=0.2)
    rng = np.random.default_rng(31)
    phi0 = rng.uniform(-0.05, 1.05, (nz, ny, nx))
    u0 = rng.normal(0, 0.02, (3, nz, ny, nx))
    orc = Model(p).init(phi0, u0)
    dn = Dense3D(nx, ny, nz, W=p.W, sigma=p.sigma, mobility=p.mobility, nu=p.nu, lam=p.lam, xi=p.xi,
                 eps_n=p.eps_n, rho_h=p.rho_heavy, rho_l=p.rho_light)
    # velocity order of the dense implementation -> the oracle's
    perm = [int(np.where((D3Q19.c == cv).all(axis=1))[0][0]) for cv in dn.c]
    g, f, J = dn.init(phi0.reshape(-1), u0.reshape(3, -1).T.copy())
    go = orc.g.reshape(19, -1).T[:, perm]
    assert np.max(np.abs(go - g)) < 1e-15
    for t in range(3):
        orc.step(1)
        g, f, J = dn.step(g, f, J)
        go = orc.g.reshape(19, -1).T[:, perm]
        fo = orc.f.reshape(19, -1).T[:, perm]
        assert np.max(np.abs(go - g)) < 1e-14, t
        assert np.max(np.abs(fo - f)) < 1e-14, t
        assert np.max(np.abs(orc.Jprev.reshape(3, -1).T - J)) < 1e-14, t


# --------------------------------------------------------------------------- invariants
def test_d3q19_total_phi_conserved():
    n = 16
    p = _case(n, n, n, rho_light=0.1, sigma=0.01, nu=0.05)
    phi0 = W.drops_phi(p, [(7.3, 8.1, 6.6, 5.0)])
    m = Model(p).init(phi0)
    V0 = m.phi().sum()
    m.step(300)
    assert abs(m.phi().sum() - V0) / V0 < 2e-13


def test_d3q19_centred_drop_keeps_its_mirror_symmetries():
    n = 12
    p = _case(n, n, n, rho_light=0.1, sigma=0.01, nu=0.05)
    c = (n - 1) / 2
    z, y, x = np.meshgrid(*(np.arange(n, dtype=float),) * 3, indexing="ij")
    # an ellipsoid-ish drop, mirror-symmetric about each mid-plane but with no rotation symmetry
    phi0 = W.drops_phi(p, [(c, c, c, 3.5)]) * (1 + 0.03 * np.cos(2 * np.pi * (x - c) / n)
                                               + 0.02 * np.cos(2 * np.pi * (z - c) / n))
    m = Model(p).init(phi0)
    m.step(60)
    F = m.fields()
    ph, u = F["phi"], F["u"]
    for ax in range(3):
        flip = np.flip(ph, axis=2 - ax)
        assert np.max(np.abs(ph - flip)) < 1e-13, ax
        # the velocity component along the mirror's normal is odd, the others even
        for d in range(3):
            sign = -1.0 if d == ax else 1.0
            assert np.max(np.abs(u[d] - sign * np.flip(u[d], axis=2 - ax))) < 1e-14, (ax, d)
    assert np.max(np.abs(u)) > 1e-6          # the flow is not trivially zero


# --------------------------------------------------------------------------- textbook limits
def _amplitude(field, phase):
    """Amplitude of the sin/cos(phase) mode of a real field."""
    s, c = np.sin(phase), np.cos(phase)
    return np.hypot((field * s).sum() / (s * s).sum(), (field * c).sum() / (c * c).sum())


def _shear_wave_rate(shape, kvec, avec, nu=0.1, steps=400):
    nx, ny, nz = shape
    p = _case(nx, ny, nz, rho_light=1.0, nu=nu)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    K = [2 * np.pi * kvec[0] / nx, 2 * np.pi * kvec[1] / ny, 2 * np.pi * kvec[2] / nz]
    phase = K[0] * x + K[1] * y + K[2] * z
    a = np.asarray(avec, float) / np.linalg.norm(avec)
    assert abs(a @ np.array(K)) < 1e-14                      # transverse wave
    u0 = 0.01 * a[:, None, None, None] * np.sin(phase)[None]
    m = Model(p).init(np.zeros((nz, ny, nx)), u0)

    def amp():
        u = m.fields()["u"]
        return _amplitude(np.tensordot(a, u, axes=(0, 0)), phase)
    a0 = amp()
    m.step(steps)
    a1 = amp()
    k2 = sum(v * v for v in K)
    return -np.log(a1 / a0) / steps / (p.nu * k2)


# Each wave exercises one independent component of the traceless stress, so every f row
# that should relax at 1 / tau_f is seen by some wave:
# u_x(z) and u_z(x): p_xz; u_y(x): p_xy; u_z(y): p_yz; a y-z diagonal wave with u along
# (0, 1, -1): the normal-stress difference p_yy - p_zz only; an x-y diagonal wave with u
# along (1, -1, 0): p_xx - p_yy, which mixes 2 p_xx - p_yy - p_zz and p_yy - p_zz.
SHEAR_WAVES = {
    "ux_along_z": ((1, 1, 48), (0, 0, 1), (1, 0, 0)),
    "uz_along_x": ((48, 1, 1), (1, 0, 0), (0, 0, 1)),
    "uy_along_x": ((48, 1, 1), (1, 0, 0), (0, 1, 0)),
    "uz_along_y": ((1, 48, 1), (0, 1, 0), (0, 0, 1)),
    "yz_diagonal": ((1, 32, 32), (0, 1, 1), (0, 1, -1)),
    "xy_diagonal": ((32, 32, 1), (1, 1, 0), (1, -1, 0)),
}


@pytest.mark.parametrize("name", list(SHEAR_WAVES))
def test_d3q19_shear_wave_decays_at_the_viscous_rate(name):
    shape, k, a = SHEAR_WAVES[name]
    assert abs(_shear_wave_rate(shape, k, a) - 1) < 5e-3


def _phase_mode(shape, kvec, u=(0.0, 0.0, 0.0), steps=300):
    """A small phase-field mode with sigma = 0 and W -> infinity, so that only the
    lambda M lap(phi) part of Eq. 17's flux acts (and advection by u)."""
    nx, ny, nz = shape
    p = _case(nx, ny, nz, W=1e9, sigma=0.0, mobility=0.1, rho_light=1.0)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    K = np.array([2 * np.pi * kvec[0] / nx, 2 * np.pi * kvec[1] / ny, 2 * np.pi * kvec[2] / nz])
    phase = K[0] * x + K[1] * y + K[2] * z
    phi0 = 0.5 + 0.01 * np.sin(phase)
    u0 = np.broadcast_to(np.asarray(u, float)[:, None, None, None], (3, nz, ny, nx)).copy()
    m = Model(p).init(phi0, u0)

    def coef():
        ph = m.phi() - 0.5
        return complex((ph * np.sin(phase)).sum(), (ph * np.cos(phase)).sum())
    c0 = coef()
    m.step(steps)
    c1 = coef()
    rate = -np.log(abs(c1) / abs(c0)) / steps / (p.lam * p.mobility * (K @ K))
    # a mode sin(k.x - w t) has coefficient pair rotating by the angle w t = k.u t
    shift = np.angle(c1 / c0) % (2 * np.pi)
    return rate, shift, float(K @ np.asarray(u, float)) * steps


@pytest.mark.parametrize("k", [(0, 0, 1), (1, 0, 1)], ids=["z", "xz"])
def test_d3q19_phase_field_diffuses_at_lambda_M_k2(k):
    rate, _, _ = _phase_mode((32, 4, 32), k)
    assert abs(rate - 1) < 5e-3


@pytest.mark.parametrize("shape,k", [((48, 2, 2), (1, 0, 0)), ((2, 48, 2), (0, 1, 0)), ((2, 2, 48), (0, 0, 1)),
                                     ((48, 2, 48), (1, 0, 1))], ids=["x", "y", "z", "xz"])
def test_d3q19_phase_field_is_carried_by_the_flow(shape, k):
    u = (0.03, -0.02, 0.04)
    _, shift, want = _phase_mode(shape, k, u=u, steps=200)
    # the mode's coefficient pair turns by -k.u t; the tolerance covers the O(k^2)
    # dispersion of the discrete advection
    assert abs(shift - (-want) % (2 * np.pi)) < 5e-3 * abs(want), (shift, want)


@pytest.mark.slow
def test_d3q19_laplace_law_sphere_classical_limit():
    # lambda = 0 (classical C-H): a drop at rest has the pressure jump 2 sigma / R of a
    # sphere, twice the 2D jump; two radii check the 1 / R scaling.
    res = {}
    for R in (5.0, 7.0):
        n = 20
        p = _case(n, n, n, sigma=0.01, mobility=0.1, rho_light=0.1, nu=0.3, lam=0.0)
        c = (n - 1) / 2
        m = Model(p).init(W.drops_phi(p, [(c, c, c, R)]))
        m.step(1000)
        pr = m.fields()["p"]
        z, y, x = np.meshgrid(*(np.arange(n),) * 3, indexing="ij")
        r = np.sqrt((x - c) ** 2 + (y - c) ** 2 + (z - c) ** 2)
        res[R] = (pr[r < R / 2].mean() - pr[r > R + 3].mean()) / (2 * p.sigma / R)
    for R, v in res.items():
        assert abs(v - 1) < 0.08, res
    assert abs(res[5.0] / res[7.0] - 1) < 0.05, res


# --------------------------------------------------------------------------- planted mistakes
def test_planted_rate_row_mistakes_are_caught(monkeypatch):
    """Swap one of the oracle's D3Q19 relaxation rows for a neighbour and check that the
    pins above notice: f's p_ww row (11) for the 4th-order row 10, and g's z flux row (7)
    for the 3rd-order row 16."""
    good = oracle_lattice.default_rates

    def swap(which, old, new):
        def rates(lat, tau, w):
            s = good(lat, tau, w)
            if lat.name == "D3Q19" and w == which:
                s[old], s[new] = s[new], s[old]
            return s
        return rates

    import oracle.model as om
    monkeypatch.setattr(om, "default_rates", swap("f", 11, 10))
    assert abs(_shear_wave_rate(*SHEAR_WAVES["yz_diagonal"][:1], *SHEAR_WAVES["yz_diagonal"][1:]) - 1) > 0.05
    monkeypatch.setattr(om, "default_rates", swap("g", 7, 16))
    rate, _, _ = _phase_mode((32, 4, 32), (0, 0, 1))
    assert abs(rate - 1) > 0.05


# --------------------------------------------------------------------------- walls bounding y
@pytest.mark.parametrize("srt", [True, False], ids=["srt", "mrt"])
def test_d3q19_couette_between_moving_walls(srt):
    """Walls at y = -1/2 and ny - 1/2 moving -U and +U along x (half-way bounce-back with
    the moving-wall term): the steady flow is the linear Couette profile, exactly for a
    single relaxation time (every rate of f at 1 / tau_f) and to the lattice's
    second-order accuracy with the default multiple rates."""
    ny, U = 16, 0.01
    p = _case(3, ny, 3, wall_y=True, wall_u_bottom=(-U, 0, 0), wall_u_top=(U, 0, 0), nu=0.5, rho_light=1.0)
    if srt:
        tf = 0.5 + 3 * p.nu
        p = p.replace(s_f=tuple([1 / tf] * 19))
    m = Model(p).init(np.zeros((3, ny, 3)))
    m.step(3000)
    u = m.fields()["u"]
    y = np.arange(ny)
    exact = -U + 2 * U * (y + 0.5) / ny
    err = np.max(np.abs(u[0] - exact[None, :, None])) / U
    assert err < (1e-9 if srt else 2e-2)
    assert np.max(np.abs(u[1])) < 1e-12 * U and np.max(np.abs(u[2])) < 1e-12 * U


def test_d3q19_walls_conserve_phi_and_mirror_a_drop():
    """A drop midway between walls at rest: the total of phi is conserved to round-off
    (bounce-back returns every population), and the field stays mirror symmetric about
    the channel's mid-plane."""
    p = _case(16, 14, 12, wall_y=True, sigma=0.005, nu=0.05, rho_light=0.2)
    phi0 = W.drops_phi(p, [(7.5, 6.5, 5.5, 4.0)])
    m = Model(p).init(phi0)
    s0 = m.phi().sum()
    m.step(200)
    phi = m.phi()
    assert abs(phi.sum() - s0) < 2e-13 * s0
    assert np.max(np.abs(phi - phi[:, ::-1, :])) < 1e-12
