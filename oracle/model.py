"""The oracle's time step: the paper's Sect. 3 equations, written out in numpy.

TEST INFRASTRUCTURE ONLY (see the package docstring).

State per node: phase-field populations g_i, hydrodynamic populations f_i (both
already streamed, i.e. at time t), and the previous step's phi u used by the
backward time difference.  Arrays have shape (Q, nz, ny, nx) or (D, nz, ny, nx);
2D cases use nz = 1 and velocities with a zero z component.

One step, in the only order in which every quantity depends on time-t values:
  1. phi = sum_i g_i                                   (Eq. 35)
  2. rho(phi), clipped phi, psi                        (Eq. 37 and the clipping rule after it)
  3. grad phi, lap phi, grad psi                       (Eqs. 39, 40)
  4. chemical potential, surface-tension force         (Eq. 2; F_s = mu grad phi, Sect. 2)
  5. velocity and pressure                             (Eqs. 28, 29) or the prescribed vortex (Eqs. 43, 44)
  6. time derivative of phi u                          (backward difference, Sect. 3.2)
  7. g: equilibrium, source, MRT collision             (Eqs. 31, 32, 33)
  8. f: equilibrium, forcing, MRT collision            (Eqs. 21, 22, 23, 25)
  9. streaming, with bounce-back walls when present
Readings of points the paper leaves open are stated where they are used.

Works with complex128 arrays too (complex-step differentiation): the clip acts on
the real part, and every other operation is analytic.
"""
from __future__ import annotations

import numpy as np

from .lattice import default_rates, lattice_for, stress_rows


def _clip01(phi):
    """phi_clip = min(max(0, phi), 1), applied to the real part (Sect. 3.2, after Eq. 37)."""
    re = np.real(phi)
    out = np.where(re < 0.0, 0.0 * phi, phi)
    out = np.where(re > 1.0, 0.0 * phi + 1.0, out)
    return out


def min_image(d, n, periodic):
    """Displacement wrapped to [-n/2, n/2) along a periodic axis."""
    if not periodic:
        return d
    return d - n * np.floor((d + 0.5 * n) / n)


class Model:
    """One case of the coupled (or prescribed-velocity) phase-field LB model.

    ``sigma`` and ``mobility`` may be overridden (e.g. by complex numbers for
    complex-step derivatives); everything else comes from the ``CaseParams``.
    ``normal_tau`` only affects complex-step derivatives: see ``unit_normal``.
    """

    def __init__(self, p, dtype=np.float64, sigma=None, mobility=None, normal_tau=0.0):
        self.p = p
        self.normal_tau = float(normal_tau)
        self.lat = lat = lattice_for(p.lattice)
        self.dtype = dtype
        self.cs2 = lat.cs2
        sig = p.sigma if sigma is None else sigma
        mob = p.mobility if mobility is None else mobility
        # Sect. 2, after Eq. 1: beta = 12 sigma / W, kappa = 3 sigma W / 2.
        self.beta = 12.0 * sig / p.W
        self.kappa = 1.5 * sig * p.W
        # Eq. 34: M = cs^2 (tau_g - 1/2);  Eq. 27 with mu = rho nu: nu = cs^2 (tau_f - 1/2).
        self.tau_g = 0.5 + mob / self.cs2
        self.tau_f = 0.5 + p.nu / self.cs2
        # Unequal viscosities of the two phases (Sect. 4.1 names the dynamic viscosity
        # ratio mu_l / mu_g): tau_f follows Eq. 27 node by node (see tau_f_of).
        nu_l = getattr(p, "nu_light", None)
        self.visc = nu_l is not None and nu_l != p.nu
        self.mu_heavy = p.rho_heavy * p.nu
        self.mu_light = p.rho_light * (p.nu if nu_l is None else nu_l)
        # global volume correction (an ablation, not the paper's model: see global_source)
        self.mass_fix = float(getattr(p, "mass_fix", 0.0))
        self.V_ref = None
        sg = default_rates(lat, self.tau_g, "g")
        sf = default_rates(lat, self.tau_f, "f")
        if p.s_g:
            sg = [v if v != 0 else d for v, d in zip(p.s_g, sg)]
        if p.s_f:
            sf = [v if v != 0 else d for v, d in zip(p.s_f, sf)]
        self.Sg = np.diag(np.array(sg, dtype=dtype))
        self.Sf = np.diag(np.array(sf, dtype=dtype))
        self.M = lat.M.astype(dtype)
        self.Minv = np.linalg.inv(lat.M).astype(dtype)
        self.I = np.eye(lat.Q, dtype=dtype)
        self.shape = (p.nz, p.ny, p.nx)
        Q, D = lat.Q, lat.D
        self.g = np.zeros((Q,) + self.shape, dtype=dtype)
        self.f = np.zeros((Q,) + self.shape, dtype=dtype)
        self.Jprev = np.zeros((D,) + self.shape, dtype=dtype)
        self.t = 0
        self.cvec = lat.c[:, :D].astype(np.float64)      # (Q, D)

    # ------------------------------------------------------------------ stencils
    def wet_ghost(self, edge, side):
        """phi of the ghost row behind a wall (side 0: bottom, 1: top) from the edge row's
        phi_e.  The equilibrium profile (Eqs. 4-5) has |grad phi| = (4 / W) phi (1 - phi);
        where the interface meets the wall at the contact angle theta (measured in the
        heavy phase), the normal derivative of phi into the fluid is then
        -(4 / W) cos(theta) phi (1 - phi).  Taken as the one-sided difference across the
        half-way wall with phi at the edge node: phi_g = phi_e + (4 / W) cos(theta)
        phi_e (1 - phi_e).  theta = 90 degrees (cos = 0) gives the mirror phi_g = phi_e.
        (A reading: the paper states no boundary conditions.)"""
        p = self.p
        cw = getattr(p, "wall_cos_bottom" if side == 0 else "wall_cos_top", 0.0)
        if cw == 0.0:
            return edge
        return edge + 4.0 / p.W * cw * edge * (1.0 - edge)

    def _pad(self, a, wet=False):
        """One ghost layer: periodic axes wrap; wall axes (y) mirror the first interior
        node across the half-way wall, i.e. zero normal gradient (a reading: the paper
        does not state its boundary conditions).  wet: a is phi, and the ghost rows are
        the wetting ghosts of the edge rows (wet_ghost)."""
        a = np.pad(a, ((1, 1), (0, 0), (0, 0)), mode="wrap")
        a = np.pad(a, ((0, 0), (1, 1), (0, 0)), mode="edge" if self.p.wall_y else "wrap")
        if wet and self.p.wall_y:
            a[:, 0, :] = self.wet_ghost(a[:, 1, :], 0)
            a[:, -1, :] = self.wet_ghost(a[:, -2, :], 1)
        a = np.pad(a, ((0, 0), (0, 0), (1, 1)), mode="wrap")
        return a

    def _at(self, ap, ci):
        nz, ny, nx = self.shape
        cx, cy, cz = (int(v) for v in ci)
        return ap[1 + cz:1 + cz + nz, 1 + cy:1 + cy + ny, 1 + cx:1 + cx + nx]

    def _grad_padded(self, ap):
        lat = self.lat
        out = np.zeros((lat.D,) + self.shape, dtype=ap.dtype)
        for i in range(1, lat.Q):
            nb = self._at(ap, lat.c[i])
            for d in range(lat.D):
                if lat.c[i, d] != 0:
                    out[d] = out[d] + lat.w[i] * lat.c[i, d] * nb / self.cs2
        return out

    def grad(self, a, wet=False):
        """Isotropic gradient, Eq. 39: sum_{i != 0} w_i c_i a(x + c_i) / cs^2 (wet: a is phi,
        with wetting ghosts behind walls)."""
        return self._grad_padded(self._pad(a, wet))

    def grad_psi(self, phi):
        """Gradient (Eq. 39) of psi (Eq. 37), with psi of the wetting ghosts behind walls."""
        return self._grad_padded(self.psi_of(self._pad(phi, wet=True)))

    def lap(self, a, wet=False):
        """Isotropic Laplacian, Eq. 40: sum_{i != 0} 2 w_i [a(x + c_i) - a(x)] / cs^2 (wet: a
        is phi, with wetting ghosts behind walls)."""
        lat = self.lat
        ap = self._pad(a, wet)
        out = np.zeros(self.shape, dtype=a.dtype)
        for i in range(1, lat.Q):
            out = out + 2.0 * lat.w[i] * (self._at(ap, lat.c[i]) - a) / self.cs2
        return out

    # ------------------------------------------------------------------ pieces
    def rho_of(self, phi):
        """Density, linear in the (unclipped) order parameter: rho_light at phi = 0 and
        rho_heavy at phi = 1 (a reading: the paper gives only the density ratio)."""
        p = self.p
        return p.rho_light + phi * (p.rho_heavy - p.rho_light)

    def tau_f_of(self, phi, rho):
        """Per-node relaxation time of f, Eq. 27: mu = rho c_s^2 (tau_f - 1/2), with the
        dynamic viscosity interpolated linearly in the (unclipped) order parameter
        between the light (phi = 0) and heavy (phi = 1) phases, as the density is (a
        reading: the paper names the viscosity ratio but not the interpolation)."""
        mu = self.mu_light + phi * (self.mu_heavy - self.mu_light)
        return 0.5 + mu / (rho * self.cs2)

    @staticmethod
    def smooth_volume_terms(phi):
        """H(phi_c) = phi_c^2 (3 - 2 phi_c), a smooth step that counts the volume enclosed by
        the phi = 1/2 level (it is flat at 0 and 1, so small bulk shifts of phi do not
        count), and the interface indicator delta(phi_c) = 4 phi_c (1 - phi_c), which is
        W |grad phi| of the equilibrium profile (Eq. 5)."""
        pc = _clip01(phi)
        return pc * pc * (3.0 - 2.0 * pc), 4.0 * pc * (1.0 - pc)

    def volume(self, phi=None):
        """V = sum_x H(phi_c): the volume the global correction holds."""
        return self.smooth_volume_terms(self.phi() if phi is None else phi)[0].sum()

    def global_source(self, phi):
        """The correction of the kind the paper's introduction describes (Wang et al.): a
        source added at every interface node, in proportion to the interface indicator,
        whose total makes up a rate r of the volume lost since the reference state:
        S(x) = kappa delta(x), kappa = r (V_ref - V(t)) / sum delta.  The paper states no
        formula; this form is a reading.  Returns S (zero without the correction)."""
        if self.mass_fix == 0.0:
            return None
        H, delta = self.smooth_volume_terms(phi)
        sd = delta.sum()
        kappa = self.mass_fix * (self.V_ref - H.sum()) / sd if np.real(sd) > 0 else 0.0 * sd
        return kappa * delta

    def psi_of(self, phi):
        """Regularised signed distance, Eq. 37, evaluated on the clipped phi."""
        p = self.p
        pc = _clip01(phi)
        return p.W / 4.0 * np.log((pc + p.xi) / (1.0 - pc + p.xi))

    def s_i(self, u):
        """Eq. 23: s_i(u) = w_i [c_i.u / cs^2 + (c_i.u)^2 / (2 cs^4) - u.u / (2 cs^2)], shape (Q, ...)."""
        cu = np.tensordot(self.cvec, u, axes=(1, 0))            # (Q, ...)
        uu = (u * u).sum(axis=0)
        w = self.lat.w.reshape((-1,) + (1,) * uu.ndim)
        cs2 = self.cs2
        return w * (cu / cs2 + cu * cu / (2.0 * cs2 * cs2) - uu / (2.0 * cs2))

    def prescribed_u(self, t):
        """Single-vortex velocity of Eqs. 43-44 at step t, node (i, j) at (x, y) = (i, j);
        L is the box side along the sine's own axis, t counts steps (a reading of the
        garbled time scaling after Eq. 44)."""
        p = self.p
        nz, ny, nx = self.shape
        x = np.arange(nx, dtype=np.float64)[None, None, :]
        y = np.arange(ny, dtype=np.float64)[None, :, None]
        ct = np.cos(np.pi * t / p.T)
        u = np.zeros((self.lat.D,) + self.shape, dtype=self.dtype)
        u[0] = p.U0 * np.sin(np.pi * x / nx) ** 2 * np.sin(2.0 * np.pi * y / ny) * ct
        u[1] = -p.U0 * np.sin(np.pi * y / ny) ** 2 * np.sin(2.0 * np.pi * x / nx) * ct
        return u

    def fields(self):
        """Every nodal quantity of the current state (time t), steps 1-5 above."""
        p, lat, cs2 = self.p, self.lat, self.cs2
        phi = self.g.sum(axis=0)                                   # Eq. 35
        rho = self.rho_of(phi)
        psi = self.psi_of(phi)                                     # Eq. 37
        sech2 = 1.0 - np.tanh(2.0 * psi / p.W) ** 2                # factor in Eq. 32
        gphi = self.grad(phi, wet=True)                            # Eq. 39
        lphi = self.lap(phi, wet=True)                             # Eq. 40
        gpsi = self.grad_psi(phi)
        mu = 4.0 * self.beta * phi * (phi - 1.0) * (phi - 0.5) - self.kappa * lphi   # Eq. 2
        Fs = mu * gphi                                             # F_s = mu grad phi (Sect. 2)
        grho = (p.rho_heavy - p.rho_light) * gphi
        if p.mode == "coupled":
            j = np.tensordot(self.cvec.T, self.f, axes=(1, 0))     # sum_i c_i f_i
            u = (j + 0.5 * Fs) / rho                               # Eq. 28 (dt = 1)
            w0 = lat.w[0]
            s0 = self.s_i(u)[0]
            press = cs2 / (1.0 - w0) * (self.f[1:].sum(axis=0) + 0.5 * (u * grho).sum(axis=0)
                                        + rho * s0)                # Eq. 29
        else:
            u = self.prescribed_u(self.t)
            press = np.zeros_like(phi)
        return dict(phi=phi, rho=rho, psi=psi, sech2=sech2, gphi=gphi, lphi=lphi, gpsi=gpsi,
                    mu=mu, Fs=Fs, grho=grho, u=u, p=press)

    def g_equilibrium(self, phi, mu, u):
        """Eq. 31: g0 = phi + (w0 - 1)(mu + lambda phi); gi = wi (mu + lambda phi) + wi ci.(phi u)/cs^2."""
        lat, cs2 = self.lat, self.cs2
        H = mu + self.p.lam * phi
        w = lat.w.reshape((-1,) + (1,) * phi.ndim)
        cphiu = np.tensordot(self.cvec, phi * u, axes=(1, 0))
        geq = w * H + w * cphiu / cs2
        geq[0] = phi + (lat.w[0] - 1.0) * H
        return geq

    def g_source(self, V):
        """Eq. 32 written as G_i = w_i c_i . V with
        V = d_t(phi u) / cs^2 + (lambda / W) [1 - tanh^2(2 psi / W)] n."""
        w = self.lat.w.reshape((-1,) + (1,) * (V.ndim - 1))
        return w * np.tensordot(self.cvec, V, axes=(1, 0))

    def unit_normal(self, gpsi):
        """grad psi / |grad psi|, with |grad psi| = sqrt(|grad psi|^2 + eps_n^2) (a reading: the
        paper does not say what to do where psi is flat).

        With complex arrays and normal_tau > 0, the normal is held at its real value (no
        derivative) where |Re grad psi| < normal_tau: away from the interface psi
        saturates, |grad psi| falls towards eps_n, and the derivative of n there, with
        gain lambda / |grad psi| per step, is rounding-driven and grows without bound
        over long runs.  The value of n is unchanged; only derivatives see the cut."""
        n2 = (gpsi * gpsi).sum(axis=0)
        n = gpsi / np.sqrt(n2 + self.p.eps_n ** 2)
        if self.normal_tau > 0.0 and np.iscomplexobj(n):
            mag2 = (np.real(gpsi) ** 2).sum(axis=0)
            n = np.where(mag2[None] < self.normal_tau ** 2, np.real(n) + 0j, n)
        return n

    def f_equilibrium(self, press, rho, u):
        """Eq. 22: f0 = (w0 - 1) p / cs^2 + rho s0(u); fi = wi p / cs^2 + rho si(u)."""
        lat, cs2 = self.lat, self.cs2
        w = lat.w.reshape((-1,) + (1,) * rho.ndim)
        feq = w * press / cs2 + rho * self.s_i(u)
        feq[0] = (lat.w[0] - 1.0) * press / cs2 + rho * self.s_i(u)[0]
        return feq

    def f_forcing(self, u, grho, Fs):
        """Eq. 21, term by term:
        F_i = w_i [u.grad rho + c_i.F / cs^2 + (u grad rho):(c_i c_i - cs^2 I) / cs^2]."""
        lat, cs2 = self.lat, self.cs2
        w = lat.w.reshape((-1,) + (1,) * (u.ndim - 1))
        ug = (u * grho).sum(axis=0)
        cF = np.tensordot(self.cvec, Fs, axes=(1, 0))
        cu = np.tensordot(self.cvec, u, axes=(1, 0))
        cg = np.tensordot(self.cvec, grho, axes=(1, 0))
        contraction = cu * cg - cs2 * ug          # (u grad rho) : (c c - cs^2 I)
        return w * (ug + cF / cs2 + contraction / cs2)

    def mrt(self, pop, eq, src, S):
        """Moment-space collision, Eqs. 25/33: m* = m - S (m - m_eq) + (I - S/2) src_bar,
        back to velocity space with M^{-1}.  S is the diagonal rate matrix, or an array of
        rates per moment row and node, shape (Q, ...) like pop."""
        Q = self.lat.Q
        shp = pop.shape
        m = self.M @ pop.reshape(Q, -1)
        meq = self.M @ eq.reshape(Q, -1)
        sb = self.M @ src.reshape(Q, -1)
        if S.shape == (Q, Q):
            mstar = m - S @ (m - meq) + (self.I - 0.5 * S) @ sb
        else:
            s = S.reshape(Q, -1)
            mstar = m - s * (m - meq) + (1.0 - 0.5 * s) * sb
        return (self.Minv @ mstar).reshape(shp)

    def f_rates(self, phi, rho):
        """Rates of the f collision: the constant S^f, or with unequal viscosities the
        same rates per node with the stress rows at 1 / tau_f(phi) (Eq. 27)."""
        if not self.visc:
            return self.Sf
        Q = self.lat.Q
        s = np.broadcast_to(np.diag(self.Sf).reshape((Q,) + (1,) * phi.ndim), (Q,) + phi.shape).copy()
        s = s.astype(np.result_type(phi, s))
        tau = self.tau_f_of(phi, rho)
        for k in stress_rows(self.lat):
            s[k] = 1.0 / tau
        return s

    # ------------------------------------------------------------------ streaming
    def stream(self, post, rho=None, moving=False):
        """Pull streaming pop_i(x, t+1) = post_i(x - c_i).  With walls bounding y at
        y = -1/2 and y = ny - 1/2, a population whose source lies behind a wall is the
        node's own opposite post-collision population (half-way bounce-back); for f the
        moving-wall term + 2 w_i rho (c_i . u_wall) / cs^2 is added (rho of the node at
        the collision time).  A reading: the paper states no boundary conditions."""
        lat, p = self.lat, self.p
        out = np.empty_like(post)
        for i in range(lat.Q):
            cx, cy, cz = (int(v) for v in lat.c[i])
            out[i] = np.roll(post[i], shift=(cz, cy, cx), axis=(0, 1, 2))
        if p.wall_y:
            ny = self.shape[1]
            for i in range(lat.Q):
                cy = int(lat.c[i, 1])
                if cy == 0:
                    continue
                row = 0 if cy > 0 else ny - 1
                uw = np.array(p.wall_u_bottom if cy > 0 else p.wall_u_top)[: lat.D]
                val = post[lat.opp[i]][:, row, :]
                if moving:
                    cu = float(np.dot(lat.c[i, : lat.D], uw))
                    if cu != 0.0:
                        val = val + 2.0 * lat.w[i] * rho[:, row, :] * cu / self.cs2
                out[i][:, row, :] = val
        return out

    # ------------------------------------------------------------------ public
    def init(self, phi0, u0=None):
        """Initial state (a reading: the paper only says u = p = 0 initially):
        g = g_eq(phi0, mu0, u0), f = f_eq(p = 0, rho(phi0), u0), previous phi u = phi0 u0."""
        p, lat = self.p, self.lat
        phi0 = np.asarray(phi0).reshape(self.shape).astype(self.dtype)
        if p.mode == "vortex":
            u0 = self.prescribed_u(0)
        elif u0 is None:
            u0 = np.zeros((lat.D,) + self.shape, dtype=self.dtype)
        else:
            u0 = np.asarray(u0).reshape((lat.D,) + self.shape).astype(self.dtype)
        mu0 = 4.0 * self.beta * phi0 * (phi0 - 1.0) * (phi0 - 0.5) - self.kappa * self.lap(phi0, wet=True)
        self.g = self.g_equilibrium(phi0, mu0, u0)
        if p.mode == "coupled":
            self.f = self.f_equilibrium(np.zeros_like(phi0), self.rho_of(phi0), u0)
        else:
            self.f = np.zeros_like(self.g)
        self.Jprev = phi0 * u0
        self.t = 0
        self.set_reference_volume()
        return self

    def set_reference_volume(self):
        """V_ref of the global correction: the volume of the current state."""
        self.V_ref = self.volume() if self.mass_fix != 0.0 else None
        return self

    def step(self, n=1):
        p, lat, cs2 = self.p, self.lat, self.cs2
        for _ in range(int(n)):
            F = self.fields()
            phi, u = F["phi"], F["u"]
            J = phi * u
            dJ = J - self.Jprev                                   # backward difference, dt = 1
            self.Jprev = J
            V = dJ / cs2 + (p.lam / p.W) * F["sech2"] * self.unit_normal(F["gpsi"])
            G = self.g_source(V)                                  # Eq. 32
            geq = self.g_equilibrium(phi, F["mu"], u)             # Eq. 31
            gstar = self.mrt(self.g, geq, G, self.Sg)             # Eq. 33
            S = self.global_source(phi)
            if S is not None:                                     # g_i += w_i S
                gstar = gstar + self.lat.w.reshape((-1,) + (1,) * phi.ndim) * S
            if p.mode == "coupled":
                feq = self.f_equilibrium(F["p"], F["rho"], u)     # Eqs. 22, 23
                Fi = self.f_forcing(u, F["grho"], F["Fs"])        # Eq. 21
                fstar = self.mrt(self.f, feq, Fi, self.f_rates(phi, F["rho"]))   # Eq. 25
                self.f = self.stream(fstar, rho=F["rho"], moving=True)
            self.g = self.stream(gstar)
            self.t += 1
        return self

    def phi(self):
        return self.g.sum(axis=0)

    def observables(self):
        return observables_from_phi(self.p, self.phi())


def label_geometry(p):
    """Reference centres of the observation labels and the periodicity of each axis.

    With no centres given, one label covers the domain, referred to its centre.
    Every node belongs to the label whose centre is nearest (minimum image along
    periodic axes; the first one on ties).
    """
    cents = list(p.label_centres) or [((p.nx - 1) / 2.0, (p.ny - 1) / 2.0, (p.nz - 1) / 2.0)]
    periodic = (True, not p.wall_y, True)
    return np.array(cents, dtype=np.float64), periodic


def observables_from_phi(p, phi):
    """Per-label volume reductions of a phase field: sum phi, #(phi >= 1/2),
    sum phi d, sum phi d d^T (d: displacement from the label centre), non-finite flag.

    Returns a dict of arrays with leading dimension = number of labels; the second
    moments are ordered xx, yy, zz, xy, xz, yz.
    """
    cents, periodic = label_geometry(p)
    nz, ny, nx = p.nz, p.ny, p.nx
    phi = np.asarray(phi).reshape(nz, ny, nx)
    X = np.arange(nx, dtype=np.float64)[None, None, :] + np.zeros((nz, ny, nx))
    Y = np.arange(ny, dtype=np.float64)[None, :, None] + np.zeros((nz, ny, nx))
    Z = np.arange(nz, dtype=np.float64)[:, None, None] + np.zeros((nz, ny, nx))
    disp = []
    for (cx, cy, cz) in cents:
        disp.append((min_image(X - cx, nx, periodic[0]),
                     min_image(Y - cy, ny, periodic[1]),
                     min_image(Z - cz, nz, periodic[2])))
    d2 = np.stack([dx * dx + dy * dy + dz * dz for dx, dy, dz in disp])
    label = np.argmin(d2, axis=0)
    L = len(cents)
    res = {k: [] for k in ("sum_phi", "count_half", "sum_phi_d", "sum_phi_dd", "nonfinite")}
    for k in range(L):
        m = label == k
        dx, dy, dz = (a[m] for a in disp[k])
        ph = phi[m]
        res["sum_phi"].append(ph.sum())
        res["count_half"].append(int((np.real(ph) >= 0.5).sum()))
        res["sum_phi_d"].append([(ph * dx).sum(), (ph * dy).sum(), (ph * dz).sum()])
        res["sum_phi_dd"].append([(ph * dx * dx).sum(), (ph * dy * dy).sum(), (ph * dz * dz).sum(),
                                  (ph * dx * dy).sum(), (ph * dx * dz).sum(), (ph * dy * dz).sum()])
        res["nonfinite"].append(int(not np.all(np.isfinite(ph))))
    return {k: np.array(v) for k, v in res.items()}


def derived_observables(obs, cents=None):
    """Volume, centroid offset and deformation D = (sqrt(l+) - sqrt(l-)) / (sqrt(l+) + sqrt(l-))
    from the eigenvalues l+- of the phi-weighted in-plane (x, y) second-moment tensor
    about the phi-weighted centroid (analytic in the inputs, for complex-step use)."""
    V = obs["sum_phi"]
    c = obs["sum_phi_d"] / V[:, None]
    dd = obs["sum_phi_dd"] / V[:, None]
    ixx = dd[:, 0] - c[:, 0] * c[:, 0]
    iyy = dd[:, 1] - c[:, 1] * c[:, 1]
    ixy = dd[:, 3] - c[:, 0] * c[:, 1]
    tr = ixx + iyy
    disc = np.sqrt(((ixx - iyy) / 2.0) ** 2 + ixy * ixy)
    lp, lm = tr / 2.0 + disc, tr / 2.0 - disc
    with np.errstate(invalid="ignore"):
        D = (np.sqrt(lp) - np.sqrt(lm)) / (np.sqrt(lp) + np.sqrt(lm))
    return dict(volume=V, centroid=c, D=D, count_half=obs["count_half"])


def observables_by_labels(phi, labels, nlabels):
    """Volume reductions of a phase field over caller-given labels: for each label l the
    sums over the nodes with labels == l of phi, of #(phi >= 1/2), of phi x and of
    phi x x^T (x = the node's position (i, j, k), moments about the origin), and whether
    phi is non-finite somewhere; nodes with a negative label belong to no label.  Second
    moments are ordered xx, yy, zz, xy, xz, yz."""
    phi = np.asarray(phi)
    labels = np.asarray(labels).reshape(phi.shape)
    nz, ny, nx = phi.shape
    Z, Y, X = np.meshgrid(np.arange(nz, dtype=np.float64), np.arange(ny, dtype=np.float64),
                          np.arange(nx, dtype=np.float64), indexing="ij")
    res = {k: [] for k in ("sum_phi", "count_half", "sum_phi_d", "sum_phi_dd", "nonfinite")}
    for k in range(nlabels):
        m = labels == k
        ph, x, y, z = phi[m], X[m], Y[m], Z[m]
        res["sum_phi"].append(ph.sum())
        res["count_half"].append(int((np.real(ph) >= 0.5).sum()))
        res["sum_phi_d"].append([(ph * x).sum(), (ph * y).sum(), (ph * z).sum()])
        res["sum_phi_dd"].append([(ph * x * x).sum(), (ph * y * y).sum(), (ph * z * z).sum(),
                                  (ph * x * y).sum(), (ph * x * z).sum(), (ph * y * z).sum()])
        res["nonfinite"].append(int(not np.all(np.isfinite(ph))))
    return {k: np.array(v) for k, v in res.items()}
