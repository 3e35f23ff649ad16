"""Dense brute-force implementation of one model step, for tiny grids only.

A second, deliberately different CPU implementation of the paper's Sect. 3 step,
used to pin the oracle: every node is visited in a Python loop, neighbours come from
explicit index arithmetic, the stencils (Eqs. 39, 40) and the streaming are dense
matrices, and the collision is the velocity-space MRT operator of Eqs. 20/30,
M^{-1} S M, built with ``np.linalg.inv``.  It shares no code with ``oracle/``.
"""
from __future__ import annotations

import numpy as np

CS2 = 1.0 / 3.0


def d2q9_tables():
    c = np.array([[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1], [1, 1], [-1, 1], [-1, -1], [1, -1]])
    w = np.array([4 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 36, 1 / 36, 1 / 36, 1 / 36])
    cx, cy = c[:, 0].astype(float), c[:, 1].astype(float)
    c2 = cx * cx + cy * cy
    M = np.array([np.ones(9), -4 + 3 * c2, 4 - 10.5 * c2 + 4.5 * c2 * c2, cx, (-5 + 3 * c2) * cx,
                  cy, (-5 + 3 * c2) * cy, cx * cx - cy * cy, cx * cy])
    return c, w, M


class Dense2D:
    def __init__(self, nx, ny, *, W, sigma, mobility, nu, lam, xi, eps_n, rho_h, rho_l,
                 wall_y=False, ub=(0.0, 0.0), ut=(0.0, 0.0), mode="coupled", U0=0.0, T=1.0,
                 s_g=None, s_f=None, nu_l=None):
        self.nx, self.ny, self.N = nx, ny, nx * ny
        self.c, self.w, self.M = d2q9_tables()
        self.W, self.lam, self.xi, self.eps = W, lam, xi, eps_n
        self.beta, self.kappa = 12 * sigma / W, 1.5 * sigma * W
        self.rho_h, self.rho_l = rho_h, rho_l
        self.wall_y, self.ub, self.ut = wall_y, np.array(ub), np.array(ut)
        self.mode, self.U0, self.T = mode, U0, T
        tg, tf = 0.5 + 3 * mobility, 0.5 + 3 * nu
        sg = s_g if s_g is not None else [1, 1, 1, 1 / tg, 1 / tg, 1 / tg, 1 / tg, 1, 1]
        sf = s_f if s_f is not None else [1, 1, 1, 1, 1, 1, 1, 1 / tf, 1 / tf]
        Minv = np.linalg.inv(self.M)
        self.Ag = Minv @ np.diag(sg) @ self.M
        self.Bg = Minv @ (np.eye(9) - 0.5 * np.diag(sg)) @ self.M
        self.Af = Minv @ np.diag(sf) @ self.M
        self.Bf = Minv @ (np.eye(9) - 0.5 * np.diag(sf)) @ self.M
        # unequal viscosities: at each node the stress rows relax at 1 / tau_f with
        # tau_f = 1/2 + mu / (rho cs^2), mu linear in phi between the two phases (Eq. 27)
        self.Minv, self.sf = Minv, list(sf)
        self.mu_h, self.mu_l = rho_h * nu, rho_l * (nu if nu_l is None else nu_l)
        self.visc = nu_l is not None and nu_l != nu
        self.opp = [int(np.where((self.c == -ci).all(axis=1))[0][0]) for ci in self.c]
        self._build_stencils()

    def idx(self, x, y):
        return x + self.nx * y

    def neighbour(self, x, y, cx, cy):
        """Index of x + c for the stencils: x wraps; y wraps, or (walls) clamps to the
        first interior row, the mirror image across the half-way wall."""
        xn = (x + cx) % self.nx
        yn = y + cy
        if self.wall_y:
            yn = min(max(yn, 0), self.ny - 1)
        else:
            yn %= self.ny
        return self.idx(xn, yn)

    def _build_stencils(self):
        N = self.N
        self.Gx, self.Gy, self.L = np.zeros((N, N)), np.zeros((N, N)), np.zeros((N, N))
        for y in range(self.ny):
            for x in range(self.nx):
                k = self.idx(x, y)
                for i in range(1, 9):
                    j = self.neighbour(x, y, *self.c[i])
                    self.Gx[k, j] += self.w[i] * self.c[i, 0] / CS2
                    self.Gy[k, j] += self.w[i] * self.c[i, 1] / CS2
                    self.L[k, j] += 2 * self.w[i] / CS2
                    self.L[k, k] -= 2 * self.w[i] / CS2

    def vortex_u(self, t):
        u = np.zeros((self.N, 2))
        for y in range(self.ny):
            for x in range(self.nx):
                ct = np.cos(np.pi * t / self.T)
                u[self.idx(x, y), 0] = self.U0 * np.sin(np.pi * x / self.nx) ** 2 * np.sin(2 * np.pi * y / self.ny) * ct
                u[self.idx(x, y), 1] = -self.U0 * np.sin(np.pi * y / self.ny) ** 2 * np.sin(2 * np.pi * x / self.nx) * ct
        return u

    def step(self, g, f, J, t):
        """g, f: (N, 9); J: (N, 2).  Returns the next (g, f, J)."""
        c, w = self.c, self.w
        phi = g.sum(axis=1)
        rho = self.rho_l + (self.rho_h - self.rho_l) * phi
        pc = np.clip(phi, 0.0, 1.0)
        a, b = pc + self.xi, 1 - pc + self.xi
        psi = self.W / 4 * np.log(a / b)
        th = np.tanh(2 * psi / self.W)
        gphi = np.stack([self.Gx @ phi, self.Gy @ phi], axis=1)
        gpsi = np.stack([self.Gx @ psi, self.Gy @ psi], axis=1)
        lphi = self.L @ phi
        mu = 4 * self.beta * phi * (phi - 1) * (phi - 0.5) - self.kappa * lphi
        Fs = mu[:, None] * gphi
        grho = (self.rho_h - self.rho_l) * gphi
        if self.mode == "coupled":
            j = f @ c
            u = (j + 0.5 * Fs) / rho[:, None]
        else:
            u = self.vortex_u(t)
        gs, fs = np.empty_like(g), np.empty_like(f)
        Jn = phi[:, None] * u
        for k in range(self.N):
            uk = u[k]
            dJ = Jn[k] - J[k]
            nrm = gpsi[k] / np.sqrt(gpsi[k] @ gpsi[k] + self.eps ** 2)
            V = dJ / CS2 + self.lam / self.W * (1 - th[k] ** 2) * nrm
            H = mu[k] + self.lam * phi[k]
            geq = np.array([w[i] * H + w[i] * (c[i] @ (phi[k] * uk)) / CS2 for i in range(9)])
            geq[0] = phi[k] + (w[0] - 1) * H
            G = np.array([w[i] * (c[i] @ V) for i in range(9)])
            # Eq. 30 with the MRT operator and Eq. 33's (I - S/2) on the source
            gs[k] = g[k] - self.Ag @ (g[k] - geq) + self.Bg @ G
            if self.mode == "coupled":
                s = np.array([w[i] * ((c[i] @ uk) / CS2 + (c[i] @ uk) ** 2 / (2 * CS2 ** 2) - uk @ uk / (2 * CS2))
                              for i in range(9)])
                press = CS2 / (1 - w[0]) * (f[k, 1:].sum() + 0.5 * uk @ grho[k] + rho[k] * s[0])
                feq = w * press / CS2 + rho[k] * s
                feq[0] = (w[0] - 1) * press / CS2 + rho[k] * s[0]
                Fi = np.array([w[i] * (uk @ grho[k] + (c[i] @ Fs[k]) / CS2
                                       + (np.outer(uk, grho[k]) * (np.outer(c[i], c[i]) - CS2 * np.eye(2))).sum() / CS2)
                               for i in range(9)])
                Af, Bf = self.Af, self.Bf
                if self.visc:
                    tau = 0.5 + (self.mu_l + phi[k] * (self.mu_h - self.mu_l)) / (rho[k] * CS2)
                    sk = np.diag(self.sf[:7] + [1 / tau, 1 / tau])
                    Af = self.Minv @ sk @ self.M
                    Bf = self.Minv @ (np.eye(9) - 0.5 * sk) @ self.M
                fs[k] = f[k] - Af @ (f[k] - feq) + Bf @ Fi
            else:
                fs[k] = f[k]
        # streaming as a dense permutation (plus bounce-back), Q N x Q N
        P = np.zeros((9 * self.N, 9 * self.N))
        wall_add = np.zeros(9 * self.N)
        for y in range(self.ny):
            for x in range(self.nx):
                k = self.idx(x, y)
                for i in range(9):
                    sx, sy = x - c[i, 0], y - c[i, 1]
                    if self.wall_y and (sy < 0 or sy >= self.ny):
                        P[9 * k + i, 9 * k + self.opp[i]] = 1.0
                        uw = self.ub if sy < 0 else self.ut
                        wall_add[9 * k + i] = 2 * w[i] * rho[k] * (c[i] @ uw) / CS2
                    else:
                        P[9 * k + i, 9 * self.idx(sx % self.nx, sy % self.ny) + i] = 1.0
        gn = (P @ gs.reshape(-1)).reshape(self.N, 9)
        fn = P @ fs.reshape(-1)
        if self.mode == "coupled":
            fn = fn + wall_add
        return gn, fn.reshape(self.N, 9), Jn

    def init(self, phi0, u0):
        c, w = self.c, self.w
        lphi = self.L @ phi0
        mu = 4 * self.beta * phi0 * (phi0 - 1) * (phi0 - 0.5) - self.kappa * lphi
        rho = self.rho_l + (self.rho_h - self.rho_l) * phi0
        g, f = np.zeros((self.N, 9)), np.zeros((self.N, 9))
        for k in range(self.N):
            H = mu[k] + self.lam * phi0[k]
            for i in range(9):
                g[k, i] = w[i] * H + w[i] * (c[i] @ (phi0[k] * u0[k])) / CS2
                cu = c[i] @ u0[k]
                s = w[i] * (cu / CS2 + cu * cu / (2 * CS2 ** 2) - u0[k] @ u0[k] / (2 * CS2))
                f[k, i] = rho[k] * s if self.mode == "coupled" else 0.0
            g[k, 0] = phi0[k] + (w[0] - 1) * H
        return g, f, phi0[:, None] * u0


# ---------------------------------------------------------------------------- 3D
def d3q19_velocities():
    """The 19 velocities of {-1, 0, 1}^3 with |c|^2 <= 2, enumerated in lexicographic order
    (not the oracle's order), with the standard weights 1/3, 1/18, 1/36 by |c|^2."""
    import itertools
    c = np.array([v for v in itertools.product((-1, 0, 1), repeat=3) if sum(a * a for a in v) <= 2])
    c2 = (c * c).sum(axis=1)
    w = np.select([c2 == 0, c2 == 1, c2 == 2], [1 / 3, 1 / 18, 1 / 36])
    return c, w


def _projector(vectors):
    """Euclidean orthogonal projector onto the span of the given vectors (rows)."""
    u, sv, _ = np.linalg.svd(np.array(vectors, dtype=float).T, full_matrices=False)
    q = u[:, sv > 1e-10 * sv[0]]
    return q @ q.T


class Dense3D:
    """One model step on a tiny periodic 3D grid, built without the moment basis.

    The multiple-relaxation-time operator of Eqs. 25/33 is M^{-1} S M.  With a basis whose
    rows are mutually orthogonal, and rates that are 1 except on one subspace, it equals
    I + (s - 1) P, with P the orthogonal projector onto that subspace.  The subspaces are
    spanned here straight from their defining polynomials: for g the first- and
    third-order axial fluxes c_a and |c|^2 c_a (a = x, y, z), relaxing at 1/tau_g; for f
    the traceless second-order tensor c_a c_b - delta_ab |c|^2 / 3, relaxing at 1/tau_f
    (Eq. 27).  Streaming is a dense permutation matrix, the stencils of Eqs. 39-40 are
    dense matrices, and every node is visited in a Python loop."""

    def __init__(self, nx, ny, nz, *, W, sigma, mobility, nu, lam, xi, eps_n, rho_h, rho_l):
        self.n = (nx, ny, nz)
        self.N = nx * ny * nz
        self.c, self.w = d3q19_velocities()
        self.Q = len(self.w)
        self.W, self.lam, self.xi, self.eps = W, lam, xi, eps_n
        self.beta, self.kappa = 12 * sigma / W, 1.5 * sigma * W
        self.rho_h, self.rho_l = rho_h, rho_l
        c = self.c.astype(float)
        c2 = (c * c).sum(axis=1)
        flux = [c[:, a] for a in range(3)] + [c2 * c[:, a] for a in range(3)]
        stress = [c[:, a] * c[:, b] - (a == b) * c2 / 3 for a in range(3) for b in range(3)]
        tg, tf = 0.5 + 3 * mobility, 0.5 + 3 * nu
        I = np.eye(self.Q)
        self.Ag = I + (1 / tg - 1) * _projector(flux)
        self.Af = I + (1 / tf - 1) * _projector(stress)
        self.Bg = I - 0.5 * self.Ag
        self.Bf = I - 0.5 * self.Af
        self._build()

    def idx(self, x, y, z):
        nx, ny, _ = self.n
        return x + nx * (y + ny * z)

    def _build(self):
        nx, ny, nz = self.n
        N, Q, c, w = self.N, self.Q, self.c, self.w
        self.G = np.zeros((3, N, N))
        self.L = np.zeros((N, N))
        self.P = np.zeros((Q * N, Q * N))
        for z in range(nz):
            for y in range(ny):
                for x in range(nx):
                    k = self.idx(x, y, z)
                    for i in range(Q):
                        cx, cy, cz = c[i]
                        nb = self.idx((x + cx) % nx, (y + cy) % ny, (z + cz) % nz)
                        src = self.idx((x - cx) % nx, (y - cy) % ny, (z - cz) % nz)
                        self.P[Q * k + i, Q * src + i] = 1.0
                        if cx == cy == cz == 0:
                            continue
                        for d in range(3):
                            self.G[d, k, nb] += w[i] * c[i, d] / CS2
                        self.L[k, nb] += 2 * w[i] / CS2
                        self.L[k, k] -= 2 * w[i] / CS2

    def step(self, g, f, J):
        """g, f: (N, Q) in this class's velocity order; J: (N, 3).  Returns the next state."""
        c, w, Q = self.c.astype(float), self.w, self.Q
        rest = int(np.where((self.c == 0).all(axis=1))[0][0])
        phi = g.sum(axis=1)
        rho = self.rho_l + (self.rho_h - self.rho_l) * phi
        pc = np.clip(phi, 0.0, 1.0)
        psi = self.W / 4 * np.log((pc + self.xi) / (1 - pc + self.xi))
        th = np.tanh(2 * psi / self.W)
        gphi = np.stack([self.G[d] @ phi for d in range(3)], axis=1)
        gpsi = np.stack([self.G[d] @ psi for d in range(3)], axis=1)
        mu = 4 * self.beta * phi * (phi - 1) * (phi - 0.5) - self.kappa * (self.L @ phi)
        Fs = mu[:, None] * gphi
        grho = (self.rho_h - self.rho_l) * gphi
        u = (f @ c + 0.5 * Fs) / rho[:, None]
        Jn = phi[:, None] * u
        gs, fs = np.empty_like(g), np.empty_like(f)
        for k in range(self.N):
            uk = u[k]
            nrm = gpsi[k] / np.sqrt(gpsi[k] @ gpsi[k] + self.eps ** 2)
            V = (Jn[k] - J[k]) / CS2 + self.lam / self.W * (1 - th[k] ** 2) * nrm
            H = mu[k] + self.lam * phi[k]
            geq = np.array([w[i] * H + w[i] * (c[i] @ Jn[k]) / CS2 for i in range(Q)])
            geq[rest] = phi[k] + (w[rest] - 1) * H
            G = np.array([w[i] * (c[i] @ V) for i in range(Q)])
            gs[k] = g[k] - self.Ag @ (g[k] - geq) + self.Bg @ G
            s = np.array([w[i] * ((c[i] @ uk) / CS2 + (c[i] @ uk) ** 2 / (2 * CS2 ** 2) - uk @ uk / (2 * CS2))
                          for i in range(Q)])
            moving = [i for i in range(Q) if i != rest]
            press = CS2 / (1 - w[rest]) * (f[k, moving].sum() + 0.5 * uk @ grho[k] + rho[k] * s[rest])
            feq = w * press / CS2 + rho[k] * s
            feq[rest] = (w[rest] - 1) * press / CS2 + rho[k] * s[rest]
            Fi = np.array([w[i] * (uk @ grho[k] + (c[i] @ Fs[k]) / CS2
                                   + (np.outer(uk, grho[k]) * (np.outer(c[i], c[i]) - CS2 * np.eye(3))).sum() / CS2)
                           for i in range(Q)])
            fs[k] = f[k] - self.Af @ (f[k] - feq) + self.Bf @ Fi
        gn = (self.P @ gs.reshape(-1)).reshape(self.N, Q)
        fn = (self.P @ fs.reshape(-1)).reshape(self.N, Q)
        return gn, fn, Jn

    def init(self, phi0, u0):
        c, w, Q = self.c.astype(float), self.w, self.Q
        rest = int(np.where((self.c == 0).all(axis=1))[0][0])
        mu = 4 * self.beta * phi0 * (phi0 - 1) * (phi0 - 0.5) - self.kappa * (self.L @ phi0)
        rho = self.rho_l + (self.rho_h - self.rho_l) * phi0
        g, f = np.zeros((self.N, Q)), np.zeros((self.N, Q))
        for k in range(self.N):
            H = mu[k] + self.lam * phi0[k]
            for i in range(Q):
                g[k, i] = w[i] * H + w[i] * (c[i] @ (phi0[k] * u0[k])) / CS2
                cu = c[i] @ u0[k]
                f[k, i] = rho[k] * w[i] * (cu / CS2 + cu * cu / (2 * CS2 ** 2) - u0[k] @ u0[k] / (2 * CS2))
            g[k, rest] = phi0[k] + (w[rest] - 1) * H
        return g, f, phi0[:, None] * u0
