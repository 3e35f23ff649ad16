"""Seeded, synthetic inputs shared by the CPU oracle tests, the GPU tests and the bench.

This module holds case parameters and initial fields only: none of the lattice
Boltzmann arithmetic lives here, so the oracle (``oracle/``) and the HIP library
(``paper_2505_10899_amd``) can both be fed from it without sharing any code of the
method itself.

Initial phase fields are the equilibrium hyperbolic-tangent profile of the paper's
Sect. 2 (Eq. 4), phi = 1/2 [1 + tanh(2 s / W)], with s the signed distance to the
interface (positive inside the heavy phase).  Several drops are superposed as in the
two-droplet initialisation of Sect. 4.1.

Node (i, j, k) sits at position (x, y, z) = (i, j, k) in lattice units.  Walls, when
present, bound the y axis half-way between nodes: at y = -1/2 and y = ny - 1/2.
"""
from __future__ import annotations

import dataclasses
import json
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

LATTICES = ("D2Q9", "D3Q19")
STORAGES = ("fp64", "fp32", "fp16s")
MODES = ("coupled", "vortex")


@dataclasses.dataclass
class CaseParams:
    """One simulation case, in lattice units (dx = dt = 1).

    Every physical quantity the paper's problem statement names (Sects. 2-4):
    interface width W, surface tension sigma, mobility M, penalty constant lambda,
    regulariser xi, the two densities and the kinematic viscosity; plus choices the
    paper leaves open (boundary type, relaxation rates other than the four it
    fixes, the normal regulariser eps_n).
    """

    nx: int
    ny: int
    nz: int = 1
    lattice: str = "D2Q9"
    storage: str = "fp64"
    mode: str = "coupled"
    wall_y: bool = False                       # bounce-back walls bounding y
    wall_u_bottom: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    wall_u_top: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    wall_cos_bottom: float = 0.0               # cos(contact angle) of the bottom wall, angle in the
    wall_cos_top: float = 0.0                  # heavy phase (0: 90 degrees, mirror stencil ghosts)
    W: float = 4.0
    sigma: float = 0.01
    mobility: float = 0.1
    lam: float = 0.5                           # penalty constant (Sect. 2, after Eq. 6)
    mass_fix: float = 0.0                      # rate of a global volume correction (0: none)
    xi: float = 1e-10                          # regulariser in Eq. 37
    eps_n: float = 1e-12                       # |grad psi| regulariser of the unit normal
    rho_heavy: float = 1.0                     # density where phi = 1
    rho_light: float = 1.0                     # density where phi = 0
    nu: float = 0.1                            # kinematic viscosity (tau_f = 1/2 + nu / cs^2); of the
                                               # heavy phase when nu_light is given
    nu_light: Optional[float] = None           # kinematic viscosity of the light phase (None: nu)
    s_g: Optional[Tuple[float, ...]] = None    # None: default MRT rates for g
    s_f: Optional[Tuple[float, ...]] = None    # None: default MRT rates for f
    U0: float = 0.0                            # prescribed single-vortex amplitude (Eqs. 43-44)
    T: float = 1.0                             # prescribed single-vortex period, in steps
    label_centres: List[Tuple[float, float, float]] = dataclasses.field(default_factory=list)

    @property
    def n_nodes(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def dim(self) -> int:
        return 2 if self.lattice == "D2Q9" else 3

    def replace(self, **kw) -> "CaseParams":
        return dataclasses.replace(self, **kw)

    def to_json(self) -> dict:
        return dataclasses.asdict(self)


# ---------------------------------------------------------------------------
# initial fields
# ---------------------------------------------------------------------------

def _axis_coords(n: int) -> np.ndarray:
    return np.arange(n, dtype=np.float64)


def _min_image(d: np.ndarray, n: int, periodic: bool) -> np.ndarray:
    if not periodic:
        return d
    return d - n * np.round(d / n)


def drops_phi(p: CaseParams, drops: Sequence[Tuple[float, float, float, float]]) -> np.ndarray:
    """Sum of tanh drops (Eq. 4 profile; Sect. 4.1 superposition).

    ``drops`` holds (cx, cy, cz, R).  Distances use the minimum image along periodic
    axes.  Returns phi with shape (nz, ny, nx), float64.
    """
    z = _axis_coords(p.nz)[:, None, None]
    y = _axis_coords(p.ny)[None, :, None]
    x = _axis_coords(p.nx)[None, None, :]
    phi = np.zeros((p.nz, p.ny, p.nx))
    for (cx, cy, cz, R) in drops:
        dx = _min_image(x - cx, p.nx, True)
        dy = _min_image(y - cy, p.ny, not p.wall_y)
        dz = _min_image(z - cz, p.nz, True) if p.nz > 1 else 0.0 * z
        r = np.sqrt(dx * dx + dy * dy + dz * dz)
        phi = phi + 0.5 * (1.0 + np.tanh(2.0 * (R - r) / p.W))
    return phi


def cylinder_phi(p: CaseParams, cx: float, cy: float, R0: float, eps: float, wavelength: float) -> np.ndarray:
    """Liquid column along z with radius R(z) = R0 (1 + eps cos(2 pi z / wavelength))."""
    z = _axis_coords(p.nz)[:, None, None]
    y = _axis_coords(p.ny)[None, :, None]
    x = _axis_coords(p.nx)[None, None, :]
    dx = _min_image(x - cx, p.nx, True)
    dy = _min_image(y - cy, p.ny, True)
    r = np.sqrt(dx * dx + dy * dy)
    Rz = R0 * (1.0 + eps * np.cos(2.0 * np.pi * z / wavelength))
    return 0.5 * (1.0 + np.tanh(2.0 * (Rz - r) / p.W))


def slab_phi(p: CaseParams, y0: float, y1: float) -> np.ndarray:
    """Flat heavy slab between y0 < y < y1 (two tanh interfaces, periodic in y)."""
    y = _axis_coords(p.ny)[None, :, None] + 0.0 * _axis_coords(p.nx)[None, None, :]
    y = np.broadcast_to(y, (p.nz, p.ny, p.nx))
    s = np.minimum(y - y0, y1 - y)
    return 0.5 * (1.0 + np.tanh(2.0 * s / p.W))


def couette_u(p: CaseParams) -> np.ndarray:
    """Linear shear profile matching the two moving walls (x-velocity only), shape (D, nz, ny, nx)."""
    ub, ut = p.wall_u_bottom[0], p.wall_u_top[0]
    y = _axis_coords(p.ny)
    ux = ub + (ut - ub) * (y + 0.5) / p.ny
    u = np.zeros((p.dim, p.nz, p.ny, p.nx))
    u[0] = ux[None, :, None]
    return u


# ---------------------------------------------------------------------------
# the workloads
# ---------------------------------------------------------------------------

def two_droplets(storage: str = "fp64", scale: int = 1) -> Tuple[CaseParams, np.ndarray, None]:
    """Two static drops in gas: 128x128 periodic, R = 24 at (40, 64) and R = 8 at (96, 64),
    W = 4, density ratio 10, M = 0.1, sigma = 0.01, nu = 0.1, u = p = 0.

    ``scale`` multiplies the box and the geometry (scale = 32 gives a 4096x4096 box).
    """
    s = int(scale)
    p = CaseParams(nx=128 * s, ny=128 * s, W=4.0, sigma=0.01, mobility=0.1, nu=0.1,
                   rho_heavy=1.0, rho_light=0.1, storage=storage,
                   label_centres=[(40.0 * s, 64.0 * s, 0.0), (96.0 * s, 64.0 * s, 0.0)])
    phi0 = drops_phi(p, [(40.0 * s, 64.0 * s, 0.0, 24.0 * s), (96.0 * s, 64.0 * s, 0.0, 8.0 * s)])
    return p, phi0, None


def single_vortex(storage: str = "fp64", L: int = 256, T: float = 8000.0) -> Tuple[CaseParams, np.ndarray, None]:
    """Phase field under the prescribed single vortex of Eqs. 43-44: L x L periodic,
    disk R = 0.15 L at (0.5 L, 0.75 L), W = 4, M = 0.02, sigma = 0.01, U0 = 0.04."""
    p = CaseParams(nx=L, ny=L, mode="vortex", W=4.0, sigma=0.01, mobility=0.02,
                   U0=0.04, T=float(T), storage=storage)
    phi0 = drops_phi(p, [(0.5 * L, 0.75 * L, 0.0, 0.15 * L)])
    return p, phi0, None


def rayleigh_plateau(storage: str = "fp32", nx: int = 96, ny: int = 96, nz: int = 384,
                     R0: float = 16.0) -> Tuple[CaseParams, np.ndarray, None]:
    """3D liquid column, D3Q19, periodic: R(z) = R0 (1 + 0.1 cos(2 pi z / nz)), axis at the
    box centre, W = 4, density ratio 10, sigma = 0.005, nu = 0.05, M = 0.1."""
    p = CaseParams(nx=nx, ny=ny, nz=nz, lattice="D3Q19", W=4.0, sigma=0.005, mobility=0.1,
                   nu=0.05, rho_heavy=1.0, rho_light=0.1, storage=storage)
    phi0 = cylinder_phi(p, nx / 2.0, ny / 2.0, R0, 0.1, float(nz))
    return p, phi0, None


def shear_droplet(storage: str = "fp64", nx: int = 512, ny: int = 256, R: float = 48.0,
                  U: float = 0.02, Ca: float = 0.2, Re: float = 0.5) -> Tuple[CaseParams, np.ndarray, np.ndarray]:
    """Drop in Couette flow between walls moving at -U (bottom) and +U (top), periodic in x,
    density ratio 1.  Shear rate 2U/ny; viscosity from Re = rate R^2 / nu, sigma from
    Ca = nu rate R / sigma (rho = 1).  Initial velocity is the linear Couette profile."""
    rate = 2.0 * U / ny
    nu = rate * R * R / Re
    sigma = nu * rate * R / Ca
    p = CaseParams(nx=nx, ny=ny, wall_y=True, wall_u_bottom=(-U, 0.0, 0.0), wall_u_top=(U, 0.0, 0.0),
                   W=4.0, sigma=sigma, mobility=0.1, nu=nu, rho_heavy=1.0, rho_light=1.0,
                   storage=storage, label_centres=[((nx - 1) / 2.0, (ny - 1) / 2.0, 0.0)])
    phi0 = drops_phi(p, [((nx - 1) / 2.0, (ny - 1) / 2.0, 0.0, R)])
    return p, phi0, couette_u(p)


# ---------------------------------------------------------------------------
# the paper's four test problems at their own sizes (Sect. 4), with lam = 0 giving the
# classical model they are compared with.  Common parameters of Sect. 4.1: W = 3,
# density and viscosity ratio 1, M = 0.1, sigma = 0.01; the rest (radii, wall speed,
# viscosity) is not stated and takes the readings noted per builder.
# ---------------------------------------------------------------------------

def paper_two_drops(lam: float = 0.5, storage: str = "fp64", r1: float = 24.0,
                    r2: float = 8.0) -> Tuple[CaseParams, np.ndarray, None]:
    """Sect. 4.1: two drops centred on the base (y = 0) of a 200 x 100 box at x = 80 and
    x = 160 (periodic, so each drop also wraps across y = 0); radii not given (24 and 8
    here, the large and small drops of the two-drop case); nu = 0.1.  Labels: the two
    centres."""
    p = CaseParams(nx=200, ny=100, W=3.0, sigma=0.01, mobility=0.1, nu=0.1, rho_heavy=1.0, rho_light=1.0,
                   lam=lam, storage=storage, label_centres=[(80.0, 0.0, 0.0), (160.0, 0.0, 0.0)])
    return p, drops_phi(p, [(80.0, 0.0, 0.0, r1), (160.0, 0.0, 0.0, r2)]), None


def paper_vortex(lam: float = 0.5, storage: str = "fp64", n: int = 6) -> Tuple[CaseParams, np.ndarray, None]:
    """Sect. 4.2: disk R = 45 at (0.5 L, 0.75 L) in a 200 x 200 box under Eqs. 43-44 with
    U0 = 0.04 and T = n L / U0 (n = 6: 30000 steps)."""
    L = 200
    p = CaseParams(nx=L, ny=L, mode="vortex", W=3.0, sigma=0.01, mobility=0.1, U0=0.04, T=n * L / 0.04,
                   lam=lam, storage=storage)
    return p, drops_phi(p, [(0.5 * L, 0.75 * L, 0.0, 45.0)]), None


def paper_shear_drop(lam: float = 0.5, storage: str = "fp64", r: float = 8.0,
                     U: float = 0.02) -> Tuple[CaseParams, np.ndarray, np.ndarray]:
    """Sect. 4.4: drop of radius 8 at the centre of a 128 x 64 box between walls moving
    at -U and +U (U not given: 0.02, the wall speed of the shear cases); nu = 0.1; initial
    velocity the Couette profile."""
    p = CaseParams(nx=128, ny=64, W=3.0, sigma=0.01, mobility=0.1, nu=0.1, rho_heavy=1.0, rho_light=1.0, lam=lam,
                   wall_y=True, wall_u_bottom=(-U, 0.0, 0.0), wall_u_top=(U, 0.0, 0.0), storage=storage,
                   label_centres=[(63.5, 31.5, 0.0)])
    return p, drops_phi(p, [(63.5, 31.5, 0.0, r)]), couette_u(p)


def paper_rayleigh_plateau_2d(lam: float = 0.5, storage: str = "fp64") -> Tuple[CaseParams, np.ndarray, None]:
    """Sect. 4.3: the layer of Eq. 45, phi = 1/2 [1 + tanh(2 (a - y + 0.05 cos x) / W)], on
    (0, 2 pi) x (0, pi) with 256 x 128 nodes and a = 0.15, fluid at rest.  Readings: a and
    the 0.05 amplitude are in the box's units, so 128 / pi nodes per unit (a = 6.1 nodes,
    amplitude 2.0 nodes); W = 3 lattice units (Sect. 4.1's common value); half-way walls at
    y = 0 and y = pi (node rows 0 and 127 lie half a node inside them), x periodic; node
    (i, j) sits at (x, y) = ((i + 1/2) h, (j + 1/2) h) with h = pi / 128."""
    nx, ny = 256, 128
    h = np.pi / ny
    p = CaseParams(nx=nx, ny=ny, W=3.0, sigma=0.01, mobility=0.1, nu=0.1, rho_heavy=1.0, rho_light=1.0, lam=lam,
                   wall_y=True, storage=storage)
    x = (np.arange(nx, dtype=np.float64) + 0.5) * h
    y = (np.arange(ny, dtype=np.float64) + 0.5) * h
    s = (0.15 - y[:, None] + 0.05 * np.cos(x)[None, :]) / h          # signed distance in nodes
    phi0 = (0.5 * (1.0 + np.tanh(2.0 * s / p.W)))[None]
    return p, phi0, None


BATCH_SEED = 10899


def batch_cases(n_cases: int = 512, seed: int = BATCH_SEED, storage: str = "fp16s",
                side_lo: int = 64, side_hi: int = 512):
    """Independent D2Q9 drop cases of uneven sizes (the batched workload).

    Per case, from numpy's PCG64(seed): nx and ny log-uniform in [side_lo, side_hi]
    (independent); radius uniform in [0.1, 0.3] x min(nx, ny); density ratio
    log-uniform in [1, 100]; static (periodic) or shear (walls +-0.02) with
    probability 1/2 each; W = 4, M = 0.1, sigma = 0.01, nu = 0.1.  The drop sits at
    the box centre.  Returns a list of (params, phi0, u0) and the JSON-able case list.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    table = []
    lo, hi = math.log(side_lo), math.log(side_hi)
    for k in range(n_cases):
        nx = int(round(math.exp(rng.uniform(lo, hi))))
        ny = int(round(math.exp(rng.uniform(lo, hi))))
        R = float(rng.uniform(0.1, 0.3)) * min(nx, ny)
        ratio = math.exp(rng.uniform(0.0, math.log(100.0)))
        shear = bool(rng.uniform() < 0.5)
        cx, cy = (nx - 1) / 2.0, (ny - 1) / 2.0
        p = CaseParams(nx=nx, ny=ny, W=4.0, sigma=0.01, mobility=0.1, nu=0.1,
                       rho_heavy=1.0, rho_light=1.0 / ratio, storage=storage,
                       wall_y=shear,
                       wall_u_bottom=(-0.02, 0.0, 0.0) if shear else (0.0, 0.0, 0.0),
                       wall_u_top=(0.02, 0.0, 0.0) if shear else (0.0, 0.0, 0.0),
                       label_centres=[(cx, cy, 0.0)])
        phi0 = drops_phi(p, [(cx, cy, 0.0, R)])
        u0 = couette_u(p) if shear else None
        out.append((p, phi0, u0))
        table.append({"nx": nx, "ny": ny, "R": R, "ratio": ratio, "shear": shear})
    return out, table


def batch_case_list_json(n_cases: int = 512, seed: int = BATCH_SEED) -> str:
    _, table = batch_cases(n_cases, seed)
    return json.dumps(table)


# ---------------------------------------------------------------------------
# FP64 free-run parity cases: drops and columns placed off the lattice nodes
# ---------------------------------------------------------------------------

def offnode_parity_cases():
    """Cases for the 1000-step FP64 free-run parity check, name -> (params, phi0, u0, steps).

    Every drop centre (and the column axis) lies off the lattice nodes and off the
    half-node mirror lines.  A centre on a node makes grad psi vanish there by symmetry,
    so the unit normal of Eq. 32 is set by rounding and any two correct implementations
    drift apart; off-node, the oracle run against itself with phi0 perturbed by 1e-15
    stays within about 6e-15 on phi after 1000 steps.  Covered: the two-drop case at
    its full 128 x 128 size, moving walls, the prescribed vortex, the classical model
    (lambda = 0), relaxation rates off their defaults, and a D3Q19 column (24 x 24 x 96,
    200 steps)."""
    out = {}
    p = CaseParams(nx=128, ny=128, W=4.0, sigma=0.01, mobility=0.1, nu=0.1, rho_heavy=1.0, rho_light=0.1,
                   label_centres=[(40.37, 64.41, 0.0), (96.23, 63.71, 0.0)])
    out["two_droplets_128"] = (p, drops_phi(p, [(40.37, 64.41, 0.0, 24.0), (96.23, 63.71, 0.0, 8.0)]), None, 1000)
    p, _, u0 = shear_droplet(nx=66, ny=20, R=6.0, U=0.02, Ca=0.2, Re=0.5)
    p = p.replace(rho_light=0.5, label_centres=[(32.31, 9.17, 0.0)])
    out["walls_moving"] = (p, drops_phi(p, [(32.31, 9.17, 0.0, 6.0)]), u0, 1000)
    p = CaseParams(nx=50, ny=50, mode="vortex", W=4.0, sigma=0.01, mobility=0.02, U0=0.04, T=40.0)
    out["vortex"] = (p, drops_phi(p, [(25.3, 37.2, 0.0, 7.5)]), None, 1000)
    p = CaseParams(nx=64, ny=64, lam=0.0, rho_light=0.2, sigma=0.02)
    out["classical_lambda0"] = (p, drops_phi(p, [(31.77, 31.21, 0.0, 10.0)]), None, 1000)
    p = CaseParams(nx=64, ny=20, rho_light=0.3, s_g=(0, 1.3, 1.1, 0, 0, 0, 0, 1.2, 1.1),
                   s_f=(1.0, 1.2, 1.3, 1.1, 1.2, 1.1, 1.2, 0, 0))
    out["mrt_rates"] = (p, drops_phi(p, [(31.63, 9.28, 0.0, 6.0)]), None, 1000)
    p = CaseParams(nx=24, ny=24, nz=96, lattice="D3Q19", W=4.0, sigma=0.005, mobility=0.1, nu=0.05,
                   rho_heavy=1.0, rho_light=0.1)
    out["d3q19_column"] = (p, cylinder_phi(p, 11.63, 12.27, 6.0, 0.1, 96.0), None, 200)
    return out
