"""Lattice tables for the oracle (test infrastructure only).

D2Q9 follows the paper's Sect. 3 literally: velocities from the closed form of
Eq. 19, weights 4/9, 1/9, 1/36, c_s^2 = 1/3, and the transformation matrix of
Eq. 24 typed in row by row.

D3Q19 is not in the paper (it treats two-dimensional flows only).  For the 3D
workload the oracle uses the standard D3Q19 velocity set with weights 1/3, 1/18,
1/36 and the orthogonal moment basis of d'Humieres et al. (2002), built here by
evaluating that basis' published polynomials at the velocities.
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass(frozen=True)
class Lattice:
    name: str
    D: int
    c: np.ndarray          # (Q, 3) integer velocities, z component 0 in 2D
    w: np.ndarray          # (Q,) weights
    M: np.ndarray          # (Q, Q) transformation matrix, rows are moments
    opp: np.ndarray        # (Q,) index of -c_i
    cs2: float = 1.0 / 3.0

    @property
    def Q(self) -> int:
        return int(self.c.shape[0])


def _opposites(c: np.ndarray) -> np.ndarray:
    opp = np.empty(len(c), dtype=np.int64)
    for i, ci in enumerate(c):
        matches = [j for j, cj in enumerate(c) if np.all(cj == -ci)]
        assert len(matches) == 1
        opp[i] = matches[0]
    return opp


def _d2q9() -> Lattice:
    # Eq. 19: i = 0 rest; i = 1..4 axis directions at angle (i-1) pi/2; i = 5..8 diagonals
    # of length sqrt(2) at angle (2i-9) pi/4.
    c = np.zeros((9, 3))
    for i in range(1, 5):
        a = (i - 1) * np.pi / 2.0
        c[i, :2] = (np.cos(a), np.sin(a))
    for i in range(5, 9):
        a = (2 * i - 9) * np.pi / 4.0
        c[i, :2] = (np.sqrt(2.0) * np.cos(a), np.sqrt(2.0) * np.sin(a))
    c = np.rint(c).astype(np.int64)
    w = np.array([4.0 / 9.0] + [1.0 / 9.0] * 4 + [1.0 / 36.0] * 4)
    # Eq. 24, row order rho, e, epsilon, j_x, q_x, j_y, q_y, p_xx, p_xy.
    M = np.array([
        [1, 1, 1, 1, 1, 1, 1, 1, 1],
        [-4, -1, -1, -1, -1, 2, 2, 2, 2],
        [4, -2, -2, -2, -2, 1, 1, 1, 1],
        [0, 1, 0, -1, 0, 1, -1, -1, 1],
        [0, -2, 0, 2, 0, 1, -1, -1, 1],
        [0, 0, 1, 0, -1, 1, 1, -1, -1],
        [0, 0, -2, 0, 2, 1, 1, -1, -1],
        [0, 1, -1, 1, -1, 0, 0, 0, 0],
        [0, 0, 0, 0, 0, 1, -1, 1, -1],
    ], dtype=np.float64)
    return Lattice("D2Q9", 2, c, w, M, _opposites(c))


def _d3q19() -> Lattice:
    c = [(0, 0, 0),
         (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
         (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0),
         (1, 0, 1), (-1, 0, -1), (1, 0, -1), (-1, 0, 1),
         (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)]
    c = np.array(c, dtype=np.int64)
    c2 = (c * c).sum(axis=1)
    w = np.where(c2 == 0, 1.0 / 3.0, np.where(c2 == 1, 1.0 / 18.0, 1.0 / 36.0))
    cx, cy, cz = (c[:, k].astype(np.float64) for k in range(3))
    c2 = c2.astype(np.float64)
    # d'Humieres et al. (2002) polynomial basis, in their order:
    # rho, e, eps, jx, qx, jy, qy, jz, qz, 3pxx, 3pixx, pww, piww, pxy, pyz, pxz, mx, my, mz
    rows = [
        np.ones(19),
        19.0 * c2 - 30.0,
        (21.0 * c2 * c2 - 53.0 * c2 + 24.0) / 2.0,
        cx, (5.0 * c2 - 9.0) * cx,
        cy, (5.0 * c2 - 9.0) * cy,
        cz, (5.0 * c2 - 9.0) * cz,
        3.0 * cx * cx - c2, (3.0 * c2 - 5.0) * (3.0 * cx * cx - c2),
        cy * cy - cz * cz, (3.0 * c2 - 5.0) * (cy * cy - cz * cz),
        cx * cy, cy * cz, cx * cz,
        (cy * cy - cz * cz) * cx, (cz * cz - cx * cx) * cy, (cx * cx - cy * cy) * cz,
    ]
    M = np.array(rows, dtype=np.float64)
    return Lattice("D3Q19", 3, c, w, M, _opposites(c))


D2Q9 = _d2q9()
D3Q19 = _d3q19()


def lattice_for(name: str) -> Lattice:
    return {"D2Q9": D2Q9, "D3Q19": D3Q19}[name]


def stress_rows(lat: Lattice):
    """The moment rows of f that carry the traceless stress (they relax at 1/tau_f,
    Eq. 27): p_xx and p_xy of Eq. 24 in D2Q9; 3p_xx, p_ww, p_xy, p_yz, p_xz in D3Q19."""
    return (7, 8) if lat.name == "D2Q9" else (9, 11, 13, 14, 15)


def default_rates(lat: Lattice, tau: float, which: str):
    """Diagonal relaxation rates.

    The paper fixes only tau_g = 1/s_3 = 1/s_5 (Eq. 34) and tau_f = 1/s_7 = 1/s_8
    (Eq. 27) for D2Q9.  The reading used here (listed with the other readings of the
    paper in the design notes): for g every odd (flux) moment relaxes at 1/tau_g, so
    that the source term's (I - S/2) factor of Eq. 33 equals the scalar factor of
    Eq. 30; for f the shear-stress moments relax at 1/tau_f; every other rate is 1.
    """
    s = [1.0 + 0.0 * tau] * lat.Q
    if which == "f":
        rows = stress_rows(lat)
    else:
        rows = (3, 4, 5, 6) if lat.name == "D2Q9" else (3, 4, 5, 6, 7, 8)
    for r in rows:
        s[r] = 1.0 / tau
    return s
