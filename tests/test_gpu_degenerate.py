"""GPU checks of the degenerate states the method has: a single uniform phase (phi = 0,
phi = 1, or a uniform mixture) at rest is a fixed point of the step.  Its gradients
vanish, so does the unit normal (n = 0 / sqrt(0 + eps_n^2)) and with it the level-set
source, and the populations sit at their equilibrium.  Every storage and both lattices,
with periodic faces and (D2Q9) walls at rest, must keep phi at its value and u at zero,
with no NaN from the regularised normal or the clipped signed distance.
"""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _v():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_10899_amd import vclb
    return vclb


TOL = {"fp64": (1e-13, 1e-14), "fp32": (1e-6, 1e-8), "fp16s": (1e-5, 1e-9)}


@pytest.mark.parametrize("value", [0.0, 1.0, 0.3])
@pytest.mark.parametrize("storage", ["fp64", "fp32", "fp16s"])
@pytest.mark.parametrize("geom", ["d2q9", "d2q9_walls", "d3q19"])
def test_uniform_phase_is_a_fixed_point(geom, storage, value):
    v = _v()
    if geom == "d3q19":
        p = W.CaseParams(nx=20, ny=12, nz=8, lattice="D3Q19", sigma=0.005, nu=0.05, rho_light=0.1, storage=storage)
    else:
        p = W.CaseParams(nx=70, ny=33, rho_light=0.1, wall_y=geom == "d2q9_walls", storage=storage)
    phi0 = np.full((p.nz, p.ny, p.nx), value)
    c = v.Case(p).init(phi0)
    steps = 100
    c.step(steps)
    F = c.observe(v.FIELD_PHI | v.FIELD_U)
    dphi = float(np.max(np.abs(F["phi"] - value)))
    umax = float(np.max(np.abs(F["u"])))
    print(f"case: uniform phi = {value}, {geom} {storage}, {steps} steps: |phi - value| {dphi:.2e}, |u| {umax:.2e}",
          flush=True)
    sys.stdout.flush()
    assert np.all(np.isfinite(F["phi"])) and np.all(np.isfinite(F["u"]))
    tp, tu = TOL[storage]
    assert dphi <= tp and umax <= tu, (dphi, umax)
