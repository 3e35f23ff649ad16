"""GPU checks of D3Q19 cases bounded by walls in y (half-way bounce-back, tangential wall
velocities, wetting ghosts), through the fused 3D step and the plain path:

- one step from the oracle's exact state matches the oracle node by node, in sections
  that cover the rows exactly, overhang the last row, or reach past both walls;
- 200 free FP64 steps match the oracle to 1e-12 on phi, rho and u;
- FP32 and FP16S storage stay close to the FP64 oracle and keep the total of phi.
"""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import Model

pytestmark = pytest.mark.gpu


def _v():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_10899_amd import vclb
    return vclb


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _channel(storage="fp64", cb=0.4, ct=-0.2):
    """A drop resting near the bottom wall of a 20 x 13 x 16 channel, centre off the
    nodes; walls moving (-0.01, 0, 0.005) and (0.01, 0, -0.005)."""
    p = W.CaseParams(nx=20, ny=13, nz=16, lattice="D3Q19", wall_y=True, wall_u_bottom=(-0.01, 0.0, 0.005),
                     wall_u_top=(0.01, 0.0, -0.005), wall_cos_bottom=cb, wall_cos_top=ct, sigma=0.005, nu=0.05,
                     rho_light=0.3, storage=storage, label_centres=[(9.7, 3.2, 7.6)])
    return p, W.drops_phi(p, [(9.7, 3.2, 7.6, 4.5)]), None


@pytest.mark.parametrize("tile", [None, (16, 6, 16), (64, 10, 4)], ids=["default", "past_both_walls", "past_x"])
@pytest.mark.parametrize("plain", [False, True], ids=["fused", "plain"])
def test_walls3d_one_step_parity(plain, tile):
    _v()
    from test_gpu_parity import one_step_parity
    p, phi0, u0 = _channel()
    say(f"case: D3Q19 walls, {'plain' if plain else 'fused'}, tile {tile}")
    m = Model(p).init(phi0, u0)
    for t in (0, 5, 30):
        while m.t < t:
            m.step(1)
        ref = Model(p)
        ref.g, ref.f, ref.Jprev, ref.t = m.g.copy(), m.f.copy(), m.Jprev.copy(), m.t
        ratio, ferr, raw = one_step_parity(p, ref, plain=plain, tile=tile)
        say(f"  t={t}: populations {raw:.2e} (error / bound {ratio:.2f}), fields {ferr:.2e}")
        assert ratio <= 1.0 and ferr <= 1e-13, t


def test_walls3d_fp64_free_run_1e12():
    v = _v()
    p, phi0, u0 = _channel()
    steps = 200
    m = Model(p).init(phi0, u0)
    m.step(steps)
    F0 = m.fields()
    c = v.Case(p).init(phi0, u0)
    c.step(steps)
    F = c.observe(v.FIELD_PHI | v.FIELD_RHO | v.FIELD_U)
    errs = {k: float(np.max(np.abs(F[k] - F0[k]))) for k in ("phi", "rho", "u")}
    say(f"case: D3Q19 walls, {steps} FP64 steps: max-abs {errs}")
    for k, e in errs.items():
        assert e <= 1e-12, (k, e)


@pytest.mark.parametrize("storage", ["fp32", "fp16s"])
def test_walls3d_reduced_precision(storage):
    v = _v()
    p, phi0, u0 = _channel(storage=storage)
    steps = 100
    m = Model(p.replace(storage="fp64")).init(phi0, u0)
    m.step(steps)
    F0 = m.fields()
    c = v.Case(p).init(phi0, u0)
    v0 = c.reduce()["sum_phi"].sum()
    c.step(steps)
    F = c.observe(v.FIELD_PHI | v.FIELD_U)
    dphi = float(np.max(np.abs(F["phi"] - F0["phi"])))
    du = float(np.max(np.abs(F["u"] - F0["u"])))
    drift = abs(c.reduce()["sum_phi"].sum() - v0) / v0
    say(f"case: D3Q19 walls {storage}, {steps} steps: |dphi| {dphi:.2e}, |du| {du:.2e}, drift {drift:.2e}")
    tol = {"fp32": (2e-5, 2e-6, 1e-6), "fp16s": (3e-3, 3e-4, 1e-5)}[storage]
    assert dphi <= tol[0] and du <= tol[1] and drift <= tol[2]


@pytest.mark.parametrize("storage", ["fp32", "fp16s"])
def test_walls3d_sections_agree_bit_for_bit(storage):
    """The same 20 steps in sections of 256 lanes and in the wide 768-lane sections (one
    workgroup per CU, staged planes) give the same state bit for bit."""
    import torch
    v = _v()
    p, phi0, u0 = _channel(storage=storage)
    states = []
    for tile in [(32, 8, 8), (96, 10, 8), (16, 7, 16)]:
        c = v.Case(p, tile=tile).init(phi0, u0)
        c.step(20)
        torch.cuda.synchronize()
        states.append([x.clone() for x in c.state_device() if x is not None])
    for other in states[1:]:
        for xa, xb in zip(states[0], other):
            assert torch.equal(xa, xb)
