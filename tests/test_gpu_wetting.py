"""GPU checks of wetting walls (a contact angle on each wall, through the stencil ghosts
behind it; the paper states no boundary conditions, so the condition is a reading):

- one step from the oracle's exact state matches the oracle node by node, fused and
  plain paths, with two different angles and moving walls;
- 1000 free FP64 steps of an off-node sessile drop match the oracle to 1e-12 on phi,
  rho and u, fused and plain;
- the batched step (strips and bands) gives the oracle's state for cases of different
  angles;
- FP32 and FP16S storage stay close to the FP64 oracle and keep the total of phi.
The adjoint through wetting walls is checked in test_gpu_adjoint.py.
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


def _sessile(nx=70, ny=30, R=10.0, cb=0.5, ct=-0.3, storage="fp64", moving=True):
    """A drop on the bottom wall (centre off the nodes), contact angles acos(cb) at the
    bottom and acos(ct) at the top, walls moving -+0.01 (or at rest)."""
    U = 0.01 if moving else 0.0
    xc = nx / 2 + 0.37
    p = W.CaseParams(nx=nx, ny=ny, wall_y=True, wall_u_bottom=(-U, 0.0, 0.0), wall_u_top=(U, 0.0, 0.0),
                     wall_cos_bottom=cb, wall_cos_top=ct, rho_light=0.5, sigma=0.01, nu=0.1, storage=storage,
                     label_centres=[(xc, 2.0, 0.0)])
    x = np.arange(nx)[None, None, :]
    y = np.arange(ny)[None, :, None]
    d = R - np.sqrt((x - xc) ** 2 + (y + 0.5 - 1.13) ** 2)
    phi0 = 0.5 * (1.0 + np.tanh(2.0 * d / p.W)) * np.ones((1, ny, nx))
    return p, phi0, None


@pytest.mark.parametrize("plain", [False, True], ids=["fused", "plain"])
def test_wetting_one_step_parity(plain):
    _v()
    from test_gpu_parity import one_step_parity
    p, phi0, u0 = _sessile()
    say(f"case: wetting walls cos {p.wall_cos_bottom} / {p.wall_cos_top}, {'plain' if plain else 'fused'}")
    m = Model(p).init(phi0, u0)
    for t in (0, 5, 40):
        while m.t < t:
            m.step(1)
        ref = Model(p)
        ref.g, ref.f, ref.Jprev, ref.t = m.g.copy(), m.f.copy(), m.Jprev.copy(), m.t
        ratio, ferr, raw = one_step_parity(p, ref, plain=plain)
        say(f"  t={t}: populations {raw:.2e} (error / bound {ratio:.2f}), fields {ferr:.2e}")
        assert ratio <= 1.0 and ferr <= 1e-13, t


@pytest.mark.parametrize("plain", [False, True], ids=["fused", "plain"])
def test_wetting_fp64_free_run_1e12(plain):
    v = _v()
    p, phi0, u0 = _sessile()
    steps = 1000
    m = Model(p).init(phi0, u0)
    m.step(steps)
    F0 = m.fields()
    c = v.Case(p).init(phi0, u0)
    (c.step_plain if plain else c.step)(steps)
    F = c.observe(v.FIELD_PHI | v.FIELD_RHO | v.FIELD_U)
    errs = {k: float(np.max(np.abs(F[k] - F0[k]))) for k in ("phi", "rho", "u")}
    say(f"case: wetting walls, 1000 FP64 steps, {'plain' if plain else 'fused'}: max-abs {errs}")
    for k, e in errs.items():
        assert e <= 1e-12, (k, e)


@pytest.mark.parametrize("tile", [(64, 16, 0), (128, 1024, 101)], ids=["strips", "bands"])
def test_wetting_batch_matches_the_oracle(tile):
    """Three cases of different angles (one neutral) in one batch, 200 FP64 steps."""
    v = _v()
    cases = [_sessile(nx=70, ny=30, cb=0.5, ct=-0.3), _sessile(nx=52, ny=26, R=8.0, cb=-0.6, ct=0.2, moving=False),
             _sessile(nx=40, ny=20, R=6.0, cb=0.0, ct=0.0)]
    b = v.Batch([p for p, _, _ in cases]).init([(phi0, u0) for _, phi0, u0 in cases])
    b.set_tile(tile[0], tile[1])
    b.set_schedule(tile[2])
    steps = 200
    b.step(steps)
    for k, (p, phi0, u0) in enumerate(cases):
        m = Model(p).init(phi0, u0)
        m.step(steps)
        F0 = m.fields()
        F = b.cases[k].observe(v.FIELD_PHI | v.FIELD_U)
        e = max(float(np.max(np.abs(F["phi"] - F0["phi"]))), float(np.max(np.abs(F["u"] - F0["u"]))))
        say(f"case: batch {tile}, case {k} cos {p.wall_cos_bottom}/{p.wall_cos_top}: max-abs {e:.2e}")
        assert e <= 1e-12, (k, e)


@pytest.mark.parametrize("storage", ["fp32", "fp16s"])
def test_wetting_reduced_precision(storage):
    v = _v()
    p, phi0, u0 = _sessile(storage=storage)
    steps = 200
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
    say(f"case: wetting walls {storage}, {steps} steps: |dphi| {dphi:.2e}, |du| {du:.2e}, drift {drift:.2e}")
    tol = {"fp32": (2e-5, 2e-6, 1e-6), "fp16s": (3e-3, 3e-4, 1e-5)}[storage]
    assert dphi <= tol[0] and du <= tol[1] and drift <= tol[2]
