"""GPU parity of the discrete adjoint (FP64 D2Q9 coupled) through the C ABI.

References: the oracle's complex-step derivatives (exact derivatives of the same
discrete map, oracle/gradient.py), central differences of the GPU forward run, and
the exact values conservation fixes (d sum(phi) / d phi0 = 1 at every node, zero
derivative with respect to sigma and M).  phi0 directions are r 4 phi0 (1 - phi0) with
r standard normal from PCG64(1): changes that stay off the clipped bulk, where the map
has a kink.  Both sides differentiate the unit normal only where |grad psi| >= 0.3
(the default cut; tau = 0 is the exact derivative, checked on the small case).  The
cases include walls with wetting ghosts (a sessile drop) and unequal viscosities.
"""
import sys

import numpy as np
import pytest
import torch

import workloads as W
from oracle import gradient as OG

pytestmark = pytest.mark.gpu

TOL = 1e-6     # relative, on every derivative


def _vclb():
    from paper_2505_10899_amd import vclb
    return vclb


def _shear():
    p, phi0, u0 = W.shear_droplet(nx=64, ny=32, R=8.0)
    return "shear64x32", p, phi0, u0, 120, 16


def _drops():
    p, _, _ = W.two_droplets(scale=1)
    p = p.replace(nx=64, ny=48, label_centres=[(20.0, 24.0, 0.0), (46.0, 22.0, 0.0)])
    phi0 = W.drops_phi(p, [(20.0, 24.0, 0.0, 10.0), (46.0, 22.0, 0.0, 5.0)])
    return "drops64x48", p, phi0, None, 60, 0


def _wetting():
    """A drop on the bottom wall of a 64 x 32 channel, walls moving -+0.01 and wetting at
    contact angles acos(0.5) and acos(-0.3): the wetting ghosts enter the derivative."""
    from test_oracle_gradient import _sessile
    p, phi0, u0, n = _sessile()
    return "sessile64x32", p, phi0, u0, n, 10


def _visc():
    """The 66 x 24 walled shear drop with unequal viscosities (ratio 3.75): the per-node
    stress rate of f (Eq. 27) enters the derivative."""
    from test_oracle_gradient import _visc as visc_case
    p, phi0, u0, n = visc_case()
    return "visc66x24", p, phi0, u0, n, 10


CASES = [_shear, _drops, _wetting, _visc]


def _direction(phi0, k=0):
    rng = np.random.Generator(np.random.PCG64(1))
    for _ in range(k + 1):
        r = rng.standard_normal(phi0.shape)
    return r * 4.0 * phi0 * (1.0 - phi0)


def _record(case_fn, every=None):
    v = _vclb()
    name, p, phi0, u0, n, ev = case_fn()
    print(f"[adjoint] case {name} steps {n} every {ev if every is None else every}", flush=True)
    c = v.Case(p)
    c.adjoint_record(phi0, u0, nsteps=n, every=ev if every is None else every)
    return c, p, phi0, u0, n


def _grad(c, weights):
    v = _vclb()
    raw = c.reduce_raw()
    seed = v.obs_seed(raw, c.nlabels, weights)
    dphi, ds, dm = c.adjoint_run(seed)
    torch.cuda.synchronize()
    return dphi.cpu().numpy().reshape(-1), ds, dm


def _close(got, ref, scale):
    return abs(got - ref) <= TOL * max(abs(ref), scale)


@pytest.mark.parametrize("case_fn", CASES)
def test_total_phi_adjoint_is_exact(case_fn):
    c, p, phi0, u0, n = _record(case_fn)
    w = np.zeros((c.nlabels, 5))
    w[:, 0] = 1.0
    dphi, ds, dm = _grad(c, w)
    assert np.abs(dphi - 1.0).max() < 1e-12
    V = c.derived()[:, 0].sum()
    assert abs(ds) < 1e-12 * V and abs(dm) < 1e-12 * V


@pytest.mark.parametrize("case_fn", CASES)
def test_adjoint_matches_complex_step(case_fn):
    c, p, phi0, u0, n = _record(case_fn)
    d = _direction(phi0).reshape(-1)
    cs = {wrt: OG.complex_step(p, phi0, u0, n, wrt, direction=d.reshape(phi0.shape))
          for wrt in ("sigma", "mobility", "phi0")}
    fwd = c.derived()
    ref_fwd = OG.derived_after(p, phi0, u0, n)
    assert np.allclose(fwd, ref_fwd, rtol=1e-9, atol=1e-9)
    for label in range(c.nlabels):
        for k, name in ((0, "volume"), (1, "centroid_x"), (2, "centroid_y"), (4, "D")):
            w = np.zeros((c.nlabels, 5))
            w[label, k] = 1.0
            dphi, ds, dm = _grad(c, w)
            got = {"sigma": ds, "mobility": dm, "phi0": float(dphi @ d)}
            # scale for derivatives that vanish (volume vs sigma, M; symmetric centroids)
            scale = 1e-6 * abs(fwd[label, 0]) if k == 0 else 1e-3
            for wrt, val in got.items():
                ref = cs[wrt][label, k]
                print(f"[adjoint] label {label} {name} d/d{wrt}: gpu {val:.12e} cs {ref:.12e}", flush=True)
                assert _close(val, ref, scale), (label, name, wrt, val, ref)


def test_checkpoint_interval_does_not_change_the_gradient():
    w = np.array([[0.0, 0.3, 0.0, 0.0, 1.0]])
    res = []
    for every in (1, 7, 120):
        c, *_ = _record(_shear, every=every)
        res.append(_grad(c, w))
    for r in res[1:]:
        assert np.array_equal(r[0], res[0][0]) and r[1] == res[0][1] and r[2] == res[0][2]


def test_adjoint_matches_gpu_central_differences():
    v = _vclb()
    name, p, phi0, u0, n, ev = _shear()
    c, *_ = _record(_shear)
    w = np.array([[0.0, 0.0, 0.0, 0.0, 1.0]])
    dphi, ds, dm = _grad(c, w)
    d = _direction(phi0, k=1)

    def D_at(q, ph):
        k = v.Case(q)
        k.init(ph, u0)
        k.step(n)
        return k.derived()[0, 4]

    es = 1e-5 * p.sigma
    fd_s = (D_at(p.replace(sigma=p.sigma + es), phi0) - D_at(p.replace(sigma=p.sigma - es), phi0)) / (2 * es)
    em = 1e-5 * p.mobility
    fd_m = (D_at(p.replace(mobility=p.mobility + em), phi0) - D_at(p.replace(mobility=p.mobility - em), phi0)) / (2 * em)
    e = 1e-4
    fd_p = (D_at(p, phi0 + e * d) - D_at(p, phi0 - e * d)) / (2 * e)
    print(f"[adjoint] FD sigma {fd_s:.10e} adj {ds:.10e}; M {fd_m:.10e} adj {dm:.10e}; "
          f"phi0 {fd_p:.10e} adj {float(dphi @ d.reshape(-1)):.10e}", flush=True)
    assert _close(ds, fd_s, 0.0) and _close(dm, fd_m, 0.0)
    assert _close(float(dphi @ d.reshape(-1)), fd_p, 0.0)


def test_autograd_function():
    v = _vclb()
    name, p, phi0, u0, n, ev = _shear()
    phi = torch.tensor(phi0, dtype=torch.float64, device="cuda", requires_grad=True)
    sig = torch.tensor(p.sigma, dtype=torch.float64, requires_grad=True)
    mob = torch.tensor(p.mobility, dtype=torch.float64, requires_grad=True)
    out = v.rollout(p, phi, sig, mob, nsteps=n, every=ev, u0=u0)
    assert out.shape == (1, 5)
    loss = out[0, 4] + 0.3 * out[0, 1] - 0.01 * out[0, 0]
    gphi, gs, gm = torch.autograd.grad(loss, (phi, sig, mob))
    c, *_ = _record(_shear)
    dphi, ds, dm = _grad(c, np.array([[-0.01, 0.3, 0.0, 0.0, 1.0]]))
    assert np.array_equal(gphi.detach().cpu().numpy().reshape(-1), dphi)
    assert float(gs) == ds and float(gm) == dm
    assert np.allclose(out.detach().numpy(), OG.derived_after(p, phi0, u0, n), rtol=1e-9, atol=1e-9)


def test_exact_derivative_without_the_normal_cut():
    c, p, phi0, u0, n = _record(_shear)
    d = _direction(phi0).reshape(-1)
    w = np.array([[0.0, 0.0, 0.0, 0.0, 1.0]])
    seed = _vclb().obs_seed(c.reduce_raw(), 1, w)
    dphi, ds, dm = c.adjoint_run(seed, normal_tau=0.0)
    dphi = dphi.cpu().numpy().reshape(-1)
    for wrt, val in (("sigma", ds), ("mobility", dm), ("phi0", float(dphi @ d))):
        ref = OG.complex_step(p, phi0, u0, n, wrt, direction=d.reshape(phi0.shape), tau=0.0)[0, 4]
        print(f"[adjoint] exact d D/d{wrt}: gpu {val:.12e} cs {ref:.12e}", flush=True)
        assert _close(val, ref, 1e-3)


def test_medium_case_matches_complex_step():
    """128x64 shear, 200 steps: the size at which the exact derivative is already dominated
    by bulk terms (so the normal cut matters)."""
    v = _vclb()
    p, phi0, u0 = W.shear_droplet(nx=128, ny=64, R=16.0)
    n = 200
    print("[adjoint] case shear128x64 steps 200", flush=True)
    c = v.Case(p)
    c.adjoint_record(phi0, u0, nsteps=n, every=0)
    d = _direction(phi0).reshape(-1)
    dphi, ds, dm = _grad(c, np.array([[0.0, 0.0, 0.0, 0.0, 1.0]]))
    for wrt, val in (("sigma", ds), ("mobility", dm), ("phi0", float(dphi @ d))):
        ref = OG.complex_step(p, phi0, u0, n, wrt, direction=d.reshape(phi0.shape))[0, 4]
        print(f"[adjoint] shear128x64 d D/d{wrt}: gpu {val:.12e} cs {ref:.12e}", flush=True)
        assert _close(val, ref, 1e-3)


def test_full_shear_case_against_central_differences():
    """The 512x256 shear case over 4000 steps with a checkpoint every 200: dD/dsigma, dD/dM
    and dD/dphi0 along 10 directions (PCG64(1)) against central differences of the GPU
    forward run.  At this length the differences scatter with their step e (rounding
    and truncation; e.g. 1e-4 relative for dD/dM over e = 3e-4..1e-2), so each adjoint
    value is compared with the median over several steps, within twice their spread plus
    1e-6 of the largest derivative of its kind."""
    v = _vclb()
    p, phi0, u0 = W.shear_droplet("fp64")
    n, every = 4000, 200
    print("[adjoint] case shear512x256 steps 4000 every 200", flush=True)
    c = v.Case(p)
    c.set_reduce_every(0)
    c.adjoint_record(phi0, u0, nsteps=n, every=every)
    dphi, ds, dm = _grad(c, np.array([[0.0, 0.0, 0.0, 0.0, 1.0]]))
    assert np.isfinite(dphi).all()

    def D_at(q, ph):
        k = v.Case(q)
        k.set_reduce_every(0)
        k.init(ph, u0)
        k.step(n)
        return k.derived()[0, 4]

    def central(at, steps):
        vals = np.array([(at(e) - at(-e)) / (2 * e) for e in steps])
        return float(np.median(vals)), float(vals.max() - vals.min())

    rel = (1e-2, 3e-3, 1e-3, 3e-4)
    fd_s, sp_s = central(lambda e: D_at(p.replace(sigma=p.sigma * (1 + e)), phi0), rel)
    fd_s, sp_s = fd_s / p.sigma, sp_s / p.sigma
    fd_m, sp_m = central(lambda e: D_at(p.replace(mobility=p.mobility * (1 + e)), phi0), rel)
    fd_m, sp_m = fd_m / p.mobility, sp_m / p.mobility
    print(f"[adjoint] C4 dD/dsigma adj {ds:.10e} fd {fd_s:.10e} (spread {sp_s:.1e}); "
          f"dD/dM adj {dm:.10e} fd {fd_m:.10e} (spread {sp_m:.1e})", flush=True)
    assert abs(ds - fd_s) <= 2 * sp_s + 1e-6 * abs(fd_s)
    assert abs(dm - fd_m) <= 2 * sp_m + 1e-6 * abs(fd_m)
    rng = np.random.Generator(np.random.PCG64(1))
    rows = []
    for k in range(10):
        d = rng.standard_normal(phi0.shape) * 4.0 * phi0 * (1.0 - phi0)
        fd, sp = central(lambda e: D_at(p, phi0 + e * d), (1e-2, 1e-3, 1e-4))
        adj = float(dphi @ d.reshape(-1))
        rows.append((adj, fd, sp))
        print(f"[adjoint] C4 direction {k}: adj {adj:.10e} fd {fd:.10e} spread {sp:.1e}", flush=True)
    scale = max(abs(r[1]) for r in rows)
    for adj, fd, sp in rows:
        assert abs(adj - fd) <= 2 * sp + 1e-6 * scale


def test_full_shear_case_against_oracle_complex_step():
    """The 512x256 shear case over 4000 steps with a checkpoint every 200: dD/dsigma, dD/dM
    and dD/dphi0 along the 10 PCG64(1) directions against the oracle's complex step at the
    same size and length (stored by tests/golden/make_adjoint_golden.py, the same normal
    cut), to 1e-6 relative; directions relative to the largest of the ten.  The forward D
    agrees to 1e-9."""
    import os
    v = _vclb()
    g = np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "shear512x256_adjoint_t4000.npz"))
    p, phi0, u0 = W.shear_droplet("fp64")
    n, every = int(g["nsteps"]), 200
    assert abs(float(g["normal_tau"]) - v.NORMAL_TAU) < 1e-15
    print(f"[adjoint] case shear512x256 steps {n} every {every} against the stored complex step", flush=True)
    c = v.Case(p)
    c.set_reduce_every(0)
    c.adjoint_record(phi0, u0, nsteps=n, every=every)
    D = float(c.derived()[0, 4])
    print(f"[adjoint] C4 D gpu {D:.15e} oracle {float(g['D']):.15e}", flush=True)
    assert abs(D - float(g["D"])) <= 1e-9 * abs(float(g["D"]))
    dphi, ds, dm = _grad(c, np.array([[0.0, 0.0, 0.0, 0.0, 1.0]]))
    for name, got, ref in (("sigma", ds, float(g["dD_dsigma"])), ("M", dm, float(g["dD_dM"]))):
        print(f"[adjoint] C4 dD/d{name}: gpu {got:.12e} cs {ref:.12e} rel {abs(got - ref) / abs(ref):.1e}", flush=True)
        assert _close(got, ref, 0.0), (name, got, ref)
    rng = np.random.Generator(np.random.PCG64(1))
    refs = np.asarray(g["dD_dphi0_dir"])
    scale = float(np.max(np.abs(refs)))
    for k in range(len(refs)):
        d = rng.standard_normal(phi0.shape) * 4.0 * phi0 * (1.0 - phi0)
        got = float(dphi @ d.reshape(-1))
        print(f"[adjoint] C4 direction {k}: gpu {got:.12e} cs {refs[k]:.12e} "
              f"rel to largest {abs(got - refs[k]) / scale:.1e}", flush=True)
        assert _close(got, float(refs[k]), scale), (k, got, refs[k])
