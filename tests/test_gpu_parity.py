"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

FP64 storage must match the oracle to 1e-12 max-abs on phi, rho and u; FP32 and
FP16-shifted storage are judged by relative volume drift against the FP64 oracle
(1e-6 and 1e-4 per drop).  The fused and plain GPU paths must agree bitwise.
"""
import ctypes
import os
import sys

import numpy as np
import pytest

import workloads as W
from oracle import Model

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def _v():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_10899_amd import vclb
    return vclb


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def max_abs(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))))


def run_gpu(p, phi0, u0, steps, tile=None, plain=False):
    v = _v()
    c = v.Case(p, tile=tile).init(phi0, u0)
    if plain:
        c.step_plain(steps)
    else:
        c.step(steps)
    return c


# --------------------------------------------------------------------------- full-size FP64
def test_two_droplets_fp64_1000_steps_matches_oracle():
    say("case: two droplets 128x128 fp64, 1000 steps (stored oracle result)")
    g = np.load(os.path.join(HERE, "golden", "two_droplets_fp64_t1000.npz"))
    p, phi0, u0 = W.two_droplets("fp64")
    c = run_gpu(p, phi0, u0, 1000)
    assert c.time() == 1000
    F = c.observe()
    e_phi, e_rho, e_u = max_abs(F["phi"], g["phi"]), max_abs(F["rho"], g["rho"]), max_abs(F["u"], g["u"])
    say("max-abs phi %.3e rho %.3e u %.3e p %.3e" % (e_phi, e_rho, e_u, max_abs(F["p"], g["p"])))
    assert e_phi <= 1e-12 and e_rho <= 1e-12 and e_u <= 1e-12
    assert max_abs(F["p"], g["p"]) <= 1e-12
    r = c.reduce()
    assert np.allclose(r["sum_phi"], g["sum_phi_t1000"], rtol=1e-12, atol=0)
    assert np.array_equal(r["count_half"], g["count_half"].astype(float))
    assert np.allclose(r["sum_phi_d"], g["sum_phi_d"], rtol=0, atol=1e-9)
    assert np.allclose(r["sum_phi_dd"], g["sum_phi_dd"], rtol=1e-11)
    h = c.history(500, 1)
    assert np.allclose(h["sum_phi"][0], g["sum_phi_t500"], rtol=1e-12, atol=0)


# --------------------------------------------------------------------------- small cases, many variants
def _small_case(variant):
    if variant == "periodic_ragged":
        p = W.CaseParams(nx=70, ny=37, W=4.0, sigma=0.01, mobility=0.1, nu=0.1, rho_light=0.1,
                         label_centres=[(20.0, 18.0, 0.0), (50.0, 18.0, 0.0)])
        phi0 = W.drops_phi(p, [(20, 18, 0, 9.0), (50, 18, 0, 5.0)])
        return p, phi0, None
    if variant == "walls_moving":
        p, phi0, u0 = W.shear_droplet(nx=66, ny=20, R=6.0, U=0.02, Ca=0.2, Re=0.5)
        p = p.replace(rho_light=0.5)
        return p, W.drops_phi(p, [(32.5, 9.5, 0, 6.0)]), u0
    if variant == "vortex":
        return W.single_vortex("fp64", L=50, T=40.0)
    if variant == "classical_lambda0":
        p = W.CaseParams(nx=64, ny=64, lam=0.0, rho_light=0.2, sigma=0.02)
        return p, W.drops_phi(p, [(31.5, 31.5, 0, 10.0)]), None
    if variant == "mrt_rates":
        p = W.CaseParams(nx=64, ny=20, rho_light=0.3, s_g=(0, 1.3, 1.1, 0, 0, 0, 0, 1.7, 0.9),
                         s_f=(1.2, 1.4, 1.6, 0.8, 1.5, 0.8, 1.5, 0, 0))
        return p, W.drops_phi(p, [(31.5, 9.5, 0, 6.0)]), None
    if variant == "narrow_tall":
        p = W.CaseParams(nx=3, ny=130, rho_light=0.1)
        return p, W.slab_phi(p, 30.0, 90.0), None
    raise ValueError(variant)


VARIANTS = ["periodic_ragged", "walls_moving", "vortex", "classical_lambda0", "mrt_rates", "narrow_tall"]


@pytest.mark.parametrize("variant", VARIANTS)
def test_small_cases_match_oracle(variant):
    steps = 60
    say(f"case: {variant}, fp64, {steps} steps")
    p, phi0, u0 = _small_case(variant)
    m = Model(p).init(phi0, u0)
    m.step(steps)
    F0 = m.fields()
    c = run_gpu(p, phi0, u0, steps)
    F = c.observe()
    for k in ("phi", "rho", "u", "p", "mu", "psi"):
        err = max_abs(F[k], F0[k])
        say(f"  {k}: {err:.3e}")
        assert err <= 1e-12, k
    r = c.reduce()
    o = m.observables()
    assert np.allclose(r["sum_phi"], o["sum_phi"], rtol=1e-12, atol=1e-12)
    assert np.array_equal(r["count_half"], o["count_half"].astype(float))


@pytest.mark.parametrize("storage", ["fp64", "fp32", "fp16s"])
def test_plain_path_equals_fused_bitwise(storage):
    say(f"case: plain vs fused, {storage}")
    for variant in ("periodic_ragged", "walls_moving", "vortex"):
        p, phi0, u0 = _small_case(variant)
        p = p.replace(storage=storage)
        a = run_gpu(p, phi0, u0, 50).observe()
        b = run_gpu(p, phi0, u0, 50, plain=True).observe()
        for k in a:
            assert np.array_equal(a[k], b[k]), (variant, k)


@pytest.mark.parametrize("storage", ["fp64", "fp16s"])
def test_tile_shape_does_not_change_the_state(storage):
    say(f"case: tile invariance, {storage}")
    p, phi0, u0 = _small_case("periodic_ragged")
    p = p.replace(nx=200, ny=45, storage=storage)
    phi0 = W.drops_phi(p, [(60, 20, 0, 12.0), (150, 25, 0, 7.0)])
    ref = None
    for tile in ((64, 1), (64, 7), (128, 16), (256, 45), (256, 64), (192, 5)):
        F = run_gpu(p, phi0, u0, 30, tile=tile).observe()
        if ref is None:
            ref = F
        else:
            for k in F:
                assert np.array_equal(F[k], ref[k]), (tile, k)


def test_history_and_determinism():
    say("case: per-step reductions vs oracle, determinism")
    p, phi0, u0 = _small_case("periodic_ragged")
    m = Model(p).init(phi0, u0)
    c1 = run_gpu(p, phi0, u0, 25)
    c2 = run_gpu(p, phi0, u0, 25)
    h1, h2 = c1.history(0, 25), c2.history(0, 25)
    for k in h1:
        assert np.array_equal(h1[k], h2[k]), k
    for t in range(25):
        o = m.observables()
        assert np.allclose(h1["sum_phi"][t], o["sum_phi"], rtol=1e-12, atol=1e-12)
        assert np.array_equal(h1["count_half"][t], o["count_half"].astype(float))
        assert np.allclose(h1["sum_phi_dd"][t][:, [0, 1, 3]], o["sum_phi_dd"][:, [0, 1, 3]], rtol=1e-11)
        m.step(1)
    assert np.array_equal(c1.observe()["phi"], c2.observe()["phi"])


def test_checkpoint_roundtrip_continues_bitwise():
    say("case: checkpoint save/load")
    v = _v()
    for storage in ("fp64", "fp16s"):
        p, phi0, u0 = _small_case("walls_moving")
        p = p.replace(storage=storage)
        a = run_gpu(p, phi0, u0, 17)
        blob = a.save()
        a.step(13)
        b = v.Case(p).load(blob)
        assert b.time() == 17
        b.step(13)
        fa, fb = a.observe(), b.observe()
        for k in fa:
            assert np.array_equal(fa[k], fb[k]), (storage, k)
        bad = bytearray(blob)
        bad[-1] ^= 0xFF
        with pytest.raises(v.VclbError):
            b.load(bytes(bad))


@pytest.mark.parametrize("storage,tol", [("fp32", 1e-6), ("fp16s", 1e-4)])
def test_reduced_precision_volume_drift(storage, tol):
    say(f"case: two droplets {storage}, 1000 steps, volume vs the FP64 oracle")
    g = np.load(os.path.join(HERE, "golden", "two_droplets_fp64_t1000.npz"))
    p, phi0, u0 = W.two_droplets(storage)
    c = run_gpu(p, phi0, u0, 1000)
    for t, key in ((500, "sum_phi_t500"),):
        h = c.history(t, 1)
        drift = np.abs(h["sum_phi"][0] - g[key]) / g[key]
        say(f"  t={t} relative volume error per drop {drift}")
        assert np.all(drift <= tol)
    r = c.reduce()
    drift = np.abs(r["sum_phi"] - g["sum_phi_t1000"]) / g["sum_phi_t1000"]
    F = c.observe()
    say(f"  t=1000 relative volume error per drop {drift}; max |phi - phi_oracle| {max_abs(F['phi'], g['phi']):.3e}")
    assert np.all(drift <= tol)


def test_d3q19_small_matches_oracle():
    say("case: D3Q19 16x12x20 fp64, 30 steps")
    p = W.CaseParams(nx=16, ny=12, nz=20, lattice="D3Q19", sigma=0.005, nu=0.05, rho_light=0.1)
    phi0 = W.cylinder_phi(p, 7.5, 5.5, 4.0, 0.1, 20.0)
    m = Model(p).init(phi0)
    m.step(30)
    F0 = m.fields()
    for tile in ((16, 4, 4), (32, 2, 3), (64, 1, 20)):
        c = run_gpu(p, phi0, None, 30, tile=(tile[0], tile[2], tile[1]))
        F = c.observe()
        for k in ("phi", "rho", "u", "p"):
            err = max_abs(F[k], F0[k])
            say(f"  tile {tile} {k}: {err:.3e}")
            assert err <= 1e-12, (tile, k)
    r = c.reduce()
    assert np.allclose(r["sum_phi"], m.observables()["sum_phi"], rtol=1e-12)


def test_nonfinite_phi_is_reported():
    say("case: NaN in phi0 reaches the reductions")
    import torch
    v = _v()
    p, phi0, _ = _small_case("periodic_ragged")
    phi0 = phi0.copy()
    phi0[0, 10, 10] = np.nan
    c = v.Case(p)
    d = torch.as_tensor(phi0.reshape(-1)).cuda()
    rc = v.lib().vclb_case_init(c.h, ctypes.c_void_p(d.data_ptr()), None, v.DEVICE,
                                ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0
    c.step(2)
    r = c.reduce()
    assert r["rc"] == v.VCLB_ENONFINITE and r["nonfinite"].any()
    with pytest.raises(v.VclbError):
        v.Case(p).init(phi0)
