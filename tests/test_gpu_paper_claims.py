"""The paper's qualitative claims, run through the GPU path at the test problems' own
sizes (Sect. 4), each against the classical model (lam = 0, no correction term):

- two drops at rest (Sect. 4.1): the small drop keeps its area with the correction and
  shrinks without it;
- a drop of radius 8 in shear flow on a coarse grid (Sect. 4.4): it survives with the
  correction and loses half its area without it;
- the time-reversed single vortex with n = 6 (Sect. 4.2): the disk returns closer to its
  initial shape with the correction;
- the Rayleigh-Plateau break-up (Sect. 4.3), on the benchmark's 3D liquid column (the
  planar 2D layer of Eq. 45 does not break up under either model): the column pinches
  into a drop and a satellite under both models; with the correction the volume stays
  put and the satellite keeps its size, without it both shrink.

The thresholds are set between the two models' measured values with a wide margin; the
figures themselves are not in the text, so no printed value pins these runs."""
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


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _areas(v, builder, steps, every):
    """#(phi >= 1/2) per label at steps 0, every, ..., steps - every, and at the end."""
    out = {}
    for lam in (0.5, 0.0):
        p, phi0, u0 = builder(lam)
        c = v.Case(p).init(phi0, u0)
        c.set_reduce_every(every)
        c.step(steps)
        h = np.array([c.history(t, 1)["count_half"][0] for t in range(0, steps, every)])
        out[lam] = np.vstack([h, c.reduce()["count_half"][None]])
    return out


def test_two_drops_small_drop_keeps_its_area_only_with_the_correction():
    v = _v()
    a = _areas(v, W.paper_two_drops, 100000, 10000)
    for lam in (0.5, 0.0):
        say(f"two drops, lam = {lam}: area / initial (large, small) at the end "
            f"{a[lam][-1, 0] / a[lam][0, 0]:.4f}, {a[lam][-1, 1] / a[lam][0, 1]:.4f}")
    kept = a[0.5][:, 1] / a[0.5][0, 1]
    lost = a[0.0][-1, 1] / a[0.0][0, 1]
    assert np.all(np.abs(kept - 1.0) <= 0.03)      # measured: within 2.1%
    assert lost <= 0.85                            # measured: 0.75
    assert abs(a[0.5][-1, 0] / a[0.5][0, 0] - 1.0) <= 0.02


def test_small_drop_in_shear_survives_only_with_the_correction():
    v = _v()
    a = _areas(v, W.paper_shear_drop, 100000, 10000)
    for lam in (0.5, 0.0):
        say(f"shear drop r = 8, lam = {lam}: area / initial over time {np.round(a[lam][:, 0] / a[lam][0, 0], 3).tolist()}")
    assert np.all(np.abs(a[0.5][:, 0] / a[0.5][0, 0] - 1.0) <= 0.03)   # measured: within 1%
    assert a[0.0][-1, 0] / a[0.0][0, 0] <= 0.6                         # measured: 0.42


def test_single_vortex_returns_closer_with_the_correction():
    v = _v()
    err = {}
    for lam in (0.5, 0.0):
        p, phi0, _ = W.paper_vortex(lam)
        c = v.Case(p).init(phi0, None)
        c.set_reduce_every(0)
        c.step(int(round(p.T)))
        phi = c.observe()["phi"].reshape(phi0.shape)
        err[lam] = float(np.abs(phi - phi0).sum() / (2.0 * np.pi * 45.0))
        say(f"vortex n = 6, lam = {lam}: sum |phi(T) - phi0| per unit perimeter {err[lam]:.4f}, "
            f"area {int((phi >= 0.5).sum())} of {int((phi0 >= 0.5).sum())}")
    assert err[0.5] <= 0.6 * err[0.0]                # measured: 0.70 against 1.47


def _regions_periodic_x(mask):
    """Number of connected regions of a (ny, nx) mask, periodic along x."""
    from scipy import ndimage
    lab, n = ndimage.label(mask)
    parent = list(range(n + 1))

    def root(k):
        while parent[k] != k:
            parent[k] = parent[parent[k]]
            k = parent[k]
        return k

    for a, b in zip(lab[:, 0], lab[:, -1]):
        if a > 0 and b > 0:
            parent[root(int(a))] = root(int(b))
    return len({root(k) for k in range(1, n + 1)})


def test_rayleigh_plateau_layer_2d_stays_one_layer():
    """Sect. 4.3 at the paper's own size: the layer of Eq. 45 on 256 x 128 nodes (readings in
    workloads.paper_rayleigh_plateau_2d), 100 000 steps, with the correction and without
    it.  A planar layer has no azimuthal curvature to drive a Rayleigh-Plateau break-up:
    under both models it stays one connected layer along the periodic x axis, and its
    area #(phi >= 1/2) stays within 1% of its start."""
    v = _v()
    for lam in (0.5, 0.0):
        p, phi0, u0 = W.paper_rayleigh_plateau_2d(lam)
        c = v.Case(p).init(phi0, u0)
        c.set_reduce_every(0)
        a0 = int((phi0 >= 0.5).sum())
        areas, parts = [], []
        for _ in range(10):
            c.step(10000)
            phi = c.observe(v.FIELD_PHI)["phi"][0]
            parts.append(_regions_periodic_x(phi >= 0.5))
            areas.append(int((phi >= 0.5).sum()))
        say(f"2D layer, lam = {lam}: area / initial every 10k steps {np.round(np.array(areas) / a0, 4).tolist()}, "
            f"connected regions {parts}")
        assert all(k == 1 for k in parts), lam
        assert np.all(np.abs(np.array(areas) / a0 - 1.0) <= 0.01), lam     # measured: within 0.8% (lam 0.5)


def _drop_labels(phi):
    """Host labels of the drops of a (nz, ny, nx) field: the connected regions of
    phi >= 1/2, joined across the periodic z faces (the column's axis), numbered largest
    first; every other node takes the label of the nearest region node (so that each
    drop's diffuse interface counts with it).  Returns (labels int32, count)."""
    from scipy import ndimage
    lab, n = ndimage.label(phi >= 0.5)
    parent = list(range(n + 1))

    def root(k):
        while parent[k] != k:
            parent[k] = parent[parent[k]]
            k = parent[k]
        return k

    lo, hi = lab[0], lab[-1]
    both = (lo > 0) & (hi > 0)
    for a, b in zip(lo[both], hi[both]):
        parent[root(int(a))] = root(int(b))
    roots = np.array([root(k) for k in range(n + 1)])
    lab = roots[lab]
    size = np.bincount(lab.ravel(), minlength=n + 1)
    size[0] = 0
    order = [k for k in np.argsort(-size, kind="stable") if size[k] > 0]
    renum = np.full(n + 1, -1)
    renum[order] = np.arange(len(order))
    lab = renum[lab]
    # nearest region node for the rest, on three copies stacked along the periodic z axis
    nz = phi.shape[0]
    tiled = np.concatenate([lab, lab, lab], axis=0)
    _, idx = ndimage.distance_transform_edt(tiled < 0, return_indices=True)
    near = tiled[tuple(idx)][nz:2 * nz]
    return near.astype(np.int32), len(order)


def _drops(v, c, phi):
    """Per drop, largest first: #(phi >= 1/2) and the FP64 volume sum(phi), both from the
    library's device reductions over the host's drop labels."""
    lab, n = _drop_labels(phi)
    r = c.reduce_labels(lab, n)
    return [int(x) for x in r["count_half"]], [float(x) for x in r["sum_phi"]]


def test_rayleigh_plateau_column_keeps_its_drops_only_with_the_correction():
    """96 x 96 x 384 column, R0 = 16 with a 10% perturbation over the box length (FP32):
    it pinches between steps 20 500 and 21 000 into one drop and one satellite under both
    models."""
    v = _v()
    out = {}
    for lam in (0.5, 0.0):
        p, phi0, u0 = W.rayleigh_plateau("fp32")
        c = v.Case(p.replace(lam=lam)).init(phi0, u0)
        c.set_reduce_every(0)
        vol0 = int((phi0 >= 0.5).sum())
        total0 = c.reduce()["sum_phi"].sum()
        c.step(30000)
        d30, s30 = _drops(v, c, c.observe(v.FIELD_PHI)["phi"])
        c.step(10000)
        d40, s40 = _drops(v, c, c.observe(v.FIELD_PHI)["phi"])
        out[lam] = (vol0, d30, d40)
        say(f"column, lam = {lam}: drops #(phi >= 1/2) at 30k {d30}, at 40k {d40}; volume at 40k / initial "
            f"{sum(d40) / vol0:.4f}; sum(phi) per drop at 30k {np.round(s30, 2).tolist()}, at 40k {np.round(s40, 2).tolist()}")
        # every node belongs to a drop: the drops' sum(phi) add up to the total, which is conserved
        assert abs(sum(s40) - total0) <= 1e-6 * total0
    for lam in (0.5, 0.0):
        vol0, d30, d40 = out[lam]
        assert len(d30) == 2 and len(d40) == 2, lam                      # one drop and one satellite
    vol0, d30, d40 = out[0.5]
    assert abs(sum(d40) / vol0 - 1.0) <= 0.01                            # measured: +0.3%
    assert abs(d40[1] / d30[1] - 1.0) <= 0.005                           # satellite, measured: +0.1%
    vol0, e30, e40 = out[0.0]
    assert sum(e40) / vol0 <= 0.985                                      # measured: 0.969
    assert e40[1] < e30[1]                                               # measured: -0.8% in 10k steps
    assert d40[1] >= 1.05 * e40[1]                                       # measured: 1.11


def _drop_count(phi):
    """Number of connected regions of phi >= 1/2, joined across the periodic z faces."""
    from scipy import ndimage
    lab, n = ndimage.label(phi >= 0.5)
    parent = list(range(n + 1))

    def root(k):
        while parent[k] != k:
            parent[k] = parent[parent[k]]
            k = parent[k]
        return k

    lo, hi = lab[0], lab[-1]
    both = (lo > 0) & (hi > 0)
    for a, b in zip(lo[both], hi[both]):
        parent[root(int(a))] = root(int(b))
    return len({root(k) for k in range(1, n + 1)})


def test_rayleigh_plateau_column_per_storage():
    """The column above (lam = 0.5) in FP64, FP32 and FP16S storage: the step at which it
    pinches off (found to 500 steps) and each drop's volume at step 40 000 (FP64 device sums
    over the same host labels), FP32 and FP16S against FP64, whose path matches the oracle
    to 1e-12 over free runs."""
    v = _v()
    res = {}
    for st in ("fp64", "fp32", "fp16s"):
        p, phi0, u0 = W.rayleigh_plateau(st)
        c = v.Case(p).init(phi0, u0)
        c.set_reduce_every(0)
        total0 = c.reduce()["sum_phi"].sum()
        t = 20000
        c.step(t)
        while _drop_count(c.observe(v.FIELD_PHI)["phi"]) < 2 and t < 34000:
            c.step(500)
            t += 500
        c.step(40000 - t)
        _, s = _drops(v, c, c.observe(v.FIELD_PHI)["phi"])
        res[st] = (t, s, total0)
        say(f"column {st}: pinched off by step {t}; sum(phi) per drop at 40k {np.round(s, 3).tolist()}; "
            f"total drift {abs(sum(s) - total0) / total0:.1e}")
        del c
    t64, s64, _ = res["fp64"]
    assert len(s64) == 2 and t64 < 34000
    # measured: FP32 pinches at the same check, its drops within 9e-5 of FP64's; FP16S one
    # check (500 steps) later, its drops within 6.7e-3 (the satellite)
    for st, (dt, dv) in {"fp32": (500, 1e-3), "fp16s": (1000, 2e-2)}.items():
        t, s, total0 = res[st]
        rel = [abs(a / b - 1.0) for a, b in zip(s, s64)]
        say(f"  {st} against fp64: pinch-off {t - t64:+d} steps, drop volumes {np.round(rel, 6).tolist()}")
        assert len(s) == 2 and abs(t - t64) <= dt and max(rel) <= dv, (st, t, t64, rel)
