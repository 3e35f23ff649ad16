"""The library's derived observables and their moment gradients (host arithmetic of
vclb_obs_derived / vclb_obs_seed, no GPU) against the oracle's derived_observables and
its complex-step derivative with respect to each moment."""
import ctypes

import numpy as np
import pytest

import workloads as W
from oracle.model import derived_observables, observables_from_phi


def _vclb():
    from paper_2505_10899_amd import vclb
    return vclb


def _moments():
    """Moments of an off-centre tilted ellipse (label 0) and a small disc (label 1)."""
    p = W.CaseParams(nx=96, ny=64, label_centres=[(30.0, 32.0, 0.0), (75.0, 30.0, 0.0)])
    y, x = np.mgrid[0:64, 0:96].astype(float)
    c, s = np.cos(0.4), np.sin(0.4)
    u, w = (x - 33.5) * c + (y - 30.2) * s, -(x - 33.5) * s + (y - 30.2) * c
    r1 = np.sqrt((u / 14.0) ** 2 + (w / 8.0) ** 2)
    r2 = np.hypot(x - 76.0, y - 31.0) / 6.0
    phi = 0.5 * (1 + np.tanh(2 * (1 - r1) * 8.0 / 4.0)) + 0.5 * (1 + np.tanh(2 * (1 - r2) * 6.0 / 4.0))
    return observables_from_phi(p, phi.reshape(1, 64, 96))


def _pack(o, nl):
    v = _vclb()
    arr = (v.Obs * nl)()
    for k in range(nl):
        arr[k].sum_phi = float(o["sum_phi"][k])
        arr[k].count_half = float(o["count_half"][k])
        for a in range(3):
            arr[k].sum_phi_d[a] = float(o["sum_phi_d"][k][a])
        for a in range(6):
            arr[k].sum_phi_dd[a] = float(o["sum_phi_dd"][k][a])
    return arr


def _oracle_derived(o):
    d = derived_observables(o)
    return np.column_stack([d["volume"], d["centroid"][:, 0], d["centroid"][:, 1], d["centroid"][:, 2], d["D"]])


def test_derived_matches_oracle():
    v = _vclb()
    o = _moments()
    got = v.obs_derived(_pack(o, 2), 2)
    ref = _oracle_derived(o)
    assert ref[0, 4] > 0.2 and ref[1, 4] < 0.05          # elongated ellipse, near-round disc
    assert np.allclose(got, ref, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("label", [0, 1])
def test_seed_is_the_moment_gradient(label):
    """vclb_obs_seed with a unit weight on observable k returns dO_k/dm; the reference
    is the complex-step derivative of the oracle's derived_observables in each moment."""
    v = _vclb()
    o = _moments()
    nl = 2
    h = 1e-30
    ref = np.zeros((5, 10))
    for j in range(10):
        oc = {key: np.array(val, dtype=np.complex128) for key, val in o.items() if key != "count_half"}
        oc["count_half"] = o["count_half"]
        if j == 0:
            oc["sum_phi"][label] += 1j * h
        elif j < 4:
            oc["sum_phi_d"][label][j - 1] += 1j * h
        else:
            oc["sum_phi_dd"][label][j - 4] += 1j * h
        ref[:, j] = np.imag(_oracle_derived(oc)[label]) / h
    for k in range(5):
        w = np.zeros((nl, 5))
        w[label, k] = 1.0
        seed = v.obs_seed(_pack(o, nl), nl, w)
        assert np.all(seed[1 - label] == 0.0)
        scale = np.abs(ref[k]).max() + 1e-300
        assert np.allclose(seed[label], ref[k], rtol=1e-10, atol=1e-12 * scale), (k, seed[label], ref[k])
    # linear in the weights
    w = np.array([[0.5, -1.0, 2.0, 0.0, 3.0], [0.0, 0.0, 0.0, 0.0, 0.0]])
    if label == 1:
        w = w[::-1].copy()
    seed = v.obs_seed(_pack(o, nl), nl, w)
    assert np.allclose(seed[label], w[label] @ ref, rtol=1e-10, atol=1e-12 * np.abs(w[label] @ ref).max())
