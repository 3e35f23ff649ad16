"""The label reduction that allocates nothing (vclb_reduce_static, fixed device scratch)
against vclb_reduce with the same caller labels, through the C ABI: equal bit for bit on
two calls in a row, the second on a smaller case with fewer labels (so that anything the
first call left in the shared scratch would show), and a request beyond the fixed scratch
is refused before any launch."""
import ctypes
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


def _call(v, fn, case, lab, nl):
    import torch
    t = torch.as_tensor(lab.reshape(-1), dtype=torch.int32).to(case.device).contiguous()
    arr = (v.Obs * nl)()
    rc = fn(case.h, ctypes.c_void_p(t.data_ptr()), nl, arr, None)
    torch.cuda.synchronize()
    return rc, arr


def _fields(arr, nl):
    return np.array([[a.sum_phi, a.count_half, *a.sum_phi_d, *a.sum_phi_dd, float(a.nonfinite), float(a.step),
                      float(a.label)] for a in arr[:nl]])


def _blocks(shape, size, seed):
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    b = (x // size) + ((nx + size - 1) // size) * ((y // size) + ((ny + size - 1) // size) * (z // size))
    nb = int(b.max()) + 1
    lab = np.random.default_rng(seed).permutation(nb)[b]
    lab[(x + y + z) % 11 == 0] = -1            # some nodes with no label
    return lab.astype(np.int32), nb


def test_static_scratch_reduction_matches_the_allocating_one():
    v = _v()
    L = v.lib()
    p3 = W.CaseParams(nx=48, ny=40, nz=36, lattice="D3Q19", storage="fp32", sigma=0.005, nu=0.05, rho_light=0.1)
    phi3 = W.cylinder_phi(p3, 23.3, 19.6, 8.0, 0.1, 36.0)
    p2 = W.CaseParams(nx=70, ny=45, W=4.0, sigma=0.01, rho_light=0.1)
    phi2 = W.drops_phi(p2, [(20.3, 22.1, 0, 9.0), (52.7, 20.4, 0, 6.0)])
    runs = [(p3, phi3, 9), (p2, phi2, 12)]             # the second call: fewer nodes, fewer labels
    for k, (p, phi0, size) in enumerate(runs):
        lab, nl = _blocks(phi0.shape, size, seed=k)
        say(f"case: no-alloc reduction, call {k + 1}: {p.lattice} {p.nx}x{p.ny}x{p.nz} {p.storage}, {nl} labels")
        c = v.Case(p).init(phi0)
        c.step(5)
        rc_s, a_s = _call(v, L.vclb_reduce_static, c, lab, nl)
        rc_a, a_a = _call(v, L.vclb_reduce, c, lab, nl)
        assert rc_s == v.VCLB_OK and rc_a == v.VCLB_OK, (rc_s, rc_a)
        fs, fa = _fields(a_s, nl), _fields(a_a, nl)
        assert np.array_equal(fs, fa), float(np.max(np.abs(fs - fa)))
        assert np.all(fs[:, 0] >= 0) and fs[:, 0].sum() > 0
        say(f"  equal bit for bit; total of phi over the labels {fs[:, 0].sum():.6f}")


def test_static_scratch_refuses_requests_beyond_its_size():
    v = _v()
    L = v.lib()
    p = W.CaseParams(nx=1024, ny=1024, W=4.0, sigma=0.01, rho_light=0.1)
    c = v.Case(p).init(W.drops_phi(p, [(500.3, 510.2, 0, 100.0)]))
    lab = np.zeros((1, 1024, 1024), dtype=np.int32)
    rc, _ = _call(v, L.vclb_reduce_static, c, lab, 79)       # 79 labels need more than 4 MiB here
    assert rc == v.VCLB_EINVAL
    assert b"fixed scratch" in L.vclb_last_error()
    rc, arr = _call(v, L.vclb_reduce_static, c, lab, 78)     # 78 fit
    assert rc == v.VCLB_OK
    rc2, arr2 = _call(v, L.vclb_reduce, c, lab, 78)
    assert rc2 == v.VCLB_OK and np.array_equal(_fields(arr, 78), _fields(arr2, 78))
