"""GPU checks at the largest sizes one case takes, 2^30 nodes (32768 x 32768, D2Q9), and
on either side of the 2 GiB array size up to which the periodic D3Q19 FP16S step uses
buffer resources (further below).

Such a case has planes of more than 2^29 entries, so its fused step addresses them with
64-bit offsets, and FP32 planes span more than 4 GiB.  The initial field tiles a 64 x 64
periodic drop case (centre off the nodes) 512 x 512 times.  With periodic faces every
tile of the large case sees the same neighbourhood as the small case, and the update of
a node depends only on its neighbourhood, so after a few steps (1) every tile equals
the first one bit for bit, (2) that tile matches the FP64 oracle's small case to the
storage's tolerance, and (3) the FP64 sum of phi over the 2^30 nodes is the small case's
sum times 512^2 (one tile is 3.8e-6 of it) and keeps its value over the steps.  The
fields stay on the device: the case takes about 100 GB (FP16S) or 190 GB (FP32) of the
GPU's 288 GB.
"""
import ctypes
import sys

import numpy as np
import pytest

import workloads as W
from oracle import Model

pytestmark = pytest.mark.gpu

SMALL, REPS, STEPS = 64, 512, 3
NEED_GB = {"fp16s": 140, "fp32": 230}
TOL_PHI = {"fp16s": 2e-3, "fp32": 2e-5}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _small(storage):
    c = SMALL / 2.0 + 0.37, SMALL / 2.0 + 0.41
    p = W.CaseParams(nx=SMALL, ny=SMALL, rho_light=0.1, storage=storage, label_centres=[(c[0], c[1], 0.0)])
    return p, W.drops_phi(p, [(c[0], c[1], 0.0, 14.0)])


@pytest.mark.parametrize("storage", ["fp16s", "fp32"])
def test_two_to_the_thirty_nodes_tile_by_tile(storage):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_10899_amd import vclb
    free = torch.cuda.mem_get_info()[0] / 2 ** 30
    if free < NEED_GB[storage]:
        pytest.skip(f"needs about {NEED_GB[storage]} GB of free device memory, {free:.0f} GB free")
    p_small, phi_small = _small(storage)
    n_side = SMALL * REPS
    p = p_small.replace(nx=n_side, ny=n_side, label_centres=[(n_side / 2.0 + 0.37, n_side / 2.0 + 0.41, 0.0)])
    say(f"case: {n_side} x {n_side} = {n_side * n_side} nodes, {storage}, tiled {SMALL} x {SMALL} drop, "
        f"{STEPS} fused steps")
    torch.cuda.empty_cache()
    c = vclb.Case(p)
    phi0 = torch.as_tensor(phi_small.reshape(SMALL, SMALL), device="cuda").repeat(REPS, REPS).contiguous()
    rc = vclb.lib().vclb_case_init(c.h, ctypes.c_void_p(phi0.data_ptr()), ctypes.c_void_p(0), vclb.DEVICE,
                                   vclb._stream_handle(None))
    vclb.check(rc)
    torch.cuda.synchronize()
    del phi0
    v0 = c.reduce()["sum_phi"].sum()
    c.step(STEPS)
    v1 = c.reduce()["sum_phi"].sum()
    out = torch.empty(n_side * n_side, dtype=torch.float64, device="cuda")
    vclb.check(vclb.lib().vclb_observe(c.h, vclb.FIELD_PHI, ctypes.c_void_p(out.data_ptr()), vclb.DEVICE,
                                       vclb._stream_handle(None)))
    torch.cuda.synchronize()
    tiles = out.view(REPS, SMALL, REPS, SMALL)
    first = tiles[0:1, :, 0:1, :]
    same = bool(torch.equal(tiles, first.expand_as(tiles)))
    spread = float((tiles - first).abs().max())
    tile0 = first.reshape(SMALL, SMALL).cpu().numpy()
    del out, tiles, first
    del c
    torch.cuda.empty_cache()
    m = Model(p_small.replace(storage="fp64")).init(phi_small)
    v_small = float(m.fields()["phi"].sum())
    m.step(STEPS)
    dphi = float(np.max(np.abs(tile0 - m.fields()["phi"][0])))
    drift = abs(v1 - v0) / v0
    vtile = abs(v0 - REPS * REPS * v_small) / v0
    say(f"  tiles bitwise equal: {same} (max spread {spread:.1e}); tile 0 against the FP64 oracle: {dphi:.2e}; "
        f"sum phi: initial vs 512^2 x small {vtile:.1e}, drift over {STEPS} steps {drift:.1e}")
    assert same, spread
    assert dphi <= TOL_PHI[storage], dphi
    # the stored phi carries FP32 rounding, the same in every tile (measured 2.3e-8 in
    # FP16S); one missing tile would be 3.8e-6
    assert vtile <= 2e-7 and drift <= 1e-6, (vtile, drift)


# D3Q19 FP16S: a periodic case whose arrays each span less than 2 GiB is stepped through
# buffer resources (32-bit offsets throughout); a larger one falls back to 64-bit plane
# addresses.  376 x 384 x 384 nodes put the population arrays at 2.1e9 bytes, just below
# the limit (the largest plane offset, 18 planes of ns entries, near 2^31), and
# 384 x 384 x 384 just above it.  Both tile a small periodic column 8 x 8 x 8 times: every
# tile must equal the small case stepped alone bit for bit (the two forms of the kernel
# differ only in how they address memory).
BUF3D = {"below_2GiB": ((376, 384, 384), (47, 48, 48)), "above_2GiB": ((384, 384, 384), (48, 48, 48))}


@pytest.mark.parametrize("which", list(BUF3D))
def test_d3q19_fp16s_either_side_of_the_buffer_limit(which):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_10899_amd import vclb
    (NX, NY, NZ), (sx, sy, sz) = BUF3D[which]
    reps = (NZ // sz, NY // sy, NX // sx)
    assert reps == (8, 8, 8)
    free = torch.cuda.mem_get_info()[0] / 2 ** 30
    if free < 20:
        pytest.skip(f"needs about 20 GB of free device memory, {free:.0f} GB free")
    small = W.CaseParams(nx=sx, ny=sy, nz=sz, lattice="D3Q19", sigma=0.005, nu=0.05, rho_light=0.1,
                         storage="fp16s", label_centres=[(sx / 2.0 + 0.31, sy / 2.0 + 0.27, 0.0)])
    phi_small = W.cylinder_phi(small, sx / 2.0 + 0.31, sy / 2.0 + 0.27, 9.0, 0.1, float(sz))
    big = small.replace(nx=NX, ny=NY, nz=NZ, label_centres=[(NX / 2.0, NY / 2.0, 0.0)])
    pop_bytes = 19 * ((NX * NY * NZ + 63) // 64 * 64) * 2
    say(f"case: D3Q19 FP16S {NX} x {NY} x {NZ} ({which}: population arrays {pop_bytes / 2 ** 31:.4f} x 2 GiB), "
        f"tiled {sx} x {sy} x {sz} column, {STEPS} fused steps")
    assert (pop_bytes < 2 ** 31) == (which == "below_2GiB")
    cs = vclb.Case(small).init(phi_small)
    cs.step(STEPS)
    Fs = cs.observe(vclb.FIELD_PHI | vclb.FIELD_U)
    del cs
    c = vclb.Case(big)
    phi0 = torch.as_tensor(phi_small, device="cuda").repeat(*reps).contiguous()
    vclb.check(vclb.lib().vclb_case_init(c.h, ctypes.c_void_p(phi0.data_ptr()), ctypes.c_void_p(0), vclb.DEVICE,
                                         vclb._stream_handle(None)))
    torch.cuda.synchronize()
    del phi0
    c.step(STEPS)
    n = NX * NY * NZ
    out = torch.empty(4 * n, dtype=torch.float64, device="cuda")
    vclb.check(vclb.lib().vclb_observe(c.h, vclb.FIELD_PHI | vclb.FIELD_U, ctypes.c_void_p(out.data_ptr()),
                                       vclb.DEVICE, vclb._stream_handle(None)))
    torch.cuda.synchronize()
    del c
    fields = out.view(4, reps[0], sz, reps[1], sy, reps[2], sx)
    ref = torch.as_tensor(np.concatenate([Fs["phi"][None], Fs["u"]]), device="cuda").view(4, 1, sz, 1, sy, 1, sx)
    same = bool(torch.equal(fields, ref.expand_as(fields)))
    spread = float((fields - ref).abs().max())
    say(f"  every tile bitwise equal to the small case stepped alone: {same} (max difference {spread:.1e})")
    del out, fields
    torch.cuda.empty_cache()
    assert same, spread
