"""Host-side checks of the C ABI that need no GPU: the library loads, exports every
symbol include/vclb.h declares, and rejects invalid input before any HIP call."""
import ctypes
import os
import re

import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _vclb():
    from paper_2505_10899_amd import vclb
    return vclb


def header_functions():
    text = open(os.path.join(ROOT, "include", "vclb.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(vclb_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    v = _vclb()
    L = v.lib()
    names = header_functions()
    assert len(names) >= 20
    for name in names:
        assert hasattr(L, name), name
    # the binding wraps exactly the declared entry points
    assert sorted(v.exported_symbols()) == names


def test_strerror_and_version():
    v = _vclb()
    L = v.lib()
    assert L.vclb_strerror(-1) == b"invalid argument"
    assert L.vclb_strerror(-4) == b"non-finite phi"
    assert L.vclb_version() == v.VERSION
    # the header's version, which the binding's struct layouts follow
    hdr = open(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "vclb.h")).read()
    assert f"#define VCLB_VERSION {v.VERSION}" in hdr


def _valid():
    p, _, _ = W.two_droplets()
    return p


def test_valid_params_pass():
    v = _vclb()
    for p in (_valid(), W.single_vortex()[0], W.shear_droplet()[0], W.rayleigh_plateau()[0]):
        v.validate(p)
        assert v.workspace_bytes(p) > 0


@pytest.mark.parametrize("change", [
    dict(W=0.0), dict(W=float("nan")), dict(sigma=-1.0), dict(mobility=0.0), dict(nu=-0.1),
    dict(rho_light=0.0), dict(rho_heavy=float("inf")), dict(xi=0.0), dict(lam=-0.5),
    dict(nx=0), dict(nz=2), dict(s_g=(0, 0, 0, 2.5)), dict(s_f=(0, 0, 0, 0, 0, 0, 0, -0.1)),
    dict(s_g=tuple([0.0] * 9 + [1.0])),          # rate for a moment D2Q9 does not have
    dict(mode="vortex", T=0.0),
    dict(lattice="D3Q19", mode="vortex", nz=4), dict(wall_y=True, ny=1),
    dict(label_centres=[(0, 0, 0)] * 3),
    dict(nx=65536, ny=32768),                    # 2^31 nodes: one more than the largest case
])
def test_invalid_params_rejected_without_gpu(change):
    v = _vclb()
    p = _valid().replace(**change)
    with pytest.raises(v.VclbError) as e:
        v.validate(p)
    assert e.value.code == v.VCLB_EINVAL
    # case creation validates first, before touching HIP
    h = ctypes.c_void_p()
    rc = v.lib().vclb_case_create(ctypes.byref(v.to_cparams(p)), None, 0, ctypes.byref(h))
    assert rc == v.VCLB_EINVAL and not h.value
    assert len(v.lib().vclb_last_error()) > 0


def test_largest_case_validates_with_64_bit_sizes():
    """2^31 - 1 nodes is the largest case (node indices are 32-bit inside the kernels); its
    workspace, far beyond 2^32 bytes, is sized without overflow (no HIP call)."""
    v = _vclb()
    p = _valid().replace(nx=46341, ny=46340, label_centres=[(100.0, 100.0, 0.0)])
    assert p.nx * p.ny <= 2 ** 31 - 1
    v.validate(p)
    b = {s: v.workspace_bytes(p.replace(storage=s)) for s in ("fp16s", "fp32", "fp64")}
    n = p.nx * p.ny
    # at least the populations (2 sets, A and B) and the previous phi u of every node
    assert b["fp64"] >= n * (2 * 2 * 9 * 8 + 2 * 8) > 2 ** 39
    assert b["fp16s"] < b["fp32"] < b["fp64"]


def test_workspace_grows_with_storage_precision():
    v = _vclb()
    b = {s: v.workspace_bytes(_valid().replace(storage=s)) for s in ("fp16s", "fp32", "fp64")}
    assert b["fp16s"] < b["fp32"] < b["fp64"]


def _fake_case(v, p):
    """A case on a borrowed workspace pointer: creation then makes no HIP call."""
    nbytes = v.workspace_bytes(p)
    h = ctypes.c_void_p()
    rc = v.lib().vclb_case_create(ctypes.byref(v.to_cparams(p)), ctypes.c_void_p(1 << 20), nbytes, ctypes.byref(h))
    assert rc == 0
    return h


def test_borrowed_workspace_checks():
    v = _vclb()
    p = _valid()
    h = ctypes.c_void_p()
    nbytes = v.workspace_bytes(p)
    assert v.lib().vclb_case_create(ctypes.byref(v.to_cparams(p)), ctypes.c_void_p(1 << 20), nbytes - 1,
                                    ctypes.byref(h)) == v.VCLB_ENOMEM
    assert v.lib().vclb_case_create(ctypes.byref(v.to_cparams(p)), ctypes.c_void_p((1 << 20) + 8), nbytes,
                                    ctypes.byref(h)) == v.VCLB_EINVAL


def test_step_before_init_and_bad_tiles():
    v = _vclb()
    L = v.lib()
    h = _fake_case(v, _valid())
    assert L.vclb_step(h, 1, None) == v.VCLB_ESTATE
    assert L.vclb_step(h, -1, None) == v.VCLB_EINVAL
    assert L.vclb_case_set_tile(h, 100, 8, 1) == v.VCLB_EINVAL     # not whole waves
    assert L.vclb_case_set_tile(h, 512, 8, 1) == v.VCLB_EINVAL     # above the launch bound
    assert L.vclb_case_set_tile(h, 64, 0, 1) == v.VCLB_EINVAL
    assert L.vclb_case_set_tile(h, 128, 16, 1) == 0
    assert L.vclb_case_autotune(h, None, 2, None) == v.VCLB_ESTATE      # not initialised
    assert L.vclb_case_autotune(h, None, 0, None) == v.VCLB_EINVAL
    assert L.vclb_case_autotune(None, None, 2, None) == v.VCLB_EINVAL
    bx, ty, by = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    assert L.vclb_case_get_tile(h, ctypes.byref(bx), ctypes.byref(ty), ctypes.byref(by)) == 0
    assert (bx.value, ty.value) == (128, 16)
    L.vclb_case_destroy(h)


def test_corrupt_checkpoints_rejected_before_any_copy():
    v = _vclb()
    L = v.lib()
    p = _valid()
    h = _fake_case(v, p)
    n = ctypes.c_size_t()
    assert L.vclb_state_bytes(h, ctypes.byref(n)) == 0
    good_len = n.value
    blob = ctypes.create_string_buffer(good_len)
    # truncated
    assert L.vclb_state_load(h, blob, good_len - 1, None) == v.VCLB_EINVAL
    # wrong magic
    assert L.vclb_state_load(h, blob, good_len, None) == v.VCLB_EINVAL
    assert b"checkpoint" in L.vclb_last_error()
    L.vclb_case_destroy(h)


def test_adjoint_entry_points_reject_without_gpu():
    v = _vclb()
    L = v.lib()
    p64 = W.shear_droplet(nx=64, ny=32, R=8.0)[0]
    n = ctypes.c_size_t()
    assert L.vclb_adjoint_bytes(ctypes.byref(v.to_cparams(p64)), 100, 10, ctypes.byref(n)) == 0
    # 10 checkpoints + 10 segment states of 20 doubles per node, plus 50 doubles of fields
    assert n.value >= (20 * 20 + 50) * 8 * p64.nx * p64.ny
    for q in (p64.replace(storage="fp32"), W.two_droplets()[0].replace(storage="fp16s"),
              W.single_vortex()[0], W.rayleigh_plateau(storage="fp64")[0]):
        assert L.vclb_adjoint_bytes(ctypes.byref(v.to_cparams(q)), 10, 0, ctypes.byref(n)) == v.VCLB_EINVAL
    assert L.vclb_adjoint_bytes(ctypes.byref(v.to_cparams(p64)), -1, 0, ctypes.byref(n)) == v.VCLB_EINVAL
    seed = (ctypes.c_double * 10)(1.0)
    out = (ctypes.c_double * 2)()
    h = _fake_case(v, p64)
    assert L.vclb_adjoint_run(h, seed, 0.1, None, v.DEVICE, out, None) == v.VCLB_ESTATE   # nothing recorded
    assert L.vclb_adjoint_run(h, None, 0.1, None, v.DEVICE, out, None) == v.VCLB_EINVAL
    assert L.vclb_adjoint_run(h, seed, -1.0, None, v.DEVICE, out, None) == v.VCLB_EINVAL
    assert L.vclb_adjoint_run(h, seed, float("nan"), None, v.DEVICE, out, None) == v.VCLB_EINVAL
    assert L.vclb_adjoint_record(h, None, None, v.DEVICE, 10, 0, None) == v.VCLB_EINVAL
    L.vclb_case_destroy(h)
    h = _fake_case(v, p64.replace(storage="fp32"))
    phi = (ctypes.c_double * (p64.nx * p64.ny))()
    assert L.vclb_adjoint_record(h, phi, None, v.HOST, 10, 0, None) == v.VCLB_EINVAL
    assert L.vclb_adjoint_run(h, seed, 0.1, None, v.DEVICE, out, None) == v.VCLB_EINVAL
    L.vclb_case_destroy(h)


def test_batch_entry_points_reject_null_without_gpu():
    v = _vclb()
    L = v.lib()
    out = (v.Obs * 4)()
    assert L.vclb_batch_reduce(None, out, None) == v.VCLB_EINVAL
    assert L.vclb_batch_history(None, 0, 1, out, None) == v.VCLB_EINVAL
    assert L.vclb_batch_step(None, 1, 1, None) == v.VCLB_EINVAL
    assert L.vclb_batch_balance(None, 1, 1, None, None) == v.VCLB_EINVAL
    assert L.vclb_batch_init(None, None, None, v.HOST, None) == v.VCLB_EINVAL
    cnt = ctypes.c_int32(0)
    assert L.vclb_batch_get_weights(None, None, 0, ctypes.byref(cnt)) == v.VCLB_EINVAL
    assert L.vclb_batch_set_weights(None, None, 0) == v.VCLB_EINVAL
    assert L.vclb_batch_set_reduce_every(None, 1) == v.VCLB_EINVAL


def test_bandwidth_probe_validates_before_any_hip_call():
    v = _vclb()
    L = v.lib()
    g = ctypes.c_double(0.0)
    buf = (ctypes.c_double * 8)()                       # host memory: never reached
    p = ctypes.cast(buf, ctypes.c_void_p)
    assert L.vclb_bandwidth_probe(3, p, p, 64, 1, 0, ctypes.byref(g), None) == v.VCLB_EINVAL   # mode
    assert L.vclb_bandwidth_probe(0, p, p, 64, 1, 0, None, None) == v.VCLB_EINVAL             # no result
    assert L.vclb_bandwidth_probe(0, p, p, 0, 1, 0, ctypes.byref(g), None) == v.VCLB_EINVAL   # no bytes
    assert L.vclb_bandwidth_probe(0, p, p, 40, 1, 0, ctypes.byref(g), None) == v.VCLB_EINVAL  # not 16 B
    assert L.vclb_bandwidth_probe(0, p, p, 64, 0, 0, ctypes.byref(g), None) == v.VCLB_EINVAL  # reps
    assert L.vclb_bandwidth_probe(0, None, p, 64, 1, 0, ctypes.byref(g), None) == v.VCLB_EINVAL
    assert L.vclb_bandwidth_probe(1, p, None, 64, 1, 0, ctypes.byref(g), None) == v.VCLB_EINVAL
    odd = ctypes.c_void_p(p.value + 4)
    assert L.vclb_bandwidth_probe(0, odd, p, 48, 1, 0, ctypes.byref(g), None) == v.VCLB_EINVAL  # alignment


# --------------------------------------------------------------------------- boundary types per face
def _raw(p, edit):
    v = _vclb()
    c = v.to_cparams(p)
    edit(c)
    return c


def _rc_validate(c):
    return _vclb().lib().vclb_params_validate(ctypes.byref(c))


def test_boundary_faces_validated_per_axis():
    v = _vclb()
    WALL, PER = v.WALL, v.PERIODIC
    p = _valid()
    assert _rc_validate(_raw(p, lambda c: None)) == v.VCLB_OK
    # walls on both y faces of D2Q9: supported
    def ywalls(c):
        c.bc[1][0] = c.bc[1][1] = WALL
        c.wall_u[1][0][0], c.wall_u[1][1][0] = -0.01, 0.02
    assert _rc_validate(_raw(p, ywalls)) == v.VCLB_OK
    bad = {
        "x walls": lambda c: (c.bc[0].__setitem__(0, WALL), c.bc[0].__setitem__(1, WALL)),
        "z walls": lambda c: (c.bc[2].__setitem__(0, WALL), c.bc[2].__setitem__(1, WALL)),
        "one-sided y wall": lambda c: c.bc[1].__setitem__(0, WALL),
        "unknown type": lambda c: (c.bc[1].__setitem__(0, 7), c.bc[1].__setitem__(1, 7)),
        "normal wall velocity": lambda c: (ywalls(c), c.wall_u[1][0].__setitem__(1, 0.01)),
        "non-finite wall velocity": lambda c: c.wall_u[0][1].__setitem__(2, float("nan")),
    }
    for name, edit in bad.items():
        assert _rc_validate(_raw(p, edit)) == v.VCLB_EINVAL, name
    # D3Q19: walls on the y faces, not on x or z
    q = W.rayleigh_plateau()[0]
    assert _rc_validate(_raw(q, lambda c: None)) == v.VCLB_OK
    assert _rc_validate(_raw(q, lambda c: (c.bc[1].__setitem__(0, WALL), c.bc[1].__setitem__(1, WALL)))) == v.VCLB_OK
    assert _rc_validate(_raw(q, lambda c: (c.bc[2].__setitem__(0, WALL), c.bc[2].__setitem__(1, WALL)))) == v.VCLB_EINVAL
    assert _rc_validate(_raw(q, lambda c: (c.bc[0].__setitem__(0, WALL), c.bc[0].__setitem__(1, WALL)))) == v.VCLB_EINVAL


def test_wetting_validation():
    v = _vclb()
    WALL = v.WALL
    p = _valid()

    def ywalls(c, cb=0.0, ct=0.0):
        c.bc[1][0] = c.bc[1][1] = WALL
        c.wall_cos[1][0], c.wall_cos[1][1] = cb, ct
    assert _rc_validate(_raw(p, lambda c: ywalls(c, 0.5, -1.0))) == v.VCLB_OK
    bad = {
        "cos above 1": lambda c: ywalls(c, 1.0000001, 0.0),
        "cos below -1": lambda c: ywalls(c, 0.0, -1.5),
        "non-finite cos": lambda c: ywalls(c, float("nan"), 0.0),
        "cos on a periodic face": lambda c: c.wall_cos[1].__setitem__(0, 0.5),
        "cos on x": lambda c: (ywalls(c), c.wall_cos[0].__setitem__(1, 0.2)),
    }
    for name, edit in bad.items():
        assert _rc_validate(_raw(p, edit)) == v.VCLB_EINVAL, name


def test_viscosity_ratio_validation():
    v = _vclb()
    p = _valid().replace(nu=0.3, nu_light=0.05)
    v.validate(p)
    assert v.to_cparams(p).nu_heavy == 0.3 and v.to_cparams(p).nu_light == 0.05
    v.validate(W.rayleigh_plateau()[0].replace(nu_light=0.2))
    for change in (dict(nu_light=-0.1), dict(nu_light=float("nan")),
                   dict(s_f=(0, 0, 0, 0, 0, 0, 0, 1.2, 0)),       # a stress rate fixed by hand
                   dict(mode="vortex", T=100.0)):
        with pytest.raises(v.VclbError) as e:
            v.validate(p.replace(**change))
        assert e.value.code == v.VCLB_EINVAL, change
    # rates outside the stress rows stay free
    v.validate(p.replace(s_f=(0, 1.3, 0, 0, 0, 0, 0, 0, 0)))
    # a batch with unequal viscosities in one case relaxes every case's f stress rows per
    # node, so a case beside it with a stress rate fixed by hand is refused (before HIP)
    one = [(5.0, 5.0, 0.0)]   # batched cases have one observation label
    fixed = _valid().replace(s_f=(0, 0, 0, 0, 0, 0, 0, 1.2, 1.2), label_centres=one)
    v.validate(fixed)
    arr = (v.Params * 2)(v.to_cparams(fixed), v.to_cparams(p.replace(label_centres=one)))
    h = ctypes.c_void_p()
    assert v.lib().vclb_batch_create(arr, 2, ctypes.byref(h)) == v.VCLB_EINVAL and not h.value
    assert "stress" in v.lib().vclb_last_error().decode()
    # the adjoint takes unequal viscosities too (its store size needs no HIP call)
    nb = ctypes.c_size_t()
    assert v.lib().vclb_adjoint_bytes(ctypes.byref(v.to_cparams(p)), 10, 2, ctypes.byref(nb)) == 0 and nb.value > 0


def test_global_correction_validation():
    v = _vclb()
    p = _valid().replace(mass_fix=0.5)
    v.validate(p)
    for r in (-0.1, 1.5, float("nan")):
        with pytest.raises(v.VclbError):
            v.validate(p.replace(mass_fix=r))
    arr = (v.Params * 1)(v.to_cparams(p))
    h = ctypes.c_void_p()
    assert v.lib().vclb_batch_create(arr, 1, ctypes.byref(h)) == v.VCLB_EINVAL and not h.value
    nb = ctypes.c_size_t()
    assert v.lib().vclb_adjoint_bytes(ctypes.byref(v.to_cparams(p)), 10, 2, ctypes.byref(nb)) == v.VCLB_EINVAL
