"""Python binding of libvclb.so: argument marshalling only.

Every step of the model runs in the HIP library; this module converts case
parameters to the C struct of include/vclb.h, gives the library a device workspace
allocated by torch, and passes torch's current HIP stream.  It raises if the library
is missing: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

import torch  # noqa: F401  (loads the HIP runtime the library links against, first)

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libvclb.so")

VCLB_OK, VCLB_EINVAL, VCLB_ENOMEM, VCLB_EHIP, VCLB_ENONFINITE, VCLB_ESTATE = 0, -1, -2, -3, -4, -5
D2Q9, D3Q19 = 0, 1
FP64, FP32, FP16S = 0, 1, 2
COUPLED, PRESCRIBED_VORTEX = 0, 1
PERIODIC, WALL = 0, 1
HOST, DEVICE = 0, 1
FIELD_PHI, FIELD_RHO, FIELD_U, FIELD_P, FIELD_MU, FIELD_PSI = 0x1, 0x2, 0x4, 0x8, 0x10, 0x20
MAX_LABELS = 2
HISTORY = 4096


class VclbError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"vclb error {code}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [
        ("lattice", ctypes.c_int32), ("storage", ctypes.c_int32), ("mode", ctypes.c_int32),
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("bc", (ctypes.c_int32 * 2) * 3), ("nlabels", ctypes.c_int32),
        ("wall_u", ((ctypes.c_double * 3) * 2) * 3),
        ("wall_cos", (ctypes.c_double * 2) * 3),
        ("W", ctypes.c_double), ("sigma", ctypes.c_double), ("mobility", ctypes.c_double),
        ("lam", ctypes.c_double), ("mass_fix", ctypes.c_double), ("xi", ctypes.c_double),
        ("eps_n", ctypes.c_double),
        ("rho_heavy", ctypes.c_double), ("rho_light", ctypes.c_double),
        ("nu_heavy", ctypes.c_double), ("nu_light", ctypes.c_double),
        ("s_g", ctypes.c_double * 19), ("s_f", ctypes.c_double * 19),
        ("U0", ctypes.c_double), ("T", ctypes.c_double),
        ("label_centre", (ctypes.c_double * 3) * MAX_LABELS),
    ]


class Obs(ctypes.Structure):
    _fields_ = [
        ("sum_phi", ctypes.c_double), ("count_half", ctypes.c_double),
        ("sum_phi_d", ctypes.c_double * 3), ("sum_phi_dd", ctypes.c_double * 6),
        ("step", ctypes.c_int64), ("nonfinite", ctypes.c_int32), ("label", ctypes.c_int32),
    ]


_lib = None

# (name, restype, argtypes) of every entry point of include/vclb.h
_P = ctypes.POINTER
_SIGS = [
    ("vclb_strerror", ctypes.c_char_p, [ctypes.c_int]),
    ("vclb_last_error", ctypes.c_char_p, []),
    ("vclb_version", ctypes.c_int, []),
    ("vclb_params_validate", ctypes.c_int, [_P(Params)]),
    ("vclb_case_workspace_bytes", ctypes.c_int, [_P(Params), _P(ctypes.c_size_t)]),
    ("vclb_case_create", ctypes.c_int, [_P(Params), ctypes.c_void_p, ctypes.c_size_t, _P(ctypes.c_void_p)]),
    ("vclb_case_destroy", None, [ctypes.c_void_p]),
    ("vclb_case_set_tile", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    ("vclb_case_get_tile", ctypes.c_int, [ctypes.c_void_p, _P(ctypes.c_int32), _P(ctypes.c_int32), _P(ctypes.c_int32)]),
    ("vclb_case_init", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]),
    ("vclb_case_set_state", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_int64, ctypes.c_int, ctypes.c_void_p]),
    ("vclb_case_get_state", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_int, ctypes.c_void_p]),
    ("vclb_step", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]),
    ("vclb_step_plain", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]),
    ("vclb_case_set_reduce_every", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    ("vclb_case_time", ctypes.c_int, [ctypes.c_void_p, _P(ctypes.c_int64), ctypes.c_void_p]),
    ("vclb_observe", ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]),
    ("vclb_reduce", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, _P(Obs), ctypes.c_void_p]),
    ("vclb_reduce_static", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, _P(Obs),
                                          ctypes.c_void_p]),
    ("vclb_history", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, _P(Obs), ctypes.c_void_p]),
    ("vclb_state_bytes", ctypes.c_int, [ctypes.c_void_p, _P(ctypes.c_size_t)]),
    ("vclb_batch_create", ctypes.c_int, [_P(Params), ctypes.c_int32, _P(ctypes.c_void_p)]),
    ("vclb_batch_destroy", None, [ctypes.c_void_p]),
    ("vclb_batch_case", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, _P(ctypes.c_void_p)]),
    ("vclb_batch_nodes", ctypes.c_int, [ctypes.c_void_p, _P(ctypes.c_int64)]),
    ("vclb_bandwidth_probe", ctypes.c_int, [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                             ctypes.c_int32, ctypes.c_int32, _P(ctypes.c_double), ctypes.c_void_p]),
    ("vclb_bandwidth_probe_ex", ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                                ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int32,
                                                _P(ctypes.c_double), ctypes.c_void_p]),
    ("vclb_batch_init", ctypes.c_int, [ctypes.c_void_p, _P(ctypes.c_void_p), _P(ctypes.c_void_p), ctypes.c_int,
                                        ctypes.c_void_p]),
    ("vclb_batch_set_tile", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32]),
    ("vclb_batch_get_tile", ctypes.c_int, [ctypes.c_void_p, _P(ctypes.c_int32), _P(ctypes.c_int32), _P(ctypes.c_int32)]),
    ("vclb_batch_set_reduce_every", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    ("vclb_batch_reduce", ctypes.c_int, [ctypes.c_void_p, _P(Obs), ctypes.c_void_p]),
    ("vclb_case_autotune", ctypes.c_int, [ctypes.c_void_p, ctypes.c_char_p, ctypes.c_int32, ctypes.c_void_p]),
    ("vclb_batch_history", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, _P(Obs), ctypes.c_void_p]),
    ("vclb_batch_set_schedule", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    ("vclb_batch_get_schedule", ctypes.c_int, [ctypes.c_void_p, _P(ctypes.c_int32)]),
    ("vclb_batch_step", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p]),
    ("vclb_batch_autotune", ctypes.c_int, [ctypes.c_void_p, ctypes.c_char_p, ctypes.c_int32, ctypes.c_void_p]),
    ("vclb_batch_balance", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, _P(ctypes.c_double),
                                           ctypes.c_void_p]),
    ("vclb_batch_get_weights", ctypes.c_int, [ctypes.c_void_p, _P(ctypes.c_double), ctypes.c_int32,
                                               _P(ctypes.c_int32)]),
    ("vclb_batch_set_weights", ctypes.c_int, [ctypes.c_void_p, _P(ctypes.c_double), ctypes.c_int32]),
    ("vclb_state_save", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    ("vclb_state_load", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    ("vclb_obs_derived", ctypes.c_int, [_P(Obs), ctypes.c_int32, _P(ctypes.c_double)]),
    ("vclb_obs_seed", ctypes.c_int, [_P(Obs), ctypes.c_int32, _P(ctypes.c_double), _P(ctypes.c_double)]),
    ("vclb_adjoint_bytes", ctypes.c_int, [_P(Params), ctypes.c_int64, ctypes.c_int32, _P(ctypes.c_size_t)]),
    ("vclb_adjoint_record", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                           ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p]),
    ("vclb_adjoint_run", ctypes.c_int, [ctypes.c_void_p, _P(ctypes.c_double), ctypes.c_double, ctypes.c_void_p,
                                        ctypes.c_int, _P(ctypes.c_double), ctypes.c_void_p]),
]

DERIVED = ("volume", "centroid_x", "centroid_y", "centroid_z", "D")
SEED_FIELDS = 10
NORMAL_TAU = 0.3   # the unit normal is differentiated where |grad psi| >= NORMAL_TAU


VERSION = 20100   # VCLB_VERSION of include/vclb.h, whose struct layouts Params and Obs mirror


def lib():
    """Load libvclb.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2505_10899_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in _SIGS:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        if L.vclb_version() // 10000 != VERSION // 10000:
            raise ImportError(f"{LIB_PATH} has version {L.vclb_version()}, this binding needs {VERSION} (its "
                              "parameter layout): rebuild it with `python -m paper_2505_10899_amd.build`")
        _lib = L
    return _lib


def exported_symbols():
    return [s[0] for s in _SIGS]


def check(rc: int):
    if rc != VCLB_OK:
        L = lib()
        raise VclbError(rc, f"{L.vclb_strerror(rc).decode()}: {L.vclb_last_error().decode()}")


def to_cparams(p) -> Params:
    """CaseParams (workloads.CaseParams or any object with the same fields) -> C struct."""
    c = Params()
    c.lattice = {"D2Q9": D2Q9, "D3Q19": D3Q19}[p.lattice]
    c.storage = {"fp64": FP64, "fp32": FP32, "fp16s": FP16S}[p.storage]
    c.mode = {"coupled": COUPLED, "vortex": PRESCRIBED_VORTEX}[p.mode]
    c.nx, c.ny, c.nz = int(p.nx), int(p.ny), int(p.nz)
    # walls bound y (both faces) or nothing: x and z are periodic
    c.bc[1][0] = c.bc[1][1] = WALL if p.wall_y else PERIODIC
    c.nlabels = len(p.label_centres)
    for a in range(3):
        c.wall_u[1][0][a] = float(p.wall_u_bottom[a])
        c.wall_u[1][1][a] = float(p.wall_u_top[a])
    c.wall_cos[1][0] = float(getattr(p, "wall_cos_bottom", 0.0))
    c.wall_cos[1][1] = float(getattr(p, "wall_cos_top", 0.0))
    c.W, c.sigma, c.mobility = float(p.W), float(p.sigma), float(p.mobility)
    c.lam, c.xi, c.eps_n = float(p.lam), float(p.xi), float(p.eps_n)
    c.mass_fix = float(getattr(p, "mass_fix", 0.0))
    c.rho_heavy, c.rho_light = float(p.rho_heavy), float(p.rho_light)
    nu_l = getattr(p, "nu_light", None)
    c.nu_heavy = float(p.nu)
    c.nu_light = float(p.nu if nu_l is None else nu_l)
    for k, v in enumerate(p.s_g or ()):
        c.s_g[k] = float(v)
    for k, v in enumerate(p.s_f or ()):
        c.s_f[k] = float(v)
    c.U0, c.T = float(p.U0), float(p.T)
    for k, cen in enumerate(p.label_centres[:MAX_LABELS]):
        for a in range(3):
            c.label_centre[k][a] = float(cen[a])
    return c


def validate(p) -> None:
    check(lib().vclb_params_validate(ctypes.byref(to_cparams(p))))


def workspace_bytes(p) -> int:
    n = ctypes.c_size_t()
    check(lib().vclb_case_workspace_bytes(ctypes.byref(to_cparams(p)), ctypes.byref(n)))
    return n.value


def _stream_handle(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Case:
    """One simulation case living on the GPU.

    Device state is a torch uint8 workspace handed to the library; calls are enqueued
    on torch's current stream (or ``stream``)."""

    def __init__(self, p, device="cuda", tile=None, _borrowed=None):
        self.p = p
        self.cp = to_cparams(p)
        self.device = torch.device(device)
        self._owner = None
        if _borrowed is not None:                 # a case owned by a Batch
            self._owner, self.h = _borrowed
        else:
            nbytes = workspace_bytes(p)
            self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            base = self.workspace.data_ptr()
            aligned = (base + 255) // 256 * 256
            h = ctypes.c_void_p()
            check(lib().vclb_case_create(ctypes.byref(self.cp), ctypes.c_void_p(aligned), nbytes, ctypes.byref(h)))
            self.h = h
        self.n = p.nx * p.ny * p.nz
        self.D = 2 if p.lattice == "D2Q9" else 3
        self.nlabels = max(1, len(p.label_centres))
        if tile is not None:
            self.set_tile(*tile)

    def __del__(self):
        try:
            if getattr(self, "h", None) and self._owner is None:
                torch.cuda.synchronize(self.device)
                lib().vclb_case_destroy(self.h)
                self.h = None
        except Exception:
            pass

    # ---------------------------------------------------------------- config
    def set_tile(self, bx, ty, by3=1):
        check(lib().vclb_case_set_tile(self.h, int(bx), int(ty), int(by3)))

    def tile(self):
        a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        check(lib().vclb_case_get_tile(self.h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return a.value, b.value, c.value

    def autotune(self, cache_path=None, steps: int = 5, stream=None):
        """Time the candidate tiles on the current state (restored afterwards) and keep the
        fastest; returns (bx, ty, by3)."""
        path = cache_path.encode() if cache_path else None
        check(lib().vclb_case_autotune(self.h, path, int(steps), _stream_handle(stream)))
        return self.tile()

    def set_reduce_every(self, every: int):
        check(lib().vclb_case_set_reduce_every(self.h, int(every)))

    # ---------------------------------------------------------------- run
    def init(self, phi0, u0=None, stream=None):
        phi = torch.as_tensor(np.ascontiguousarray(phi0, dtype=np.float64).reshape(-1)).to(self.device)
        u = None
        if u0 is not None:
            u = torch.as_tensor(np.ascontiguousarray(u0, dtype=np.float64).reshape(-1)).to(self.device)
        if not torch.isfinite(phi).all():
            raise VclbError(VCLB_ENONFINITE, "phi0 has a NaN/Inf")
        check(lib().vclb_case_init(self.h, ctypes.c_void_p(phi.data_ptr()),
                                   ctypes.c_void_p(u.data_ptr() if u is not None else 0), DEVICE,
                                   _stream_handle(stream)))
        torch.cuda.current_stream().synchronize()
        return self

    def set_state(self, g, f, J, t: int, stream=None):
        """Load a time-t state: g, f of shape (Q, nz, ny, nx), J of shape (D, nz, ny, nx)."""
        dev = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64).reshape(-1)).to(self.device)
        tg, tJ = dev(g), dev(J)
        tf = dev(f) if self.p.mode == "coupled" else None
        check(lib().vclb_case_set_state(self.h, ctypes.c_void_p(tg.data_ptr()),
                                        ctypes.c_void_p(tf.data_ptr() if tf is not None else 0),
                                        ctypes.c_void_p(tJ.data_ptr()), int(t), DEVICE, _stream_handle(stream)))
        return self

    def state_device(self, stream=None):
        """(g, f, J) of the current state, decoded to float64, as flat device tensors
        (f is None in vortex mode)."""
        Q = 9 if self.D == 2 else 19
        g = torch.empty(Q * self.n, dtype=torch.float64, device=self.device)
        J = torch.empty(self.D * self.n, dtype=torch.float64, device=self.device)
        f = torch.empty(Q * self.n, dtype=torch.float64, device=self.device) if self.p.mode == "coupled" else None
        check(lib().vclb_case_get_state(self.h, ctypes.c_void_p(g.data_ptr()),
                                        ctypes.c_void_p(f.data_ptr() if f is not None else 0),
                                        ctypes.c_void_p(J.data_ptr()), DEVICE, _stream_handle(stream)))
        torch.cuda.current_stream().synchronize()
        return g, f, J

    def get_state(self, stream=None):
        """(g, f, J) of the current state as float64 numpy arrays (f is None in vortex mode)."""
        Q = 9 if self.D == 2 else 19
        shape = (self.p.nz, self.p.ny, self.p.nx)
        g = torch.empty(Q * self.n, dtype=torch.float64, device=self.device)
        J = torch.empty(self.D * self.n, dtype=torch.float64, device=self.device)
        f = torch.empty(Q * self.n, dtype=torch.float64, device=self.device) if self.p.mode == "coupled" else None
        check(lib().vclb_case_get_state(self.h, ctypes.c_void_p(g.data_ptr()),
                                        ctypes.c_void_p(f.data_ptr() if f is not None else 0),
                                        ctypes.c_void_p(J.data_ptr()), DEVICE, _stream_handle(stream)))
        torch.cuda.current_stream().synchronize()
        g = g.cpu().numpy().reshape((Q,) + shape)
        J = J.cpu().numpy().reshape((self.D,) + shape)
        f = f.cpu().numpy().reshape((Q,) + shape) if f is not None else None
        return g, f, J

    def step(self, n: int = 1, stream=None):
        check(lib().vclb_step(self.h, int(n), _stream_handle(stream)))
        return self

    def step_plain(self, n: int = 1, stream=None):
        check(lib().vclb_step_plain(self.h, int(n), _stream_handle(stream)))
        return self

    def time(self, stream=None) -> int:
        t = ctypes.c_int64()
        check(lib().vclb_case_time(self.h, ctypes.byref(t), _stream_handle(stream)))
        return t.value

    # ---------------------------------------------------------------- observe
    def observe(self, mask: int = FIELD_PHI | FIELD_RHO | FIELD_U | FIELD_P | FIELD_MU | FIELD_PSI,
                stream=None) -> dict:
        """Fields of the current state as float64 numpy arrays shaped (nz, ny, nx) / (D, nz, ny, nx)."""
        sizes = [(FIELD_PHI, "phi", 1), (FIELD_RHO, "rho", 1), (FIELD_U, "u", self.D), (FIELD_P, "p", 1),
                 (FIELD_MU, "mu", 1), (FIELD_PSI, "psi", 1)]
        total = sum(k for b, _, k in sizes if mask & b) * self.n
        out = torch.empty(total, dtype=torch.float64, device=self.device)
        check(lib().vclb_observe(self.h, mask, ctypes.c_void_p(out.data_ptr()), DEVICE, _stream_handle(stream)))
        torch.cuda.current_stream().synchronize()
        a = out.cpu().numpy()
        shape = (self.p.nz, self.p.ny, self.p.nx)
        res, off = {}, 0
        for b, name, k in sizes:
            if mask & b:
                v = a[off: off + k * self.n]
                res[name] = v.reshape((k,) + shape) if k > 1 else v.reshape(shape)
                off += k * self.n
        return res

    def reduce_raw(self, stream=None):
        """Moments of the current state as the C array of vclb_obs (one per label)."""
        arr = (Obs * self.nlabels)()
        rc = lib().vclb_reduce(self.h, None, 0, arr, _stream_handle(stream))
        if rc not in (VCLB_OK, VCLB_ENONFINITE):
            check(rc)
        return arr

    def derived(self, stream=None) -> np.ndarray:
        """(labels, 5) array of volume, centroid offset (x, y, z) and deformation D."""
        return obs_derived(self.reduce_raw(stream), self.nlabels)

    # ---------------------------------------------------------------- adjoint (FP64 D2Q9 coupled)
    def adjoint_record(self, phi0, u0=None, nsteps: int = 0, every: int = 0, stream=None):
        """Forward pass from phi0 (and u0) over nsteps steps, keeping a state every
        `every` steps (0: ceil(sqrt(nsteps))) for vclb_adjoint_run."""
        phi = _as_device_f64(phi0, self.device)
        u = _as_device_f64(u0, self.device) if u0 is not None else None
        if not torch.isfinite(phi).all():
            raise VclbError(VCLB_ENONFINITE, "phi0 has a NaN/Inf")
        check(lib().vclb_adjoint_record(self.h, ctypes.c_void_p(phi.data_ptr()),
                                        ctypes.c_void_p(u.data_ptr() if u is not None else 0), DEVICE,
                                        int(nsteps), int(every), _stream_handle(stream)))
        return self

    def adjoint_run(self, seed, normal_tau: float = NORMAL_TAU, stream=None):
        """Backward pass for the moment weights `seed` ((labels, 10) array, see
        obs_seed), with the unit normal differentiated where |grad psi| >= normal_tau.
        Returns (dJ/dphi0 as a float64 device tensor shaped (nz, ny, nx), dJ/dsigma, dJ/dM)."""
        sd = np.ascontiguousarray(seed, dtype=np.float64).reshape(-1)
        if sd.size != self.nlabels * SEED_FIELDS:
            raise VclbError(VCLB_EINVAL, "seed must hold 10 weights per label")
        dphi = torch.empty(self.n, dtype=torch.float64, device=self.device)
        out = (ctypes.c_double * 2)()
        check(lib().vclb_adjoint_run(self.h, sd.ctypes.data_as(_P(ctypes.c_double)), float(normal_tau),
                                     ctypes.c_void_p(dphi.data_ptr()), DEVICE, out, _stream_handle(stream)))
        return dphi.reshape(self.p.nz, self.p.ny, self.p.nx), out[0], out[1]

    def reduce(self, stream=None) -> dict:
        arr = (Obs * self.nlabels)()
        rc = lib().vclb_reduce(self.h, None, 0, arr, _stream_handle(stream))
        if rc not in (VCLB_OK, VCLB_ENONFINITE):
            check(rc)
        out = _obs_to_dict(arr, self.nlabels)
        out["rc"] = rc
        return out

    def reduce_labels(self, labels, nlabels: int = 0, static: bool = False, stream=None) -> dict:
        """Volume reductions over caller labels: labels[n] (int32, shape (nz, ny, nx) or
        flat; numpy or torch; negative = no label), nlabels labels (0: max label + 1).
        Moments are about the origin (d = the node's position).  static: use the entry
        point that allocates nothing (vclb_reduce_static, fixed device scratch)."""
        lab = torch.as_tensor(labels).reshape(-1).to(device=self.device, dtype=torch.int32).contiguous()
        if lab.numel() != self.n:
            raise VclbError(VCLB_EINVAL, "one label per node")
        nl = int(nlabels) if nlabels else int(lab.max().item()) + 1
        arr = (Obs * max(1, nl))()
        fn = lib().vclb_reduce_static if static else lib().vclb_reduce
        rc = fn(self.h, ctypes.c_void_p(lab.data_ptr()), nl, arr, _stream_handle(stream))
        if rc not in (VCLB_OK, VCLB_ENONFINITE):
            check(rc)
        out = _obs_to_dict(arr, max(1, nl))
        out["rc"] = rc
        return out

    def history(self, t_first: int, count: int, stream=None) -> dict:
        arr = (Obs * (self.nlabels * count))()
        rc = lib().vclb_history(self.h, int(t_first), int(count), arr, _stream_handle(stream))
        if rc not in (VCLB_OK, VCLB_ENONFINITE):
            check(rc)
        d = _obs_to_dict(arr, self.nlabels * count)
        return {k: v.reshape((count, self.nlabels) + v.shape[1:]) for k, v in d.items()}

    # ---------------------------------------------------------------- checkpoints
    def state_bytes(self) -> int:
        n = ctypes.c_size_t()
        check(lib().vclb_state_bytes(self.h, ctypes.byref(n)))
        return n.value

    def save(self, stream=None) -> bytes:
        n = self.state_bytes()
        buf = ctypes.create_string_buffer(n)
        check(lib().vclb_state_save(self.h, buf, n, _stream_handle(stream)))
        return buf.raw

    def load(self, blob: bytes, stream=None):
        buf = ctypes.create_string_buffer(blob, len(blob))
        check(lib().vclb_state_load(self.h, buf, len(blob), _stream_handle(stream)))
        return self


def _as_device_f64(a, device):
    if isinstance(a, torch.Tensor):
        return a.detach().to(device=device, dtype=torch.float64).contiguous().reshape(-1)
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64).reshape(-1)).to(device)


def bandwidth_probe(mode: str = "copy", nbytes: int = 2 << 30, reps: int = 10, blocks: int = 0,
                    device="cuda", stream=None) -> float:
    """Achievable HBM bandwidth in GB/s (vclb_bandwidth_probe) over fresh buffers of
    nbytes: "copy" (read + write counted), "read" or "write"."""
    m = {"copy": 0, "read": 1, "write": 2}[mode]
    n = nbytes // 4
    src = torch.ones(n, dtype=torch.float32, device=device) if m != 2 else None
    dst = torch.empty(n if m != 1 else 4, dtype=torch.float32, device=device)
    g = ctypes.c_double(0.0)
    check(lib().vclb_bandwidth_probe(m, ctypes.c_void_p(dst.data_ptr()),
                                     ctypes.c_void_p(src.data_ptr() if src is not None else 0),
                                     ctypes.c_size_t(n * 4), int(reps), int(blocks), ctypes.byref(g),
                                     _stream_handle(stream)))
    return g.value


def bandwidth_probe_best(mode: str = "copy", nbytes: int = 2 << 30, reps: int = 5, device="cuda", stream=None):
    """Fastest rate (GB/s) of the probe over its kernel shapes (vclb_bandwidth_probe_ex):
    vectors in flight per lane {1, 2, 4, 8} x plain / non-temporal accesses x {2, 4, 8, 16}
    workgroups per compute unit.  Returns (GB/s, {"unroll", "nontemporal",
    "blocks_per_cu"})."""
    m = {"copy": 0, "read": 1, "write": 2}[mode]
    n = nbytes // 4
    src = torch.ones(n, dtype=torch.float32, device=device) if m != 2 else None
    dst = torch.empty(n if m != 1 else 4, dtype=torch.float32, device=device)
    ncu = torch.cuda.get_device_properties(torch.device(device)).multi_processor_count
    best, cfg = 0.0, None
    for unroll in (1, 2, 4, 8):
        for nt in (0, 1):
            for per_cu in (2, 4, 8, 16):
                g = ctypes.c_double(0.0)
                check(lib().vclb_bandwidth_probe_ex(m, unroll, nt, ctypes.c_void_p(dst.data_ptr()),
                                                    ctypes.c_void_p(src.data_ptr() if src is not None else 0),
                                                    ctypes.c_size_t(n * 4), int(reps), int(per_cu * ncu),
                                                    ctypes.byref(g), _stream_handle(stream)))
                if g.value > best:
                    best, cfg = g.value, {"unroll": unroll, "nontemporal": nt, "blocks_per_cu": per_cu}
    return best, cfg


def obs_derived(arr, nlabels: int) -> np.ndarray:
    """Derived observables (volume, centroid offset x/y/z, D) per label from vclb_obs moments."""
    out = (ctypes.c_double * (5 * nlabels))()
    check(lib().vclb_obs_derived(arr, int(nlabels), out))
    return np.array(out[:]).reshape(nlabels, 5)


def obs_seed(arr, nlabels: int, weights) -> np.ndarray:
    """Moment weights (labels, 10) of J = sum weights[l, k] * derived[l, k], linearised at arr."""
    w = np.ascontiguousarray(weights, dtype=np.float64).reshape(-1)
    if w.size != 5 * nlabels:
        raise VclbError(VCLB_EINVAL, "weights must hold 5 values per label")
    out = (ctypes.c_double * (SEED_FIELDS * nlabels))()
    check(lib().vclb_obs_seed(arr, int(nlabels), w.ctypes.data_as(_P(ctypes.c_double)), out))
    return np.array(out[:]).reshape(nlabels, SEED_FIELDS)


class _Rollout(torch.autograd.Function):
    """Derived observables after nsteps steps as a differentiable function of
    (phi0, sigma, mobility); the backward pass is the library's discrete adjoint."""

    @staticmethod
    def forward(ctx, phi0, sigma, mobility, p, nsteps, every, u0, device, normal_tau):
        q = p.replace(sigma=float(sigma), mobility=float(mobility))
        case = Case(q, device=device)
        case.adjoint_record(phi0, u0, nsteps=nsteps, every=every)
        raw = case.reduce_raw()
        ctx.case, ctx.raw, ctx.tau = case, raw, normal_tau
        ctx.shape = phi0.shape
        return torch.as_tensor(obs_derived(raw, case.nlabels), dtype=torch.float64)

    @staticmethod
    def backward(ctx, grad_out):
        case = ctx.case
        seed = obs_seed(ctx.raw, case.nlabels, grad_out.detach().cpu().numpy())
        dphi, dsig, dmob = case.adjoint_run(seed, normal_tau=ctx.tau)
        return (dphi.reshape(ctx.shape), torch.tensor(dsig, dtype=torch.float64),
                torch.tensor(dmob, dtype=torch.float64), None, None, None, None, None, None)


def rollout(p, phi0: torch.Tensor, sigma: torch.Tensor, mobility: torch.Tensor, nsteps: int, every: int = 0,
            u0=None, device="cuda", normal_tau: float = NORMAL_TAU) -> torch.Tensor:
    """(labels, 5) tensor of volume, centroid offset (x, y, z) and deformation D after
    nsteps FP64 D2Q9 coupled steps from phi0, differentiable in phi0, sigma and mobility
    (checkpoint every `every` steps; 0: ceil(sqrt(nsteps)); normal_tau: see adjoint_run)."""
    return _Rollout.apply(phi0, sigma, mobility, p, int(nsteps), int(every), u0, device, float(normal_tau))


def _obs_to_dict(arr, n) -> dict:
    return {
        "sum_phi": np.array([arr[k].sum_phi for k in range(n)]),
        "count_half": np.array([arr[k].count_half for k in range(n)]),
        "sum_phi_d": np.array([list(arr[k].sum_phi_d) for k in range(n)]),
        "sum_phi_dd": np.array([list(arr[k].sum_phi_dd) for k in range(n)]),
        "nonfinite": np.array([arr[k].nonfinite for k in range(n)]),
        "step": np.array([arr[k].step for k in range(n)]),
        "label": np.array([arr[k].label for k in range(n)]),
    }


class Batch:
    """Many independent coupled D2Q9 cases advanced together (one work-list kernel per
    step, a call's steps replayed from one hipGraph).  ``cases[k]`` is a Case view of
    case k (init, observe, reduce, history, get/set_state)."""

    def __init__(self, params_list, device="cuda"):
        n = len(params_list)
        arr = (Params * n)(*[to_cparams(p) for p in params_list])
        h = ctypes.c_void_p()
        check(lib().vclb_batch_create(arr, n, ctypes.byref(h)))
        self.h = h
        self.device = torch.device(device)
        self.params = list(params_list)
        self.cases = []
        for k, p in enumerate(self.params):
            ch = ctypes.c_void_p()
            check(lib().vclb_batch_case(self.h, k, ctypes.byref(ch)))
            self.cases.append(Case(p, device=device, _borrowed=(self, ch)))

    def __del__(self):
        try:
            if getattr(self, "h", None):
                torch.cuda.synchronize(self.device)
                for c in self.cases:
                    c.h = None
                lib().vclb_batch_destroy(self.h)
                self.h = None
        except Exception:
            pass

    def init(self, fields, stream=None):
        """Initial state of every case from a list of (phi0, u0) pairs (u0 may be None),
        in one library call."""
        if len(fields) != len(self.cases):
            raise VclbError(VCLB_EINVAL, "one (phi0, u0) pair per case")
        phis, us = [], []
        for phi0, u0 in fields:
            phi = _as_device_f64(phi0, self.device)
            if not torch.isfinite(phi).all():
                raise VclbError(VCLB_ENONFINITE, "phi0 has a NaN/Inf")
            phis.append(phi)
            us.append(_as_device_f64(u0, self.device) if u0 is not None else None)
        n = len(phis)
        pp = (ctypes.c_void_p * n)(*[t.data_ptr() for t in phis])
        up = (ctypes.c_void_p * n)(*[t.data_ptr() if t is not None else 0 for t in us])
        check(lib().vclb_batch_init(self.h, pp, up, DEVICE, _stream_handle(stream)))
        torch.cuda.current_stream().synchronize()
        return self

    def nodes(self) -> int:
        n = ctypes.c_int64()
        check(lib().vclb_batch_nodes(self.h, ctypes.byref(n)))
        return n.value

    def set_tile(self, bx, ty):
        check(lib().vclb_batch_set_tile(self.h, int(bx), int(ty)))

    def tile(self):
        a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        check(lib().vclb_batch_get_tile(self.h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return a.value, b.value, c.value

    def set_reduce_every(self, every: int):
        check(lib().vclb_batch_set_reduce_every(self.h, int(every)))

    def reduce(self, stream=None) -> dict:
        """Volume reductions of every case's current state in one call: arrays shaped
        (ncases, MAX_LABELS, ...); labels beyond a case's count are zero."""
        n = len(self.cases)
        arr = (Obs * (n * MAX_LABELS))()
        rc = lib().vclb_batch_reduce(self.h, arr, _stream_handle(stream))
        if rc not in (VCLB_OK, VCLB_ENONFINITE):
            check(rc)
        d = _obs_to_dict(arr, n * MAX_LABELS)
        out = {k: v.reshape((n, MAX_LABELS) + v.shape[1:]) for k, v in d.items()}
        out["rc"] = rc
        return out

    def history(self, t_first: int, count: int, stream=None) -> dict:
        """Recorded per-step reductions of every case, arrays shaped (count, ncases,
        MAX_LABELS, ...)."""
        n = len(self.cases)
        arr = (Obs * (count * n * MAX_LABELS))()
        rc = lib().vclb_batch_history(self.h, int(t_first), int(count), arr, _stream_handle(stream))
        if rc not in (VCLB_OK, VCLB_ENONFINITE):
            check(rc)
        d = _obs_to_dict(arr, count * n * MAX_LABELS)
        return {k: v.reshape((count, n, MAX_LABELS) + v.shape[1:]) for k, v in d.items()}

    def set_schedule(self, flat_pct: int):
        check(lib().vclb_batch_set_schedule(self.h, int(flat_pct)))

    def schedule(self) -> int:
        v = ctypes.c_int32()
        check(lib().vclb_batch_get_schedule(self.h, ctypes.byref(v)))
        return v.value

    def step(self, n: int = 1, graph: bool = True, stream=None):
        check(lib().vclb_batch_step(self.h, int(n), 1 if graph else 0, _stream_handle(stream)))
        return self

    def autotune(self, cache_path=None, steps: int = 5, stream=None):
        path = cache_path.encode() if cache_path else None
        check(lib().vclb_batch_autotune(self.h, path, int(steps), _stream_handle(stream)))
        return self.tile()

    def weights(self) -> np.ndarray:
        """Slot weights in force (ones when none are)."""
        n = ctypes.c_int32(0)
        check(lib().vclb_batch_get_weights(self.h, None, 0, ctypes.byref(n)))
        buf = (ctypes.c_double * max(1, n.value))()
        check(lib().vclb_batch_get_weights(self.h, buf, n.value, ctypes.byref(n)))
        return np.array(buf[:n.value])

    def set_weights(self, w):
        """Apply slot weights (one per slot of the current launch shape; empty clears)."""
        a = np.ascontiguousarray(w, dtype=np.float64)
        check(lib().vclb_batch_set_weights(self.h, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if a.size else None,
                                           int(a.size)))
        return self

    def balance(self, rounds: int = 3, steps: int = 3, stream=None) -> float:
        """Re-cut the runs to the measured speed of each workgroup slot (state restored);
        returns the slowest slot's time before over after."""
        g = ctypes.c_double(1.0)
        check(lib().vclb_batch_balance(self.h, int(rounds), int(steps), ctypes.byref(g), _stream_handle(stream)))
        return g.value
