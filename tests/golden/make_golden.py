"""Write the stored expected values used by the GPU parity tests.

Every value here comes from the CPU oracle (``oracle/``) run on the seeded inputs
of ``workloads``; nothing comes from the HIP library.  Re-run after any change to
the oracle's arithmetic:

    python tests/golden/make_golden.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle import Model  # noqa: E402


def two_droplets_1000():
    """Two static drops, 128 x 128 periodic, FP64, 1000 steps: phi, rho, u, p at t = 1000,
    the per-droplet reductions at t = 0, 500, 1000, and the oracle's own round-off
    envelope: the largest change of each field at t = 1000 when phi0 is perturbed by a
    relative 1e-15 (seeded normal noise)."""
    p, phi0, u0 = W.two_droplets("fp64")
    m = Model(p).init(phi0, u0)
    sums = {0: m.observables()["sum_phi"]}
    m.step(500)
    sums[500] = m.observables()["sum_phi"]
    m.step(500)
    sums[1000] = m.observables()["sum_phi"]
    F = m.fields()
    obs = m.observables()
    rng = np.random.default_rng(1)
    q = Model(p).init(phi0 * (1.0 + 1e-15 * rng.standard_normal(phi0.shape)), u0)
    q.step(1000)
    G = q.fields()
    env = {k: float(np.max(np.abs(F[k] - G[k]))) for k in ("phi", "rho", "u", "p")}
    oq = q.observables()
    env_sum = np.abs(oq["sum_phi"] - obs["sum_phi"])
    env_count = np.abs(oq["count_half"] - obs["count_half"])
    np.savez_compressed(os.path.join(HERE, "two_droplets_fp64_t1000.npz"),
                        phi=F["phi"], rho=F["rho"], u=F["u"], p=F["p"],
                        sum_phi_t0=sums[0], sum_phi_t500=sums[500], sum_phi_t1000=sums[1000],
                        count_half=obs["count_half"], sum_phi_d=obs["sum_phi_d"], sum_phi_dd=obs["sum_phi_dd"],
                        env_phi=env["phi"], env_rho=env["rho"], env_u=env["u"], env_p=env["p"],
                        env_sum_phi=env_sum, env_count_half=env_count)
    print("round-off envelope at t = 1000:", env, "per-drop sums", env_sum, "counts", env_count)


def offnode_free_runs():
    """FP64 fields phi, rho, u after each 2D case's steps in ``workloads.offnode_parity_cases``
    (drops off the lattice nodes), and the oracle's own round-off envelope there: the
    largest change of each field when phi0 is perturbed by a relative 1e-15."""
    out = {}
    for name, (p, phi0, u0, steps) in W.offnode_parity_cases().items():
        if p.lattice != "D2Q9":
            continue                      # the 3D column is run by the test itself
        m = Model(p).init(phi0, u0)
        m.step(steps)
        F = m.fields()
        rng = np.random.default_rng(1)
        q = Model(p).init(phi0 * (1.0 + 1e-15 * rng.standard_normal(phi0.shape)), u0)
        q.step(steps)
        G = q.fields()
        for k in ("phi", "rho", "u"):
            out[f"{name}__{k}"] = F[k]
            out[f"{name}__env_{k}"] = float(np.max(np.abs(F[k] - G[k])))
        out[f"{name}__steps"] = steps
        print(name, {k: out[f"{name}__env_{k}"] for k in ("phi", "rho", "u")}, flush=True)
    np.savez_compressed(os.path.join(HERE, "offnode_fp64_free_runs.npz"), **out)


if __name__ == "__main__":
    which = sys.argv[1:] or ["two_droplets_1000", "offnode_free_runs"]
    if "two_droplets_1000" in which:
        two_droplets_1000()
    if "offnode_free_runs" in which:
        offnode_free_runs()
    print("wrote", HERE)
