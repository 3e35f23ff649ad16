"""Write the oracle's reference gradients for the full-size drop-in-shear case.

The case is the 512 x 256 D2Q9 FP64 drop in shear (walls moving -+0.02, R = 48, density
ratio 1, Ca = 0.2, Re = 0.5) over 4000 steps.  The objective is the deformation D of the
drop (second-moment definition) after the last step.  Its derivatives with respect to the
surface tension sigma, the mobility M, and the initial field phi0 along ten directions
are taken by the complex step of the oracle (``oracle.gradient.complex_step``).  That
step is exact for the discrete map and uses the same normal cut (tau = 0.3) as the GPU
adjoint.  The directions are d_k = z_k 4 phi0 (1 - phi0), with z_k the k-th standard
normal field drawn from PCG64(1).

Every value comes from the CPU oracle run on the seeded inputs of ``workloads``; nothing
comes from the HIP library.  Each of the twelve complex runs takes about 40 minutes on
one core, so they run (with the forward run) in parallel worker processes:

    python tests/golden/make_adjoint_golden.py [workers]
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle import gradient as OG  # noqa: E402

NSTEPS = 4000
NDIR = 10
OUT = os.path.join(HERE, "shear512x256_adjoint_t4000.npz")


def directions(phi0):
    rng = np.random.Generator(np.random.PCG64(1))
    return [rng.standard_normal(phi0.shape) * 4.0 * phi0 * (1.0 - phi0) for _ in range(NDIR)]


def job(k):
    """k = -1: D itself; 0: d/dsigma, 1: d/dmobility, 2 + j: d/dphi0 along direction j;
    returns (k, value, seconds)."""
    try:
        from threadpoolctl import threadpool_limits
        limit = threadpool_limits(limits=1)
    except Exception:   # pragma: no cover
        limit = None
    p, phi0, u0 = W.shear_droplet("fp64")
    t0 = time.time()
    if k == -1:
        v = OG.derived_after(p, phi0, u0, NSTEPS)
    elif k == 0:
        v = OG.complex_step(p, phi0, u0, NSTEPS, "sigma")
    elif k == 1:
        v = OG.complex_step(p, phi0, u0, NSTEPS, "mobility")
    else:
        v = OG.complex_step(p, phi0, u0, NSTEPS, "phi0", direction=directions(phi0)[k - 2])
    if limit is not None:
        limit.__exit__(None, None, None)
    return k, float(v[0, 4]), time.time() - t0


def main():
    import multiprocessing as mp
    workers = int(sys.argv[1]) if len(sys.argv) > 1 else 6
    for var in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[var] = "1"
    res = {}
    with mp.get_context("fork").Pool(workers) as pool:
        for k, val, sec in pool.imap_unordered(job, range(-1, 2 + NDIR)):
            res[k] = val
            print(f"job {k}: {val:.15e} ({sec:.0f} s)", flush=True)
    np.savez(OUT, D=np.float64(res[-1]), dD_dsigma=np.float64(res[0]), dD_dM=np.float64(res[1]),
             dD_dphi0_dir=np.array([res[2 + j] for j in range(NDIR)]), nsteps=np.int64(NSTEPS),
             normal_tau=np.float64(OG.NORMAL_TAU))
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main()
