"""Writes the oracle's full-size results for the GPU full-size parity tests.

Calls only ``oracle/`` (and ``synth`` for the seeded inputs).  For each
workload (seed 0) the FP64 oracle sets up the two-level method and solves
with PCG to a 1e-10 residual reduction; the per-subdomain step
(``oracle.geneo.local_setup``) runs in a pool of forked processes, which
changes nothing in the arithmetic.  Output ``fullsize_<workload>_seed0.npz``
holds the PCG solution, the reference solution (that one refined twice with
residuals in extended precision), the iteration count, the CG-Lanczos
condition estimate, the coarse dimension and the per-subdomain eigenvector
counts.

    python tests/golden/make_fullsize_golden.py grf_512 [layers_96 laminate_128x32x24]

grf_512 (512^2 Darcy) takes a few minutes, layers_96 (96^3) and the laminate
about an hour each on 8 cores.
"""
import multiprocessing as mp
import os
import sys
import time

# one BLAS thread per pool process (set before numpy loads its BLAS)
os.environ.setdefault("OMP_NUM_THREADS", "1")
os.environ.setdefault("OPENBLAS_NUM_THREADS", os.environ["OMP_NUM_THREADS"])

import numpy as np  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import decomp, fem, geneo, pcg  # noqa: E402

_CTX = {}


def _local(j):
    c = _CTX
    return geneo.local_setup(c["prob"], c["A"], c["subs"][j], c["nev"], c["tau"], c["nev_max"],
                             True, False, "auto")


def run(name, procs):
    prob = synth.CONFIGS[name](seed=0)
    t0 = time.time()
    A, b = fem.assemble(prob)
    subs, _ = decomp.build(prob)
    nev, tau, nev_max = prob.nev, prob.tau, prob.nev_max
    if tau is not None:
        nev = None
    _CTX.update(prob=prob, A=A, subs=subs, nev=nev, tau=tau, nev_max=nev_max)
    with mp.get_context("fork").Pool(procs) as pool:
        locs = pool.map(_local, range(len(subs)), chunksize=1)
    g = geneo.setup(prob, A=A, subs=subs, nev=nev, tau=tau, nev_max=nev_max, locs=locs)
    t1 = time.time()
    res = pcg.pcg(A, b, g.apply, rtol=prob.rtol, maxit=prob.maxit)
    t2 = time.time()
    assert res.converged
    kappa = pcg.kappa_estimate(res.alphas, res.betas)
    # reference solution: two refinement steps with extended-precision
    # residuals and PCG corrections to 1e-6
    x_ref = pcg.refine(A, b, res.x, lambda r: pcg.pcg(A, r, g.apply, rtol=1e-6,
                                                      maxit=prob.maxit).x, steps=2)
    t3 = time.time()
    err = np.linalg.norm(res.x - x_ref) / np.linalg.norm(x_ref)
    print("%s: setup %.1f s, pcg %.1f s, refinement %.1f s, iters %d, kappa %.3f, nc %d, "
          "plain vs refined %.2e" % (name, t1 - t0, t2 - t1, t3 - t2, res.iters, kappa, g.nc, err),
          flush=True)
    np.savez_compressed(os.path.join(HERE, "fullsize_%s_seed0.npz" % name),
                        x=res.x, x_ref=x_ref, iters=res.iters, kappa=kappa, nc=g.nc,
                        m=np.asarray(g.m, dtype=np.int32), rtol=prob.rtol,
                        relres=res.relres)


def main():
    names = sys.argv[1:] or ["grf_512"]
    procs = int(os.environ.get("GOLDEN_PROCS", "8"))
    for name in names:
        run(name, procs)


if __name__ == "__main__":
    main()
