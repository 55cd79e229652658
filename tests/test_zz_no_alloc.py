"""pcg_solve_noalloc (the allocation-free variant of pcg_solve, for callers
that cannot allocate) against pcg_solve through the C ABI: two calls in a
row on the same GPU, the second on a smaller problem, each compared with
pcg_solve on the same handle and right-hand side (the same kernels in the
same order: the solutions agree to the bit, iterations and residuals are
equal), and the solutions against the FP64 oracle's (1e-8, iterations
+-2).  Sizes beyond the fixed array's limits are rejected."""
import numpy as np
import pytest
import torch

import synth
from gpu_common import gpu_assemble, gpu_setup, need_gpu, say
from oracle import fem, geneo, pcg

pytestmark = pytest.mark.gpu


def _solve_both(prob, nrhs, refine):
    from paper_1906_10944_amd import geneo as G
    sysm = gpu_assemble(prob)
    h = gpu_setup(sysm, prob, precision=1 if prob.precision == "mixed" else 0, refine=refine)
    n = prob.ndof
    rng = np.random.Generator(np.random.PCG64(prob.ndof))
    B = np.stack([sysm.b.cpu().numpy()] + [rng.normal(size=n) * (sysm.b.cpu().numpy() != 0)
                                          for _ in range(nrhs - 1)])
    b = torch.as_tensor(B.ravel(), dtype=torch.float64, device="cuda")
    x1 = torch.zeros_like(b)
    x2 = torch.zeros_like(b)
    i1 = G.pcg_solve(sysm.csr(), h, b, x1, rtol=1e-10, maxit=2000, nrhs=nrhs)
    i2 = G.pcg_solve_noalloc(sysm.csr(), h, b, x2, rtol=1e-10, maxit=2000, nrhs=nrhs)
    torch.cuda.synchronize()
    i1 = i1 if isinstance(i1, list) else [i1]
    i2 = i2 if isinstance(i2, list) else [i2]
    return sysm, h, B, x1.cpu().numpy().reshape(nrhs, n), x2.cpu().numpy().reshape(nrhs, n), i1, i2


def test_noalloc_matches_pcg_solve_two_calls_second_smaller():
    need_gpu()
    from paper_1906_10944_amd import geneo as G
    probs = [synth.grf_2d(seed=5, n=96, parts=3, ovl=2, inclusions=3),
             synth.channels_2d(1, n=32, parts=2, n_channels=3, nev=4)]
    # the first handle refines its solutions once (the correction solve and
    # its residual also live in the fixed array), the second does not
    for prob, nrhs, refine in zip(probs, (2, 1), (1, 0)):
        say("[noalloc]", prob.name, "ndof", prob.ndof, "nrhs", nrhs, "refine", refine)
        sysm, h, B, x1, x2, i1, i2 = _solve_both(prob, nrhs, refine)
        for k in range(nrhs):
            say("   rhs %d: pcg_solve it %d (+%d) relres %.3e | noalloc it %d (+%d) relres %.3e | "
                "max |dx| %.3e" % (k, i1[k]["iters"], i1[k]["refine_iters"], i1[k]["relres"],
                                   i2[k]["iters"], i2[k]["refine_iters"], i2[k]["relres"],
                                   np.abs(x1[k] - x2[k]).max()))
            assert i2[k]["converged"] and i2[k]["iters"] == i1[k]["iters"]
            assert i2[k]["refine_iters"] == i1[k]["refine_iters"]
            assert (i1[k]["refine_iters"] > 0) == (refine > 0)
            assert i2[k]["relres"] == i1[k]["relres"]
            assert i2[k]["true_relres"] == i1[k]["true_relres"]
            assert i2[k]["kappa_est"] == pytest.approx(i1[k]["kappa_est"], rel=1e-12)
            assert np.array_equal(x1[k], x2[k])
        # the oracle's solution of the first right-hand side
        A, b = fem.assemble(prob)
        g = geneo.setup(prob, A=A)
        ref = pcg.pcg(A, b, g.apply, rtol=1e-10)
        assert abs(i2[0]["iters"] - ref.iters) <= 2
        assert np.linalg.norm(x2[0] - ref.x) <= 1e-8 * np.linalg.norm(ref.x)
        h.close()


def test_noalloc_rejects_sizes_beyond_its_array():
    need_gpu()
    from paper_1906_10944_amd import geneo as G
    prob = synth.channels_2d(1, n=32, parts=2, n_channels=3, nev=4)
    sysm = gpu_assemble(prob)
    h = gpu_setup(sysm, prob)
    x = torch.zeros_like(sysm.b)
    with pytest.raises(G.GeneoError) as e:
        G.pcg_solve_noalloc(sysm.csr(), h, sysm.b, x, rtol=1e-10, maxit=5000)
    assert e.value.code == G.GENEO_ERR_ARG and "maxit <= 4096" in str(e.value)
    h.close()
    # 1025^2 = 1,050,625 dofs > 2^20
    big = synth.grf_2d(seed=1, n=1024, parts=32, ovl=2, inclusions=4)
    sysm = gpu_assemble(big)
    h = gpu_setup(sysm, big, precision=1)
    x = torch.zeros_like(sysm.b)
    with pytest.raises(G.GeneoError) as e:
        G.pcg_solve_noalloc(sysm.csr(), h, sysm.b, x, rtol=1e-10, maxit=100)
    assert e.value.code == G.GENEO_ERR_ARG and "n <= 1048576" in str(e.value)
    h.close()
