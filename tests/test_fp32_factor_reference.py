"""Pins of the FP32 local-factor reference that the serving test compares
mixed-precision requests with (the iteration count decided in the request's
precision): on a small channels problem, every factor is lower triangular,
reproduces its Dirichlet matrix to FP32 accuracy (L L^T = A_D within
n u_32 |L| |L|^T, entrywise) and is the FP64 oracle's factor within the
rounding of an FP32 factorisation (u_32 kappa); the oracle preconditioner
built from them still converges."""
import numpy as np

import synth
from oracle import fem, geneo, pcg
from test_gpu_serving import _fp32_local_factors

U32 = 2.0 ** -24


def test_fp32_factors_reproduce_the_dirichlet_matrices():
    p = synth.channels_2d(seed=6, n=32, parts=2, n_channels=3, nev=4, precision="mixed")
    A, b = fem.assemble(p)
    g = geneo.setup(p, A=A)
    facs = _fp32_local_factors(g, A)
    assert len(facs) == len(g.subs)
    for s, L, L64 in zip(g.subs, facs, g.chol):
        AD = geneo.dirichlet_matrix(A, s)
        n = len(AD)
        assert np.array_equal(L, np.tril(L))
        # scaled backward error of a Cholesky factorisation in FP32
        d = 1.0 / np.sqrt(np.diag(AD))
        Ls = d[:, None] * L                      # the factor of the scaled matrix
        S = d[:, None] * AD * d[None, :]
        err = np.abs(Ls @ Ls.T - S)
        bound = 4 * n * U32 * (np.abs(Ls) @ np.abs(Ls).T) + 4 * U32
        assert np.all(err <= bound)
        kappa = np.linalg.cond(S)
        rel = np.linalg.norm(Ls - d[:, None] * L64) / np.linalg.norm(d[:, None] * L64)
        assert 0 < rel <= 10 * n * U32 * kappa
    g.chol = facs
    r = pcg.pcg(A, b, g.apply, rtol=1e-10)
    assert r.converged
