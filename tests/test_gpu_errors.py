"""Failure handling of the device path, forced from the host with valid
inputs (every kernel still runs to its normal exit):

* a local Dirichlet matrix that is not SPD (one diagonal entry of A made
  negative inside subdomain 0): the factorisation records the failed pivot
  and the setup returns GENEO_ERR_LOCAL_NOT_SPD, in FP64 and in mixed mode
  (where the FP32 pivot test fails first and the FP64 refactor then fails);
* a shifted matrix A_N - sigma B that is not SPD (one diagonal entry of a
  local Neumann matrix made strongly negative inside subdomain 1): the
  setup returns GENEO_ERR_SHIFT_NOT_SPD (the pivot tests are read back
  while the first eigen sweeps are already queued);
* PCG stopped by maxit: GENEO_ERR_MAXIT with the iterations done reported;
* eigen sweeps stopped by eig_maxit: GENEO_ERR_EIGEN_NOCONV.

After each error the library keeps working: a correct setup and apply
follow on the same device.
"""
import numpy as np
import pytest
import torch

import synth
from gpu_common import gpu_apply, gpu_assemble, gpu_setup, need_gpu, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def small():
    need_gpu()
    prob = synth.grf_2d(seed=3, n=48, parts=2, ovl=2, inclusions=2)
    return prob, gpu_assemble(prob)


def _healthy(prob, sysm):
    h = gpu_setup(sysm, prob, precision=1)
    z = gpu_apply(h, sysm, np.ones(prob.ndof))
    h.close()
    assert np.all(np.isfinite(z))


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_local_matrix_not_spd(small, precision):
    from paper_1906_10944_amd import geneo as G
    prob, sysm = small
    # an interior dof of subdomain 0 (in D_0 only), its diagonal made negative
    sp_ = sysm.sub_ptr.cpu().numpy()
    idx = sysm.sub_idx.cpu().numpy()
    fl = sysm.sub_flags.cpu().numpy()
    seg = slice(sp_[0], sp_[1])
    cand = idx[seg][(fl[seg] & 1).astype(bool)]
    g = int(cand[len(cand) // 2])
    rp = sysm.A_rowptr.cpu().numpy()
    col = sysm.A_col.cpu().numpy()
    pos = rp[g] + int(np.nonzero(col[rp[g]:rp[g + 1]] == g)[0][0])
    saved = sysm.A_val[pos].item()
    sysm.A_val[pos] = -abs(saved)
    torch.cuda.synchronize()
    try:
        with pytest.raises(G.GeneoError) as e:
            gpu_setup(sysm, prob, precision=precision)
        say("[errors]", e.value)
        assert e.value.code == G.GENEO_ERR_LOCAL_NOT_SPD
        assert "subdomain 0" in str(e.value)
    finally:
        sysm.A_val[pos] = saved
        torch.cuda.synchronize()
    _healthy(prob, sysm)


def test_shifted_matrix_not_spd(small):
    from paper_1906_10944_amd import geneo as G
    prob, sysm = small
    sp_ = sysm.sub_ptr.cpu().numpy()
    rp = sysm.loc_rowptr.cpu().numpy()
    col = sysm.loc_col.cpu().numpy()
    r0, n = int(sp_[1]), int(sp_[2] - sp_[1])
    r = n // 2
    pos = int(rp[r0 + r]) + int(np.nonzero(col[rp[r0 + r]:rp[r0 + r + 1]] == r)[0][0])
    saved = sysm.an_val[pos].item()
    sysm.an_val[pos] = -1e3 * abs(saved)
    torch.cuda.synchronize()
    try:
        for precision in (1, 0):
            with pytest.raises(G.GeneoError) as e:
                gpu_setup(sysm, prob, precision=precision)
            say("[errors]", e.value)
            assert e.value.code == G.GENEO_ERR_SHIFT_NOT_SPD
            assert "subdomain 1" in str(e.value)
    finally:
        sysm.an_val[pos] = saved
        torch.cuda.synchronize()
    _healthy(prob, sysm)


def test_pcg_maxit(small):
    from paper_1906_10944_amd import geneo as G
    prob, sysm = small
    h = gpu_setup(sysm, prob, precision=1)
    x = torch.zeros_like(sysm.b)
    with pytest.raises(G.GeneoError) as e:
        G.pcg_solve(sysm.csr(), h, sysm.b, x, rtol=1e-10, maxit=3)
    assert e.value.code == G.GENEO_ERR_MAXIT
    info = G.pcg_solve(sysm.csr(), h, sysm.b, x, rtol=1e-10, maxit=3, check=False)
    assert info["iters"] == 3 and not info["converged"] and info["relres"] > 1e-10
    h.close()
    _healthy(prob, sysm)


def test_eigen_no_convergence(small):
    from paper_1906_10944_amd import geneo as G
    prob, sysm = small
    with pytest.raises(G.GeneoError) as e:
        gpu_setup(sysm, prob, precision=1, eig_maxit=1)
    say("[errors]", e.value)
    assert e.value.code == G.GENEO_ERR_EIGEN_NOCONV
    _healthy(prob, sysm)


def test_chebyshev_degree_above_six_is_rejected(small):
    """Degrees above 6 are refused before any work: the filter would let a
    floating subdomain's kernel modes outgrow the smallest wanted Ritz
    vectors by more than 1/u."""
    from paper_1906_10944_amd import geneo as G
    prob, sysm = small
    with pytest.raises(G.GeneoError) as e:
        gpu_setup(sysm, prob, precision=1, eig_cheb=7)
    assert e.value.code == G.GENEO_ERR_ARG and "eig_cheb" in str(e.value)
    h = gpu_setup(sysm, prob, precision=1, eig_cheb=6)
    h.close()
    _healthy(prob, sysm)


def test_pcg_start_cases(small):
    """The PCG start runs on the device: a zero right-hand side and an initial
    guess that already meets the tolerance both stop before the first
    iteration (converged, x untouched); the iterations run in captured
    chunks of 8 and 2, and every iteration limit, multiple of neither or
    not, stops exactly there."""
    import torch
    from paper_1906_10944_amd import geneo as G
    prob, sysm = small
    h = gpu_setup(sysm, prob, precision=1)
    A = sysm.csr()
    # b = 0, x0 = 0: nothing to do
    zero = torch.zeros_like(sysm.b)
    x = torch.zeros_like(sysm.b)
    info = G.pcg_solve(A, h, zero, x, rtol=1e-10, maxit=100)
    assert info["iters"] == 0 and info["converged"] and info["relres"] == 0.0
    assert not torch.any(x)
    # full solve from zero
    x = torch.zeros_like(sysm.b)
    full = G.pcg_solve(A, h, sysm.b, x, rtol=1e-10, maxit=500)
    assert full["converged"] and full["iters"] > 2
    # restart from the solution with a tolerance its true residual meets
    # (the recurrence residual reached 1e-10, the true one has an FP64 floor)
    x2 = x.clone()
    again = G.pcg_solve(A, h, sysm.b, x2, rtol=1e-5, maxit=500)
    say("[pcg start] full", full["iters"], "restart", again["iters"], again["relres"])
    assert again["converged"] and again["iters"] == 0
    assert torch.equal(x2, x)
    # each iteration limit below the full count stops exactly there
    for mx in (1, 2, 3, 7, 9, 10, full["iters"] - 1):
        xm = torch.zeros_like(sysm.b)
        part = G.pcg_solve(A, h, sysm.b, xm, rtol=1e-10, maxit=mx, check=False)
        assert part["iters"] == mx and not part["converged"], (mx, part)
    h.close()


def test_coarse_matrix_not_spd_repeated_subdomain(small):
    """Def. 2: A_H = Z^T A Z is SPD only for independent basis vectors.  A
    subdomain listed twice (valid index lists and local matrices, the copy
    appended at the end) gives every one of its basis vectors twice, so A_H
    is singular and the setup returns GENEO_ERR_COARSE_NOT_SPD."""
    from paper_1906_10944_amd import geneo as G
    prob, sysm = small
    sp_ = sysm.sub_ptr.cpu().numpy().astype(np.int64)
    rp = sysm.loc_rowptr.cpu().numpy().astype(np.int64)
    r0, r1 = int(sp_[0]), int(sp_[1])
    nloc, nnz = int(sp_[-1]), int(rp[-1])
    e0, e1 = int(rp[r0]), int(rp[r1])
    dev = sysm.sub_ptr.device
    i32 = lambda a: torch.as_tensor(np.asarray(a, dtype=np.int32), device=dev)
    sub_ptr = i32(np.concatenate([sp_, [nloc + (r1 - r0)]]))
    sub_idx = torch.cat([sysm.sub_idx, sysm.sub_idx[r0:r1]])
    flags = torch.cat([sysm.sub_flags, sysm.sub_flags[r0:r1]])
    pou = torch.cat([sysm.pou, sysm.pou[r0:r1]])
    loc_rowptr = i32(np.concatenate([rp, nnz + (rp[r0 + 1:r1 + 1] - e0)]))
    loc_col = torch.cat([sysm.loc_col, sysm.loc_col[e0:e1]])
    an = torch.cat([sysm.an_val, sysm.an_val[e0:e1]])
    ao = torch.cat([sysm.ao_val, sysm.ao_val[e0:e1]])
    torch.cuda.synchronize()
    subs = G.Subdomains(prob.nsub + 1, nloc + (r1 - r0), sub_ptr.data_ptr(), sub_idx.data_ptr(),
                        flags.data_ptr(), pou.data_ptr())
    An = G.CsrBatch(loc_rowptr.data_ptr(), loc_col.data_ptr(), an.data_ptr())
    Ao = G.CsrBatch(loc_rowptr.data_ptr(), loc_col.data_ptr(), ao.data_ptr())
    # a fixed count m at the widest gap of subdomain 0's spectrum (oracle),
    # so that both copies select the same invariant subspace
    from oracle import decomp, geneo as og
    s0 = decomp.build(prob)[0][0]
    AN, Ao_ = og.local_matrices(prob, s0)
    lam = og.generalized_eigen(AN, s0.mu[:, None] * Ao_ * s0.mu[None, :]).lam
    m = 1 + int(np.argmax([(lam[k + 1] - lam[k]) / lam[k + 1] for k in range(6)]))
    say("[errors] repeated subdomain, m =", m, "lam", lam[:m + 1])
    # both copies converged far below the rounding level of the pivot test
    # (their start blocks differ, so their basis vectors agree only to about
    # the eigen tolerance; at 1e-8 the Schur pivot of the copy is ~1e-16)
    for precision in (0, 1):
        opts = G.opts_from_problem(prob, precision=precision, tau=0.0, nev=m, eig_tol=1e-12)
        with pytest.raises(G.GeneoError) as e:
            G.geneo_setup(sysm.csr(), subs, An, Ao, opts)
        say("[errors]", e.value)
        assert e.value.code == G.GENEO_ERR_COARSE_NOT_SPD
    # the same lists without the copy are fine
    _healthy(prob, sysm)
