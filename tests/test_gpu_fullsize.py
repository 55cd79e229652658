"""Parity at the full size of the bench workload: 512^2 Darcy (263,169 dofs,
256 subdomains, seed 0), with the options and launch configuration the
bench times.

The oracle does not run the whole method at this size in seconds, so it
checks what it can compute one subdomain at a time, plus properties that
hold at any size:

* the whole assembled matrix and load vector;
* the one-level apply (FP64 and mixed) on residuals supported in the
  Dirichlet sets of sampled subdomains: only those subdomains and their
  neighbours contribute, and the oracle factors just those;
* eigenvalue counts, eigenvalues and coarse-basis spans of sampled
  subdomains;
* the Galerkin identity A_H = Z^T A Z for the whole coarse matrix the
  device factors (with the oracle's A);
* PCG: convergence, the true residual through the oracle's A, and the
  symmetry of the operator the device applies;
* the whole solution and the iteration count, FP64 and mixed form, against
  the oracle's full run stored by ``golden/make_fullsize_golden.py``
  (iterations within +-2, solution within 1e-8 relative).
"""
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import synth
from gpu_common import (csr_to_scipy, gpu_apply, gpu_assemble, gpu_pcg, gpu_setup, need_gpu, say,
                        kappa_spd, span_contamination)
from oracle import decomp, fem, geneo

pytestmark = pytest.mark.gpu

# spread over the 16 x 16 partition: corners, edges and interior; 135 holds
# a floating-free interior block, the others touch the physical boundary
SAMPLE = [0, 15, 135, 170, 240, 255]
U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def full():
    need_gpu()
    prob = synth.CONFIGS["grf_512"](seed=0)
    say("[fullsize] ndof", prob.ndof, "nsub", prob.nsub)
    A, b = fem.assemble(prob)
    subs, _ = decomp.build(prob)
    sysm = gpu_assemble(prob)
    return prob, A, b, subs, sysm


def _patch_residual(prob, subs, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    r = np.zeros(prob.ndof)
    for j in SAMPLE:
        idx = subs[j].dofs[subs[j].dmask]
        r[idx] = rng.normal(size=len(idx))
    return r


def _one_level_oracle(A, subs, r, unit):
    """Sum over the subdomains whose D_k meets supp(r) of R_k^T A_k^{-1} R_k r,
    and the forward-error bound of that sum when subdomain k is solved in
    precision unit[k]: sum_k 10 u_k kappa_k |A_k^{-1} R_k r|, with kappa_k the
    condition number of the diagonally scaled A_k (the device factors the
    scaled matrix)."""
    z = np.zeros_like(r)
    bound, used, kmax = 0.0, 0, 1.0
    for s in subs:
        idx = s.dofs[s.dmask]
        if not len(idx) or not np.any(r[idx]):
            continue
        AD = geneo.dirichlet_matrix(A, s)
        zk = sla.cho_solve(sla.cho_factor(AD, lower=True), r[idx])
        z[idx] += zk
        d = 1.0 / np.sqrt(np.diag(AD))
        ev = np.linalg.eigvalsh(d[:, None] * AD * d[None, :])
        kappa = ev[-1] / ev[0]
        bound += 10 * unit[s.j] * kappa * np.linalg.norm(zk)
        kmax = max(kmax, kappa)
        used += 1
    return z, bound, used, kmax


def test_fullsize_assembly(full):
    prob, A, b, subs, sysm = full
    # the device keeps the full stencil pattern (explicit zeros where the
    # Dirichlet elimination removed couplings): compare values
    Ag = csr_to_scipy(sysm.A_rowptr, sysm.A_col, sysm.A_val, prob.ndof)
    assert abs(Ag - A).max() <= 1e-13 * abs(A).max()
    bg = sysm.b.cpu().numpy()
    assert np.allclose(bg, b, rtol=1e-14, atol=1e-14 * abs(b).max())


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_fullsize_one_level_apply(full, precision):
    prob, A, b, subs, sysm = full
    from paper_1906_10944_amd import geneo as G
    r = _patch_residual(prob, subs, 21)
    h = gpu_setup(sysm, prob, precision=precision, coarse=0)
    z = gpu_apply(h, sysm, r)
    z2 = gpu_apply(h, sysm, r)  # the other walk order over the subdomains
    fp64 = G.geneo_get_local_precision(h, len(subs))
    h.close()
    assert np.array_equal(z, z2)
    if precision == 0:
        assert fp64.all()
    # each subdomain is solved with an inverse formed from a backward-stable
    # factor of its scaled matrix, in FP64 or (mixed, pivot test passed) FP32:
    # forward error O(u_k kappa_k), so the sum is within sum_k 10 u_k kappa_k
    # |z_k| of the oracle's FP64 solves (floor 1e-12 relative)
    unit = np.where(fp64 != 0, np.finfo(float).eps / 2, U32)
    zo, bound, used, kmax = _one_level_oracle(A, subs, r, unit)
    diff = np.linalg.norm(z - zo)
    tol = max(1e-12 * np.linalg.norm(zo), bound)
    say("[fullsize one-level %s] %d subdomains (%d FP64), max kappa %.3e, rel diff %.3e, "
        "bound %.3e" % ("fp64" if precision == 0 else "mixed", used, int(fp64.sum()), kmax,
                        diff / np.linalg.norm(zo), tol / np.linalg.norm(zo)))
    assert diff <= tol


@pytest.fixture(scope="module")
def bench_handle(full):
    prob, A, b, subs, sysm = full
    h = gpu_setup(sysm, prob, precision=1)   # the bench's configuration
    yield h
    h.close()


def test_fullsize_eigen_and_basis(full, bench_handle):
    prob, A, b, subs, sysm = full
    from paper_1906_10944_amd import geneo as G
    h = bench_handle
    info = G.geneo_get_setup_info(h)
    m, lam = G.geneo_get_eigenvalues(h, len(subs))
    zoff, z, _ = G.geneo_get_coarse(h, len(subs), with_ah=False)
    for j in SAMPLE:
        s = subs[j]
        AN, Ao = geneo.local_matrices(prob, s)
        ev = geneo.generalized_eigen(AN, s.mu[:, None] * Ao * s.mu[None, :])
        mj = geneo.select_count(ev.lam, nev=prob.nev, tau=prob.tau, nev_max=prob.nev_max)
        say("[fullsize eigen] subdomain", j, "m", m[j], "oracle", mj, ev.lam[:mj])
        assert m[j] == mj
        for c in range(mj):
            assert lam[j, c] == pytest.approx(ev.lam[c], rel=1e-8, abs=1e-11), (j, c)
        if mj == 0:
            continue
        Zg = z[zoff[j]:zoff[j + 1]].reshape(len(s.dofs), mj)
        kC = kappa_spd(AN + 1e-3 * (s.mu[:, None] * Ao * s.mu[None, :]))
        res = span_contamination(s.mu, ev.lam, ev.P, Zg, info["eig_max_resid"], kC)
        if res is not None:
            say("   span weight outside %.2e bound %.2e" % res)
            assert res[0] <= res[1], (j, res)


def test_fullsize_coarse_matrix_is_galerkin_product(full, bench_handle):
    prob, A, b, subs, sysm = full
    from paper_1906_10944_amd import geneo as G
    h = bench_handle
    m, _ = G.geneo_get_eigenvalues(h, len(subs))
    zoff, z, ah = G.geneo_get_coarse(h, len(subs))
    rows, cidx, vals = [], [], []
    off = 0
    for s in subs:
        mj = m[s.j]
        blk = z[zoff[s.j]:zoff[s.j + 1]].reshape(len(s.dofs), mj)
        r_, c_ = np.nonzero(blk)
        rows.append(s.dofs[r_])
        cidx.append(c_ + off)
        vals.append(blk[r_, c_])
        off += mj
    Z = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cidx))),
                      shape=(prob.ndof, off))
    AH = (Z.T @ (A @ Z)).toarray()
    say("[fullsize galerkin] n_c", off)
    assert ah.shape == AH.shape
    assert np.abs(ah - AH).max() <= 1e-12 * np.abs(AH).max()
    assert np.allclose(np.sqrt(np.asarray(Z.multiply(Z).sum(axis=0))).ravel(), 1.0, rtol=1e-12)


def test_fullsize_pcg_and_operator(full, bench_handle):
    prob, A, b, subs, sysm = full
    h = bench_handle
    x, inf = gpu_pcg(h, sysm, rtol=prob.rtol, maxit=prob.maxit)
    true_rel = np.linalg.norm(b - A @ x) / np.linalg.norm(b)
    say("[fullsize pcg] iters", inf["iters"], "relres %.3e true %.3e kappa %.1f" %
        (inf["relres"], true_rel, inf["kappa_est"]))
    assert inf["converged"] and inf["relres"] <= prob.rtol
    # the true residual of this problem has an FP64 floor near 1e-6 (its
    # conditioning); the recurrence residual is what reaches rtol
    assert true_rel <= 1e-5
    assert 1.0 < inf["kappa_est"] < 1e3
    # the operator is symmetric: y^T M^{-1} r and r^T M^{-1} y use the same
    # stored inverses and differ only by the rounding of the FP64 sums,
    # |y^T dz| <= gamma_n |y|^T |S| |r| with n ~ 1.4e3 terms per entry; for
    # these smooth inverses |S| |r| exceeds |S r| by up to ~1e3 (random signs
    # of r cancel in S r): 1.4e3 * 1.1e-16 * 1e3 ~ 2e-10 of |y| |M^{-1} r|
    rng = np.random.Generator(np.random.PCG64(31))
    r, y = rng.normal(size=prob.ndof), rng.normal(size=prob.ndof)
    zr, zy = gpu_apply(h, sysm, r), gpu_apply(h, sysm, y)
    asym = abs(y @ zr - r @ zy) / (np.linalg.norm(y) * np.linalg.norm(zr))
    say("[fullsize operator] relative asymmetry %.2e" % asym)
    assert asym <= 1e-9
    assert r @ zr > 0 and y @ zy > 0


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "fullsize_grf_512_seed0.npz")


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_fullsize_solution_matches_oracle_run(full, precision):
    """The oracle's whole FP64 run (setup and PCG to 1e-10, stored by
    golden/make_fullsize_golden.py, which calls only the oracle) against the
    device's, in the bench's launch configuration: iterations within +-2,
    the plain solution within 1e-8 of the oracle's, and the solution after
    two refinement steps within 1e-8 of the oracle's refined reference."""
    prob, A, b, subs, sysm = full
    gold = np.load(GOLDEN)
    from paper_1906_10944_amd import geneo as G
    h = gpu_setup(sysm, prob, precision=precision, refine=2)
    info = G.geneo_get_setup_info(h)
    m, _ = G.geneo_get_eigenvalues(h, len(subs))
    # the plain method on a handle without refinement
    h0 = gpu_setup(sysm, prob, precision=precision)
    x0, inf0 = gpu_pcg(h0, sysm, rtol=prob.rtol, maxit=prob.maxit)
    h0.close()
    x, inf = gpu_pcg(h, sysm, rtol=prob.rtol, maxit=prob.maxit)
    h.close()
    form = "fp64" if precision == 0 else "mixed"
    res = {}
    for key, xg, xo in (("plain", x0, gold["x"]), ("refined", x, gold["x_ref"])):
        res[key] = (np.linalg.norm(xg - xo) / np.linalg.norm(xo),
                    np.abs(xg - xo).max() / np.abs(xo).max())
    say("[fullsize solution %s] iters %d oracle %d, nc %d oracle %d, plain rel diff %.3e "
        "max-abs %.3e, refined (+%d its) rel diff %.3e max-abs %.3e, true residual %.2e" %
        (form, inf0["iters"], int(gold["iters"]), info["nc"], int(gold["nc"]), res["plain"][0],
         res["plain"][1], inf["refine_iters"], res["refined"][0], res["refined"][1],
         inf["true_relres"]))
    assert np.array_equal(m, gold["m"])
    assert abs(inf0["iters"] - int(gold["iters"])) <= 2 and inf["iters"] == inf0["iters"]
    for key in res:
        assert res[key][0] <= 1e-8 and res[key][1] <= 1e-8, (key, res[key])
