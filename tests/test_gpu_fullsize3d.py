"""Parity at full size for the two 3D workloads, one GPU, the bench's options:

* 96^3 layered Darcy (912,673 dofs, 8^3 subdomains of 12^3 elements,
  overlap 1, 12 eigenvectors, mixed precision);
* the clamped 128x32x24 laminate (319,275 dofs, 16x4x4 subdomains, overlap
  1, 24 eigenvectors: eigen block 48, mixed precision).

The oracle runs the whole method at these sizes only in hours (dense
generalised eigenproblems of order 3,375), so it checks, per workload:

* the whole assembled matrix and load vector;
* for two sampled subdomains -- one touching the Dirichlet boundary and one
  floating (no Dirichlet dof: A_N,j has the constant / the six rigid-body
  modes as kernel, the case the eigen stall rule and, for the laminate, the
  48-column eigen block serve) -- the eigenvector count, the eigenvalues
  (1e-8 relative) and the span of the coarse columns (the measured Ritz
  residual over the gap);
* the one-level apply on a residual supported in the samples' Dirichlet
  sets (only the subdomains meeting it contribute; the oracle factors just
  those), within sum_k 10 u_k kappa_k |z_k|;
* the Galerkin identity A_H = Z^T A Z for the whole coarse matrix, with the
  oracle's A;
* PCG to 1e-10: convergence, the true residual through the oracle's A, the
  Lanczos condition estimate, and the symmetry of the device's operator.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import synth
from gpu_common import (csr_to_scipy, gpu_apply, gpu_assemble, gpu_pcg, gpu_setup, need_gpu, say,
                        kappa_spd, span_contamination)
from oracle import decomp, fem, geneo

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
U64 = np.finfo(float).eps / 2

# (boundary subdomain, floating interior subdomain)
SAMPLES = {"layers_96": (0, 3 + 8 * (3 + 8 * 3)),              # corner; (3, 3, 3)
           "laminate_128x32x24": (0, 7 + 16 * (1 + 4 * 1)),  # clamped end; (7, 1, 1)
           "laminate_s20_32x8x6": (0, 2 + 4 * 1)}             # clamped end; (2, 1, 0)


@pytest.fixture(scope="module", params=["layers_96", "laminate_128x32x24",
                                        "laminate_s20_32x8x6"])
def big(request):
    need_gpu()
    prob = synth.CONFIGS[request.param](seed=0)
    say("[fullsize3d]", request.param, "ndof", prob.ndof, "nsub", prob.nsub)
    A, b = fem.assemble(prob)
    subs, _ = decomp.build(prob)
    sysm = gpu_assemble(prob)
    h = gpu_setup(sysm, prob, precision=1)
    from paper_1906_10944_amd import geneo as G
    info = G.geneo_get_setup_info(h)
    say("   setup: nc", info["nc"], "sweeps", info["eig_sweeps"], "block", info["eig_block"],
        "stalled", info["eig_stalled"], "max resid %.2e" % info["eig_max_resid"],
        "fp64 fallbacks", info["fallback_fp64"])
    yield request.param, prob, A, b, subs, sysm, h, info
    h.close()


def test_assembly(big):
    name, prob, A, b, subs, sysm, h, info = big
    Ag = csr_to_scipy(sysm.A_rowptr, sysm.A_col, sysm.A_val, prob.ndof)
    assert abs(Ag - A).max() <= 1e-13 * abs(A).max()
    assert np.allclose(sysm.b.cpu().numpy(), b, rtol=1e-14, atol=1e-14 * abs(b).max())


def test_sampled_eigen_and_span(big):
    name, prob, A, b, subs, sysm, h, info = big
    from paper_1906_10944_amd import geneo as G
    m, lam = G.geneo_get_eigenvalues(h, len(subs))
    zoff, z, _ = G.geneo_get_coarse(h, len(subs), with_ah=False)
    for j in SAMPLES[name]:
        s = subs[j]
        floating = not s.dirichlet.any()
        AN, Ao = geneo.local_matrices(prob, s)
        ev = geneo.generalized_eigen(AN, s.mu[:, None] * Ao * s.mu[None, :])
        mj = geneo.select_count(ev.lam, nev=prob.nev, tau=prob.tau, nev_max=prob.nev_max)
        say("[eigen %s] subdomain %d (%s, |N_j| %d): m %d oracle %d" %
            (name, j, "floating" if floating else "boundary", len(s.dofs), m[j], mj))
        say("   device", lam[j, :mj])
        say("   oracle", ev.lam[:mj])
        assert m[j] == mj
        if floating:   # kernel of A_N,j: constants (Darcy) or six rigid-body modes
            nker = 1 if prob.ncomp == 1 else 6
            assert np.all(np.abs(ev.lam[:nker]) < 1e-8) and ev.lam[nker] > 1e-8
        for c in range(mj):
            assert lam[j, c] == pytest.approx(ev.lam[c], rel=1e-8, abs=1e-11), (j, c)
        Zg = z[zoff[j]:zoff[j + 1]].reshape(len(s.dofs), mj)
        assert np.all(Zg[~s.dmask] == 0.0)
        kC = kappa_spd(AN + 1e-3 * (s.mu[:, None] * Ao * s.mu[None, :]))
        res = span_contamination(s.mu, ev.lam, ev.P, Zg, info["eig_max_resid"], kC)
        if res is not None:
            say("   span weight outside %.2e bound %.2e" % res)
            assert res[0] <= res[1], (j, res)


def _kappa_scaled(AD, L):
    """Condition number of D^{-1/2} A_D D^{-1/2} (D = diag A_D), by Lanczos
    on the matrix and on its inverse (through the Cholesky factor L of A_D)."""
    d = 1.0 / np.sqrt(np.diag(AD))
    S = d[:, None] * AD * d[None, :]
    n = len(d)
    hi = spla.eigsh(S, k=1, which="LA", return_eigenvectors=False, tol=1e-6)[0]
    inv = spla.LinearOperator((n, n), dtype=float,
                              matvec=lambda v: sla.cho_solve((L, True), v / d) / d)
    lo_inv = spla.eigsh(inv, k=1, which="LA", return_eigenvectors=False, tol=1e-6)[0]
    return hi * lo_inv


def test_one_level_apply_sampled(big):
    name, prob, A, b, subs, sysm, h, info = big
    from paper_1906_10944_amd import geneo as G
    rng = np.random.Generator(np.random.PCG64(41))
    r = np.zeros(prob.ndof)
    for j in SAMPLES[name]:
        idx = subs[j].dofs[subs[j].dmask]
        r[idx] = rng.normal(size=len(idx))
    h1 = gpu_setup(sysm, prob, precision=1, coarse=0)
    zg = gpu_apply(h1, sysm, r)
    fp64 = G.geneo_get_local_precision(h1, len(subs))
    h1.close()
    zo = np.zeros_like(r)
    bound, used = 0.0, 0
    for s in subs:
        idx = s.dofs[s.dmask]
        if not len(idx) or not np.any(r[idx]):
            continue
        AD = geneo.dirichlet_matrix(A, s)
        L = np.linalg.cholesky(AD)
        zk = sla.cho_solve((L, True), r[idx])
        zo[idx] += zk
        uk = U64 if fp64[s.j] else U32
        bound += 10 * uk * _kappa_scaled(AD, L) * np.linalg.norm(zk)
        used += 1
    diff = np.linalg.norm(zg - zo)
    tol = max(1e-12 * np.linalg.norm(zo), bound)
    say("[one-level %s] %d subdomains, rel diff %.3e, bound %.3e" %
        (name, used, diff / np.linalg.norm(zo), tol / np.linalg.norm(zo)))
    assert diff <= tol


def test_coarse_matrix_is_galerkin_product(big):
    name, prob, A, b, subs, sysm, h, info = big
    from paper_1906_10944_amd import geneo as G
    m, _ = G.geneo_get_eigenvalues(h, len(subs))
    zoff, z, ah = G.geneo_get_coarse(h, len(subs))
    rows, cidx, vals, off = [], [], [], 0
    for s in subs:
        mj = int(m[s.j])
        blk = z[zoff[s.j]:zoff[s.j + 1]].reshape(len(s.dofs), mj)
        r_, c_ = np.nonzero(blk)
        rows.append(s.dofs[r_])
        cidx.append(c_ + off)
        vals.append(blk[r_, c_])
        off += mj
    Z = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cidx))),
                      shape=(prob.ndof, off))
    AH = (Z.T @ (A @ Z)).toarray()
    say("[galerkin %s] n_c %d" % (name, off))
    assert ah.shape == AH.shape
    assert np.abs(ah - AH).max() <= 1e-12 * np.abs(AH).max()
    assert np.allclose(np.sqrt(np.asarray(Z.multiply(Z).sum(axis=0))).ravel(), 1.0, rtol=1e-12)


def test_pcg_and_operator(big):
    name, prob, A, b, subs, sysm, h, info = big
    x, inf = gpu_pcg(h, sysm, rtol=prob.rtol, maxit=prob.maxit)
    true_rel = np.linalg.norm(b - A @ x) / np.linalg.norm(b)
    say("[pcg %s] iters %d relres %.3e true %.3e kappa %.2f" %
        (name, inf["iters"], inf["relres"], true_rel, inf["kappa_est"]))
    assert inf["converged"] and inf["relres"] <= prob.rtol
    assert true_rel <= 1e-6
    assert 1.0 < inf["kappa_est"] < 1e3
    rng = np.random.Generator(np.random.PCG64(43))
    r, y = rng.normal(size=prob.ndof), rng.normal(size=prob.ndof)
    zr, zy = gpu_apply(h, sysm, r), gpu_apply(h, sysm, y)
    asym = abs(y @ zr - r @ zy) / (np.linalg.norm(y) * np.linalg.norm(zr))
    say("[operator %s] relative asymmetry %.2e" % (name, asym))
    assert asym <= 1e-9
    assert r @ zr > 0 and y @ zy > 0


def test_solution_matches_oracle_run(big):
    """The oracle's whole FP64 run of the workload (setup with the Lanczos
    eigen path and PCG to 1e-10, stored by golden/make_fullsize_golden.py,
    which calls only the oracle): eigenvector counts equal, iterations
    within +-2, the plain solution within 1e-8 of the oracle's and the
    solution after two refinement steps within 1e-8 of the oracle's refined
    reference."""
    import os
    name, prob, A, b, subs, sysm, h, info = big
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                        "fullsize_%s_seed0.npz" % name)
    gold = np.load(path)
    from paper_1906_10944_amd import geneo as G
    m, _ = G.geneo_get_eigenvalues(h, len(subs))
    x0, inf0 = gpu_pcg(h, sysm, rtol=prob.rtol, maxit=prob.maxit)
    h2 = gpu_setup(sysm, prob, precision=1, refine=2)
    x, inf = gpu_pcg(h2, sysm, rtol=prob.rtol, maxit=prob.maxit)
    h2.close()
    res = {}
    for key, xg, xo in (("plain", x0, gold["x"]), ("refined", x, gold["x_ref"])):
        res[key] = (np.linalg.norm(xg - xo) / np.linalg.norm(xo),
                    np.abs(xg - xo).max() / np.abs(xo).max())
    say("[solution %s] iters %d oracle %d, nc %d oracle %d, plain rel diff %.3e max-abs %.3e, "
        "refined (+%d its) rel diff %.3e max-abs %.3e" %
        (name, inf0["iters"], int(gold["iters"]), info["nc"], int(gold["nc"]), res["plain"][0],
         res["plain"][1], inf["refine_iters"], res["refined"][0], res["refined"][1]))
    assert np.array_equal(m, gold["m"])
    assert abs(inf0["iters"] - int(gold["iters"])) <= 2
    for key in res:
        assert res[key][0] <= 1e-8 and res[key][1] <= 1e-8, (key, res[key])
