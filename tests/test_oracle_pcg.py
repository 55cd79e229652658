"""Pins of the oracle's PCG and of the qualitative results the paper states
(Sec. 3 Thm. 1; Sec. 5.2; Sec. 5.3 Table 1)."""
import json
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla

import synth
from oracle import fem, geneo, pcg

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_pcg_matches_direct_solve_channels():
    p = synth.channels_2d(0)
    A, b = fem.assemble(p)
    g = geneo.setup(p, A=A)
    res = pcg.pcg(A, b, g.apply, rtol=1e-10)
    xd = spla.spsolve(A.tocsc(), b)
    assert res.converged
    assert np.linalg.norm(res.x - xd) <= 1e-8 * np.linalg.norm(xd)
    # recurrence residual agrees with the true residual
    true = np.linalg.norm(b - A @ res.x) / np.linalg.norm(b)
    assert abs(true - res.relres) <= 1e-12 + 1e-3 * res.relres


def test_exact_preconditioner_one_iteration():
    p = synth.darcy_problem("t", np.ones((9, 9)), (1, 1), 1)
    A, b = fem.assemble(p)
    lu = spla.splu(A.tocsc())
    res = pcg.pcg(A, b, lu.solve, rtol=1e-10)
    assert res.iters == 1 and res.converged


def test_single_subdomain_geneo_is_exact_inverse():
    """One subdomain: empty overlap zone, V_H = {0}, M^{-1} = A^{-1}."""
    rng = np.random.Generator(np.random.PCG64(2))
    p = synth.darcy_problem("t", np.exp(rng.normal(size=(10, 12))), (1, 1), 2, nev=4)
    A, b = fem.assemble(p)
    g = geneo.setup(p, A=A)
    assert g.nc == 0 and g.m == [0]
    assert np.all(np.isinf(g.lam[0]))
    res = pcg.pcg(A, b, g.apply)
    assert res.iters == 1


def test_lanczos_kappa_matches_preconditioned_spectrum():
    p = synth.channels_2d(0, n=24, parts=3, n_channels=3, nev=2)
    A, b = fem.assemble(p)
    g = geneo.setup(p, A=A)
    free = ~fem.dirichlet_mask(p)
    n = p.ndof
    M = np.column_stack([g.apply(e) for e in np.eye(n)])
    Af = A.toarray()
    ev = sla.eigh(Af[np.ix_(free, free)], np.linalg.inv(M[np.ix_(free, free)]),
                  eigvals_only=True)
    # random right-hand side: every eigencomponent present, so the extreme
    # Ritz values of the CG-Lanczos matrix converge to the extreme eigenvalues
    rb = np.random.Generator(np.random.PCG64(7)).normal(size=n) * free
    res = pcg.pcg(A, rb, g.apply, rtol=1e-12)
    est = pcg.kappa_estimate(res.alphas, res.betas)
    assert est == pytest.approx(ev[-1] / ev[0], rel=1e-3)


def test_thm1_bound_golden():
    d = json.load(open(os.path.join(GOLD, "thm1_bound.json")))
    for c in d["cases"]:
        k0, r = c["k0"], c["H_over_delta"]
        assert (1 + k0) * (2 + k0 * (2 * k0 + 1) * (1 + r)) == c["bound"]


def _iters(prob, **kw):
    A, b = fem.assemble(prob)
    g = geneo.setup(prob, A=A, **kw)
    res = pcg.pcg(A, b, g.apply, rtol=1e-10)
    assert res.converged
    return res.iters, pcg.kappa_estimate(res.alphas, res.betas), g


def test_geneo_flat_in_contrast_one_level_not():
    """Iterations stay flat as the contrast grows (Sec. 5.2, Fig. 4) while the
    one-level method degrades."""
    its, its1 = [], []
    for c in (1e0, 1e3, 1e6):
        p = synth.layered_2d(n=32, parts=4, ovl=2, layers=8, contrast=c, nev=4)
        i2, _, _ = _iters(p, nev=4)
        i1, _, _ = _iters(p, coarse=False)
        its.append(i2)
        its1.append(i1)
    assert max(its) - min(its) <= 4, its
    assert its1[-1] > its[-1] + 10, (its1, its)


def test_geneo_flat_in_subdomain_count_one_level_grows():
    """Table 1 trend: the one-level condition number and iteration count grow
    with the number of subdomains; GenEO's condition number stays flat."""
    its, its1, kap, kap1 = [], [], [], []
    for parts in (2, 4, 8):
        p = synth.layered_2d(n=48, parts=parts, ovl=2, layers=8, contrast=1e4, nev=6)
        i2, k2, _ = _iters(p, nev=6)
        i1, k1, _ = _iters(p, coarse=False)
        its.append(i2)
        its1.append(i1)
        kap.append(k2)
        kap1.append(k1)
    assert max(kap) / min(kap) < 1.5 and max(kap) < 10, kap
    assert max(its) - min(its) <= 8, its
    assert kap1[-1] > 5 * kap1[0] and its1[-1] > its1[0] + 20, (kap1, its1)


def test_thm1_threshold_closed_form():
    """delta_j / H_j for a 40 x 40 grid (h = 1/40) in 4 x 4 parts with
    overlap 2: interior boxes span 10 + 2 + 2 = 14 elements per side, corner
    boxes 12, edge boxes 14 x 12; delta = 2 * 2 / 40.  So tau = 4 / (14
    sqrt 2) inside, 4 / (12 sqrt 2) at the corners, 4 / sqrt(14^2 + 12^2)
    along the edges."""
    from oracle import decomp
    p = synth.layered_2d(n=40, parts=4, ovl=2, layers=8, contrast=1.0, nev=4)
    subs, _ = decomp.build(p)
    t = decomp.thm1_threshold(p, subs).reshape(4, 4)
    assert t[1, 1] == pytest.approx(0.2020305089104421, rel=1e-14)
    assert t[0, 0] == pytest.approx(0.2357022603955158, rel=1e-14)
    assert t[0, 1] == pytest.approx(0.21693045781865616, rel=1e-14)
    assert np.allclose(t, t.T) and np.allclose(t, t[::-1, ::-1])


def test_threshold_selection_and_kappa_bound():
    """Thm. 1: with m_j = #{lam < delta_j / H_j} the condition estimate stays
    under (1 + k0)[2 + k0 (2 k0 + 1) max_j (1 + H_j / delta_j)], k0 = 4."""
    from oracle import decomp
    p = synth.layered_2d(n=48, parts=4, ovl=2, layers=8, contrast=1e6, nev=16)
    subs, _ = decomp.build(p)
    tau = decomp.thm1_threshold(p, subs)
    it, kap, g = _iters(p, tau=tau, nev_max=64)
    k0 = 4
    bound = (1 + k0) * (2 + k0 * (2 * k0 + 1) * np.max(1 + 1 / tau))
    assert kap <= bound
    assert all(np.sum(l < t) == m for l, m, t in zip(g.lam, g.m, tau))
    assert max(g.m) < 64


def test_extended_residual_against_exact_rationals():
    """residual_extended carries about 64 bits: on a small system with
    ill-scaled entries it matches the exact rational residual, rounded to
    FP64, where the FP64 residual is visibly off."""
    from fractions import Fraction
    import scipy.sparse as sp
    rng = np.random.Generator(np.random.PCG64(13))
    n = 30
    M = sp.random(n, n, density=0.3, random_state=1, format="csr")
    M.data = rng.normal(size=M.nnz) * 10.0 ** rng.integers(-6, 7, size=M.nnz)
    x = rng.normal(size=n)
    b = M @ x + rng.normal(size=n) * 1e-12
    r = pcg.residual_extended(M, b, x)
    exact = []
    for i in range(n):
        s = Fraction(b[i])
        for k in range(M.indptr[i], M.indptr[i + 1]):
            s -= Fraction(M.data[k]) * Fraction(x[M.indices[k]])
        exact.append(float(s))
    exact = np.array(exact)
    # per row the terms reach |a_ij x_j| <= scale; FP64 sums err by about
    # u scale, the extended ones by about 2^-64 scale (plus the final
    # rounding of a residual of size 1e-12)
    scale = np.abs(M).max() * np.abs(x).max()
    err_ext = np.max(np.abs(r - exact))
    err_64 = np.max(np.abs((b - M @ x) - exact))
    assert err_ext <= 2.0 ** -60 * scale + 1e-27
    assert err_64 >= 100 * err_ext


def test_refined_geneo_pcg_matches_refined_sparse_lu():
    """Two independent routes to A^{-1} b on a badly conditioned layered
    problem (contrast 1e6, Neumann sides): GenEO-PCG to 1e-10 and sparse LU
    differ at the FP64 floor u kappa(A); after refinement with extended
    residuals they agree to 1e-13."""
    p = synth.layered_2d(n=40, parts=4, ovl=2, layers=8, contrast=1e6, nev=4)
    A, b = fem.assemble(p)
    g = geneo.setup(p, A=A)
    res = pcg.pcg(A, b, g.apply, rtol=1e-10)
    lu = spla.splu(A.tocsc())
    x_lu = lu.solve(b)
    x1 = pcg.refine(A, b, res.x, lambda r: pcg.pcg(A, r, g.apply, rtol=1e-6).x, steps=3)
    x2 = pcg.refine(A, b, x_lu, lu.solve, steps=3)
    nx = np.linalg.norm(x2)
    ev = np.linalg.eigvalsh(A.toarray())
    u = np.finfo(float).eps / 2
    print("kappa %.2e plain PCG vs LU %.2e refined %.2e" % (
        ev[-1] / ev[0], np.linalg.norm(res.x - x_lu) / nx, np.linalg.norm(x1 - x2) / nx))
    # attainable accuracy of refinement: about u + u_ext kappa(A)
    kappa = ev[-1] / ev[0]
    assert np.linalg.norm(x1 - x2) <= 10 * (u + 2.0 ** -64 * kappa) * nx
    assert np.linalg.norm(x1 - x2) <= 1e-2 * np.linalg.norm(res.x - x_lu)
    assert np.linalg.norm(res.x - x2) <= 10 * u * kappa * nx
