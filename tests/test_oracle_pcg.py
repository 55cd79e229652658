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


def test_pcg_matches_direct_solve_config1():
    p = synth.config1_channels(0)
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
    p = synth.config1_channels(0, n=24, parts=3, n_channels=3, nev=2)
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


def test_threshold_selection_and_kappa_bound():
    """Thm. 1: with m_j = #{lam < delta/H} the estimate stays under the bound."""
    n, parts, ovl = 48, 4, 2
    p = synth.layered_2d(n=n, parts=parts, ovl=ovl, layers=8, contrast=1e6, nev=16)
    H_over_delta = (n / parts + 2 * ovl) / ovl
    it, kap, g = _iters(p, tau=1.0 / H_over_delta, nev_max=64)
    k0 = 4
    bound = (1 + k0) * (2 + k0 * (2 * k0 + 1) * (1 + H_over_delta))
    assert kap <= bound
    assert all(np.sum(l < 1.0 / H_over_delta) == m for l, m in zip(g.lam, g.m))
