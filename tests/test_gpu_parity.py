"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Tolerances: assembly and index work are exact or within a few ulps of the
summation order (1e-13 relative); FP64 solver results within 1e-12 for the
one-level operator, 1e-8 relative for eigenvalues, solutions and the
two-level operator, PCG iterations within +-2 of the oracle.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from gpu_common import (SMALL_PROBLEMS, csr_to_scipy, gpu_apply, gpu_assemble, gpu_pcg,
                        gpu_setup, local_dense, need_gpu, say)
from oracle import decomp, fem, geneo, pcg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", params=sorted(SMALL_PROBLEMS))
def case(request):
    need_gpu()
    prob = SMALL_PROBLEMS[request.param]()
    say("[case]", request.param, "ndof", prob.ndof, "nsub", prob.nsub)
    A, b = fem.assemble(prob)
    subs, _ = decomp.build(prob)
    sysm = gpu_assemble(prob)
    return request.param, prob, A, b, subs, sysm


def test_assembly_global(case):
    name, prob, A, b, subs, sysm = case
    n = prob.ndof
    Ag = csr_to_scipy(sysm.A_rowptr, sysm.A_col, sysm.A_val, n)
    scale = abs(A).max()
    assert abs(Ag - A).max() <= 1e-13 * scale
    assert np.allclose(sysm.b.cpu().numpy(), b, rtol=1e-14, atol=1e-14 * abs(b).max())
    rp = sysm.A_rowptr.cpu().numpy()
    col = sysm.A_col.cpu().numpy()
    for r in range(0, n, max(1, n // 50)):
        seg = col[rp[r]:rp[r + 1]]
        assert np.all(np.diff(seg) > 0)


def test_subdomain_lists_and_pou(case):
    name, prob, A, b, subs, sysm = case
    sp_ = sysm.sub_ptr.cpu().numpy()
    idx = sysm.sub_idx.cpu().numpy()
    fl = sysm.sub_flags.cpu().numpy()
    pou = sysm.pou.cpu().numpy()
    assert sp_[-1] == sum(len(s.dofs) for s in subs)
    for s in subs:
        seg = slice(sp_[s.j], sp_[s.j + 1])
        assert np.array_equal(idx[seg], s.dofs)
        assert np.array_equal((fl[seg] & 1).astype(bool), s.dmask)
        assert np.array_equal((fl[seg] & 2).astype(bool), s.dirichlet)
        assert np.array_equal(pou[seg], s.mu)


def test_local_matrices(case):
    name, prob, A, b, subs, sysm = case
    for s in subs[:: max(1, len(subs) // 6)]:
        AN, Ao = geneo.local_matrices(prob, s)
        scale = np.abs(AN).max()
        assert np.abs(local_dense(sysm, s.j, "an") - AN).max() <= 1e-13 * scale
        assert np.abs(local_dense(sysm, s.j, "ao") - Ao).max() <= 1e-13 * scale


@pytest.fixture(scope="module")
def solved(case):
    name, prob, A, b, subs, sysm = case
    g = geneo.setup(prob, A=A, subs=subs, keep_eigvecs=True)
    say("[oracle] nc", g.nc)
    h = gpu_setup(sysm, prob, precision=0)
    from paper_1906_10944_amd import geneo as G
    info = G.geneo_get_setup_info(h)
    say("[gpu] setup", {k: info[k] for k in ("nc", "eig_sweeps", "eig_block", "eig_max_resid")})
    return g, h, info


def _kappa_local(A, subs):
    """Largest condition number of the diagonally scaled local Dirichlet
    matrices (the matrices both sides factor)."""
    k = 1.0
    for s in subs:
        AD = geneo.dirichlet_matrix(A, s)
        d = 1.0 / np.sqrt(np.diag(AD))
        ev = np.linalg.eigvalsh(AD * d[:, None] * d[None, :])
        k = max(k, ev[-1] / ev[0])
    return k


def test_one_level_apply(case):
    name, prob, A, b, subs, sysm = case
    g = geneo.setup(prob, A=A, subs=subs, coarse=False)
    h = gpu_setup(sysm, prob, precision=0, coarse=0)
    rng = np.random.Generator(np.random.PCG64(11))
    r = rng.normal(size=prob.ndof)
    z = gpu_apply(h, sysm, r)
    zo = g.apply_one_level(r)
    # both sides solve with a backward-stable FP64 factorisation of the same
    # scaled matrices: each forward error is O(u kappa), so they may differ
    # by that much (10 u kappa, floor 1e-12)
    tol = max(1e-12, 10 * np.finfo(float).eps / 2 * _kappa_local(A, subs))
    say("[one-level] rel diff %.3e tol %.3e" % (np.linalg.norm(z - zo) / np.linalg.norm(zo), tol))
    assert np.linalg.norm(z - zo) <= tol * np.linalg.norm(zo)


def _cut_gap(lam, m):
    if m == 0 or m >= len(lam) or not np.isfinite(lam[m]):
        return np.inf
    return (lam[m] - lam[m - 1]) / max(abs(lam[m]), 1e-300)


def test_eigenvalues(case, solved):
    name, prob, A, b, subs, sysm = case
    g, h, info = solved
    from paper_1906_10944_amd import geneo as G
    m, lam = G.geneo_get_eigenvalues(h, len(subs))
    assert list(m) == list(g.m)
    for j, s in enumerate(subs):
        lo = g.lam[j]
        for c in range(m[j]):
            assert lam[j, c] == pytest.approx(lo[c], rel=1e-8, abs=1e-11), (j, c)


def test_coarse_matrix_is_galerkin_product(case, solved):
    name, prob, A, b, subs, sysm = case
    g, h, info = solved
    from paper_1906_10944_amd import geneo as G
    zoff, z, ah = G.geneo_get_coarse(h, len(subs))
    nc = info["nc"]
    if nc == 0:
        return
    cols, off = [], 0
    rows, cidx, vals = [], [], []
    m, _ = G.geneo_get_eigenvalues(h, len(subs))
    for s in subs:
        mj = m[s.j]
        blk = z[zoff[s.j]:zoff[s.j + 1]].reshape(len(s.dofs), mj)
        r_, c_ = np.nonzero(blk)
        rows.append(s.dofs[r_])
        cidx.append(c_ + off)
        vals.append(blk[r_, c_])
        off += mj
    Z = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cidx))),
                      shape=(prob.ndof, nc))
    AH = (Z.T @ (A @ Z)).toarray()
    assert np.abs(ah - AH).max() <= 1e-12 * np.abs(AH).max()
    # columns unit l2 and supported on D_j
    assert np.allclose(np.sqrt(np.asarray(Z.multiply(Z).sum(axis=0))).ravel(), 1.0, rtol=1e-12)
    # span agrees with the oracle's wherever the cut is not degenerate; the
    # angle between the spans is bounded by (Ritz residual)/(gap) in the
    # shift-inverted problem, nu = 1/(lam - sigma), residual <= eig_tol * nu_1
    Zo = g.Z.toarray()
    eig_tol, sigma = 1e-10, -1e-3
    off = 0
    for s in subs:
        mj = m[s.j]
        lo = g.lam[s.j]
        if mj and _cut_gap(lo, mj) > 1e-6:
            bound = _span_bound(lo, mj, eig_tol, sigma) + 1e-10
            Zg = Z[:, off:off + mj].toarray()
            Zoj = Zo[:, off:off + mj]
            Q, _ = np.linalg.qr(Zg)
            err = np.linalg.norm(Zoj - Q @ (Q.T @ Zoj)) / np.linalg.norm(Zoj)
            assert err <= bound, (s.j, err, bound)
        off += mj


def _span_bound(lam, m, eig_tol=1e-10, sigma=-1e-3):
    """Heuristic angle bound between computed and exact span of the first m
    basis vectors: Ritz residual over the gap in the shift-inverted problem
    (Davis-Kahan), with a factor 100 for sqrt(m) and for the change of
    variables p = G^{-T} y, z = X p."""
    if m == 0 or m >= len(lam) or not np.isfinite(lam[m]):
        return 1e-12
    nu = 1.0 / (np.asarray(lam[:m + 1]) - sigma)
    return 100 * eig_tol * nu[0] / (nu[m - 1] - nu[m])


def test_two_level_apply(case, solved):
    name, prob, A, b, subs, sysm = case
    g, h, info = solved
    degenerate = any(_cut_gap(l, mm) <= 1e-6 for l, mm in zip(g.lam, g.m))
    rng = np.random.Generator(np.random.PCG64(12))
    r = rng.normal(size=prob.ndof)
    z = gpu_apply(h, sysm, r)
    zo = g.apply(r)
    bound = max(_span_bound(l, mm) for l, mm in zip(g.lam, g.m))
    tol = 1e-3 if degenerate else max(1e-9, 10 * bound)
    say("[two-level apply]", name, "rel diff", np.linalg.norm(z - zo) / np.linalg.norm(zo),
        "tol", tol)
    assert np.linalg.norm(z - zo) <= tol * np.linalg.norm(zo)
    # symmetry of the operator the GPU applies
    y = rng.normal(size=prob.ndof)
    zy = gpu_apply(h, sysm, y)
    assert abs(y @ z - r @ zy) <= 1e-12 * np.linalg.norm(y) * np.linalg.norm(z) * 10


def _lam_min(A):
    import scipy.sparse.linalg as spla
    if A.shape[0] <= 6000:
        return np.linalg.eigvalsh(A.toarray())[0]
    return spla.eigsh(A.tocsc(), k=1, sigma=0, which="LM", return_eigenvectors=False)[0]


def _check_solution(prob, A, b, sysm, h, apply_ref, tag):
    """Iterations within +-2 and solution within 1e-8 of the oracle at a
    1e-10 residual reduction, where the problem's conditioning determines
    the solution that well.  Two solutions x_g (of the device system A_g,
    b_g) and x_o (of A, b) with residuals r_g, r_o differ by at most
    (|r_g| + |r_o| + |A_g - A| |x| + |b_g - b|) / lambda_min(A); the
    tolerance is max(1e-8 |x_o|, that bound)."""
    x, inf = gpu_pcg(h, sysm, rtol=1e-10)
    ref = pcg.pcg(A, b, apply_ref, rtol=1e-10)
    say("[pcg %s]" % tag, prob.name, "gpu it", inf["iters"], "oracle it", ref.iters,
        "kappa", inf["kappa_est"], pcg.kappa_estimate(ref.alphas, ref.betas))
    assert inf["converged"]
    Ag = csr_to_scipy(sysm.A_rowptr, sysm.A_col, sysm.A_val, prob.ndof)
    bg = sysm.b.cpu().numpy()
    rg = np.linalg.norm(bg - Ag @ x)
    ro = np.linalg.norm(b - A @ ref.x)
    fro = np.sqrt((Ag.multiply(Ag)).sum())
    # the device residual is the recurrence's, up to the rounding floor of A x
    assert rg <= 2e-10 * np.linalg.norm(bg) + 1e-15 * fro * np.linalg.norm(x)
    nx = np.linalg.norm(ref.x)
    dA = (Ag - A)
    dA = np.sqrt((dA.multiply(dA)).sum())
    bound = (rg + ro + dA * nx + np.linalg.norm(bg - b)) / _lam_min(A)
    diff = np.linalg.norm(x - ref.x)
    say("   rel diff %.2e  bound %.2e" % (diff / nx, bound / nx))
    assert diff <= max(1e-8 * nx, 1.01 * bound)
    return inf, ref


def test_pcg_fp64(case, solved):
    name, prob, A, b, subs, sysm = case
    g, h, info = solved
    inf, ref = _check_solution(prob, A, b, sysm, h, g.apply, "fp64")
    assert abs(inf["iters"] - ref.iters) <= 2


def test_pcg_mixed(case):
    name, prob, A, b, subs, sysm = case
    g = geneo.setup(prob, A=A, subs=subs)
    h = gpu_setup(sysm, prob, precision=1)
    from paper_1906_10944_amd import geneo as G
    info = G.geneo_get_setup_info(h)
    say("[mixed] fallback subdomains", info["fallback_fp64"])
    inf, ref = _check_solution(prob, A, b, sysm, h, g.apply, "mixed")
    assert inf["iters"] <= ref.iters + 4
