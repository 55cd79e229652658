"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Tolerances:
* assembly and index work: exact, or within a few ulps of the summation
  order (1e-13 relative);
* one-level operator: 10 u kappa of the scaled local matrices (both sides
  solve with backward-stable FP64 factors), normwise and element-wise;
* eigenvalues: 1e-8 relative;
* coarse basis: each device column, written in the oracle's C-orthonormal
  eigenvectors (C = A_N - sigma B), has no more weight outside the selected
  eigenspace (extended through the end of a cluster the cut splits) than
  the device's measured Ritz residual over the measured gap allows
  (Davis-Kahan in the shift-inverted operator);
* two-level operator: the oracle's formula (Def. 2) evaluated with the
  device's basis, to the rounding of the two solves (10 u kappa);
* PCG: solution within 1e-8 relative (normwise and element-wise) of the
  oracle's at a 1e-10 residual reduction, and iterations within +-2, for
  the FP64 and the mixed form; and the solutions after two refinement
  steps (residuals in double-double / extended precision) within 1e-8 of
  each other too.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from gpu_common import (SMALL_PROBLEMS, csr_to_scipy, gpu_apply, gpu_assemble, gpu_pcg,
                        gpu_setup, kappa_spd, local_dense, need_gpu, say,
                        span_contamination, kappa_local)
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
    """Both sides sum every entry's element contributions in ascending
    element order from the same closed-form Darcy element matrix: the Darcy
    matrices agree bit for bit; the elasticity ones (quadrature on both
    sides, different operation orders) to rounding."""
    name, prob, A, b, subs, sysm = case
    n = prob.ndof
    Ag = csr_to_scipy(sysm.A_rowptr, sysm.A_col, sysm.A_val, n)
    scale = abs(A).max()
    if prob.ncomp == 1:
        assert abs(Ag - A).max() == 0.0
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
        tol = 0.0 if prob.ncomp == 1 else 1e-13 * scale
        assert np.abs(local_dense(sysm, s.j, "an") - AN).max() <= tol
        assert np.abs(local_dense(sysm, s.j, "ao") - Ao).max() <= tol


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


@pytest.mark.parametrize("form", [1, 2], ids=["triangular", "inverse"])
def test_one_level_apply(case, form):
    """Both forms of the device's local solves (substitution with the banded
    factors, product with the symmetric inverses) against the oracle."""
    name, prob, A, b, subs, sysm = case
    g = geneo.setup(prob, A=A, subs=subs, coarse=False)
    h = gpu_setup(sysm, prob, precision=0, coarse=0, local_solve=form)
    rng = np.random.Generator(np.random.PCG64(11))
    r = rng.normal(size=prob.ndof)
    z = gpu_apply(h, sysm, r)
    zo = g.apply_one_level(r)
    # both sides solve with a backward-stable FP64 factorisation of the same
    # scaled matrices: each forward error is O(u kappa), so they may differ
    # by that much (10 u kappa, floor 1e-12)
    tol = max(1e-12, 10 * np.finfo(float).eps / 2 * kappa_local(A, subs))
    mx = np.abs(z - zo).max() / np.abs(zo).max()
    say("[one-level] rel diff %.3e max-abs %.3e tol %.3e" %
        (np.linalg.norm(z - zo) / np.linalg.norm(zo), mx, tol))
    assert np.linalg.norm(z - zo) <= tol * np.linalg.norm(zo)
    assert mx <= tol


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


def _gpu_basis(h, subs, nc):
    """Device coarse basis as dense blocks over N_j, and as a global sparse Z."""
    from paper_1906_10944_amd import geneo as G
    zoff, z, ah = G.geneo_get_coarse(h, len(subs))
    m, _ = G.geneo_get_eigenvalues(h, len(subs))
    blocks, rows, cidx, vals, off = [], [], [], [], 0
    for s in subs:
        mj = int(m[s.j])
        blk = z[zoff[s.j]:zoff[s.j + 1]].reshape(len(s.dofs), mj)
        blocks.append(blk)
        r_, c_ = np.nonzero(blk)
        rows.append(s.dofs[r_])
        cidx.append(c_ + off)
        vals.append(blk[r_, c_])
        off += mj
    return blocks, rows, cidx, vals, ah, m


def _zsparse(prob, rows, cidx, vals, nc):
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cidx))),
                         shape=(prob.ndof, nc))


def test_coarse_matrix_is_galerkin_product(case, solved):
    name, prob, A, b, subs, sysm = case
    g, h, info = solved
    nc = info["nc"]
    if nc == 0:
        return
    blocks, rows, cidx, vals, ah, m = _gpu_basis(h, subs, nc)
    Z = _zsparse(prob, rows, cidx, vals, nc)
    AH = (Z.T @ (A @ Z)).toarray()
    assert np.abs(ah - AH).max() <= 1e-12 * np.abs(AH).max()
    # columns unit l2 and supported on D_j
    assert np.allclose(np.sqrt(np.asarray(Z.multiply(Z).sum(axis=0))).ravel(), 1.0, rtol=1e-12)
    for s, blk in zip(subs, blocks):
        assert np.all(blk[~s.dmask] == 0.0)


def test_coarse_basis_spans_geneo_eigenspace(case, solved):
    """Def. 4 with the shift-invert solve of Sec. 4.4: every device column
    lies in X times the oracle's wanted eigenspace (through the end of a
    cluster the cut splits) up to the measured Ritz residual over the gap
    (``gpu_common.span_contamination``)."""
    name, prob, A, b, subs, sysm = case
    g, h, info = solved
    nc = info["nc"]
    if nc == 0:
        return
    blocks, *_ = _gpu_basis(h, subs, nc)
    worst = 0.0
    for s, blk in zip(subs, blocks):
        if blk.shape[1] == 0:
            continue
        AN, Ao = geneo.local_matrices(prob, s)
        kC = kappa_spd(AN + 1e-3 * (s.mu[:, None] * Ao * s.mu[None, :]))
        res = span_contamination(s.mu, g.lam[s.j], g.eigvecs[s.j], blk, info["eig_max_resid"], kC)
        if res is None:
            continue
        out, bound = res
        worst = max(worst, out / bound)
        assert out <= bound, (s.j, blk.shape[1], out, bound)
    say("[span]", name, "r_meas %.2e worst fraction of bound %.3f" % (info["eig_max_resid"], worst))


def _cond(M):
    ev = np.linalg.eigvalsh(0.5 * (M + M.T))
    return ev[-1] / ev[0]


def test_two_level_apply(case, solved):
    """M^{-1} r = R_H^T A_H^{-1} R_H r + sum_j R_j^T A_j^{-1} R_j r (Def. 2),
    the oracle's formula evaluated with the device's coarse basis (whose
    span is checked above).  Both sides solve with backward-stable FP64
    factors (the device with explicit symmetric inverses), so the parts
    differ by 10 u kappa of their matrices."""
    name, prob, A, b, subs, sysm = case
    g, h, info = solved
    nc = info["nc"]
    rng = np.random.Generator(np.random.PCG64(12))
    r = rng.normal(size=prob.ndof)
    z = gpu_apply(h, sysm, r)
    u = np.finfo(float).eps / 2
    z1 = g.apply_one_level(r)
    zc = np.zeros_like(z1)
    kH = 1.0
    if nc:
        _, rows, cidx, vals, ah, m = _gpu_basis(h, subs, nc)
        Z = _zsparse(prob, rows, cidx, vals, nc)
        AH = (Z.T @ (A @ Z)).toarray()
        AH = 0.5 * (AH + AH.T)
        zc = Z @ np.linalg.solve(AH, Z.T @ r)
        kH = _cond(AH)
    zo = z1 + zc
    kl = kappa_local(A, subs)
    tol_abs = 10 * u * (kl * np.linalg.norm(z1) + kH * np.linalg.norm(zc)) \
        + 1e-13 * np.linalg.norm(zo)
    diff = np.linalg.norm(z - zo)
    say("[two-level apply] %s rel diff %.3e tol %.3e (kappa_loc %.2e kappa_H %.2e) "
        "max-abs %.3e" % (name, diff / np.linalg.norm(zo), tol_abs / np.linalg.norm(zo), kl, kH,
                          np.abs(z - zo).max() / np.abs(zo).max()))
    assert tol_abs <= 1e-6 * np.linalg.norm(zo)
    assert diff <= tol_abs
    assert np.abs(z - zo).max() <= tol_abs / np.linalg.norm(zo) * np.abs(zo).max()
    # symmetry of the operator the GPU applies
    y = rng.normal(size=prob.ndof)
    zy = gpu_apply(h, sysm, y)
    assert abs(y @ z - r @ zy) <= 1e-12 * np.linalg.norm(y) * np.linalg.norm(z) * 10


def _check_solution(prob, A, b, sysm, h, apply_ref, tag, precision):
    """At a 1e-10 residual reduction: iterations within +-2 of the oracle's
    and the solution within 1e-8 relative (2-norm and max-abs) of the
    oracle's.  Then with two refinement steps on both sides (residuals in
    double-double on the device, in extended precision in the oracle): the
    refined solutions within 1e-8 as well, which holds whatever the
    conditioning of A (a plain FP64 solve is only accurate to about
    u kappa(A))."""
    x, inf = gpu_pcg(h, sysm, rtol=1e-10)
    ref = pcg.pcg(A, b, apply_ref, rtol=1e-10)
    say("[pcg %s]" % tag, prob.name, "gpu it", inf["iters"], "oracle it", ref.iters,
        "kappa", inf["kappa_est"], pcg.kappa_estimate(ref.alphas, ref.betas))
    assert inf["converged"]
    assert abs(inf["iters"] - ref.iters) <= 2
    Ag = csr_to_scipy(sysm.A_rowptr, sysm.A_col, sysm.A_val, prob.ndof)
    bg = sysm.b.cpu().numpy()
    fro = np.sqrt((Ag.multiply(Ag)).sum())
    # the device residual is the recurrence's, up to the rounding floor of A x
    assert np.linalg.norm(bg - Ag @ x) <= 2e-10 * np.linalg.norm(bg) + 1e-15 * fro * np.linalg.norm(x)
    x_ref = pcg.refine(A, b, ref.x, lambda r: pcg.pcg(A, r, apply_ref, rtol=1e-6).x, steps=2)
    h2 = gpu_setup(sysm, prob, precision=precision, refine=2)
    xr, infr = gpu_pcg(h2, sysm, rtol=1e-10)
    h2.close()
    assert infr["iters"] == inf["iters"]
    out = {}
    for key, xg, xo in (("plain", x, ref.x), ("refined", xr, x_ref)):
        nx = np.linalg.norm(xo)
        diff = np.linalg.norm(xg - xo) / nx
        mx = np.abs(xg - xo).max() / np.abs(xo).max()
        out[key] = (diff, mx)
    say("   plain: rel diff %.2e max-abs %.2e | refined (+%d its): rel diff %.2e max-abs %.2e "
        "| plain vs refined oracle %.2e" % (out["plain"] + (infr["refine_iters"],) + out["refined"]
                                           + (np.linalg.norm(ref.x - x_ref) / np.linalg.norm(x_ref),)))
    for key in out:
        assert out[key][0] <= 1e-8 and out[key][1] <= 1e-8, (key, out[key])
    return inf, ref


def test_pcg_fp64(case, solved):
    name, prob, A, b, subs, sysm = case
    g, h, info = solved
    _check_solution(prob, A, b, sysm, h, g.apply, "fp64", 0)


def test_pcg_mixed(case):
    name, prob, A, b, subs, sysm = case
    g = geneo.setup(prob, A=A, subs=subs)
    h = gpu_setup(sysm, prob, precision=1)
    from paper_1906_10944_amd import geneo as G
    info = G.geneo_get_setup_info(h)
    say("[mixed] fallback subdomains", info["fallback_fp64"])
    _check_solution(prob, A, b, sysm, h, g.apply, "mixed", 1)
