"""Pins of the oracle's GenEO eigenproblem, coarse space and preconditioner
(Sec. 3 eq. (4), Def. 2, Def. 4; Sec. 4.3-4.5)."""
import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import decomp, fem, geneo


def _rng(s):
    return np.random.Generator(np.random.PCG64(s))


def _spd(n, rng, cond=1e3):
    Q, _ = np.linalg.qr(rng.normal(size=(n, n)))
    return (Q * np.logspace(0, np.log10(cond), n)) @ Q.T


def test_shift_invert_matches_library_pencil_solver():
    rng = _rng(0)
    A, B = _spd(30, rng), _spd(30, rng, 1e2)
    ev = geneo.generalized_eigen(A, B)
    ref = sla.eigh(A, B, eigvals_only=True)
    assert np.allclose(ev.lam, ref, rtol=1e-9)
    for k in range(30):
        p = ev.P[:, k]
        assert np.linalg.norm(A @ p - ev.lam[k] * B @ p) <= 1e-9 * np.linalg.norm(A @ p)


def test_singular_B_reciprocal_pencil():
    """Finite eigenvalues of A p = lam B p with B PSD of rank r are the
    reciprocals of the positive eigenvalues of B p = mu A p (A SPD)."""
    rng = _rng(1)
    n, r = 25, 9
    A = _spd(n, rng)
    F = rng.normal(size=(n, r))
    B = F @ F.T
    ev = geneo.generalized_eigen(A, B)
    mu = sla.eigh(B, A, eigvals_only=True)[::-1][:r]
    assert np.sum(np.isfinite(ev.lam)) == r
    assert np.allclose(ev.lam[:r], 1.0 / mu, rtol=1e-8)


def _small_darcy(parts=3, n=12, ovl=2, contrast=1e4, seed=0):
    rng = _rng(seed)
    k = np.where(rng.uniform(size=(n, n)) < 0.2, contrast, 1.0)
    return synth.darcy_problem("t", k, (parts, parts), ovl, nev=4)


def _local(prob, j):
    subs, _ = decomp.build(prob)
    s = subs[j]
    AN, Ao = geneo.local_matrices(prob, s)
    B = s.mu[:, None] * Ao * s.mu[None, :]
    return s, AN, Ao, B


@pytest.mark.parametrize("j", [0, 4])
def test_sylvester_inertia_counts(j):
    p = _small_darcy()
    s, AN, Ao, B = _local(p, j)
    ev = geneo.generalized_eigen(AN, B)
    for tau in (1e-3, 0.05, 0.2, 0.7, 3.0):
        neg = int(np.sum(np.linalg.eigvalsh(AN - tau * B) < 0))
        assert neg == int(np.sum(ev.lam < tau)), tau


def test_eigen_residuals_and_B_orthonormality():
    p = _small_darcy()
    s, AN, Ao, B = _local(p, 4)
    ev = geneo.generalized_eigen(AN, B)
    fin = np.isfinite(ev.lam)
    Pf = ev.P[:, fin]
    for k in range(Pf.shape[1]):
        x = Pf[:, k]
        r = AN @ x - ev.lam[k] * (B @ x)
        # normwise backward error of the pair
        bound = (np.linalg.norm(AN, 2) + ev.lam[k] * np.linalg.norm(B, 2)) * np.linalg.norm(x)
        assert np.linalg.norm(r) <= 1e-12 * bound
    assert np.all(ev.lam[fin] >= -1e-12)
    G = Pf.T @ (AN - geneo.SIGMA * B) @ Pf
    assert np.allclose(G, np.eye(G.shape[0]), atol=1e-9)


def test_darcy_kernel_floating_vs_boundary_subdomains():
    p = _small_darcy(parts=3)
    subs, _ = decomp.build(p)
    for s in subs:
        AN, Ao = geneo.local_matrices(p, s)
        B = s.mu[:, None] * Ao * s.mu[None, :]
        ev = geneo.generalized_eigen(AN, B)
        floating = not s.dirichlet.any()
        if floating:
            assert abs(ev.lam[0]) < 1e-10 and ev.lam[1] > 1e-4
            v = ev.P[:, 0] / np.linalg.norm(ev.P[:, 0])
            assert np.allclose(np.abs(v), 1 / np.sqrt(len(v)), rtol=1e-8)
        else:
            assert ev.lam[0] > 1e-4
    assert sum(not s.dirichlet.any() for s in subs) == 1   # centre of 3x3


def _rbm_local(prob, dofs):
    nn = [n + 1 for n in prob.ne]
    k = dofs[::3] // 3
    x = (k % nn[0]) * prob.h[0]
    y = ((k // nn[0]) % nn[1]) * prob.h[1]
    z = (k // (nn[0] * nn[1])) * prob.h[2]
    o, zr = np.ones_like(x), np.zeros_like(x)
    modes = [(o, zr, zr), (zr, o, zr), (zr, zr, o), (-y, x, zr), (zr, -z, y), (z, zr, -x)]
    return np.array([np.stack(m, 1).ravel() for m in modes]).T


def _small_laminate(nx=12):
    p4 = synth.laminate_3d(ne=(nx, 2, 5), parts=(3, 1, 1), nev=8)
    return p4


def test_elasticity_floating_subdomain_has_six_zero_modes():
    p = _small_laminate()
    subs, _ = decomp.build(p)
    s = subs[1]                        # middle part: not touching x = 0
    assert not s.dirichlet.any()
    AN, Ao = geneo.local_matrices(p, s)
    B = s.mu[:, None] * Ao * s.mu[None, :]
    ev = geneo.generalized_eigen(AN, B)
    assert np.sum(np.abs(ev.lam) < 1e-8) == 6 and ev.lam[6] > 1e-5
    R = _rbm_local(p, s.dofs)
    Q, _ = np.linalg.qr(ev.P[:, :6])
    assert np.linalg.norm(R - Q @ (Q.T @ R)) <= 1e-8 * np.linalg.norm(R)
    s0 = subs[0]                       # clamped part
    AN0, Ao0 = geneo.local_matrices(p, s0)
    ev0 = geneo.generalized_eigen(AN0, s0.mu[:, None] * Ao0 * s0.mu[None, :])
    assert ev0.lam[0] > 1e-5


def _dense_Z(g):
    return g.Z.toarray()


def test_coarse_space_contains_weighted_kernel():
    p = _small_darcy(parts=3)
    g = geneo.setup(p, nev=2)
    Z = _dense_Z(g)
    for s in g.subs:
        if s.dirichlet.any():
            continue
        v = np.zeros(p.ndof)
        v[s.dofs] = s.mu                        # R_j^T X_j 1
        c, *_ = np.linalg.lstsq(Z, v, rcond=None)
        assert np.linalg.norm(v - Z @ c) <= 1e-10 * np.linalg.norm(v)


def test_coarse_space_contains_weighted_rigid_body_modes():
    p = _small_laminate()
    g = geneo.setup(p, nev=7)
    Z = _dense_Z(g)
    s = g.subs[1]
    R = _rbm_local(p, s.dofs)
    for k in range(6):
        v = np.zeros(p.ndof)
        v[s.dofs] = s.mu * R[:, k]
        c, *_ = np.linalg.lstsq(Z, v, rcond=None)
        assert np.linalg.norm(v - Z @ c) <= 1e-9 * np.linalg.norm(v)


def test_coarse_matrix_brute_force_sparsity_and_local_formula():
    p = _small_darcy(parts=3)
    g = geneo.setup(p, nev=3)
    Z = _dense_Z(g)
    Ad = g.A.toarray()
    assert np.allclose(g.AH, Z.T @ Ad @ Z, rtol=0, atol=1e-12 * np.abs(g.AH).max())
    off = geneo.coarse_offsets(g.m)
    subs = g.subs
    for i in range(len(subs)):
        for j in range(len(subs)):
            blk = g.AH[off[i]:off[i + 1], off[j]:off[j + 1]]
            adjacent = len(np.intersect1d(subs[i].dofs, subs[j].dofs)) > 0
            if not adjacent:
                assert np.all(blk == 0.0)
            else:
                # phi_i^T A_j phi_j with the Neumann matrix of subdomain j (Sec. 4.5)
                AN, _ = geneo.local_matrices(p, subs[j])
                Zi = Z[subs[j].dofs, off[i]:off[i + 1]]
                Zj = Z[subs[j].dofs, off[j]:off[j + 1]]
                assert np.allclose(Zi.T @ AN @ Zj, blk, atol=1e-11 * np.abs(g.AH).max())


def test_dirichlet_matrix_two_routes():
    p = _small_darcy(parts=3)
    A, _ = fem.assemble(p)
    subs, _ = decomp.build(p)
    for s in subs:
        AD = geneo.dirichlet_matrix(A, s)
        AN, _ = geneo.local_matrices(p, s)
        d = s.dmask
        assert np.allclose(AD, AN[np.ix_(d, d)], rtol=1e-14, atol=0)


def test_preconditioner_symmetric_positive_and_basis_invariant():
    p = _small_darcy(parts=3)
    g = geneo.setup(p, nev=3)
    rng = _rng(5)
    x, y = rng.normal(size=p.ndof), rng.normal(size=p.ndof)
    free = ~fem.dirichlet_mask(p)
    x[~free] = 0
    y[~free] = 0
    a, b = x @ g.apply(y), y @ g.apply(x)
    assert abs(a - b) <= 1e-12 * (abs(a) + abs(b))
    assert x @ g.apply(x) > 0
    z0 = g.apply(y)
    # rescale and flip basis columns: the span, hence M^{-1}, is unchanged
    sc = rng.uniform(0.1, 10.0, g.nc) * rng.choice([-1.0, 1.0], g.nc)
    g.Z = g.Z @ np.diag(sc)
    import scipy.sparse as sp
    g.Z = sp.csr_matrix(g.Z)
    AH = (g.Z.T @ (g.A @ g.Z)).toarray()
    g.LH = np.linalg.cholesky(0.5 * (AH + AH.T))
    assert np.linalg.norm(g.apply(y) - z0) <= 1e-12 * np.linalg.norm(z0)


def test_selection_rules():
    lam = np.array([0.0, 0.01, 0.05, 0.099, 0.1, 0.3, np.inf])
    assert geneo.select_count(lam, nev=3) == 3
    assert geneo.select_count(lam, nev=10) == 6
    assert geneo.select_count(lam, tau=0.1, nev_max=16) == 4
    assert geneo.select_count(lam, tau=0.1, nev_max=2) == 2
    assert geneo.select_count(np.full(4, np.inf), nev=3) == 0


def test_basis_vectors_normalised_signed_supported():
    p = _small_darcy(parts=3)
    g = geneo.setup(p, nev=3)
    Z = _dense_Z(g)
    assert np.allclose(np.linalg.norm(Z, axis=0), 1.0, rtol=1e-14)
    off = geneo.coarse_offsets(g.m)
    for s in g.subs:
        blk = Z[:, off[s.j]:off[s.j + 1]]
        outside = np.setdiff1d(np.arange(p.ndof), s.dofs[s.dmask])
        assert np.all(blk[outside] == 0.0)
        for k in range(blk.shape[1]):
            i = np.argmax(np.abs(blk[:, k]))
            assert blk[i, k] > 0


def test_coarse_cholesky_rejects_repeated_basis_vector():
    """A_H is SPD iff the columns of Z are independent (Def. 2): a repeated
    column makes it singular, and the factor must say so whatever sign the
    rounding leaves on the vanishing pivot."""
    p = synth.channels_2d(0, n=16, parts=2, n_channels=2, nev=3)
    A, _ = fem.assemble(p)
    g = geneo.setup(p, A=A)
    Z = g.Z.toarray()
    L = geneo.coarse_cholesky(g.AH)
    assert np.allclose(L @ L.T, g.AH, rtol=0, atol=1e-13 * np.abs(g.AH).max())
    for k in (0, g.nc // 2, g.nc - 1):
        Zd = np.column_stack([Z, Z[:, k]])
        AHd = Zd.T @ (A @ Zd)
        with pytest.raises(np.linalg.LinAlgError):
            geneo.coarse_cholesky(0.5 * (AHd + AHd.T))
