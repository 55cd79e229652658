"""GenEO coarse space and two-level additive Schwarz (oracle; test infrastructure).

Steps, in the paper's order and notation:

1. local matrices (Sec. 4.3): the Neumann matrix A_j of subdomain j (all
   elements of Omega_j, Dirichlet conditions only on the physical boundary,
   none on subdomain boundaries), the overlap matrix A_j^o (only the
   elements of the overlap zone), X_j = diag(mu_j); and the Dirichlet matrix
   of the one-level method, A_j = R_j A R_j^T (Sec. 3), taken from the
   global matrix on D_j;
2. the generalised eigenproblem A_j p = lambda X_j A_j^o X_j p (Sec. 4.3,
   the discrete form of eq. (4)), solved with the shift-and-invert spectral
   transformation of Sec. 4.4: for a shift sigma < 0 the matrix
   C = A_j - sigma B_j (B_j = X_j A_j^o X_j) is SPD, C^{-1} B_j x = nu x has
   the same eigenvectors and nu = 1/(lambda - sigma).  The dense symmetric
   form G^{-1} B_j G^{-T} y = nu y with C = G G^T, p = G^{-T} y, is solved
   with a library symmetric eigensolver;
   Above LANCZOS_MIN_N local dofs only the wanted end of the spectrum is
   computed, by implicitly restarted Lanczos (ARPACK, as in Sec. 4.4) on the
   same symmetric operator;
3. selection of the m_j smallest eigenvalues (Def. 4): a fixed count, or the
   count below a threshold capped at a maximum (Thm. 1, the threshold rule);
4. coarse basis vectors X_j p, normalised in the l2 norm (Sec. 4.4);
5. the coarse matrix A_H = R_H A R_H^T = Z^T A Z (Def. 2, Sec. 4.5) and its
   Cholesky factor (a pivot at or below n_c eps max_k (A_H)_kk counts as
   singular);
6. the two-level additive Schwarz operator (acting as the identity on the
   eliminated Dirichlet dofs, which lie in no D_j and have unit rows)
   M^{-1} = R_H^T A_H^{-1} R_H + sum_j R_j^T A_j^{-1} R_j (Def. 2).

Readings where the paper is silent: sigma = -1e-3 (any sigma < 0 gives the
same eigenpairs, only conditioning changes); eigenvalues with
nu <= 1e-14 max(nu) are infinite (B_j is singular); ties in lambda keep
ascending index order; the sign of each basis vector makes its largest
entry in magnitude positive (lowest index among ties) -- M^{-1} depends only
on span(Z), so sign and scale never change an iterate in exact arithmetic.

Pins (tests/test_oracle_geneo.py): scipy's generalised eigensolver on SPD
pencils, Sylvester inertia counts of A_j - tau B_j, eigen residuals,
lambda = 0 with the constant (Darcy) or the six rigid-body modes
(elasticity) as kernel of floating subdomains and no zero eigenvalue for
subdomains touching the Dirichlet boundary, the coarse space containing
X_j times that kernel, A_H against a brute-force dense Z^T A Z and the local
formula phi_i^T A_i phi_j, symmetry of M^{-1}, and M^{-1} = A^{-1} for a
single subdomain.
"""
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import fem, decomp

SIGMA = -1e-3
NU_ZERO_REL = 1e-14


# ------------------------------------------------------------ local matrices

def local_matrices(prob, sub):
    """Dense (A_N, A_o) of one subdomain over N_j (local numbering = sorted dofs)."""
    n = len(sub.dofs)
    gdofs = fem.element_dofs(prob)

    def build(elems):
        M = np.zeros((n, n))
        if len(elems) == 0:
            return M
        Ke = fem.element_matrices(prob, elems)
        ld = np.searchsorted(sub.dofs, gdofs[elems])   # N_j is sorted
        assert np.all(sub.dofs[ld] == gdofs[elems])
        for e in range(len(elems)):
            M[np.ix_(ld[e], ld[e])] += Ke[e]
        return M

    AN = build(sub.elems)
    Ao = build(sub.overlap_elems)
    # same (homogeneous Dirichlet) boundary treatment as the global matrix
    d = sub.dirichlet
    for M in (AN, Ao):
        M[d, :] = 0.0
        M[:, d] = 0.0
        M[d, d] = 1.0
    return AN, Ao


def dirichlet_matrix(A, sub):
    """A_j = R_j A R_j^T on D_j, read from the global sparse matrix."""
    idx = sub.dofs[sub.dmask]
    return A[idx][:, idx].toarray()


# ------------------------------------------------------------- eigenproblem

@dataclass
class EigenResult:
    lam: np.ndarray      # ascending; inf where nu vanishes
    P: np.ndarray        # columns = eigenvectors p over N_j (B-normalised for finite lam)


def generalized_eigen(AN, B, sigma=SIGMA):
    """All eigenpairs of AN p = lam B p via shift-and-invert (Sec. 4.4)."""
    C = AN - sigma * B
    G = np.linalg.cholesky(C)                        # C = G G^T
    W = sla.solve_triangular(G, B, lower=True)       # G^{-1} B
    S = sla.solve_triangular(G, W.T, lower=True)     # G^{-1} B G^{-T} (B symmetric)
    S = 0.5 * (S + S.T)
    nu, Y = np.linalg.eigh(S)                        # ascending nu
    nu, Y = nu[::-1], Y[:, ::-1]                     # descending nu = ascending lam
    numax = max(nu[0], 0.0)
    finite = nu > NU_ZERO_REL * numax if numax > 0 else np.zeros(len(nu), bool)
    lam = np.full(len(nu), np.inf)
    lam[finite] = sigma + 1.0 / nu[finite]
    P = sla.solve_triangular(G.T, Y, lower=False)    # p = G^{-T} y
    order = np.argsort(lam, kind="stable")
    return EigenResult(lam=lam[order], P=P[:, order])


LANCZOS_MIN_N = 1500


def generalized_eigen_lanczos(AN, B, k, sigma=SIGMA):
    """The k smallest eigenpairs of AN p = lam B p through the same
    shift-and-invert transform (Sec. 4.4), by implicitly restarted Lanczos
    (ARPACK, the solver the paper uses) on S = G^{-1} B G^{-T} for its k
    largest eigenvalues nu = 1 / (lam - sigma), to machine precision.  Used
    for large subdomains, where the full spectrum costs too much; returns
    the same quantities as :func:`generalized_eigen` for the k pairs."""
    import scipy.sparse.linalg as spla
    n = AN.shape[0]
    C = AN - sigma * B
    G = np.linalg.cholesky(C)
    Bs = sp.csr_matrix(B)

    def S(v):
        w = sla.solve_triangular(G, v, lower=True, trans="T")      # G^{-T} v
        return sla.solve_triangular(G, Bs @ w, lower=True)         # G^{-1} B G^{-T} v

    op = spla.LinearOperator((n, n), matvec=S, dtype=np.float64)
    v0 = np.ones(n) / np.sqrt(n)
    nu, Y = spla.eigsh(op, k=k, which="LA", tol=0.0, v0=v0, ncv=min(n, max(2 * k + 1, 48)))
    order = np.argsort(-nu, kind="stable")                        # descending nu
    nu, Y = nu[order], Y[:, order]
    numax = max(nu[0], 0.0)
    finite = nu > NU_ZERO_REL * numax if numax > 0 else np.zeros(len(nu), bool)
    lam = np.full(len(nu), np.inf)
    lam[finite] = sigma + 1.0 / nu[finite]
    P = sla.solve_triangular(G, Y, lower=True, trans="T")         # p = G^{-T} y
    order = np.argsort(lam, kind="stable")
    return EigenResult(lam=lam[order], P=P[:, order])


def select_count(lam, nev=None, tau=None, nev_max=None):
    """m_j: a fixed count, or #{lam < tau} capped at nev_max (finite lam only)."""
    nfin = int(np.sum(np.isfinite(lam)))
    if tau is None:
        return min(int(nev), nfin)
    return min(int(nev_max), int(np.sum(lam < tau)), nfin)


def basis_vectors(mu, P):
    """Coarse basis X_j p / ||X_j p||_2 with the sign convention of this module."""
    Z = mu[:, None] * P
    nrm = np.linalg.norm(Z, axis=0)
    Z = Z / np.where(nrm > 0, nrm, 1.0)[None, :]
    for k in range(Z.shape[1]):
        i = int(np.argmax(np.abs(Z[:, k])))   # first index of the max magnitude
        if Z[i, k] < 0:
            Z[:, k] = -Z[:, k]
    return Z


# --------------------------------------------------------- full setup/apply

@dataclass
class GenEO:
    prob: object
    A: sp.csr_matrix
    subs: list
    chol: list = field(default_factory=list)      # Cholesky factors of A_j (D_j)
    lam: list = field(default_factory=list)       # per-subdomain eigenvalues
    m: list = field(default_factory=list)         # per-subdomain counts
    Z: sp.csr_matrix = None                       # N x n_c coarse basis
    AH: np.ndarray = None
    LH: np.ndarray = None

    @property
    def nc(self):
        return 0 if self.Z is None else self.Z.shape[1]

    def _uncovered(self):
        """Dofs in no D_j: the eliminated Dirichlet dofs, whose rows of A are
        unit rows; the operator acts as the identity on them."""
        cov = np.zeros(len(self.A.indptr) - 1, dtype=bool)
        for s in self.subs:
            cov[s.dofs[s.dmask]] = True
        return ~cov

    def apply(self, r):
        """z = M_AS,2^{-1} r (Def. 2), identity on the eliminated dofs."""
        z = self.apply_one_level(r)
        if self.nc:
            rH = self.Z.T @ r
            yH = sla.cho_solve((self.LH, True), rH)
            z += self.Z @ yH
        return z

    def apply_one_level(self, r):
        z = np.zeros_like(r)
        for s, L in zip(self.subs, self.chol):
            idx = s.dofs[s.dmask]
            if len(idx):
                z[idx] += sla.cho_solve((L, True), r[idx])
        unc = self._uncovered()
        z[unc] = r[unc]
        return z


def local_setup(prob, A, s, nev, tau, nev_max, coarse, keep_eigvecs, eig_method):
    """Everything one subdomain contributes: the Cholesky factor of its
    Dirichlet matrix A_j (Sec. 3), its eigenvalues (Sec. 4.3-4.4), the count
    m_j (Def. 4 / Thm. 1) and its coarse basis block (Sec. 4.4)."""
    AD = dirichlet_matrix(A, s)
    L = np.linalg.cholesky(AD) if len(AD) else np.zeros((0, 0))
    if not coarse:
        return L, np.zeros(0), 0, None, None
    AN, Ao = local_matrices(prob, s)
    B = s.mu[:, None] * Ao * s.mu[None, :]
    lanczos = eig_method == "lanczos" or (eig_method == "auto" and
                                           len(s.dofs) > LANCZOS_MIN_N)
    want = nev if tau is None else nev_max
    if lanczos and want + 8 < len(s.dofs) - 1:
        ev = generalized_eigen_lanczos(AN, B, want + 8)
    else:
        ev = generalized_eigen(AN, B)
    mj = select_count(ev.lam, nev=nev, tau=tau, nev_max=nev_max)
    Zj = basis_vectors(s.mu, ev.P[:, :mj]) if mj else None
    return L, ev.lam, mj, (ev.P if keep_eigvecs else None), Zj


def setup(prob, A=None, nev=None, tau=None, nev_max=None, coarse=True,
          subs=None, keep_eigvecs=False, eig_method="auto", locs=None):
    """Build the two-level preconditioner of ``prob`` (options default to the
    problem's own).  ``eig_method``: "full" spectrum, "lanczos" for the
    wanted pairs only, or "auto" (Lanczos above LANCZOS_MIN_N local dofs).
    ``locs``: the :func:`local_setup` results of every subdomain, if they
    were computed elsewhere (e.g. in parallel processes); else computed
    here, one subdomain after the other."""
    if A is None:
        A, _ = fem.assemble(prob)
    if subs is None:
        subs, _ = decomp.build(prob)
    if nev is None and tau is None:
        nev, tau, nev_max = prob.nev, prob.tau, prob.nev_max
    g = GenEO(prob=prob, A=A, subs=subs)
    g.eigvecs = [] if keep_eigvecs else None
    if locs is None:
        # tau: one threshold, or one per subdomain (e.g. delta_j / H_j, Thm. 1)
        taus = [None if tau is None else (float(tau) if np.isscalar(tau) else float(tau[s.j]))
                for s in subs]
        locs = [local_setup(prob, A, s, nev, t, nev_max, coarse, keep_eigvecs, eig_method)
                for s, t in zip(subs, taus)]
    cols = []
    for s, (L, lam, mj, P, Zj) in zip(subs, locs):
        g.chol.append(L)
        g.lam.append(lam)
        g.m.append(mj)
        if keep_eigvecs:
            g.eigvecs.append(P)
        if mj:
            cols.append((s, Zj))
    if coarse and cols:
        rows, cidx, vals = [], [], []
        off = 0
        for s, Zj in cols:
            r_, c_ = np.nonzero(Zj)
            rows.append(s.dofs[r_])
            cidx.append(c_ + off)
            vals.append(Zj[r_, c_])
            off += Zj.shape[1]
        g.Z = sp.csr_matrix((np.concatenate(vals),
                             (np.concatenate(rows), np.concatenate(cidx))),
                            shape=(prob.ndof, off))
        AH = (g.Z.T @ (A @ g.Z)).toarray()
        g.AH = 0.5 * (AH + AH.T)
        g.LH = coarse_cholesky(g.AH)
    return g


def coarse_cholesky(AH):
    """Cholesky factor of A_H (Def. 2).  A_H is SPD exactly when the basis
    vectors are linearly independent; a pivot at or below
    n_c * eps * max_k (A_H)_kk (what rounding alone leaves where the exact
    pivot vanishes, e.g. for a repeated basis vector) is taken as singular."""
    nc = AH.shape[0]
    try:
        L = np.linalg.cholesky(AH)
    except np.linalg.LinAlgError as e:
        raise np.linalg.LinAlgError("coarse matrix is not SPD") from e
    tol = nc * np.finfo(np.float64).eps * np.max(np.diag(AH))
    if np.min(np.diag(L)) ** 2 <= tol:
        raise np.linalg.LinAlgError("coarse matrix is numerically singular")
    return L


def coarse_offsets(m):
    return np.concatenate([[0], np.cumsum(m)]).astype(np.int64)
