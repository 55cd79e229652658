"""Preconditioned conjugate gradients (oracle; test infrastructure).

Textbook Hestenes-Stiefel PCG as used for every experiment of Sec. 5,
stopped on a residual reduction: x_0 = 0 and the iteration stops as soon as
||b - A x_k||_2 (the recurrence residual) is at most rtol * ||b||_2.  The
iteration count is the number of products with A.  The condition number
reported beside iterations (Table 1, Table 2) is estimated from the CG
coefficients through the Lanczos tridiagonal matrix
T_kk = 1/alpha_k + beta_{k-1}/alpha_{k-1}, T_{k,k+1} = sqrt(beta_k)/alpha_k.

Beside it, iterative refinement with residuals in extended precision, for
reference solutions of badly conditioned systems, where a plain FP64
solve is only accurate to about u kappa(A).

Pins (tests/test_oracle_pcg.py): agreement with a sparse direct solve,
exact termination in one step when the preconditioner is A^{-1}, the true
residual matching the recurrence residual, the Lanczos estimate against
the eigenvalues of the preconditioned operator on a small case, the
extended residual against exact rational arithmetic, and refined GenEO-PCG
against refined sparse LU (two independent routes to A^{-1} b).
"""
from dataclasses import dataclass, field

import numpy as np


@dataclass
class PCGResult:
    x: np.ndarray
    iters: int
    converged: bool
    relres: float
    alphas: list = field(default_factory=list)
    betas: list = field(default_factory=list)
    resid: list = field(default_factory=list)


def pcg(A, b, apply_M, rtol=1e-10, maxit=2000):
    x = np.zeros_like(b)
    r = b.copy()
    bnorm = np.linalg.norm(b)
    res = PCGResult(x=x, iters=0, converged=False, relres=1.0)
    if bnorm == 0.0:
        res.converged, res.relres = True, 0.0
        return res
    z = apply_M(r)
    p = z.copy()
    rz = r @ z
    for k in range(1, maxit + 1):
        q = A @ p
        alpha = rz / (p @ q)
        x += alpha * p
        r -= alpha * q
        res.alphas.append(alpha)
        rn = np.linalg.norm(r)
        res.resid.append(rn / bnorm)
        res.iters = k
        if rn <= rtol * bnorm:
            res.converged = True
            break
        z = apply_M(r)
        rz_new = r @ z
        beta = rz_new / rz
        res.betas.append(beta)
        rz = rz_new
        p = z + beta * p
    res.x = x
    res.relres = res.resid[-1] if res.resid else 0.0
    return res


def lanczos_tridiagonal(alphas, betas):
    """The k x k Lanczos matrix of k CG steps."""
    k = len(alphas)
    T = np.zeros((k, k))
    for i in range(k):
        T[i, i] = 1.0 / alphas[i] + (betas[i - 1] / alphas[i - 1] if i > 0 else 0.0)
        if i + 1 < k:
            T[i, i + 1] = T[i + 1, i] = np.sqrt(betas[i]) / alphas[i]
    return T


def kappa_estimate(alphas, betas):
    if len(alphas) == 0:
        return 1.0
    ev = np.linalg.eigvalsh(lanczos_tridiagonal(alphas, betas[:len(alphas) - 1]))
    return float(ev[-1] / ev[0])


def residual_extended(A, b, x):
    """b - A x with every product and sum in extended precision (numpy's
    longdouble: the x87 80-bit format here, unit roundoff 2^-64), rounded
    to FP64 once at the end."""
    A = A.tocsr()
    ld = np.longdouble
    prod = A.data.astype(ld) * np.asarray(x, dtype=ld)[A.indices]
    rows = np.add.reduceat(prod, A.indptr[:-1]) if prod.size else np.zeros(A.shape[0], ld)
    rows[np.diff(A.indptr) == 0] = 0
    return (np.asarray(b, dtype=ld) - rows).astype(np.float64)


def refine(A, b, x, solve, steps=2):
    """Iterative refinement (Wilkinson; see Higham, Accuracy and Stability
    of Numerical Algorithms, ch. 12): r = b - A x in extended precision,
    d = solve(r) in FP64, x += d, ``steps`` times.  The residual's extra
    precision moves the attainable forward error from u kappa(A) (FP64
    residuals) towards u."""
    x = np.array(x, dtype=np.float64)
    for _ in range(steps):
        r = residual_extended(A, b, x)
        if not np.any(r):
            break
        x = x + solve(r)
    return x
