"""Plant plausible mistakes in the oracle (on the CPU) and check that the
pins catch them: a wrong sign of the shift, a dropped partition-of-unity
weight in the eigenproblem, a dropped operator in the coarse matrix, a
wrong PoU count, an inverted CG coefficient.  Each planted mistake must
make at least one pin fail."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synth
from oracle import decomp, fem, geneo, pcg


def _prob():
    rng = np.random.Generator(np.random.PCG64(0))
    k = np.where(rng.uniform(size=(12, 12)) < 0.2, 1e4, 1.0)
    return synth.darcy_problem("t", k, (3, 3), 2, nev=3)


def pin_inertia_of_setup(prob):
    """#neg(A_N - tau X A^o X) == #{lam < tau} for the setup's eigenvalues,
    with B built here from its definition."""
    A, _ = fem.assemble(prob)
    subs, _ = decomp.build(prob)
    g = geneo.setup(prob, A=A, subs=subs)
    for s, lam in zip(subs, g.lam):
        AN, Ao = geneo.local_matrices(prob, s)
        B = np.diag(s.mu) @ Ao @ np.diag(s.mu)
        for tau in (0.05, 0.3, 1.0):
            if np.sum(np.linalg.eigvalsh(AN - tau * B) < 0) != np.sum(lam < tau):
                return False
    return True


def pin_kernel_eigenvalue_zero(prob):
    subs, _ = decomp.build(prob)
    s = [x for x in subs if not x.dirichlet.any()][0]
    AN, Ao = geneo.local_matrices(prob, s)
    ev = geneo.generalized_eigen(AN, s.mu[:, None] * Ao * s.mu[None, :])
    return abs(ev.lam[0]) < 1e-10


def pin_coarse_brute_force(prob):
    A, _ = fem.assemble(prob)
    g = geneo.setup(prob, A=A)
    Z = g.Z.toarray()
    return np.allclose(g.AH, Z.T @ A.toarray() @ Z, atol=1e-12 * np.abs(g.AH).max())


def pin_pou_sum(prob):
    subs, _ = decomp.build(prob)
    tot = decomp.pou_sum(prob, subs)
    d = fem.dirichlet_mask(prob)
    return np.max(np.abs(tot[~d] - 1.0)) <= 1e-15


def pin_pcg_direct(prob):
    A, b = fem.assemble(prob)
    g = geneo.setup(prob, A=A)
    r = pcg.pcg(A, b, g.apply, rtol=1e-10, maxit=300)
    xd = spla.spsolve(A.tocsc(), b)
    return r.converged and np.linalg.norm(r.x - xd) <= 1e-8 * np.linalg.norm(xd)


PINS = [pin_inertia_of_setup, pin_kernel_eigenvalue_zero, pin_coarse_brute_force,
        pin_pou_sum, pin_pcg_direct]


def test_pins_hold_on_the_real_oracle():
    p = _prob()
    for pin in PINS:
        assert pin(p), pin.__name__


def _caught(monkeypatch_ctx):
    p = _prob()
    results = []
    for pin in PINS:
        try:
            results.append(pin(p))
        except Exception:
            results.append(False)
    return not all(results)


def test_wrong_shift_sign_is_caught(monkeypatch):
    orig = geneo.generalized_eigen

    def bad(AN, B, sigma=geneo.SIGMA):
        ev = orig(AN, B, sigma)
        fin = np.isfinite(ev.lam)
        ev.lam[fin] = ev.lam[fin] - 2 * sigma      # lam = -sigma + 1/nu
        return ev
    monkeypatch.setattr(geneo, "generalized_eigen", bad)
    assert _caught(monkeypatch)


def test_dropped_pou_weight_in_B_is_caught(monkeypatch):
    orig = geneo.local_matrices

    def bad_setup_local(prob, sub):
        AN, Ao = orig(prob, sub)
        return AN, Ao / np.where(np.outer(sub.mu, sub.mu) > 0, np.outer(sub.mu, sub.mu), 1.0)
    monkeypatch.setattr(geneo, "local_matrices", bad_setup_local)
    # the pin builds B from the definition with the unmodified weights
    p = _prob()
    monkeypatch.setattr(geneo, "local_matrices", orig)
    A, _ = fem.assemble(p)
    subs, _ = decomp.build(p)
    monkeypatch.setattr(geneo, "local_matrices", bad_setup_local)
    g = geneo.setup(p, A=A, subs=subs)
    monkeypatch.setattr(geneo, "local_matrices", orig)
    ok = True
    for s, lam in zip(subs, g.lam):
        AN, Ao = geneo.local_matrices(p, s)
        B = np.diag(s.mu) @ Ao @ np.diag(s.mu)
        for tau in (0.05, 0.3, 1.0):
            ok &= np.sum(np.linalg.eigvalsh(AN - tau * B) < 0) == np.sum(lam < tau)
    assert not ok


def test_dropped_operator_in_coarse_matrix_is_caught(monkeypatch):
    orig = geneo.setup

    def bad(prob, **kw):
        g = orig(prob, **kw)
        if g.Z is not None:
            g.AH = (g.Z.T @ g.Z).toarray()
        return g
    monkeypatch.setattr(geneo, "setup", bad)
    assert _caught(monkeypatch)


def test_wrong_pou_count_is_caught(monkeypatch):
    orig = decomp.build

    def bad(prob):
        subs, mult = orig(prob)
        for s in subs:
            s.mu = np.where(s.mu > 0, 1.0 / (1.0 / np.where(s.mu > 0, s.mu, 1.0) + 1.0), 0.0)
        return subs, mult
    monkeypatch.setattr(decomp, "build", bad)
    assert _caught(monkeypatch)


def test_inverted_cg_coefficient_is_caught(monkeypatch):
    def bad_pcg(A, b, apply_M, rtol=1e-10, maxit=2000):
        x = np.zeros_like(b)
        r = b.copy()
        z = apply_M(r)
        p = z.copy()
        rz = r @ z
        res = pcg.PCGResult(x=x, iters=0, converged=False, relres=1.0)
        for k in range(1, maxit + 1):
            q = A @ p
            alpha = rz / (p @ q)
            x += alpha * p
            r -= alpha * q
            res.iters = k
            if np.linalg.norm(r) <= rtol * np.linalg.norm(b):
                res.converged = True
                break
            z = apply_M(r)
            rz_new = r @ z
            beta = rz / rz_new          # inverted
            rz = rz_new
            p = z + beta * p
        res.x = x
        return res
    monkeypatch.setattr(pcg, "pcg", bad_pcg)
    assert _caught(monkeypatch)


# ---------------------------------------------- elasticity element mutations
def _elasticity_pins_hold():
    """The closed-form elasticity pins of test_oracle_fem, run as booleans."""
    import test_oracle_fem as T
    ok = True
    for which in ("ply", "ply90", "resin", "random"):
        try:
            T.test_elasticity_element_energy_of_linear_fields(which)
        except AssertionError:
            ok = False
    for which in ("resin", "ply", "ply90"):
        try:
            T.test_elasticity_uniaxial_bar_closed_form(which)
        except AssertionError:
            ok = False
    return ok


def test_elasticity_pins_hold_on_the_real_oracle():
    assert _elasticity_pins_hold()


def test_tensorial_shear_strain_is_caught(monkeypatch):
    """Shear rows of the strain matrix halved (tensorial instead of
    engineering shear): the kernel and patch pins still pass, the energy
    pin must not."""
    orig = fem.strain_matrix

    def bad(grad_phys):
        B = orig(grad_phys)
        B[3:, :] *= 0.5
        return B
    monkeypatch.setattr(fem, "strain_matrix", bad)
    assert not _elasticity_pins_hold()


def test_scaled_shear_modulus_is_caught(monkeypatch):
    orig = fem.elasticity_element_matrix

    def bad(h, C):
        C2 = np.array(C, dtype=float)
        C2[3:, 3:] *= 2.0
        return orig(h, C2)
    monkeypatch.setattr(fem, "elasticity_element_matrix", bad)
    assert not _elasticity_pins_hold()


def test_dropped_poisson_coupling_is_caught(monkeypatch):
    orig = fem.elasticity_element_matrix

    def bad(h, C):
        C2 = np.array(C, dtype=float)
        C2[:3, :3] = np.diag(np.diag(C2[:3, :3]))
        return orig(h, C2)
    monkeypatch.setattr(fem, "elasticity_element_matrix", bad)
    assert not _elasticity_pins_hold()


# ---------------------------------------------- serendipity brick mutations

def _s20_pins():
    """The serendipity pins of tests/test_oracle_s20.py, all at once."""
    import test_oracle_s20 as T
    try:
        T.test_shape_functions_interpolate_and_sum_to_one()
        T.test_shape_functions_reproduce_quadratics()
        T.test_element_rigid_modes_span_the_kernel()
        T.test_element_energy_of_linear_fields()
        T.test_element_energy_of_quadratic_fields()
        T.test_consistent_load_closed_form()
    except AssertionError:
        return False
    return True


def test_s20_pins_hold_on_the_real_oracle():
    assert _s20_pins()


def test_s20_wrong_vertex_shape_function_is_caught(monkeypatch):
    """Vertex functions with (c . xi - 1) instead of (c . xi - 2)."""
    real = fem.s20_shape_and_grad

    def wrong(xi):
        N, dN = real(xi)
        off = fem.s20_offsets()[:8] - 1
        for a in range(8):
            t = np.prod(1.0 + off[a] * xi)
            N[a] += t / 8.0
        return N, dN
    monkeypatch.setattr(fem, "s20_shape_and_grad", wrong)
    assert not _s20_pins()


def test_s20_two_point_rule_is_caught(monkeypatch):
    """The 2-point Gauss rule (exact for Q1 products, not for the
    serendipity brick's degree-4 integrands)."""
    monkeypatch.setattr(fem, "_G3", np.array([-1.0 / np.sqrt(3.0), 1.0 / np.sqrt(3.0), 0.0]))
    monkeypatch.setattr(fem, "_W3", np.array([1.0, 1.0, 0.0]))
    assert not _s20_pins()
