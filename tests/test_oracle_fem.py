"""Pins of the oracle's Q1 discretisation (Sec. 2, eqs. (2)-(3))."""
import json
import os

import numpy as np
import pytest

import synth
from oracle import fem

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def _node(prob, *c):
    nn = [n + 1 for n in prob.ne]
    k, s = 0, 1
    for ax, x in enumerate(c):
        k += x * s
        s *= nn[ax]
    return k


@pytest.mark.parametrize("n", [8, 13])
def test_2d_stencil_closed_form(n):
    g = _gold("q1_stencils.json")["2d"]
    p = synth.darcy_problem("t", np.ones((n, n)), (1, 1), 1)
    A = fem.assemble_neumann(p).toarray()
    c = _node(p, 4, 5)
    assert A[c, c] == pytest.approx(g["center"], rel=1e-14)
    for dx in (-1, 0, 1):
        for dy in (-1, 0, 1):
            if dx == dy == 0:
                continue
            kind = "corner" if dx and dy else "edge"
            assert A[c, _node(p, 4 + dx, 5 + dy)] == pytest.approx(g[kind], rel=1e-14)
    assert np.count_nonzero(np.abs(A[c]) > 1e-15) == 9


def test_2d_element_matrix_closed_form():
    g = _gold("q1_stencils.json")["element_2d"]
    K = fem.darcy_element_matrix((0.25, 0.25))
    # vertices 0:(0,0) 1:(1,0) 2:(0,1) 3:(1,1)
    assert np.allclose(np.diag(K), g["diag"], rtol=1e-14)
    assert K[0, 1] == pytest.approx(g["edge"]) and K[0, 2] == pytest.approx(g["edge"])
    assert K[0, 3] == pytest.approx(g["opposite"]) and K[1, 2] == pytest.approx(g["opposite"])


@pytest.mark.parametrize("n", [6, 9])
def test_3d_stencil_closed_form(n):
    g = _gold("q1_stencils.json")["3d"]
    h = 1.0 / n
    p = synth.darcy_problem("t", np.ones((n, n, n)), (1, 1, 1), 1)
    A = fem.assemble_neumann(p).tocsr()
    c = _node(p, 3, 3, 2)
    row = A[c].toarray().ravel()
    names = {0: "center_over_h", 1: "face_over_h", 2: "edge_over_h", 3: "corner_over_h"}
    for dx in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dz in (-1, 0, 1):
                nz = (dx != 0) + (dy != 0) + (dz != 0)
                v = row[_node(p, 3 + dx, 3 + dy, 2 + dz)]
                assert v == pytest.approx(g[names[nz]] * h, abs=1e-15)


def test_neumann_row_sums_vanish_with_variable_kappa():
    rng = np.random.Generator(np.random.PCG64(3))
    k = np.exp(rng.normal(size=(7, 9)))
    p = synth.darcy_problem("t", k, (1, 1), 1)
    A = fem.assemble_neumann(p)
    assert np.max(np.abs(A @ np.ones(p.ndof))) < 1e-13 * np.max(k)
    assert abs(A - A.T).max() <= 1e-15 * np.max(k)


def test_total_load_equals_f_times_volume():
    p = synth.darcy_problem("t", np.ones((5, 7)), (1, 1), 1, load=3.0)
    fe = fem.element_load(p)
    assert fe.sum() == pytest.approx(3.0 * 1.0, rel=1e-14)


def test_dirichlet_elimination():
    p = synth.channels_2d(0, n=16, parts=2, n_channels=2)
    A, b = fem.assemble(p)
    d = fem.dirichlet_mask(p)
    Ad = A.toarray()
    assert np.array_equal(Ad, Ad.T)
    assert np.all(Ad[d][:, d] == np.eye(d.sum()))
    assert np.all(Ad[d][:, ~d] == 0) and np.all(b[d] == 0)
    assert np.all(b[~d] > 0)


def _manufactured_error(n):
    p = synth.darcy_problem("t", np.ones((n, n)), (1, 1), 1)

    def f(x):
        return 2 * np.pi ** 2 * np.sin(np.pi * x[:, 0]) * np.sin(np.pi * x[:, 1])

    A, b = fem.assemble(p, f=f)
    import scipy.sparse.linalg as spla
    u = spla.spsolve(A.tocsc(), b)
    xs = np.arange(n + 1) / n
    X, Y = np.meshgrid(xs, xs, indexing="xy")
    ex = (np.sin(np.pi * X) * np.sin(np.pi * Y)).ravel()
    return np.max(np.abs(u - ex))


def test_manufactured_solution_second_order():
    e = [_manufactured_error(n) for n in (8, 16, 32)]
    assert e[0] / e[1] > 3.5 and e[1] / e[2] > 3.5
    assert e[2] < 5e-3


def _rbm(coords):
    x, y, z = coords.T
    o, zr = np.ones_like(x), np.zeros_like(x)
    modes = [(o, zr, zr), (zr, o, zr), (zr, zr, o),
             (-y, x, zr), (zr, -z, y), (z, zr, -x)]
    return np.array([np.stack(m, axis=1).ravel() for m in modes]).T


def test_elasticity_element_kernel_is_rigid_body_modes():
    ply = synth.ply_stiffness(160.0, 10.0, 10.0, 5.0, 5.0, 5.0, 0.3, 0.3, 0.3)
    for C in (ply, synth.rotate_z90(ply), synth.isotropic_stiffness(4.0, 0.35)):
        K = fem.elasticity_element_matrix((1.0, 0.7, 1.3), C)
        ev = np.linalg.eigvalsh(K)
        assert np.sum(np.abs(ev) < 1e-10 * ev[-1]) == 6
        assert ev[6] > 1e-6 * ev[-1]
        off = np.array([[(a >> i) & 1 for i in range(3)] for a in range(8)], float)
        R = _rbm(off * np.array([1.0, 0.7, 1.3]))
        assert np.max(np.abs(K @ R)) < 1e-12 * ev[-1]


def test_elasticity_patch_test():
    C = synth.ply_stiffness(160.0, 10.0, 10.0, 5.0, 5.0, 5.0, 0.3, 0.3, 0.3)
    ne = (4, 3, 3)
    Cs = np.broadcast_to(C, (3, 3, 4, 6, 6))
    p = synth.elasticity_problem("t", Cs, ne, (1, 1, 1), 1, dirichlet=0,
                                 load=(0.0, 0.0, 0.0), h=(0.5, 1.0, 2.0))
    A = fem.assemble_neumann(p)
    nn = [n + 1 for n in ne]
    k = np.arange(p.nnodes)
    ix, iy, iz = k % nn[0], (k // nn[0]) % nn[1], k // (nn[0] * nn[1])
    coords = np.stack([ix * 0.5, iy * 1.0, iz * 2.0], axis=1)
    rng = np.random.Generator(np.random.PCG64(1))
    Gm = rng.normal(size=(3, 3))
    u = (coords @ Gm.T).ravel()
    r = (A @ u).reshape(-1, 3)
    inner = (ix > 0) & (ix < ne[0]) & (iy > 0) & (iy < ne[1]) & (iz > 0) & (iz < ne[2])
    assert np.max(np.abs(r[inner])) < 1e-11 * np.max(np.abs(A.data)) * np.max(np.abs(u))
    # six-dimensional kernel of the free assembled operator
    R = _rbm(coords)
    assert np.max(np.abs(A @ R)) < 1e-11 * np.max(np.abs(A.data)) * np.max(np.abs(R))


# ------------------------------------------------ elasticity constitutive pins
# Sec. 2, eq. (3): the bilinear form integrates C eps(u) : eps(v).  The pins
# below fix the strain-displacement map (engineering shear, Voigt order 11,
# 22, 33, 23, 13, 12) and the constitutive coupling independently of the
# oracle's strain matrix: the six-zero-mode and patch pins above hold for
# any symmetric C and any scaling of the shear rows.

def _engineering_strain(G):
    """Voigt strain of the linear field u(x) = G x, written out from the
    definition eps_ij = (G_ij + G_ji) / 2 with engineering shear 2 eps_ij."""
    return np.array([G[0, 0], G[1, 1], G[2, 2],
                     G[1, 2] + G[2, 1], G[0, 2] + G[2, 0], G[0, 1] + G[1, 0]])


def _random_spd_voigt(seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    M = rng.normal(size=(6, 6))
    return M @ M.T + 6.0 * np.eye(6)


@pytest.mark.parametrize("which", ["ply", "ply90", "resin", "random"])
def test_elasticity_element_energy_of_linear_fields(which):
    """For u = G x the strain is constant, 2-point Gauss is exact, and the
    element energy is u^T K_e u = vol * eps(G)^T C eps(G)."""
    ply = synth.ply_stiffness(160.0, 10.0, 10.0, 5.0, 5.0, 5.0, 0.3, 0.3, 0.3)
    C = {"ply": ply, "ply90": synth.rotate_z90(ply),
         "resin": synth.isotropic_stiffness(4.0, 0.35), "random": _random_spd_voigt(5)}[which]
    h = np.array([0.8, 1.1, 0.6])
    K = fem.elasticity_element_matrix(h, C)
    off = np.array([[(a >> i) & 1 for i in range(3)] for a in range(8)], float) * h
    rng = np.random.Generator(np.random.PCG64(17))
    for _ in range(6):
        G = rng.normal(size=(3, 3))
        u = (off @ G.T).ravel()            # vertex-major, 3 components
        eps = _engineering_strain(G)
        exact = np.prod(h) * eps @ C @ eps
        assert u @ K @ u == pytest.approx(exact, rel=1e-12)
    # pure shear fields excite only the shear block of C
    for (i, j, v) in ((0, 1, 5), (0, 2, 4), (1, 2, 3)):
        G = np.zeros((3, 3))
        G[i, j] = 1.0
        u = (off @ G.T).ravel()
        assert u @ K @ u == pytest.approx(np.prod(h) * C[v, v], rel=1e-12)


def _bar_nodal_traction(prob, sigma0):
    """Consistent nodal loads of the uniform tractions +-sigma0 e_x on the
    end faces x = 0 and x = L of a box: each bilinear face element passes a
    quarter of its force to each of its four nodes."""
    nx, ny, nz = prob.ne
    hx, hy, hz = prob.h
    f = np.zeros((prob.nnodes, 3))
    wy = np.full(ny + 1, hy)
    wy[[0, -1]] = hy / 2
    wz = np.full(nz + 1, hz)
    wz[[0, -1]] = hz / 2
    for iz in range(nz + 1):
        for iy in range(ny + 1):
            w = wy[iy] * wz[iz]
            k0 = 0 + (nx + 1) * (iy + (ny + 1) * iz)
            k1 = nx + (nx + 1) * (iy + (ny + 1) * iz)
            f[k0, 0] -= sigma0 * w
            f[k1, 0] += sigma0 * w
    return f.ravel()


@pytest.mark.parametrize("which", ["resin", "ply", "ply90"])
def test_elasticity_uniaxial_bar_closed_form(which):
    """A bar pulled by end tractions sigma0, held only against rigid motions
    (six single-component supports), is in uniaxial stress: its displacement
    is u = diag(eps_1, eps_2, eps_3) x with eps from the engineering
    constants (eps_1 = sigma0 / E_x, eps_2 = -nu_xy sigma0 / E_x, ...), which
    Q1 reproduces exactly."""
    E1, E2, E3, G12, nu12, nu13, nu23 = 160.0, 10.0, 10.0, 5.0, 0.3, 0.3, 0.3
    ply = synth.ply_stiffness(E1, E2, E3, G12, G12, G12, nu12, nu13, nu23)
    sigma0 = 0.37
    if which == "resin":
        E, nu = 4.0, 0.35
        C = synth.isotropic_stiffness(E, nu)
        eps = sigma0 / E * np.array([1.0, -nu, -nu])
    elif which == "ply":
        C = ply
        eps = sigma0 / E1 * np.array([1.0, -nu12, -nu13])
    else:   # fibre along y: pulled across the fibres, nu_21 = nu_12 E2 / E1
        C = synth.rotate_z90(ply)
        eps = sigma0 / E2 * np.array([1.0, -nu12 * E2 / E1, -nu23])
    ne, h = (6, 2, 3), (0.5, 0.4, 0.3)
    Cs = np.broadcast_to(C, (ne[2], ne[1], ne[0], 6, 6))
    p = synth.elasticity_problem("bar", Cs, ne, (1, 1, 1), 1, dirichlet=0,
                                 load=(0.0, 0.0, 0.0), h=h)
    K = fem.assemble_neumann(p).tocsr()
    f = _bar_nodal_traction(p, sigma0)
    # supports: node (0,0,0) all components, (L,0,0) y and z, (0,H,0) z
    nx, ny = ne[0], ne[1]
    fixed = [0, 1, 2, 3 * nx + 1, 3 * nx + 2, 3 * (nx + 1) * ny + 2]
    free = np.setdiff1d(np.arange(p.ndof), fixed)
    import scipy.sparse.linalg as spla
    u = np.zeros(p.ndof)
    u[free] = spla.spsolve(K[free][:, free].tocsc(), f[free])
    k = np.arange(p.nnodes)
    coords = np.stack([(k % (nx + 1)) * h[0], ((k // (nx + 1)) % (ny + 1)) * h[1],
                       (k // ((nx + 1) * (ny + 1))) * h[2]], axis=1)
    exact = (coords * eps[None, :]).ravel()
    assert np.max(np.abs(u - exact)) <= 1e-11 * np.max(np.abs(exact))
    # the supports carry no reaction: the end tractions are self-equilibrated
    assert np.max(np.abs((K @ exact - f))) <= 1e-11 * sigma0


@pytest.mark.parametrize("h", [(0.25, 0.25), (0.1, 0.37), (1.0 / 96, 1.0 / 96, 1.0 / 96),
                               (0.5, 1.0, 2.0)])
def test_closed_form_darcy_element_matrix_matches_quadrature(h):
    """The closed-form element matrix the assembly uses and the 2-point
    Gauss rule (exact for it) agree to rounding, and both have (near) zero
    row sums."""
    Kq = fem.darcy_element_matrix(h)
    Kc = fem.darcy_element_matrix_exact(h)
    scale = np.abs(Kq).max()
    assert np.max(np.abs(Kq - Kc)) <= 4e-16 * scale
    assert np.max(np.abs(Kc.sum(axis=1))) <= 4e-16 * scale
    assert np.array_equal(Kc, Kc.T)


def test_assembly_sums_contributions_in_element_order():
    """Each entry is the sum of its element contributions added in ascending
    element order from 0 (the order the device uses), for a field with
    contributions of very different sizes."""
    rng = np.random.Generator(np.random.PCG64(21))
    k = 10.0 ** rng.uniform(-6, 6, size=(5, 6))
    p = synth.darcy_problem("t", k, (1, 1), 1, dirichlet=0)
    A = fem.assemble_neumann(p).tolil()
    Ao, _ = fem.assemble(p)
    Kc = fem.darcy_element_matrix_exact(p.h)
    dofs = fem.element_dofs(p)
    ref = {}
    for e in range(p.nelem):
        for a in range(4):
            for b in range(4):
                key = (dofs[e, a], dofs[e, b])
                ref[key] = ref.get(key, 0.0) + k.ravel()[e] * Kc[a, b]
    for (i, j), v in ref.items():
        assert Ao[i, j] == v          # bitwise
