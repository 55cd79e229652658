"""Pins of the oracle's 20-node serendipity bricks (the element of the
paper's composite experiments, Sec. 5.3), against closed forms written out
here independently of the oracle's formulas:

* the shape functions interpolate (Kronecker delta at the 20 nodes), sum
  to one, reproduce every complete quadratic, and their gradients match
  central differences;
* the element matrix: symmetric, the six rigid-body modes span its kernel,
  and the energy of linear and quadratic displacement fields equals the
  integral of eps^T C eps over the brick in closed form (cross terms of an
  anisotropic C included);
* the consistent load: -V/8 at the vertices, V/6 at the edge midpoints;
* the mesh: node count, lattice positions of every element's nodes, face
  nodes shared with the neighbour; the partition of unity and |N_j|;
* a patch test on the assembled Neumann operator.
"""
import itertools

import numpy as np
import pytest

import synth
from oracle import decomp, fem

RNG = np.random.Generator(np.random.PCG64(20))


def _nodes_ref():
    # reference coordinates in [-1, 1]^3 of the 20 nodes, from the offsets
    return fem.s20_offsets().astype(float) - 1.0


def test_offsets_are_the_vertices_and_edge_midpoints():
    off = fem.s20_offsets()
    assert off.shape == (20, 3)
    assert len({tuple(o) for o in off}) == 20
    odd = (off % 2).sum(axis=1)
    assert np.all(odd[:8] == 0) and np.all(odd[8:] == 1)
    # every edge midpoint is the mean of two vertices one edge apart
    verts = {tuple(o) for o in off[:8]}
    for o in off[8:]:
        ax = int(np.flatnonzero(o % 2)[0])
        a, b = o.copy(), o.copy()
        a[ax], b[ax] = 0, 2
        assert tuple(a) in verts and tuple(b) in verts


def test_shape_functions_interpolate_and_sum_to_one():
    X = _nodes_ref()
    M = np.array([fem.s20_shape_and_grad(x)[0] for x in X])
    assert np.allclose(M, np.eye(20), atol=1e-15)
    for _ in range(20):
        xi = RNG.uniform(-1, 1, 3)
        N, dN = fem.s20_shape_and_grad(xi)
        assert abs(N.sum() - 1.0) < 1e-14
        assert np.allclose(dN.sum(axis=0), 0.0, atol=1e-14)


def test_shape_functions_reproduce_quadratics():
    X = _nodes_ref()
    monos = [lambda p, e=e: np.prod(p ** np.array(e), axis=-1)
             for e in itertools.product(range(3), repeat=3) if sum(e) <= 2]
    assert len(monos) == 10
    for f in monos:
        vals = f(X)
        for _ in range(5):
            xi = RNG.uniform(-1, 1, 3)
            N, _ = fem.s20_shape_and_grad(xi)
            assert abs(N @ vals - f(xi)) < 1e-13


def test_shape_gradients_match_central_differences():
    for _ in range(5):
        xi = RNG.uniform(-0.9, 0.9, 3)
        _, dN = fem.s20_shape_and_grad(xi)
        e = 1e-6
        for i in range(3):
            d = np.zeros(3)
            d[i] = e
            fd = (fem.s20_shape_and_grad(xi + d)[0] - fem.s20_shape_and_grad(xi - d)[0]) / (2 * e)
            assert np.allclose(dN[:, i], fd, atol=1e-8)


def _aniso_C():
    A = RNG.normal(size=(6, 6))
    return A @ A.T + 6 * np.eye(6)


H = np.array([1.5, 0.75, 1.25])


def _nodal(u):
    """Nodal vector (node-major, 3 comps) of a displacement field u(x) on the
    brick [0, hx] x [0, hy] x [0, hz]."""
    X = fem.s20_offsets() * (H[None, :] / 2.0)
    return np.concatenate([u(x) for x in X])


def test_element_rigid_modes_span_the_kernel():
    K = fem.s20_element_matrix(H, _aniso_C())
    assert np.allclose(K, K.T, rtol=0, atol=1e-12 * abs(K).max())
    modes = [lambda x: np.array([1.0, 0, 0]), lambda x: np.array([0, 1.0, 0]),
             lambda x: np.array([0, 0, 1.0]), lambda x: np.array([-x[1], x[0], 0]),
             lambda x: np.array([0, -x[2], x[1]]), lambda x: np.array([x[2], 0, -x[0]])]
    R = np.stack([_nodal(m) for m in modes], axis=1)
    assert np.abs(K @ R).max() <= 1e-12 * abs(K).max()
    ev = np.linalg.eigvalsh(K)
    assert np.sum(ev < 1e-10 * ev.max()) == 6


def test_element_energy_of_linear_fields():
    """u = G x: eps = (G11, G22, G33, G23+G32, G13+G31, G12+G21) constant,
    energy = vol * eps^T C eps."""
    C = _aniso_C()
    K = fem.s20_element_matrix(H, C)
    vol = np.prod(H)
    for _ in range(5):
        G = RNG.normal(size=(3, 3))
        u = _nodal(lambda x: G @ x)
        eps = np.array([G[0, 0], G[1, 1], G[2, 2], G[1, 2] + G[2, 1], G[0, 2] + G[2, 0],
                        G[0, 1] + G[1, 0]])
        assert u @ K @ u == pytest.approx(vol * eps @ C @ eps, rel=1e-12)


def test_element_energy_of_quadratic_fields():
    """u = (x y, 0, 0): eps11 = y, g12 = x, the rest zero; energy =
    C11 int y^2 + 2 C16 int x y + C66 int x^2 over the brick, and
    u = (0, 0, z^2): eps33 = 2 z, energy = 4 C33 int z^2."""
    C = _aniso_C()
    K = fem.s20_element_matrix(H, C)
    hx, hy, hz = H
    ix2, iy2, iz2 = hx ** 3 / 3 * hy * hz, hy ** 3 / 3 * hx * hz, hz ** 3 / 3 * hx * hy
    ixy = hx ** 2 / 2 * hy ** 2 / 2 * hz
    u = _nodal(lambda x: np.array([x[0] * x[1], 0.0, 0.0]))
    e = C[0, 0] * iy2 + 2 * C[0, 5] * ixy + C[5, 5] * ix2
    assert u @ K @ u == pytest.approx(e, rel=1e-12)
    u = _nodal(lambda x: np.array([0.0, 0.0, x[2] ** 2]))
    assert u @ K @ u == pytest.approx(4 * C[2, 2] * iz2, rel=1e-12)


def test_consistent_load_closed_form():
    p = synth.laminate_s20(ne=(2, 2, 1), parts=(1, 1, 1))
    fe = fem.element_load(p).reshape(p.nelem, 20, 3)
    vol = np.prod(p.h)
    load = np.array(p.load)
    assert np.allclose(fe[:, :8, :], -vol / 8 * load, rtol=0, atol=1e-15)
    assert np.allclose(fe[:, 8:, :], vol / 6 * load, rtol=0, atol=1e-15)


def _count_lattice(nb):
    """Nodes of a brick mesh of nb bricks per axis: the vertices and one node
    per edge, counted directly."""
    v = np.prod([n + 1 for n in nb])
    return v + sum(nb[a] * v // (nb[a] + 1) for a in range(3))


def test_mesh_nodes_and_shared_faces():
    p = synth.laminate_s20(ne=(3, 2, 2), parts=(1, 1, 1))
    assert p.nnodes == _count_lattice(p.ne) == len(fem.s20_node_coords(p))
    en = fem.element_nodes(p)
    xyz = fem.s20_node_coords(p)
    off = fem.s20_offsets()
    for e in range(p.nelem):
        ex, ey, ez = e % 3, (e // 3) % 2, e // 6
        assert np.array_equal(xyz[en[e]], 2 * np.array([ex, ey, ez])[None, :] + off)
    # bricks 0 and 1 (neighbours along x) share the 8 nodes of their face
    assert len(set(en[0]) & set(en[1])) == 8


def test_partition_of_unity_and_set_sizes():
    p = synth.laminate_s20(ne=(6, 4, 3), parts=(3, 2, 1), ovl=1)
    subs, _ = decomp.build(p)
    tot = decomp.pou_sum(p, subs)
    d = fem.dirichlet_mask(p)
    assert np.max(np.abs(tot[~d] - 1.0)) <= 1e-15 and np.all(tot[d] == 0.0)
    for s in subs:
        nb = [hi - lo for lo, hi in s.ebox]
        assert len(s.dofs) == 3 * _count_lattice(nb)


def test_patch_test_linear_field():
    """In one material, a linear displacement field is in equilibrium at
    every node inside a brick mesh (no load): the Neumann operator maps it
    to zero there."""
    C = np.broadcast_to(_aniso_C(), (3, 3, 3, 6, 6))    # one material
    p = synth.elasticity_problem("patch", C, (3, 3, 3), (1, 1, 1), 1, dirichlet=0,
                                 load=(0.0, 0.0, 0.0), h=(1.0, 1.0, 1.0), element="s20")
    A = fem.assemble_neumann(p)
    xyz = fem.s20_node_coords(p) / 2.0        # unit bricks
    G = RNG.normal(size=(3, 3))
    u = (xyz @ G.T).ravel()
    r = (A @ u).reshape(-1, 3)
    inner = np.all((xyz > 0) & (xyz < 3), axis=1)
    assert inner.sum() > 0
    assert np.abs(r[inner]).max() <= 1e-11 * np.abs(A.data).max() * np.abs(u).max()
