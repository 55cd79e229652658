"""Q1 and 20-node serendipity finite elements on a structured box grid
(oracle; test infrastructure).

Discretises the Darcy form (Sec. 2, eq. (2)) and the linear-elasticity form
(Sec. 2, eq. (3), no traction term) with a conforming space of continuous
(tri)linear Q1 functions, as the paper's Sec. 5.2 experiments use Q1
elements.  Element integrals use the tensor 2-point Gauss rule, which is
exact for products of Q1 gradients with a constant coefficient; the Darcy
element matrix is taken in its closed form (1D stiffness and mass factors),
which is that integral up to rounding.  Every global and local matrix entry
sums its element contributions in ascending element order, from zero.

Homogeneous Dirichlet conditions (``u = 0`` on the flagged faces) are
imposed by symmetric elimination: the row and column of a constrained degree
of freedom are zeroed, its diagonal set to 1 and its load to 0.  With zero
boundary data the free unknowns are exactly those of the eliminated system.

Pins (tests/test_oracle_fem.py): closed-form Q1 stencils, zero row sums of
the Neumann operator, O(h^2) nodal convergence to a manufactured solution,
the six rigid-body modes spanning the kernel of a free elasticity element, a
patch test, the element energy of every linear field (vol * eps^T C eps with
engineering shear strains, written out independently of the strain matrix)
and a bar in uniaxial stress whose displacement follows from the engineering
constants (E, nu) in closed form.
"""
import itertools

import numpy as np
import scipy.sparse as sp

_G = np.array([0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0)])  # on [0,1]
_W = np.array([0.5, 0.5])


def _local_offsets(dim):
    """Offsets of the 2^d element vertices, vertex a <-> bits (x, y, z) of a."""
    return np.array([[(a >> i) & 1 for i in range(dim)] for a in range(2 ** dim)])


def _shape_and_grad(dim, xi):
    """Q1 shape values and reference gradients at a point xi of [0,1]^d."""
    off = _local_offsets(dim)
    nv = len(off)
    phi = np.ones(nv)
    grad = np.ones((nv, dim))
    for a in range(nv):
        for i in range(dim):
            f = xi[i] if off[a, i] else 1.0 - xi[i]
            phi[a] *= f
            for j in range(dim):
                if j == i:
                    grad[a, j] *= 1.0 if off[a, i] else -1.0
                else:
                    grad[a, j] *= f
    return phi, grad


def quadrature(dim):
    """Tensor Gauss points on [0,1]^d and their weights."""
    pts, wts = [], []
    for idx in itertools.product(range(2), repeat=dim):
        pts.append([_G[i] for i in idx])
        wts.append(np.prod([_W[i] for i in idx]))
    return np.array(pts), np.array(wts)


def darcy_element_matrix_exact(h):
    """The same element matrix in closed form.  With the 1D stiffness
    k(i, j) = +-1 and the 1D mass m(i, j) = (1/3, 1/6) = mi / 6 (mi = 2, 1),

        K_ab = 6^{1-d} sum_x (prod_{y != x} h_y / h_x) k(a_x, b_x) prod_{y != x} mi(a_y, b_y),

    evaluated in this order: the ratio of the edge lengths, times the
    integer factor (a power of two, exact), summed over the axes in order,
    divided by 6^{d-1} once.  Every step but the ratios and the final
    division is exact, so the rows sum to zero up to those two roundings."""
    h = np.asarray(h, dtype=np.float64)
    dim = len(h)
    off = _local_offsets(dim)
    nv = 2 ** dim
    K = np.zeros((nv, nv))
    for a in range(nv):
        for b in range(nv):
            s = 0.0
            for ax in range(dim):
                c = 1.0
                for o in range(dim):
                    if o != ax:
                        c = c * h[o]
                c = c / h[ax]
                f = 1 if off[a, ax] == off[b, ax] else -1
                for o in range(dim):
                    if o != ax:
                        f *= 2 if off[a, o] == off[b, o] else 1
                s = s + c * float(f)
            K[a, b] = s / (6.0 ** (dim - 1))
    return K


def darcy_element_matrix(h):
    """Element matrix of int grad v . grad w over one box element, kappa = 1,
    by the tensor 2-point Gauss rule."""
    h = np.asarray(h, dtype=np.float64)
    dim = len(h)
    pts, wts = quadrature(dim)
    vol = np.prod(h)
    K = np.zeros((2 ** dim, 2 ** dim))
    for x, w in zip(pts, wts):
        _, g = _shape_and_grad(dim, x)
        g = g / h[None, :]
        K += w * vol * g @ g.T
    return K


def strain_matrix(grad_phys):
    """6 x 24 strain-displacement matrix (Voigt 11,22,33,23,13,12; engineering shear)."""
    nv = grad_phys.shape[0]
    B = np.zeros((6, 3 * nv))
    for a in range(nv):
        dx, dy, dz = grad_phys[a]
        c = 3 * a
        B[0, c + 0] = dx
        B[1, c + 1] = dy
        B[2, c + 2] = dz
        B[3, c + 1], B[3, c + 2] = dz, dy
        B[4, c + 0], B[4, c + 2] = dz, dx
        B[5, c + 0], B[5, c + 1] = dy, dx
    return B


def elasticity_element_matrix(h, C):
    """Element matrix of int C eps(v):eps(w) over one box element (3D)."""
    h = np.asarray(h, dtype=np.float64)
    pts, wts = quadrature(3)
    vol = np.prod(h)
    K = np.zeros((24, 24))
    for x, w in zip(pts, wts):
        _, g = _shape_and_grad(3, x)
        B = strain_matrix(g / h[None, :])
        K += w * vol * B.T @ C @ B
    return K


# --------------------------------------------- 20-node serendipity bricks
#
# The quadratic serendipity brick (the element of the paper's composite
# experiments, Sec. 5.3): nodes at the 8 vertices and the 12 edge midpoints.
# Nodes of a mesh of ne bricks live on the lattice of half-edge steps,
# coordinates 0 .. 2 ne per axis, at the points with at most one odd
# coordinate; they are numbered lexicographically (x fastest) over those
# points, which keeps the matrices banded.  Element integrals use the tensor
# 3-point Gauss rule, exact for the products of the shape gradients (degree
# at most 4 per coordinate) with a constant coefficient.

_G3 = np.array([-np.sqrt(0.6), 0.0, np.sqrt(0.6)])  # on [-1, 1]
_W3 = np.array([5.0, 8.0, 5.0]) / 9.0


def s20_offsets():
    """Local nodes as lattice offsets in {0, 1, 2}^3: the 8 vertices (bit i of
    the index = coordinate i), then the midpoints of the edges along x, y
    and z (4 each, the other two coordinates in bit order)."""
    corners = [[2 * ((a >> i) & 1) for i in range(3)] for a in range(8)]
    edges = []
    for ax in range(3):
        o1, o2 = [o for o in range(3) if o != ax]
        for b in range(4):
            o = [0, 0, 0]
            o[ax] = 1
            o[o1] = 2 * (b & 1)
            o[o2] = 2 * (b >> 1)
            edges.append(o)
    return np.array(corners + edges)


def s20_shape_and_grad(xi):
    """Serendipity shape values and gradients at xi in the reference brick
    [-1, 1]^3: a vertex node at c in {-1, 1}^3 has
    N = (c . xi - 2) prod_i (1 + c_i xi_i) / 8, an edge midpoint with c_a = 0
    has N = (1 - xi_a^2) prod_{i != a} (1 + c_i xi_i) / 4."""
    off = s20_offsets()
    N = np.zeros(20)
    dN = np.zeros((20, 3))
    for a, o in enumerate(off):
        c = o - 1
        t = 1.0 + c * xi
        if np.all(c != 0):
            s = float(np.dot(c, xi)) - 2.0
            p = t[0] * t[1] * t[2]
            N[a] = p * s / 8.0
            for i in range(3):
                pi = np.prod([t[j] for j in range(3) if j != i])
                dN[a, i] = (c[i] * pi * s + p * c[i]) / 8.0
        else:
            ax = int(np.flatnonzero(c == 0)[0])
            q = 1.0 - xi[ax] ** 2
            o1, o2 = [i for i in range(3) if i != ax]
            N[a] = q * t[o1] * t[o2] / 4.0
            dN[a, ax] = -2.0 * xi[ax] * t[o1] * t[o2] / 4.0
            dN[a, o1] = q * c[o1] * t[o2] / 4.0
            dN[a, o2] = q * c[o2] * t[o1] / 4.0
    return N, dN


def s20_quadrature():
    """Tensor 3-point Gauss points on [-1, 1]^3 and their weights (sum 8)."""
    pts, wts = [], []
    for idx in itertools.product(range(3), repeat=3):
        pts.append([_G3[i] for i in reversed(idx)])
        wts.append(np.prod([_W3[i] for i in idx]))
    return np.array(pts), np.array(wts)


def s20_element_matrix(h, C):
    """Element matrix of int C eps(v):eps(w) over one serendipity brick,
    dofs node-major (3 per node)."""
    h = np.asarray(h, dtype=np.float64)
    pts, wts = s20_quadrature()
    jac = np.prod(h) / 8.0
    K = np.zeros((60, 60))
    for x, w in zip(pts, wts):
        _, dN = s20_shape_and_grad(x)
        B = strain_matrix(dN * (2.0 / h)[None, :])
        K += w * jac * B.T @ C @ B
    return K


def s20_node_count_before(ne, x, y, z):
    """Node number of lattice point (x, y, z) (vectorised): the valid points
    (at most one odd coordinate) before it in lexicographic order."""
    nx, ny = ne[0], ne[1]
    even_layer = (ny + 1) * (2 * nx + 1) + ny * (nx + 1)
    odd_layer = (nx + 1) * (ny + 1)
    x, y, z = (np.asarray(v, dtype=np.int64) for v in (x, y, z))
    base = (z + 1) // 2 * even_layer + z // 2 * odd_layer
    ev = (z % 2) == 0
    # even z: rows y' < y hold 2 nx + 1 (even y') or nx + 1 (odd y') points
    in_even = (y + 1) // 2 * (2 * nx + 1) + y // 2 * (nx + 1) + np.where(y % 2 == 0, x, x // 2)
    in_odd = y // 2 * (nx + 1) + x // 2
    return base + np.where(ev, in_even, in_odd)


def s20_node_coords(prob):
    """Lattice coordinates (nnodes, 3) of the nodes, in node order."""
    L = [2 * n + 1 for n in prob.ne]
    z, y, x = np.meshgrid(np.arange(L[2]), np.arange(L[1]), np.arange(L[0]), indexing="ij")
    x, y, z = x.ravel(), y.ravel(), z.ravel()
    keep = (x % 2) + (y % 2) + (z % 2) <= 1
    return np.stack([x[keep], y[keep], z[keep]], axis=1)


def voigt_full(c21):
    """Symmetric 6x6 matrix from its 21 upper-triangle entries (row major)."""
    C = np.zeros((6, 6))
    C[np.triu_indices(6)] = c21
    return C + np.triu(C, 1).T


def element_nodes(prob):
    """(nelem, 2^d) global node numbers of every element, vertex order as in
    :func:`_local_offsets` (serendipity: (nelem, 20), order of
    :func:`s20_offsets`)."""
    ne = prob.ne
    if getattr(prob, "element", "q1") == "s20":
        ez, ey, ex = np.meshgrid(*[np.arange(n) for n in reversed(ne)], indexing="ij")
        ex, ey, ez = ex.ravel(), ey.ravel(), ez.ravel()
        off = s20_offsets()
        return np.stack([s20_node_count_before(ne, 2 * ex + o[0], 2 * ey + o[1], 2 * ez + o[2])
                         for o in off], axis=1)
    dim = prob.dim
    nn = [n + 1 for n in ne]
    grids = np.meshgrid(*[np.arange(n) for n in reversed(ne)], indexing="ij")
    # grids[...] indexed [iz,iy,ix]; flatten in C order -> e = ix + nx*(iy+...)
    eidx = [g.ravel() for g in reversed(grids)]  # eidx[a] = coordinate on axis a
    off = _local_offsets(dim)
    nodes = np.zeros((prob.nelem, 2 ** dim), dtype=np.int64)
    for a in range(2 ** dim):
        k = np.zeros(prob.nelem, dtype=np.int64)
        stride = 1
        for ax in range(dim):
            k += (eidx[ax] + off[a, ax]) * stride
            stride *= nn[ax]
        nodes[:, a] = k
    return nodes


def element_dofs(prob):
    """(nelem, 2^d * ncomp) global dof numbers, element vertex-major."""
    nodes = element_nodes(prob)
    if prob.ncomp == 1:
        return nodes
    c = prob.ncomp
    return (nodes[:, :, None] * c + np.arange(c)[None, None, :]).reshape(len(nodes), -1)


def element_matrices(prob, elems=None):
    """Element matrices of the given elements (all by default), shape
    (len(elems), ndofe, ndofe)."""
    if elems is None:
        elems = np.arange(prob.nelem)
    elems = np.asarray(elems)
    if prob.ncomp == 1:
        Kref = darcy_element_matrix_exact(prob.h)
        return prob.coeff[elems][:, None, None] * Kref[None]
    coeff = prob.coeff[elems]
    uniq, inv = np.unique(coeff, axis=0, return_inverse=True)
    kmat = s20_element_matrix if getattr(prob, "element", "q1") == "s20" \
        else elasticity_element_matrix
    Ku = np.array([kmat(prob.h, voigt_full(c)) for c in uniq])
    return Ku[inv.ravel()]


def element_load(prob, f=None):
    """Element load vectors int f phi_a; ``f`` is the constant body load of
    ``prob`` unless a callable f(x) -> (ncomp,) values is given."""
    dim, c = prob.dim, prob.ncomp
    if getattr(prob, "element", "q1") == "s20":
        # int N_a over the brick by the 3-point rule, times the load
        assert f is None
        pts, wts = s20_quadrature()
        jac = np.prod(np.asarray(prob.h)) / 8.0
        ia = np.zeros(20)
        for x, w in zip(pts, wts):
            ia += w * jac * s20_shape_and_grad(x)[0]
        load = np.asarray(prob.load, dtype=np.float64)
        out = np.broadcast_to(ia[None, :, None] * load[None, None, :], (prob.nelem, 20, c))
        return out.reshape(prob.nelem, 20 * c).copy()
    pts, wts = quadrature(dim)
    h = np.asarray(prob.h)
    vol = np.prod(h)
    nodes = element_nodes(prob)
    nv = 2 ** dim
    out = np.zeros((prob.nelem, nv, c))
    if f is None:
        load = np.asarray(prob.load, dtype=np.float64)
        for x, w in zip(pts, wts):
            phi, _ = _shape_and_grad(dim, x)
            out += w * vol * phi[None, :, None] * load[None, None, :]
    else:
        # element origin from its vertex 0
        nn = [n + 1 for n in prob.ne]
        k0 = nodes[:, 0]
        coords = []
        for ax in range(dim):
            coords.append((k0 % nn[ax]) * h[ax])
            k0 = k0 // nn[ax]
        origin = np.stack(coords, axis=1)
        for x, w in zip(pts, wts):
            phi, _ = _shape_and_grad(dim, x)
            fx = np.asarray(f(origin + x[None, :] * h[None, :]), dtype=np.float64)
            fx = fx.reshape(prob.nelem, c)
            out += w * vol * phi[None, :, None] * fx[:, None, :]
    return out.reshape(prob.nelem, nv * c)


def dirichlet_mask(prob):
    """Boolean mask over dofs: True where a homogeneous Dirichlet condition holds."""
    if getattr(prob, "element", "q1") == "s20":
        xyz = s20_node_coords(prob)
        m = np.zeros(prob.nnodes, dtype=bool)
        for ax in range(3):
            if prob.dirichlet >> (2 * ax) & 1:
                m |= xyz[:, ax] == 0
            if prob.dirichlet >> (2 * ax + 1) & 1:
                m |= xyz[:, ax] == 2 * prob.ne[ax]
        return np.repeat(m, prob.ncomp)
    nn = [n + 1 for n in prob.ne]
    coords = np.meshgrid(*[np.arange(n) for n in reversed(nn)], indexing="ij")
    coords = [g.ravel() for g in reversed(coords)]
    m = np.zeros(prob.nnodes, dtype=bool)
    for ax in range(prob.dim):
        if prob.dirichlet >> (2 * ax) & 1:
            m |= coords[ax] == 0
        if prob.dirichlet >> (2 * ax + 1) & 1:
            m |= coords[ax] == prob.ne[ax]
    return np.repeat(m, prob.ncomp)


def eliminate(A, b, dmask):
    """Symmetric elimination of zero Dirichlet data: zero rows/cols, unit diagonal."""
    keep = sp.diags((~dmask).astype(np.float64))
    A2 = (keep @ A @ keep + sp.diags(dmask.astype(np.float64))).tocsr()
    A2.sum_duplicates()
    A2.sort_indices()
    b2 = None if b is None else np.where(dmask, 0.0, b)
    return A2, b2


def _sum_in_element_order(prob, rows, cols, vals):
    """CSR matrix whose entry (i, j) is the sum of the contributions to it,
    added in the order they come (ascending element), starting from 0."""
    pat = sp.csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(prob.ndof, prob.ndof))
    pat.sum_duplicates()
    pat.sort_indices()
    n = np.int64(prob.ndof)
    allkey = np.repeat(np.arange(prob.ndof, dtype=np.int64), np.diff(pat.indptr)) * n \
        + pat.indices.astype(np.int64)
    pos = np.searchsorted(allkey, rows.astype(np.int64) * n + cols.astype(np.int64))
    data = np.zeros(pat.nnz)
    np.add.at(data, pos, vals)      # in the order of vals, from 0
    return sp.csr_matrix((data, pat.indices, pat.indptr), shape=pat.shape)


def assemble(prob, f=None):
    """Global CSR stiffness matrix and load vector with Dirichlet elimination.
    Each entry sums its element contributions in ascending element order."""
    dofs = element_dofs(prob)
    Ke = element_matrices(prob)
    nd = dofs.shape[1]
    rows = np.repeat(dofs, nd, axis=1).ravel()
    cols = np.tile(dofs, (1, nd)).ravel()
    A = _sum_in_element_order(prob, rows, cols, Ke.ravel())
    fe = element_load(prob, f)
    b = np.bincount(dofs.ravel(), weights=fe.ravel(), minlength=prob.ndof)
    return eliminate(A, b, dirichlet_mask(prob))


def assemble_neumann(prob, f=None):
    """Global matrix without any boundary condition (for kernel/row-sum pins)."""
    dofs = element_dofs(prob)
    Ke = element_matrices(prob)
    nd = dofs.shape[1]
    rows = np.repeat(dofs, nd, axis=1).ravel()
    cols = np.tile(dofs, (1, nd)).ravel()
    return _sum_in_element_order(prob, rows, cols, Ke.ravel())
