"""Problem descriptions for the paper-shaped workloads.

A :class:`Problem` is plain data: a structured grid of Q1 elements on a box,
the per-element coefficient, which boundary faces carry homogeneous
Dirichlet conditions, the constant body load, the box partition into
subdomains with its overlap width, and the GenEO / PCG options.

Conventions shared by every consumer (stated once here):

* elements ``e = ix + nx*(iy + ny*iz)``; nodes ``k = ix + (nx+1)*(iy +
  (ny+1)*iz)``; degrees of freedom ``k*ncomp + c``;
* element ``e`` has side lengths ``h`` (per axis) and sits at
  ``[ix*hx, (ix+1)*hx] x ...``;
* Darcy coefficient: one ``kappa`` per element; elasticity: 21 entries of
  the symmetric 6x6 Voigt stiffness per element (upper triangle, row major,
  Voigt order 11, 22, 33, 23, 13, 12 with engineering shear strains);
* ``dirichlet`` is a bitmask over faces, bit ``2*axis + side`` (side 0 is the
  face at coordinate 0, side 1 the far face);
* ``parts[a]`` subdomains along axis ``a``; the first ``ne[a] % parts[a]``
  parts get one extra element; each part is then widened by ``ovl`` element
  layers on both sides, clipped to the grid.
"""
from dataclasses import dataclass, field
from typing import Optional, Tuple

import numpy as np

from . import fields as F

ALL_FACES_2D = 0b1111
ALL_FACES_3D = 0b111111


@dataclass
class Problem:
    name: str
    dim: int
    ncomp: int
    ne: Tuple[int, ...]
    h: Tuple[float, ...]
    parts: Tuple[int, ...]
    ovl: int
    coeff: np.ndarray                 # (nelem,) or (nelem, 21), float64
    dirichlet: int                    # face bitmask
    load: Tuple[float, ...]           # constant body load per component
    nev: int = 8                      # fixed number of eigenvectors (if tau is None)
    tau: Optional[float] = None       # threshold: take lambda < tau ...
    nev_max: Optional[int] = None     # ... capped at nev_max
    precision: str = "fp64"           # "fp64" or "mixed"
    pou: str = "constant"             # partition of unity: "constant" or "sarkis"
    element: str = "q1"               # "q1" (trilinear) or "s20" (20-node serendipity
                                      # bricks, 3D elasticity)
    rtol: float = 1e-10
    maxit: int = 2000
    meta: dict = field(default_factory=dict)

    @property
    def nelem(self):
        return int(np.prod(self.ne))

    @property
    def nnodes(self):
        corners = int(np.prod([n + 1 for n in self.ne]))
        if self.element == "q1":
            return corners
        # serendipity bricks: the vertices and one node per element edge
        edges = sum(self.ne[ax] * corners // (self.ne[ax] + 1) for ax in range(3))
        return corners + edges

    @property
    def ndof(self):
        return self.nnodes * self.ncomp

    @property
    def nsub(self):
        return int(np.prod(self.parts))

    def __post_init__(self):
        self.ne = tuple(int(n) for n in self.ne)
        self.h = tuple(float(x) for x in self.h)
        self.parts = tuple(int(p) for p in self.parts)
        self.coeff = np.ascontiguousarray(self.coeff, dtype=np.float64)
        assert self.dim in (2, 3) and len(self.ne) == self.dim
        assert len(self.h) == self.dim and len(self.parts) == self.dim
        assert self.ncomp in (1, 3)
        if self.ncomp == 1:
            assert self.coeff.shape == (self.nelem,)
        else:
            assert self.dim == 3 and self.coeff.shape == (self.nelem, 21)
        assert len(self.load) == self.ncomp
        assert self.pou in ("constant", "sarkis")
        assert self.element in ("q1", "s20")
        if self.element == "s20":
            assert self.dim == 3 and self.ncomp == 3 and self.pou == "constant"
        for n, p in zip(self.ne, self.parts):
            assert 1 <= p <= n


def darcy_problem(name, kappa, parts, ovl, dirichlet=None, load=1.0, h=None,
                  **opts):
    """Darcy problem from an element coefficient array indexed ``[iz,iy,ix]``."""
    kappa = np.asarray(kappa, dtype=np.float64)
    ne = tuple(reversed(kappa.shape))
    dim = len(ne)
    if h is None:
        h = tuple(1.0 / n for n in ne)
    if dirichlet is None:
        dirichlet = ALL_FACES_2D if dim == 2 else ALL_FACES_3D
    return Problem(name=name, dim=dim, ncomp=1, ne=ne, h=h, parts=parts,
                   ovl=ovl, coeff=kappa.ravel(), dirichlet=dirichlet,
                   load=(float(load),), **opts)


def elasticity_problem(name, cvoigt, ne, parts, ovl, dirichlet, load, h,
                       **opts):
    """Elasticity problem from per-element 6x6 Voigt stiffnesses ``[iz,iy,ix,6,6]``."""
    cvoigt = np.asarray(cvoigt, dtype=np.float64)
    iu = np.triu_indices(6)
    coeff = cvoigt[..., iu[0], iu[1]].reshape(-1, 21)
    return Problem(name=name, dim=3, ncomp=3, ne=ne, h=h, parts=parts,
                   ovl=ovl, coeff=coeff, dirichlet=dirichlet, load=load,
                   **opts)


# ------------------------------------------------------------- configs ---

def channels_2d(seed=0, n=64, parts=4, ovl=2, nev=8, precision="fp64",
                     n_channels=6):
    """2D Darcy, unit square, u=0 on the boundary, f=1, k=1e6 channels."""
    k, starts = F.channel_field(n, n_channels=n_channels, seed=seed,
                                first_row=2, last_row=n - 4)
    p = darcy_problem("channels_%d" % n, k, (parts, parts), ovl,
                      nev=nev, precision=precision)
    p.meta["channel_rows"] = starts.tolist()
    p.meta["seed"] = seed
    return p


def grf_2d(seed=0, n=512, parts=16, ovl=2, tau=0.1, nev_max=16,
                precision="mixed", inclusions=24):
    """2D Darcy, k = exp(GRF) with discs of k=1e6; threshold selection."""
    g = F.grf_exponential_2d(n, var=4.0, corr=0.05, seed=seed)
    k = np.exp(g)
    if inclusions:
        k[F.inclusions_2d(n, count=inclusions, seed=seed + 1000)] = 1e6
    p = darcy_problem("grf_%d" % n, k, (parts, parts), ovl,
                      tau=tau, nev_max=nev_max, nev=nev_max,
                      precision=precision)
    p.meta["seed"] = seed
    return p


def layers_3d(seed=0, n=96, parts=8, ovl=1, nev=12, precision="mixed"):
    """3D Darcy on the unit cube with random-thickness z-layers of high contrast."""
    kz = F.z_layers_3d(n, seed=seed)
    k = np.broadcast_to(kz[:, None, None], (n, n, n)).copy()
    p = darcy_problem("layers_%d" % n, k, (parts, parts, parts), ovl,
                      nev=nev, precision=precision)
    p.meta["seed"] = seed
    return p


def laminate_stack():
    """z-stack of the synthetic laminate: (material, thickness in elements).

    Four-element plies alternately at 0 and 90 degrees about z, separated by
    one-element isotropic resin layers: 5 plies + 4 resin = 24 elements.
    """
    stack = []
    for i in range(5):
        stack.append(("ply0" if i % 2 == 0 else "ply90", 4))
        if i < 4:
            stack.append(("resin", 1))
    return stack


def laminate_3d(seed=0, ne=(128, 32, 24), parts=(16, 4, 4), ovl=1,
                     nev=24, precision="mixed"):
    """3D anisotropic elasticity of a clamped laminate under a body load.

    Moduli in GPa, element size 1; clamped (all three components) at x=0;
    load (0, 0, -1) per unit volume.  ``seed`` is unused (the stack is fixed)
    and kept only for a uniform signature.
    """
    ply = F.ply_stiffness(160.0, 10.0, 10.0, 5.0, 5.0, 5.0, 0.3, 0.3, 0.3)
    mats = {"ply0": ply, "ply90": F.rotate_z90(ply),
            "resin": F.isotropic_stiffness(4.0, 0.35)}
    nx, ny, nz = ne
    stack = laminate_stack()
    zmat = []
    for m, t in stack:
        zmat += [m] * t
    assert len(zmat) >= nz
    C = np.empty((nz, ny, nx, 6, 6))
    for iz in range(nz):
        C[iz] = mats[zmat[iz]]
    p = elasticity_problem("laminate_%dx%dx%d" % tuple(ne), C, ne, parts, ovl,
                           dirichlet=0b000001, load=(0.0, 0.0, -1.0),
                           h=(1.0, 1.0, 1.0), nev=nev, precision=precision)
    p.meta["seed"] = seed
    return p


def laminate_s20(seed=0, ne=(32, 8, 6), parts=(4, 2, 1), ovl=1, nev=16, precision="mixed"):
    """The clamped laminate of :func:`laminate_3d` on 20-node serendipity
    bricks (the element of the paper's composite experiments, Sec. 5.3):
    the same materials, clamp and load; one-element plies alternating 0 and
    90 degrees, each followed by a one-element resin layer; unit elements.
    The default, 32 x 8 x 6 bricks, has 23,175 dofs, near the 30,000 of the
    paper's composite plate.  ``seed`` is unused (the stack is fixed)."""
    ply = F.ply_stiffness(160.0, 10.0, 10.0, 5.0, 5.0, 5.0, 0.3, 0.3, 0.3)
    mats = [ply, F.isotropic_stiffness(4.0, 0.35), F.rotate_z90(ply)]
    nx, ny, nz = ne
    C = np.empty((nz, ny, nx, 6, 6))
    for iz in range(nz):
        # ply 0, resin, ply 90, resin, ply 0, ...
        C[iz] = mats[0] if iz % 4 == 0 else mats[2] if iz % 4 == 2 else mats[1]
    p = elasticity_problem("laminate_s20_%dx%dx%d" % tuple(ne), C, ne, parts, ovl,
                           dirichlet=0b000001, load=(0.0, 0.0, -1.0),
                           h=(1.0, 1.0, 1.0), nev=nev, precision=precision,
                           element="s20")
    p.meta["seed"] = seed
    return p


def layered_2d(n=40, parts=4, ovl=2, layers=8, contrast=1e6, nev=4,
               precision="fp64", dirichlet=0b1100):
    """2D Darcy with ``layers`` equally thick horizontal layers of alternating
    k = 1 and k = contrast (the paper's layered robustness study, scaled).

    By default only the bottom and top faces are Dirichlet and the sides are
    Neumann, as in the paper's structured Darcy examples, so the stiff layers
    are not anchored on the sides.
    """
    assert n % layers == 0
    t = n // layers
    kz = np.array([1.0 if (i // t) % 2 == 0 else contrast for i in range(n)])
    k = np.broadcast_to(kz[:, None], (n, n)).copy()
    return darcy_problem("layered_%d_%d" % (n, layers), k, (parts, parts), ovl,
                         dirichlet=dirichlet, nev=nev, precision=precision)


# the full-size workloads, by name
CONFIGS = {
    "channels_64": channels_2d,
    "grf_512": grf_2d,
    "layers_96": layers_3d,
    "laminate_128x32x24": laminate_3d,
    "laminate_s20_32x8x6": laminate_s20,
}
