"""Overlapping subdomains and the partition of unity (oracle; test infrastructure).

Follows Sec. 3 and Sec. 4.3 of the paper:

* a non-overlapping partition into boxes of elements is widened by ``ovl``
  element layers (one layer = the elements sharing a vertex with the current
  set, which for boxes is one element per side, clipped to the grid);
* the overlap zone of subdomain j is the set of its elements that also lie
  in another subdomain (Sec. 3); equivalently, elements counted at least
  twice when every subdomain adds a one per element (Sec. 4.3);
* ``N_j`` are the dofs of the closed subdomain, ``I_j`` those not on the
  artificial (interior) part of its boundary, ``D_j`` those of ``I_j`` that
  are not constrained by the Dirichlet condition;
* the partition of unity is the piecewise constant one: with c_k the number
  of subdomains having dof k in ``I_j``, mu_{j,k} = 1/c_k on ``D_j`` and 0
  elsewhere -- zero at Dirichlet dofs and on subdomain boundaries, summing to
  one over j at every free dof (Sec. 4.3; Def. 3); or, for problems with
  ``pou == "sarkis"``, the smooth one of Fig. 1 (right): weights
  proportional to the distance from each subdomain's artificial boundary.

Pins (tests/test_oracle_decomp.py): closed-form set sizes, maximal cover
count k0 = 2^d, the partition of unity summing to 1 at every free dof and
vanishing where required, and the overlap zone matching its set definition;
for the Sarkis weights the linear ramp across a strip of overlap in closed
form, equality with the piecewise-constant weights at overlap 1, and the
same sum and support pins.
"""
from dataclasses import dataclass

import numpy as np

from . import fem


def part_ranges(n, parts):
    """Element ranges [lo, hi) of a near-equal split of n elements into parts;
    the first n % parts parts get one extra element."""
    base, extra = divmod(n, parts)
    sizes = [base + (1 if p < extra else 0) for p in range(parts)]
    lo = np.concatenate([[0], np.cumsum(sizes)[:-1]])
    return [(int(l), int(l + s)) for l, s in zip(lo, sizes)]


@dataclass
class Subdomain:
    j: int
    ebox: tuple          # per axis (elo, ehi), overlapping element range
    elems: np.ndarray    # global element ids in the box
    dofs: np.ndarray     # N_j, sorted global dofs
    interior: np.ndarray  # bool over N_j: in I_j (not on artificial boundary)
    dirichlet: np.ndarray  # bool over N_j: constrained dof
    mu: np.ndarray       # partition-of-unity weights over N_j
    overlap_elems: np.ndarray  # global element ids of the overlap zone

    @property
    def dmask(self):
        """D_j as a mask over N_j."""
        return self.interior & ~self.dirichlet


def subdomain_boxes(prob):
    """Overlapping element boxes, subdomain j = px + Px*(py + Py*pz)."""
    per_axis = []
    for ax in range(prob.dim):
        rng = part_ranges(prob.ne[ax], prob.parts[ax])
        per_axis.append([(max(0, lo - prob.ovl), min(prob.ne[ax], hi + prob.ovl))
                         for lo, hi in rng])
    boxes = []
    for idx in np.ndindex(*reversed(prob.parts)):
        pidx = tuple(reversed(idx))  # (px, py[, pz])
        boxes.append(tuple(per_axis[ax][pidx[ax]] for ax in range(prob.dim)))
    return boxes


def _box_ids(lo, hi, strides):
    """Flattened ids of the integer box prod [lo_a, hi_a) with the given strides."""
    ids = np.zeros(1, dtype=np.int64)
    for ax in reversed(range(len(lo))):
        r = np.arange(lo[ax], hi[ax], dtype=np.int64) * strides[ax]
        ids = (ids[:, None] + r[None, :]).ravel()
    return ids


def build(prob):
    """All subdomains of ``prob`` with their sets, overlap zones and weights."""
    dim, c = prob.dim, prob.ncomp
    ne = prob.ne
    nn = [n + 1 for n in ne]
    estr = np.cumprod([1] + list(ne[:-1]))
    nstr = np.cumprod([1] + nn[:-1])
    boxes = subdomain_boxes(prob)
    dmask_glob = fem.dirichlet_mask(prob)

    # element multiplicity: every subdomain adds one on each of its elements
    mult = np.zeros(prob.nelem, dtype=np.int64)
    for b in boxes:
        mult[_box_ids([x[0] for x in b], [x[1] for x in b], estr)] += 1

    s20 = getattr(prob, "element", "q1") == "s20"
    if s20:
        # serendipity nodes: lattice of half-edge steps (coordinates scaled by 2)
        xyz = fem.s20_node_coords(prob)
    subs = []
    icount = np.zeros(prob.ndof, dtype=np.int64)
    for j, b in enumerate(boxes):
        lo = [x[0] for x in b]
        hi = [x[1] for x in b]
        elems = _box_ids(lo, hi, estr)
        if s20:
            inbox = np.ones(prob.nnodes, dtype=bool)
            for ax in range(dim):
                inbox &= (xyz[:, ax] >= 2 * lo[ax]) & (xyz[:, ax] <= 2 * hi[ax])
            nodes = np.flatnonzero(inbox)
            coords = [xyz[nodes, ax] for ax in range(dim)]
            sc = 2
        else:
            nodes = _box_ids(lo, [h + 1 for h in hi], nstr)
            coords = []
            k = nodes.copy()
            for ax in range(dim):
                coords.append(k % nn[ax])
                k //= nn[ax]
            sc = 1
        # artificial boundary: box face strictly inside the grid
        art = np.zeros(len(nodes), dtype=bool)
        for ax in range(dim):
            if lo[ax] > 0:
                art |= coords[ax] == sc * lo[ax]
            if hi[ax] < ne[ax]:
                art |= coords[ax] == sc * hi[ax]
        if c == 1:
            dofs = nodes
            interior = ~art
        else:
            dofs = (nodes[:, None] * c + np.arange(c)[None, :]).ravel()
            interior = np.repeat(~art, c)
        order = np.argsort(dofs, kind="stable")
        dofs, interior = dofs[order], interior[order]
        icount[dofs[interior]] += 1
        subs.append(Subdomain(j=j, ebox=b, elems=elems, dofs=dofs,
                              interior=interior,
                              dirichlet=dmask_glob[dofs], mu=None,
                              overlap_elems=elems[mult[elems] >= 2]))
    if getattr(prob, "pou", "constant") == "sarkis":
        _sarkis_weights(prob, subs, boxes)
        return subs, mult
    for s in subs:
        d = s.dmask
        mu = np.zeros(len(s.dofs))
        mu[d] = 1.0 / icount[s.dofs[d]]
        s.mu = mu
    return subs, mult


def artificial_distance(prob, box, nodes):
    """Distance of the given nodes of box Omega_j from the artificial part of
    its boundary (the faces of the box that lie inside Omega), in physical
    units; +inf for a box without such faces.  For a point of a box the
    nearest point of a face lies on the face's plane, so this is the
    smallest distance to the planes of the artificial faces."""
    nn = [n + 1 for n in prob.ne]
    k = np.asarray(nodes).copy()
    d = np.full(len(k), np.inf)
    for ax in range(prob.dim):
        x = k % nn[ax]
        k //= nn[ax]
        lo, hi = box[ax]
        if lo > 0:
            d = np.minimum(d, (x - lo) * prob.h[ax])
        if hi < prob.ne[ax]:
            d = np.minimum(d, (hi - x) * prob.h[ax])
    return d


def _sarkis_weights(prob, subs, boxes):
    """Smooth partition of unity of Sarkis type (Fig. 1 right): the weight of
    subdomain j at node x is d_j(x) / sum_i d_i(x), with d_i the distance
    of x from the artificial boundary of Omega_i (zero on it, and zero for
    the subdomains not containing x); zero at Dirichlet dofs.  A box without
    artificial faces (one subdomain) has weight 1."""
    c = prob.ncomp
    dist = []
    total = np.zeros(prob.nnodes)
    for s, b in zip(subs, boxes):
        nodes = s.dofs[::c] // c
        d = artificial_distance(prob, b, nodes)
        d = np.where(np.isinf(d), 1.0, d)
        dist.append(d)
        np.add.at(total, nodes, d)
    for s, d in zip(subs, dist):
        nodes = s.dofs[::c] // c
        mu = np.repeat(d / np.where(total[nodes] > 0, total[nodes], 1.0), c)
        s.mu = np.where(s.dmask, mu, 0.0)


def pou_sum(prob, subs):
    """sum_j R_j^T mu_j as a global vector."""
    out = np.zeros(prob.ndof)
    for s in subs:
        np.add.at(out, s.dofs, s.mu)
    return out


def thm1_threshold(prob, subs):
    """delta_j / H_j of Thm. 1 for every subdomain: H_j = diam(Omega_j), the
    diagonal of its element box; delta_j the width of its overlap zone, the
    strips of 2 * ovl element layers along each artificial face (ovl from
    the subdomain's own extension, ovl from the neighbour's), in the
    smallest edge length."""
    delta = 2 * prob.ovl * min(prob.h)
    out = np.zeros(len(subs))
    for s in subs:
        ext = [(hi - lo) * prob.h[ax] for ax, (lo, hi) in enumerate(s.ebox)]
        out[s.j] = delta / np.sqrt(np.sum(np.square(ext)))
    return out
