"""Pins of the oracle's overlapping decomposition and partition of unity
(Sec. 3; Def. 3; Sec. 4.3)."""
import itertools

import numpy as np
import pytest

import synth
from oracle import decomp, fem


@pytest.mark.parametrize("n,parts", [(64, 4), (10, 3), (7, 7), (100, 16)])
def test_near_equal_split(n, parts):
    r = decomp.part_ranges(n, parts)
    sizes = [hi - lo for lo, hi in r]
    assert sum(sizes) == n and max(sizes) - min(sizes) <= 1
    assert r[0][0] == 0 and r[-1][1] == n
    assert all(r[i][1] == r[i + 1][0] for i in range(parts - 1))
    assert sizes == sorted(sizes, reverse=True)


def _sizes_formula(n, parts, ovl, p):
    """Closed-form node counts along one axis for part p (|N|, |I|, |D|)."""
    lo, hi = decomp.part_ranges(n, parts)[p]
    elo, ehi = max(0, lo - ovl), min(n, hi + ovl)
    nN = ehi - elo + 1
    nI = nN - (elo > 0) - (ehi < n)
    nD = nI - (elo == 0) - (ehi == n)   # all faces Dirichlet
    return nN, nI, nD


@pytest.mark.parametrize("n,parts,ovl", [(64, 4, 2), (30, 3, 1), (17, 4, 2)])
def test_set_sizes_closed_form_2d(n, parts, ovl):
    p = synth.darcy_problem("t", np.ones((n, n)), (parts, parts), ovl)
    subs, _ = decomp.build(p)
    for s in subs:
        px, py = s.j % parts, s.j // parts
        fx = _sizes_formula(n, parts, ovl, px)
        fy = _sizes_formula(n, parts, ovl, py)
        assert len(s.dofs) == fx[0] * fy[0]
        assert s.interior.sum() == fx[1] * fy[1]
        assert s.dmask.sum() == fx[2] * fy[2]


def test_config_table_sizes():
    """|N_j| interior / corner and |D_j| of the paper-shaped configurations."""
    cases = [((64, 64), (4, 4), 2, 441, 361, 361),
             ((512, 512), (16, 16), 2, 1369, 1225, 1225),
             ((96, 96, 96), (8, 8, 8), 1, 3375, 2744, 2197)]
    for ne, parts, ovl, nint, ncorner, dint in cases:
        tot_n, tot_d = 1, 1
        for n, P in zip(ne, parts):
            f_int = _sizes_formula(n, P, ovl, 1)
            f_cor = _sizes_formula(n, P, ovl, 0)
            tot_n *= f_int[0]
            tot_d *= f_int[2]
        assert tot_n == nint and tot_d == dint
        c = 1
        for n, P in zip(ne, parts):
            c *= _sizes_formula(n, P, ovl, 0)[0]
        assert c == ncorner


@pytest.mark.parametrize("dim", [2, 3])
def test_pou_sums_to_one_and_vanishes(dim):
    if dim == 2:
        p = synth.darcy_problem("t", np.ones((13, 11)), (3, 2), 2)
    else:
        p = synth.darcy_problem("t", np.ones((7, 6, 8)), (2, 2, 3), 1)
    subs, _ = decomp.build(p)
    d = fem.dirichlet_mask(p)
    tot = decomp.pou_sum(p, subs)
    assert np.max(np.abs(tot[~d] - 1.0)) <= 1e-15
    assert np.all(tot[d] == 0.0)
    allowed = {1.0 / c for c in range(1, 2 ** dim + 1)}
    for s in subs:
        assert np.all(s.mu[~s.interior] == 0.0)
        assert np.all(s.mu[s.dirichlet] == 0.0)
        assert np.all(s.mu[s.dmask] > 0.0)
        assert all(min(abs(v - a) for a in allowed) < 1e-15 for v in s.mu[s.dmask])


def test_pou_elasticity_neumann_faces():
    ply = synth.isotropic_stiffness(4.0, 0.35)
    p = synth.elasticity_problem("t", np.broadcast_to(ply, (4, 3, 8, 6, 6)),
                                 (8, 3, 4), (2, 1, 2), 1, dirichlet=1,
                                 load=(0, 0, -1.0), h=(1, 1, 1))
    subs, _ = decomp.build(p)
    tot = decomp.pou_sum(p, subs)
    d = fem.dirichlet_mask(p)
    assert np.max(np.abs(tot[~d] - 1.0)) <= 1e-15 and np.all(tot[d] == 0)


@pytest.mark.parametrize("dim", [2, 3])
def test_cover_count_and_overlap_zone(dim):
    if dim == 2:
        p = synth.darcy_problem("t", np.ones((12, 12)), (3, 3), 1)
    else:
        p = synth.darcy_problem("t", np.ones((8, 8, 8)), (2, 2, 2), 1)
    subs, mult = decomp.build(p)
    assert mult.max() == 2 ** dim          # k0 of Sec. 3
    member = [set(s.elems.tolist()) for s in subs]
    for s in subs:
        # set definition of the overlap zone: in Omega_j and in some other Omega_i
        brute = sorted(e for e in member[s.j]
                       if any(e in member[i] for i in range(len(subs)) if i != s.j))
        assert brute == sorted(s.overlap_elems.tolist())


def test_single_subdomain_has_no_overlap():
    p = synth.darcy_problem("t", np.ones((6, 6)), (1, 1), 2)
    subs, mult = decomp.build(p)
    assert len(subs) == 1 and len(subs[0].overlap_elems) == 0
    assert np.all(subs[0].mu[subs[0].dmask] == 1.0)


def test_box_ids_enumeration():
    strides = [1, 10, 100]
    ids = decomp._box_ids([1, 2, 3], [3, 4, 5], strides)
    brute = sorted(x + 10 * y + 100 * z for x, y, z in
                   itertools.product(range(1, 3), range(2, 4), range(3, 5)))
    assert ids.tolist() == brute


# ------------------------------------------------- Sarkis partition of unity
def _sarkis(prob):
    prob.pou = "sarkis"
    subs, _ = decomp.build(prob)
    return subs


def test_sarkis_linear_ramp_across_overlap_strip():
    """Two subdomains side by side in x with overlap 2: the parts are
    [0, 8) and [8, 16), widened to [0, 10) and [6, 16).  Across the strip of
    nodes x = 6 .. 10 the left weight is (10 - x) / 4 in closed form (the
    distance to x = 10 over the sum of the distances to x = 10 and x = 6);
    1 to the left of it, 0 to the right; the same on every row."""
    p = synth.darcy_problem("t", np.ones((5, 16)), (2, 1), 2, dirichlet=0)
    subs = _sarkis(p)
    s = subs[0]
    x = (s.dofs % 17).astype(float)
    expect = np.clip((10.0 - x) / 4.0, 0.0, 1.0)
    assert np.allclose(s.mu, expect, rtol=0, atol=1e-15)
    tot = decomp.pou_sum(p, subs)
    assert np.allclose(tot, 1.0, rtol=0, atol=1e-15)


def test_sarkis_equals_piecewise_constant_at_overlap_one():
    """With one element layer of overlap every node of the strip is at
    distance 0 or h from each artificial boundary, so the distance weights
    are the counting weights 1/c_k."""
    rng = np.random.Generator(np.random.PCG64(8))
    for shape, parts in (((12, 15), (3, 4)), ((6, 7, 8), (2, 2, 3))):
        k = np.exp(rng.normal(size=shape))
        p = synth.darcy_problem("t", k, parts, 1)
        const, _ = decomp.build(p)
        sark = _sarkis(synth.darcy_problem("t", k, parts, 1))
        for a, b in zip(const, sark):
            assert np.allclose(a.mu, b.mu, rtol=1e-15, atol=0)


@pytest.mark.parametrize("shape,parts,ovl,dirichlet", [((24, 24), (3, 3), 3, 0b1111),
                                                        ((10, 9, 8), (2, 3, 2), 2, 0b000011),
                                                        ((20, 12), (4, 2), 2, 0b0101)])
def test_sarkis_sums_to_one_and_vanishes_where_required(shape, parts, ovl, dirichlet):
    p = synth.darcy_problem("t", np.ones(shape), parts, ovl, dirichlet=dirichlet)
    subs = _sarkis(p)
    d = fem.dirichlet_mask(p)
    tot = decomp.pou_sum(p, subs)
    assert np.max(np.abs(tot[~d] - 1.0)) <= 1e-15
    assert np.all(tot[d] == 0.0)
    for s in subs:
        assert np.all(s.mu[~s.dmask] == 0.0)      # artificial boundary and Dirichlet
        assert np.all((s.mu >= 0.0) & (s.mu <= 1.0))
        assert np.all(s.mu[s.dmask & ~s.dirichlet] > 0.0)


def test_sarkis_elasticity_components_share_weights():
    C = synth.isotropic_stiffness(4.0, 0.35)
    p = synth.elasticity_problem("t", np.broadcast_to(C, (4, 4, 8, 6, 6)), (8, 4, 4), (2, 1, 1),
                                 2, dirichlet=1, load=(0.0, 0.0, -1.0), h=(1.0, 1.0, 1.0))
    subs = _sarkis(p)
    for s in subs:
        m = s.mu.reshape(-1, 3)
        assert np.all(m[:, 0] == m[:, 1]) and np.all(m[:, 0] == m[:, 2])
    tot = decomp.pou_sum(p, subs)
    assert np.max(np.abs(tot[~fem.dirichlet_mask(p)] - 1.0)) <= 1e-15
