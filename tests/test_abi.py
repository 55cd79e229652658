"""The C-ABI library loads and exports every entry point its header declares;
host-only entry points (sizes, defaults, messages) work without a GPU."""
import os
import re

import numpy as np
import pytest

import synth
from oracle import decomp, fem

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "geneo.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = set(re.findall(r"\b((?:geneo|pcg)_[a-z0-9_]+)\s*\(", txt))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    import ctypes
    from paper_1906_10944_amd import geneo as G
    L = G.lib()
    names = _declared()
    assert "geneo_setup" in names and "geneo_apply" in names and "pcg_solve" in names
    for n in names:
        assert hasattr(L, n), n
        assert isinstance(getattr(L, n), ctypes._CFuncPtr)


def test_version_and_messages():
    from paper_1906_10944_amd import geneo as G
    assert "gfx950" in G.geneo_version()
    assert G.geneo_strerror(0) == "ok"
    assert "not SPD" in G.geneo_strerror(5)


def test_default_opts():
    from paper_1906_10944_amd import geneo as G
    o = G.geneo_default_opts()
    assert o.sigma == -1e-3 and o.nev == 8 and o.coarse == 1 and o.precision == 0
    # the last fields too: a layout mismatch between the header and the
    # binding would show here
    assert o.eig_stall == 10 and o.eig_floor == 1e-6 and o.eig_cheb == 4 and o.symv_tiles == 0


@pytest.mark.parametrize("make", [
    lambda: synth.channels_2d(0),
    lambda: synth.channels_2d(0, n=30, parts=3, n_channels=3, ovl=1),
    lambda: synth.darcy_problem("t", np.ones((7, 9, 10)), (2, 2, 3), 1),
    lambda: synth.laminate_3d(ne=(16, 4, 5), parts=(4, 1, 1)),
    lambda: synth.laminate_s20(ne=(6, 4, 3), parts=(3, 2, 1)),
    lambda: synth.laminate_s20(ne=(5, 3, 4), parts=(2, 1, 2), ovl=2),
])
def test_q1_sizes_match_oracle(make):
    from paper_1906_10944_amd import geneo as G
    p = make()
    s = G.geneo_q1_sizes(G.grid_from_problem(p))
    A = fem.assemble_neumann(p)
    subs, _ = decomp.build(p)
    assert s["ndof"] == p.ndof
    assert s["nnz"] == A.nnz
    assert s["nsub"] == len(subs)
    assert s["nloc"] == sum(len(x.dofs) for x in subs)
    assert s["nmax"] == max(len(x.dofs) for x in subs)
    # the batched local pattern: the couplings within each N_j
    assert s["nnz_loc"] == sum(A[x.dofs][:, x.dofs].nnz for x in subs)


def test_q1_sizes_rejects_bad_grids():
    from paper_1906_10944_amd import geneo as G
    p = synth.channels_2d(0)
    g = G.grid_from_problem(p)
    g.ovl = 0
    with pytest.raises(G.GeneoError) as e:
        G.geneo_q1_sizes(g)
    assert e.value.code == 1
    g = G.grid_from_problem(p)
    g.parts[0] = 100
    with pytest.raises(G.GeneoError):
        G.geneo_q1_sizes(g)
    # serendipity bricks are 3D elasticity only
    g = G.grid_from_problem(p)
    g.element = G.GENEO_ELEM_S20
    with pytest.raises(G.GeneoError):
        G.geneo_q1_sizes(g)


def test_error_codes_match_the_header():
    """The binding's error constants are the header's enum values."""
    from paper_1906_10944_amd import geneo as G
    txt = open(os.path.join(ROOT, "include", "geneo.h")).read()
    found = dict((m.group(1), int(m.group(2)))
                 for m in re.finditer(r"\b(GENEO_(?:OK|ERR_[A-Z_]+))\s*=\s*(\d+)", txt))
    assert found["GENEO_OK"] == G.GENEO_OK == 0
    for name, code in found.items():
        if name != "GENEO_OK":
            assert getattr(G, name) == code and G.ERRORS[code] == name
