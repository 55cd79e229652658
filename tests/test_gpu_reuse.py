"""Setups on reused device blocks.

The library keeps the device blocks of destroyed handles and finished
setups and hands them to the next setup of a similar size; such blocks
still hold the previous operator's data.  An operator built on them must
equal, bit for bit, the same operator built on blocks fresh from the
driver: no kernel may read device memory it has not written.  The stale
data comes from a different problem on the same mesh (another coefficient
field, so other eigenvectors, coarse sizes and fallback sets)."""
import numpy as np
import pytest
import synth

from gpu_common import gpu_apply, gpu_assemble, gpu_pcg, gpu_setup, kappa_local, need_gpu, say

pytestmark = pytest.mark.gpu


def _run(sysm, prob, precision, r):
    h = gpu_setup(sysm, prob, precision=precision)
    z1 = gpu_apply(h, sysm, r)
    z2 = gpu_apply(h, sysm, r)  # consecutive applies walk the subdomains in opposite orders
    x, info = gpu_pcg(h, sysm)
    h.close()
    return z1, z2, x, info["iters"]


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_reused_blocks_give_the_same_operator(precision):
    need_gpu()
    from paper_1906_10944_amd import geneo as G
    pb = synth.grf_2d(seed=3, n=48, parts=2, ovl=2, inclusions=2)
    pa = synth.grf_2d(seed=4, n=48, parts=2, ovl=2, inclusions=2)
    sb, sa = gpu_assemble(pb), gpu_assemble(pa)
    r = np.random.default_rng(7).standard_normal(pb.ndof)
    G.geneo_trim()
    say("[reuse] precision", precision, "fresh blocks")
    ref = _run(sb, pb, precision, r)
    assert np.array_equal(ref[0], ref[1])
    say("[reuse] stale blocks of another coefficient field")
    _run(sa, pa, precision, r)
    again = _run(sb, pb, precision, r)
    say("[reuse] stale blocks of the same operator")
    third = _run(sb, pb, precision, r)
    for got in (again, third):
        for a, b in zip(got[:3], ref[:3]):
            assert np.array_equal(a, b)
        assert got[3] == ref[3]
    G.geneo_trim()


def test_symv_tiles_give_the_same_operator():
    """The tiles per wavefront of the local symmetric products (forced, or
    chosen by timing) change the work split, never the arithmetic."""
    need_gpu()
    from paper_1906_10944_amd import geneo as G
    prob = synth.grf_2d(seed=3, n=48, parts=2, ovl=2, inclusions=2)
    sysm = gpu_assemble(prob)
    r = np.random.default_rng(9).standard_normal(prob.ndof)
    outs = {}
    for tiles in (8, 16, 32, 0):
        h = gpu_setup(sysm, prob, precision=1, symv_tiles=tiles)
        used = G.geneo_get_setup_info(h)["symv_tiles"]
        assert used == tiles or (tiles == 0 and used in (8, 16, 32))
        outs[tiles] = gpu_apply(h, sysm, r)
        h.close()
        say("[symv tiles]", tiles, "->", used)
    for tiles in (16, 32, 0):
        assert np.array_equal(outs[tiles], outs[8])


def test_sweep_flags_read_late_or_at_once_give_the_same_operator():
    """The host reads the eigen sweeps' convergence flags one sweep late
    (per-kernel timing off) or after every sweep (timing on); the extra
    sweep enqueued in the first case finds every subdomain inactive and
    changes nothing: eigenvalues, sweep counts and the operator agree bit
    for bit."""
    need_gpu()
    from paper_1906_10944_amd import geneo as G
    prob = synth.grf_2d(seed=3, n=48, parts=2, ovl=2, inclusions=2)
    sysm = gpu_assemble(prob)
    r = np.random.default_rng(11).standard_normal(prob.ndof)
    L = G.lib()
    outs = []
    for timing in (0, 1, 0):
        L.geneo_prof_enable(timing)
        try:
            h = gpu_setup(sysm, prob, precision=1)
        finally:
            L.geneo_prof_enable(0)
        info = G.geneo_get_setup_info(h)
        m, lam = G.geneo_get_eigenvalues(h, prob.nsub)
        outs.append((info["eig_sweeps"], m, lam, gpu_apply(h, sysm, r)))
        h.close()
        say("[sweep flags] timing", timing, "sweeps", info["eig_sweeps"], "nc", int(m.sum()))
    for got in outs[1:]:
        assert got[0] == outs[0][0]
        for a, b in zip(got[1:], outs[0][1:]):
            assert np.array_equal(a, b)


@pytest.mark.parametrize("nev,tau", [(4, None), (None, 0.1), (24, None)],
                         ids=["b16", "b32", "b48"])
def test_every_eigen_solve_kernel_gives_the_same_operator(nev, tau):
    """The eigen sweeps' triangular solves have four kernels (two tile rows
    per wavefront, or one with deeper load pipelines; 8 or 4 wavefronts per
    subdomain), each also on 16-column blocks with b / 16 workgroups per
    subdomain; all form the same sums in the same order, and the setup
    times them and keeps the fastest.
    Forced every way (and tuned), the sweep count, the eigenvalues, the
    coarse basis and the operator agree bit for bit."""
    need_gpu()
    from paper_1906_10944_amd import geneo as G
    prob = synth.grf_2d(seed=3, n=48, parts=2, ovl=2, inclusions=2)
    if tau is None:
        prob.tau, prob.nev = None, nev
    sysm = gpu_assemble(prob)
    r = np.random.default_rng(13).standard_normal(prob.ndof)
    outs = []
    never, always = -1, prob.nsub
    for v, sp in ((1, never), (2, never), (3, never), (4, never), (1, always), (2, always),
                  (3, always), (4, always), (0, 0)):
        h = gpu_setup(sysm, prob, precision=1, eig_solve=v, eig_split=sp)
        info = G.geneo_get_setup_info(h)
        m, lam = G.geneo_get_eigenvalues(h, prob.nsub)
        zoff, z, ah = G.geneo_get_coarse(h, prob.nsub)
        outs.append((info["eig_sweeps"], m, lam, z, ah, gpu_apply(h, sysm, r)))
        say("[eig solve] forced", v, sp, "used", info["eig_solve"], info["eig_split"], "block",
            info["eig_block"], "sweeps", info["eig_sweeps"])
        assert info["eig_block"] == {4: 16, None: 32, 24: 48}[nev]
        if v:
            # b = 48 unsplit has only the one-row kernels (2 and 4)
            assert info["eig_solve"] == (v if info["eig_block"] <= 32 or v % 2 == 0 else v + 1)
        if sp == never or info["eig_block"] == 16:
            assert info["eig_split"] == 0
        elif sp == always:
            assert info["eig_split"] == prob.nsub
        h.close()
    for got in outs[1:]:
        assert got[0] == outs[0][0]
        for a, b in zip(got[1:], outs[0][1:]):
            assert np.array_equal(a, b)


@pytest.mark.parametrize("case", ["layers3d_mixed", "layers3d_fp64", "laminate_mixed",
                                  "grf36_fp64"])
def test_envelope_gives_the_same_operator_as_dense(case):
    """The factorisations and the eigen solves skip the tiles outside each
    matrix's envelope (zero in the factors: no fill-in reaches them).  The
    products skipped are exact zeros, so the operator equals the dense
    computation's bit for bit: sweeps, eigenvalues, coarse basis and
    matrix, apply and PCG solution.  The 2D case has more than 32
    subdomains, so its factorisations take the batched kernels (with fewer,
    the shifted ones and the FP64 refactors take the tile-column steps, as
    does the coarse matrix)."""
    need_gpu()
    from paper_1906_10944_amd import geneo as G
    prob, prec = {
        "layers3d_mixed": (lambda: synth.layers_3d(seed=4, n=24, parts=2, ovl=1, nev=6), 1),
        "layers3d_fp64": (lambda: synth.layers_3d(seed=4, n=24, parts=2, ovl=1, nev=6), 0),
        "laminate_mixed": (lambda: synth.laminate_3d(ne=(16, 4, 5), parts=(4, 1, 1), nev=8), 1),
        "grf36_fp64": (lambda: synth.grf_2d(seed=7, n=96, parts=6, ovl=2, inclusions=3), 0),
    }[case]
    prob = prob()
    sysm = gpu_assemble(prob)
    r = np.random.default_rng(17).standard_normal(prob.ndof)
    outs = []
    for env in (0, 1, 2):
        h = gpu_setup(sysm, prob, precision=prec, envelope=env)
        info = G.geneo_get_setup_info(h)
        m, lam = G.geneo_get_eigenvalues(h, prob.nsub)
        zoff, z, ah = G.geneo_get_coarse(h, prob.nsub)
        x, inf = gpu_pcg(h, sysm)
        outs.append((info["eig_sweeps"], inf["iters"], m, lam, z, ah, gpu_apply(h, sysm, r), x))
        say("[envelope]", case, "envelope", env, "sweeps", info["eig_sweeps"], "nc", int(m.sum()),
            "fp64 local", info["fallback_fp64"], "iters", inf["iters"])
        h.close()
    for o in outs[1:]:
        assert outs[0][:2] == o[:2]
        for a, b in zip(outs[0][2:], o[2:]):
            assert np.array_equal(a, b)


@pytest.mark.parametrize("case", ["layers3d_mixed", "laminate_s20"])
def test_shifted_steps_match_the_batched_factorisation(case):
    """The shifted factorisations by tile-column steps (one launch per step
    over all subdomains) and by one workgroup per matrix differ in rounding
    order only: the same eigenvector counts, eigenvalues within 1e-8
    relative, PCG iterations within one and solutions within 1e-8."""
    need_gpu()
    from paper_1906_10944_amd import geneo as G
    prob = {
        "layers3d_mixed": lambda: synth.layers_3d(seed=4, n=24, parts=2, ovl=1, nev=6),
        "laminate_s20": lambda: synth.laminate_s20(ne=(8, 4, 3), parts=(2, 2, 1), nev=8),
    }[case]()
    sysm = gpu_assemble(prob)
    outs = []
    for steps in (-1, 1):
        h = gpu_setup(sysm, prob, precision=1, shifted_steps=steps)
        m, lam = G.geneo_get_eigenvalues(h, prob.nsub)
        x, inf = gpu_pcg(h, sysm)
        outs.append((m, lam, inf["iters"], x))
        say("[shifted steps]", case, steps, "nc", int(m.sum()), "iters", inf["iters"])
        h.close()
    (m0, l0, i0, x0), (m1, l1, i1, x1) = outs
    assert np.array_equal(m0, m1)
    for j in range(prob.nsub):
        k = int(m0[j])
        assert np.allclose(l0[j, :k], l1[j, :k], rtol=1e-8, atol=1e-12), j
    assert abs(i0 - i1) <= 1
    assert np.linalg.norm(x0 - x1) <= 1e-8 * np.linalg.norm(x0)


@pytest.mark.parametrize("case", ["layers3d_mixed", "laminate_fp64", "grf36_mixed", "laminate_s20"])
def test_local_solve_forms_agree(case):
    """The apply's local solves by substitution with the banded factors and
    by the product with the symmetric inverses agree to rounding: the same
    setup (eigenvalues and coarse matrix bit for bit: the form only changes
    the apply), one-level and two-level applies within twice the O(u kappa)
    bound of each, PCG iterations within two (the applies differ by O(u
    kappa), which on an ill-conditioned mixed-precision case moves the count)
    and solutions within 1e-8."""
    need_gpu()
    from paper_1906_10944_amd import geneo as G
    prob, prec = {
        "layers3d_mixed": (lambda: synth.layers_3d(seed=4, n=24, parts=2, ovl=1, nev=6), 1),
        "laminate_fp64": (lambda: synth.laminate_3d(ne=(16, 4, 5), parts=(4, 1, 1), nev=8), 0),
        "grf36_mixed": (lambda: synth.grf_2d(seed=7, n=96, parts=6, ovl=2, inclusions=3), 1),
        "laminate_s20": (lambda: synth.laminate_s20(ne=(8, 4, 3), parts=(2, 2, 1), nev=8), 1),
    }[case]
    prob = prob()
    sysm = gpu_assemble(prob)
    r = np.random.default_rng(23).standard_normal(prob.ndof)
    outs = []
    for form in (G.GENEO_LOCAL_TRIANGULAR, G.GENEO_LOCAL_INVERSE):
        h1 = gpu_setup(sysm, prob, precision=prec, coarse=0, local_solve=form)
        z1 = gpu_apply(h1, sysm, r)
        h1.close()
        h = gpu_setup(sysm, prob, precision=prec, local_solve=form)
        info = G.geneo_get_setup_info(h)
        assert info["local_solve"] == form
        m, lam = G.geneo_get_eigenvalues(h, prob.nsub)
        _, _, ah = G.geneo_get_coarse(h, prob.nsub)
        x, inf = gpu_pcg(h, sysm)
        outs.append((m, lam, ah, z1, gpu_apply(h, sysm, r), inf["iters"], x))
        say("[local form]", case, form, "iters", inf["iters"])
        h.close()
    (m0, l0, a0, z10, z0, i0, x0), (m1, l1, a1, z11, z1, i1, x1) = outs
    assert np.array_equal(m0, m1) and np.array_equal(l0, l1) and np.array_equal(a0, a1)
    # each form is within O(u kappa) of the exact local solves (u of the
    # factors' precision, kappa of the scaled local matrices): 2 x 10 u kappa
    from oracle import decomp, fem
    A, _ = fem.assemble(prob)
    subs, _ = decomp.build(prob)
    u = 2.0 ** -24 if prec else 2.0 ** -53
    tol = max(1e-12, 20 * u * kappa_local(A, subs))
    say("   one-level %.2e two-level %.2e tol %.2e" % (
        np.linalg.norm(z10 - z11) / np.linalg.norm(z11), np.linalg.norm(z0 - z1) / np.linalg.norm(z1), tol))
    assert np.linalg.norm(z10 - z11) <= tol * np.linalg.norm(z11)
    assert np.linalg.norm(z0 - z1) <= tol * np.linalg.norm(z1)
    assert abs(i0 - i1) <= 2
    assert np.linalg.norm(x0 - x1) <= 1e-8 * np.linalg.norm(x1)
