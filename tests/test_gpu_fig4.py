"""The robustness study of Sec. 5.2 (Fig. 4, right), scaled to one GPU, and
the eigenvalue threshold of Thm. 1 on the device.

Fig. 4 (right): Darcy on a square with 40 horizontal layers of equal
thickness alternating k = 1 and k = contrast, 8 x 8 subdomains with an
overlap of two elements, so that each subdomain holds five layers; the
paper reports that the condition number stays flat as the contrast grows
exactly when every subdomain contributes at least four eigenvectors, and
grows without bound with fewer.  Here: 200 x 200 Q1 elements (the paper
uses 800 x 800; each subdomain is 25 x 25 elements and holds five layers
either way), Dirichlet conditions on the bottom and top, Neumann on the
sides, contrasts 1e0 .. 1e6 and m = 2 .. 5, condition numbers from the
device's CG-Lanczos estimate, checked against the oracle at the largest
contrast.

Thm. 1: m_j = #{lambda < delta_j / H_j} per subdomain (thresholds from
geneo_q1_thm1_tau, checked against the oracle's), selected on the device;
the counts match the oracle's and the condition estimate stays under the
theorem's bound.
"""
import numpy as np
import pytest

import synth
from gpu_common import gpu_assemble, gpu_pcg, gpu_setup, need_gpu, say
from oracle import decomp, fem, geneo, pcg

pytestmark = pytest.mark.gpu

CONTRASTS = (1e0, 1e2, 1e4, 1e6)
MS = (2, 3, 4, 5)
# The paper's claim is about large contrast: with m >= 4 the condition
# number stays bounded as the contrast grows, with m <= 3 it grows in
# proportion to the contrast.  Checked over the last two decades of the
# sweep (1e4 -> 1e6):
FLAT_RATIO = 1.6     # m >= 4: kappa(1e6) / kappa(1e4) at most this, kappa < KAPPA_MAX
KAPPA_MAX = 100.0
GROWTH_RATIO = 50.0  # m <= 3: kappa(1e6) / kappa(1e4) at least this


def _fig4(contrast, m):
    return synth.layered_2d(n=200, parts=8, ovl=2, layers=40, contrast=contrast, nev=m)


@pytest.fixture(scope="module")
def sweep():
    need_gpu()
    out = {}
    for c in CONTRASTS:
        sysm = gpu_assemble(_fig4(c, 4))
        for m in MS:
            p = _fig4(c, m)
            h = gpu_setup(sysm, p)
            x, inf = gpu_pcg(h, sysm, rtol=1e-10)
            h.close()
            assert inf["converged"]
            out[(c, m)] = (inf["iters"], inf["kappa_est"])
        say("[fig4] contrast %.0e: %s" % (c, "  ".join(
            "m=%d it %d kappa %.2f" % ((m,) + out[(c, m)]) for m in MS)))
    return out


def test_fig4_kappa_bounded_with_four_or_more_vectors(sweep):
    for m in (4, 5):
        k = [sweep[(c, m)][1] for c in CONTRASTS]
        assert k[-1] / k[-2] <= FLAT_RATIO and max(k) < KAPPA_MAX, (m, k)


def test_fig4_kappa_grows_with_fewer_than_four_vectors(sweep):
    for m in (2, 3):
        k = [sweep[(c, m)][1] for c in CONTRASTS]
        assert all(k[i + 1] >= k[i] for i in range(len(k) - 1)), (m, k)
        assert k[-1] / k[-2] >= GROWTH_RATIO, (m, k)


@pytest.mark.parametrize("m", [3, 4])
def test_fig4_against_oracle(sweep, m):
    """m = 3 cuts every subdomain's spectrum at a wide gap: the coarse space
    is unique and the condition estimates are compared (to 1e-6).  The
    iteration count is compared within +-2 plus the spread that a 1e-10
    relative perturbation of the oracle's own coarse basis produces: the
    64 subdomains' first discarded eigenpairs leave a tight cluster of
    small eigenvalues in the preconditioned operator, and the number of
    steps CG spends on that cluster (at kappa ~ 5e5, to 1e-10) depends on
    how tightly it clusters, a property below any eigen solver's
    tolerance (a 1e-12 perturbation of the basis already moves the
    oracle's count, while its kappa is unchanged to 1e-9).  m = 4
    cuts a pair of equal eigenvalues (the mirror-symmetric overlap strips of
    interior subdomains, checked here on the oracle's spectra): both sides
    hold a valid GenEO space, not the same one, so the comparison is the
    solution, with both condition numbers bounded."""
    p = _fig4(CONTRASTS[-1], m)
    A, b = fem.assemble(p)
    g = geneo.setup(p, A=A)
    ref = pcg.pcg(A, b, g.apply, rtol=1e-10)
    ko = pcg.kappa_estimate(ref.alphas, ref.betas)
    it, kg = sweep[(CONTRASTS[-1], m)]
    gaps = [(l[m] - l[m - 1]) / l[m] for l in g.lam]
    say("[fig4 oracle] m=%d contrast %.0e: device it %d kappa %.4f | oracle it %d kappa %.4f | "
        "smallest relative gap at the cut %.2e" % (m, CONTRASTS[-1], it, kg, ref.iters, ko,
                                                   min(gaps)))
    if m == 3:
        assert min(gaps) > 1e-3
        rng = np.random.Generator(np.random.PCG64(7))
        Zp = g.Z.copy()
        Zp.data = Zp.data * (1.0 + 1e-10 * rng.standard_normal(len(Zp.data)))
        g.Z = Zp
        AH = (Zp.T @ (A @ Zp)).toarray()
        g.AH = 0.5 * (AH + AH.T)
        g.LH = geneo.coarse_cholesky(g.AH)
        refp = pcg.pcg(A, b, g.apply, rtol=1e-10)
        spread = abs(refp.iters - ref.iters)
        say("   oracle with its coarse basis perturbed by 1e-10: it %d kappa %.4f (spread %d)" %
            (refp.iters, pcg.kappa_estimate(refp.alphas, refp.betas), spread))
        assert abs(it - ref.iters) <= 2 + spread
        assert kg == pytest.approx(ko, rel=1e-6)
    else:
        assert min(gaps) < 1e-6
        sysm = gpu_assemble(p)
        h = gpu_setup(sysm, p)
        x, inf = gpu_pcg(h, sysm, rtol=1e-10)
        h.close()
        err = np.linalg.norm(x - ref.x) / np.linalg.norm(ref.x)
        say("   solution rel diff %.2e" % err)
        assert err <= 1e-8
        assert kg < KAPPA_MAX and ko < KAPPA_MAX


def test_thm1_threshold_rule_on_device():
    need_gpu()
    from paper_1906_10944_amd import geneo as G
    p = synth.layered_2d(n=48, parts=4, ovl=2, layers=8, contrast=1e6, nev=16)
    subs, _ = decomp.build(p)
    tau_o = decomp.thm1_threshold(p, subs)
    tau_g = G.geneo_q1_thm1_tau(G.grid_from_problem(p), p.nsub)
    assert np.allclose(tau_g, tau_o, rtol=1e-15, atol=0)
    sysm = gpu_assemble(p)
    opts = G.with_tau_sub(G.opts_from_problem(p, nev_max=32), tau_g)
    h = G.geneo_setup(sysm.csr(), sysm.subdomains(), sysm.neumann(), sysm.overlap(), opts)
    m, lam = G.geneo_get_eigenvalues(h, p.nsub)
    x, inf = gpu_pcg(h, sysm, rtol=1e-10)
    h.close()
    A, b = fem.assemble(p)
    g = geneo.setup(p, A=A, subs=subs, tau=tau_o, nev_max=32)
    ref = pcg.pcg(A, b, g.apply, rtol=1e-10)
    k0 = 4
    bound = (1 + k0) * (2 + k0 * (2 * k0 + 1) * np.max(1 + 1 / tau_o))
    say("[thm1] m_j", list(m), "device it %d kappa %.3f | oracle it %d | bound %.0f" %
        (inf["iters"], inf["kappa_est"], ref.iters, bound))
    assert list(m) == list(g.m)
    assert inf["converged"] and abs(inf["iters"] - ref.iters) <= 2
    assert inf["kappa_est"] <= bound
