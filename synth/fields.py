"""Coefficient-field generators (seeded, element-centre sampled).

The paper's own fields (the channel/"skyscraper" picture of its structured
Darcy example, the 40-layer robustness study, the composite stacking data)
exist only as figures or external references, so these generators are the
synthetic stand-ins.  Arrays are indexed ``[iz, iy, ix]`` (``[iy, ix]`` in
2D) and flattened in C order, i.e. element ``e = ix + nx*(iy + ny*iz)``.
"""
import numpy as np


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


# ---------------------------------------------------------------- Darcy ---

def channel_field(n, n_channels=6, width=2, k_high=1e6, k_low=1.0, seed=0,
                  first_row=2, last_row=None):
    """Horizontal high-permeability channels on an ``n x n`` element grid.

    Channel start rows are drawn uniformly from ``[first_row, last_row]`` and
    redrawn until no two channels touch (at least one background row between
    them).  Each channel spans every column.
    """
    rng = _rng(seed)
    if last_row is None:
        last_row = n - width - 2
    if last_row - first_row + 1 < n_channels * (width + 1) - width:
        raise ValueError("channels do not fit without touching")
    while True:
        starts = np.sort(rng.choice(np.arange(first_row, last_row + 1),
                                    size=n_channels, replace=False))
        if n_channels < 2 or np.all(np.diff(starts) >= width + 1):
            break
    k = np.full((n, n), k_low)
    for s in starts:
        k[s:s + width, :] = k_high
    return k, starts


def grf_exponential_2d(n, var=4.0, corr=0.05, seed=0, pad=2):
    """Stationary Gaussian field with covariance ``var*exp(-r/corr)``.

    Sampled at element centres of the unit square (spacing ``1/n``) by
    circulant embedding on a ``pad*n`` periodic torus; the padding doubles
    until the embedding's spectrum is non-negative to ``1e-10`` relative.
    """
    rng = _rng(seed)
    h = 1.0 / n
    while True:
        m = pad * n
        idx = np.arange(m)
        d = np.minimum(idx, m - idx) * h
        r = np.sqrt(d[:, None] ** 2 + d[None, :] ** 2)
        lam = np.fft.fft2(var * np.exp(-r / corr)).real
        if lam.min() >= -1e-10 * lam.max():
            break
        pad *= 2
    lam = np.clip(lam, 0.0, None)
    xi = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
    y = np.fft.fft2(np.sqrt(lam / (m * m)) * xi)
    return np.ascontiguousarray(y.real[:n, :n])


def inclusions_2d(n, count=24, rmin=0.01, rmax=0.03, seed=0):
    """Boolean mask of elements whose centre lies in one of ``count`` discs.

    Disc centres are uniform on the unit square, radii uniform in
    ``[rmin, rmax]``.
    """
    rng = _rng(seed)
    c = rng.uniform(0.0, 1.0, size=(count, 2))
    rad = rng.uniform(rmin, rmax, size=count)
    xc = (np.arange(n) + 0.5) / n
    X, Y = np.meshgrid(xc, xc, indexing="xy")  # X[iy, ix] = x(ix)
    mask = np.zeros((n, n), dtype=bool)
    for (cx, cy), r in zip(c, rad):
        mask |= (X - cx) ** 2 + (Y - cy) ** 2 <= r * r
    return mask


def z_layers_3d(nz, tmin=2, tmax=6, kmin_exp=4.0, kmax_exp=6.0, seed=0):
    """Per-``iz`` coefficient of a layered medium.

    Layer thicknesses are uniform integers in ``[tmin, tmax]``; layers
    alternate between ``k = 1`` (the first) and ``k = 10**U(kmin_exp,
    kmax_exp)``; the last layer is truncated at ``nz``.
    """
    rng = _rng(seed)
    kz = np.empty(nz)
    z, layer = 0, 0
    while z < nz:
        t = int(rng.integers(tmin, tmax + 1))
        val = 1.0 if layer % 2 == 0 else 10.0 ** rng.uniform(kmin_exp, kmax_exp)
        kz[z:min(nz, z + t)] = val
        z += t
        layer += 1
    return kz


# ----------------------------------------------------------- elasticity ---

def voigt_upper(C):
    """The 21 upper-triangle entries of a symmetric 6x6 Voigt matrix, row major."""
    iu = np.triu_indices(6)
    return np.asarray(C, dtype=np.float64)[iu]


def isotropic_stiffness(E, nu):
    """6x6 Voigt stiffness (engineering shear strains) of an isotropic solid."""
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    mu = E / (2 * (1 + nu))
    C = np.zeros((6, 6))
    C[:3, :3] = lam
    C[0, 0] = C[1, 1] = C[2, 2] = lam + 2 * mu
    C[3, 3] = C[4, 4] = C[5, 5] = mu
    return C


def ply_stiffness(E1, E2, E3, G12, G13, G23, nu12, nu13, nu23):
    """6x6 Voigt stiffness of an orthotropic ply from its engineering constants.

    Voigt order (11, 22, 33, 23, 13, 12); built by inverting the compliance.
    """
    S = np.zeros((6, 6))
    S[0, 0], S[1, 1], S[2, 2] = 1 / E1, 1 / E2, 1 / E3
    S[0, 1] = S[1, 0] = -nu12 / E1
    S[0, 2] = S[2, 0] = -nu13 / E1
    S[1, 2] = S[2, 1] = -nu23 / E2
    S[3, 3], S[4, 4], S[5, 5] = 1 / G23, 1 / G13, 1 / G12
    return np.linalg.inv(S)


def rotate_z90(C):
    """Stiffness of a ply turned 90 degrees about z (material axes 1 and 2 swap)."""
    p = [1, 0, 2, 4, 3, 5]
    return np.asarray(C)[np.ix_(p, p)]
