"""Independent 3-D reference integration for the oracle's pins: Becke's fuzzy-cell partition of space
among the atoms (A. D. Becke, J. Chem. Phys. 88, 2547 (1988)), each atom's cell integrated on a
spherical product grid about that atom.  Nothing here comes from the oracle: Slater functions and
real spherical harmonics are built from scipy.special.sph_harm_y, and the Coulomb potential of an
auxiliary Slater function from scipy's regularised incomplete gamma functions.

Partition: for atoms i, j at distances r_i, r_j from a point and R_ij apart, mu_ij = (r_i - r_j) / R_ij,
three passes of p(mu) = 1.5 mu - 0.5 mu^3, s_ij = (1 - p) / 2; cell weight w_i = prod_j s_ij /
sum_k prod_j s_kj.  Each w_i vanishes at every other nucleus to high order, so the cusps of functions
centred there do not reach the grid of atom i.
Grid of atom i: r = alpha (1 + x) / (1 - x) on Gauss-Legendre nodes x (dr = 2 alpha / (1 - x)^2 dx),
Gauss-Legendre nodes in cos(theta), equally spaced phi (exact for trigonometric polynomials below
n_phi).  Test infrastructure only.
"""
import math

import numpy as np
from scipy import special

PI = math.pi


def real_ylm(l, m, d):
    """Real spherical harmonic of the direction of d (rows): sqrt(2) (-1)^m Re/Im of the complex one
    with the Condon-Shortley phase, for m > 0 / m < 0; the complex one for m = 0."""
    r = np.linalg.norm(d, axis=-1)
    ct = np.clip(d[..., 2] / np.where(r > 0, r, 1.0), -1.0, 1.0)
    th = np.arccos(ct)
    ph = np.arctan2(d[..., 1], d[..., 0])
    am = abs(m)
    Yc = special.sph_harm_y(l, am, th, ph)
    if m == 0:
        return Yc.real
    if m > 0:
        return math.sqrt(2) * (-1) ** am * Yc.real
    return math.sqrt(2) * (-1) ** am * Yc.imag


def _norm(n, zeta):
    return (2 * zeta) ** (n + 0.5) / math.sqrt(math.factorial(2 * n))


def sto(fn, centre, p):
    """Normalised Slater function N r^(n-1) e^(-zeta r) Y_lm (eq. 1); fn = (n, l, m, zeta)."""
    n, l, m, z = int(fn[0]), int(fn[1]), int(fn[2]), float(fn[3])
    d = p - centre
    r = np.linalg.norm(d, axis=-1)
    return _norm(n, z) * r ** (n - 1) * np.exp(-z * r) * real_ylm(l, m, d)


def sto_potential(fn, centre, p):
    """Coulomb potential of the Slater function fn at points p:
    4 pi / (2l+1) N Y_lm [r^-(l+1) int_0^r s^(n+l+1) e^(-zeta s) ds + r^l int_r^inf s^(n-l) e^(-zeta s) ds],
    the two radial integrals as lower and upper incomplete gamma functions of zeta r."""
    n, l, m, z = int(fn[0]), int(fn[1]), int(fn[2]), float(fn[3])
    d = p - centre
    r = np.linalg.norm(d, axis=-1)
    x = z * r
    k1, k2 = n + l + 2, n - l + 1
    inner = special.gamma(k1) * special.gammainc(k1, x) / z ** k1
    outer = special.gamma(k2) * special.gammaincc(k2, x) / z ** k2
    return 4 * PI / (2 * l + 1) * _norm(n, z) * real_ylm(l, m, d) * (r ** (-l - 1) * inner + r ** l * outer)


def becke_grid(centres, n_r=80, n_theta=40, n_phi=80, alpha=1.0):
    """Points (N x 3) and weights (N) of the partitioned multi-centre grid."""
    centres = np.asarray(centres, dtype=float)
    x, wx = np.polynomial.legendre.leggauss(n_r)
    r = alpha * (1 + x) / (1 - x)
    wr = 2 * alpha / (1 - x) ** 2 * wx * r * r
    ct, wt = np.polynomial.legendre.leggauss(n_theta)
    st = np.sqrt(1 - ct * ct)
    ph = (np.arange(n_phi) + 0.5) * 2 * PI / n_phi
    dirs = np.stack([np.outer(st, np.cos(ph)), np.outer(st, np.sin(ph)), np.outer(ct, np.ones(n_phi))],
                    axis=-1).reshape(-1, 3)
    w_ang = np.outer(wt, np.full(n_phi, 2 * PI / n_phi)).reshape(-1)
    nc = len(centres)
    R = np.linalg.norm(centres[:, None] - centres[None], axis=-1)
    pts, wts = [], []
    for i, c in enumerate(centres):
        p = c + (r[:, None, None] * dirs[None]).reshape(-1, 3)
        w = (wr[:, None] * w_ang[None]).reshape(-1)
        dist = np.linalg.norm(p[:, None, :] - centres[None], axis=-1)
        cell = np.ones((p.shape[0], nc))
        for a in range(nc):
            for b in range(nc):
                if a == b:
                    continue
                mu = (dist[:, a] - dist[:, b]) / R[a, b]
                for _ in range(3):
                    mu = 1.5 * mu - 0.5 * mu ** 3
                cell[:, a] *= 0.5 * (1 - mu)
        pts.append(p)
        wts.append(w * cell[:, i] / cell.sum(axis=1))
    return np.concatenate(pts), np.concatenate(wts)
