"""Seeded synthetic workloads: geometries, STO basis lists, auxiliary lists and grid specs.

This module only draws inputs.  It contains none of the integration method's arithmetic, and both the
HIP library and the CPU oracle consume what it produces (as plain arrays), so a bug here cannot make the
two sides agree by accident.

Recipe (the paper prints no worked inputs, so every workload is synthetic):
  * Units are bohr and hartree.
  * Exponents are stratified log-uniform per (atom, l) channel: with c shells in the channel,
    zeta_k = exp(ln lo + (ln hi - ln lo) * (k + u_k) / c), u_k ~ U(0.25, 0.75), so no two shells of a
    channel are near-duplicates and S and (P|Q) stay positive definite.  This mimics the even-tempered
    construction of Section 3 of the paper.
  * Shells of a channel are sorted by descending zeta; basis principal quantum numbers are
    n = l + 1 + (k mod (n_max - l)); auxiliary functions use n = l + 1.
  * Every m = -l..l of a shell is enumerated (Section 3: all m degrees of freedom).
  * Auxiliary exponent ranges run from twice the atom's smallest basis exponent to twice its largest
    (Section 3: aux exponents come from sums of pairs of basis exponents), unless the workload states
    them.  The quadruple-zeta-sized sets reach four times the largest instead and spread their shells
    over l = 0..4 as (10, 8, 7, 6, 6) per heavy atom and (7, 5, 4, 3, 3) per H, which keeps adjacent
    exponents of a channel about 1.5x apart: the Coulomb metric of the triatomic QZ job then has its
    smallest eigenvalue at 1.2e-6 (of 373) on its 96x96x48-point grids, against -1.9e-6 with 16 s
    shells over twice the basis range (exactly, 2.5e-12: so close to singular that the quadrature
    error of those grids made it indefinite).
  * Grid sizes: the workloads are quoted in quadrature points per axis; with Q = 4 Gauss-Legendre
    points per cell and axis the cell counts are points / 4.
  * Seeds: numpy PCG64 from SeedSequence(15204).spawn(5)[i] for workload i (0-based).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

SEED_BASE = 15204
BOHR_PER_ANGSTROM = 1.8897261246

# shell counts per l (s, p, d, f, g, h, i) for each basis family
SHELLS = {
    "H": {
        "DZ": (2, 1),
        "TZ": (3, 2),
        "QZ": (8, 4, 2),
        "5Z": (11, 5, 3, 2),
        "auxDZ": (4, 2, 1),
        "auxTZ": (8, 3, 2),
        "auxQZ": (7, 5, 4, 3, 3),
        "aux5Z": (16, 9, 7, 6, 5),
    },
    "heavy": {
        "DZ": (4, 2, 1),
        "TZ": (6, 3, 2),
        "QZ": (11, 5, 3, 2),
        "5Z": (14, 6, 4, 3, 2),
        "auxDZ": (7, 4, 2, 1, 1),
        "auxTZ": (14, 6, 4, 2, 1),
        "auxQZ": (10, 8, 7, 6, 6),
        "aux5Z": (27, 12, 10, 8, 5, 3, 2),
    },
}

# basis exponent ranges per element (lo, hi)
ZETA_RANGE = {1: (0.4, 4.0), 6: (0.3, 10.0), 7: (0.3, 11.0), 8: (0.3, 12.0), 9: (0.3, 13.0), 17: (0.25, 18.0)}
BOHR_PER_ANGSTROM = 1.8897261246


@dataclasses.dataclass
class GridSpec:
    """Cells per axis (paper N_mu, N_nu, N_phi), GL points per axis per cell (Q), third-centre split."""
    n_mu: int
    n_nu: int
    n_phi: int
    q: int = 4
    n_sp: int = 3
    c1_scale: float = 2.3
    c1_exp: float = 0.25

    def as_tuple(self):
        return (self.n_mu, self.n_nu, self.n_phi, self.q, self.n_sp, self.c1_scale, self.c1_exp)


@dataclasses.dataclass
class Job:
    """One integral job: geometry + basis + aux basis + grid spec (problem statement of Section 2)."""
    name: str
    xyz: np.ndarray            # (n_atoms, 3) bohr
    Z: np.ndarray              # (n_atoms,) nuclear charges
    basis: np.ndarray          # (n_bf, 5): atom, n, l, m, zeta  (float64 array)
    aux: np.ndarray            # (n_aux, 5)
    grid: GridSpec
    pair_grids: Dict[Tuple[int, int], GridSpec] = dataclasses.field(default_factory=dict)
    precision: str = "fp64"    # "fp64" or "mixed"

    @property
    def n_atoms(self):
        return int(self.xyz.shape[0])

    @property
    def n_bf(self):
        return int(self.basis.shape[0])

    @property
    def n_aux(self):
        return int(self.aux.shape[0])

    def spec_for(self, a: int, b: int) -> GridSpec:
        key = (min(a, b), max(a, b))
        return self.pair_grids.get(key, self.grid)


def rng_for(workload_index: int) -> np.random.Generator:
    ss = np.random.SeedSequence(SEED_BASE).spawn(5)[workload_index]
    return np.random.Generator(np.random.PCG64(ss))


def _channel_zetas(rng: np.random.Generator, c: int, lo: float, hi: float) -> List[float]:
    u = rng.uniform(0.25, 0.75, size=c)
    k = np.arange(c)
    z = np.exp(math.log(lo) + (math.log(hi) - math.log(lo)) * (k + u) / c)
    return sorted(z.tolist(), reverse=True)


def make_shells(rng, atom: int, shells_per_l: Sequence[int], lo: float, hi: float,
                n_max: Optional[int], aux: bool) -> List[Tuple[int, int, int, int, float]]:
    """Functions (atom, n, l, m, zeta) for all shells of one atom; m runs -l..l within each shell."""
    out = []
    for l, c in enumerate(shells_per_l):
        if c == 0:
            continue
        zs = _channel_zetas(rng, c, lo, hi)
        nm = n_max if n_max is not None else len(shells_per_l)
        for k, z in enumerate(zs):
            if aux:
                n = l + 1
            else:
                span = max(nm - l, 1)
                n = l + 1 + (k % span)
            for m in range(-l, l + 1):
                out.append((atom, n, l, m, z))
    return out


def _as_array(funcs) -> np.ndarray:
    return np.array([[f[0], f[1], f[2], f[3], f[4]] for f in funcs], dtype=np.float64).reshape(-1, 5)


def _kind(Z):
    return "H" if Z == 1 else "heavy"


def build_basis(rng, Z: Sequence[int], family: str, aux_family: str, n_max: Optional[int],
                aux_ranges=None, basis_ranges=None):
    basis, aux = [], []
    for a, z in enumerate(Z):
        lo, hi = (basis_ranges or ZETA_RANGE)[int(z)]
        basis += make_shells(rng, a, SHELLS[_kind(z)][family], lo, hi, n_max, aux=False)
    for a, z in enumerate(Z):
        if aux_ranges is not None:
            alo, ahi = aux_ranges[int(z)]
        else:
            lo, hi = (basis_ranges or ZETA_RANGE)[int(z)]
            alo, ahi = 2 * lo, (4 if aux_family == "auxQZ" else 2) * hi
        aux += make_shells(rng, a, SHELLS[_kind(z)][aux_family], alo, ahi, None, aux=True)
    return _as_array(basis), _as_array(aux)


# ---------------------------------------------------------------------------------------------
# The five workloads
# ---------------------------------------------------------------------------------------------

def diatomic_small() -> Job:
    """Two H nuclei 1.4 bohr apart on z; 1s, 2s, 2p per atom; 12 aux per atom; one 40x40x16-point grid."""
    rng = rng_for(0)
    xyz = np.array([[0.0, 0.0, 0.7], [0.0, 0.0, -0.7]])
    Z = np.array([1.0, 1.0])
    basis, aux = [], []
    for a in range(2):
        basis += make_shells(rng, a, (2, 1), 0.5, 3.0, 2, aux=False)
    for a in range(2):
        aux += make_shells(rng, a, (4, 1, 1), 0.8, 6.0, None, aux=True)
    return Job("diatomic_H2_40x40x16", xyz, Z, _as_array(basis), _as_array(aux),
               GridSpec(10, 10, 4, 4, 3))


def triatomic_geometry(bond=1.8, angle_deg=104.0):
    h = math.radians(angle_deg) / 2.0
    return np.array([[0.0, 0.0, 0.0],
                     [bond * math.sin(h), 0.0, bond * math.cos(h)],
                     [-bond * math.sin(h), 0.0, bond * math.cos(h)]])


def triatomic_qz(points_per_axis=(96, 96, 48)) -> Job:
    """Bent Z=(8,1,1), bond 1.8 bohr, 104 degrees; O 55 / H 30 functions; aux 3x (l<=4); 96x96x48 grids."""
    rng = rng_for(1)
    Z = np.array([8.0, 1.0, 1.0])
    basis, aux = build_basis(rng, Z.astype(int), "QZ", "auxQZ", n_max=4)
    g = GridSpec(points_per_axis[0] // 4, points_per_axis[1] // 4, points_per_axis[2] // 4, 4, 3)
    return Job("triatomic_QZ_96x96x48", triatomic_geometry(), Z, basis, aux, g, precision="fp64")


def triatomic_5z(points_per_axis=(128, 128, 64)) -> Job:
    """Same shape, O 91 / H 55 functions (l<=4), aux 3x (l<=6), 128x128x64 grids, mixed precision."""
    rng = rng_for(2)
    Z = np.array([8.0, 1.0, 1.0])
    basis, aux = build_basis(rng, Z.astype(int), "5Z", "aux5Z", n_max=None)
    g = GridSpec(points_per_axis[0] // 4, points_per_axis[1] // 4, points_per_axis[2] // 4, 4, 3)
    return Job("triatomic_5Z_128x128x64", triatomic_geometry(), Z, basis, aux, g, precision="mixed")


# 1,3-propanediyl template (angstrom, Table S2 of the paper's supporting information)
_PROPANEDIYL = [
    (6, (1.278, 0.0, 0.2597)), (6, (0.0, 0.0, -0.5852)), (6, (-1.278, 0.0, 0.2597)),
    (1, (1.325, -0.8846, 0.9073)), (1, (1.325, 0.8846, 0.9073)),
    (1, (0.0, 0.8776, -1.246)), (1, (0.0, -0.8776, -1.246)),
    (1, (-1.325, -0.8846, 0.9073)), (1, (-1.325, 0.8846, 0.9073)),
]


def hydrocarbon_geometry(rng, cc=2.9, ch=2.05, jitter=0.05):
    t = np.array([p for _, p in _PROPANEDIYL]) * BOHR_PER_ANGSTROM
    Z = np.array([z for z, _ in _PROPANEDIYL], dtype=float)
    out = t.copy()
    mid = t[1]
    for c in (0, 2):
        d = t[c] - mid
        out[c] = mid + cc * d / np.linalg.norm(d)
    for h in range(3, 9):
        parent = min(range(3), key=lambda c: np.linalg.norm(t[h] - t[c]))
        d = t[h] - t[parent]
        out[h] = out[parent] + ch * d / np.linalg.norm(d)
    out = out + rng.uniform(-jitter, jitter, size=out.shape)
    return out, Z


def hydrocarbon9(points_choices=(64, 80, 96, 112, 128)) -> Job:
    """9-atom C3H6-shaped molecule, C 55 / H 30 functions, aux 3x, 36 pair grids of 64..128 points/axis.

    Auxiliary exponents span 4x the element's basis range at both ends: with the lower end at 2x, the
    most diffuse auxiliary functions of neighbouring atoms (2-3 bohr apart) are so nearly dependent in
    the Coulomb metric that the grids' quadrature error leaves (P|Q) indefinite (smallest eigenvalue
    -5e-6 of 870); from 4x up it is positive definite (smallest eigenvalue 6e-9 of 190)."""
    rng = rng_for(3)
    xyz, Z = hydrocarbon_geometry(rng)
    aux_ranges = {int(z): (4 * ZETA_RANGE[int(z)][0], 4 * ZETA_RANGE[int(z)][1]) for z in set(Z.astype(int).tolist())}
    basis, aux = build_basis(rng, Z.astype(int), "QZ", "auxQZ", n_max=4, aux_ranges=aux_ranges)
    pair_grids = {}
    n = len(Z)
    for a in range(n):
        for b in range(a + 1, n):
            p = rng.choice(points_choices, size=3)
            pair_grids[(a, b)] = GridSpec(int(p[0]) // 4, int(p[1]) // 4, int(p[2]) // 4, 4, 3)
    return Job("hydrocarbon9_QZ", xyz, Z, basis, aux, GridSpec(24, 24, 24, 4, 3), pair_grids,
               precision="mixed")


def random_molecule(rng, max_atoms=12, families=("DZ", "TZ", "QZ"),
                    axis_points=(48, 64, 80, 96, 112, 128), min_dist=1.8) -> Job:
    """One serving request: random tree-grown molecule, random basis family, random per-pair grids."""
    n = int(rng.integers(2, max_atoms + 1))
    Z = rng.choice([1, 6, 7, 8], size=n).astype(float)
    xyz = np.zeros((n, 3))
    placed = 1
    while placed < n:
        parent = int(rng.integers(0, placed))
        r = rng.uniform(1.8, 3.0)
        v = rng.normal(size=3)
        v /= np.linalg.norm(v)
        cand = xyz[parent] + r * v
        d = np.linalg.norm(xyz[:placed] - cand, axis=1)
        d[parent] = np.inf
        if np.all(d >= min_dist):
            xyz[placed] = cand
            placed += 1
    fam = str(rng.choice(list(families)))
    basis, aux = build_basis(rng, Z.astype(int), fam, "aux" + fam, n_max=4)
    pair_grids = {}
    for a in range(n):
        for b in range(a + 1, n):
            p = rng.choice(axis_points, size=3)
            pair_grids[(a, b)] = GridSpec(int(p[0]) // 4, int(p[1]) // 4, int(p[2]) // 4, 4, 3)
    return Job(f"request_{n}atoms_{fam}", xyz, Z, basis, aux, GridSpec(16, 16, 16, 4, 3), pair_grids,
               precision="mixed")


def serving_stream(n_requests=1100, rate_per_s=50.0, max_atoms=12, families=("DZ", "TZ", "QZ"),
                   axis_points=(48, 64, 80, 96, 112, 128)):
    """Poisson arrivals of random molecules; returns [(arrival_time_s, Job)]."""
    rng = rng_for(4)
    t = 0.0
    out = []
    for _ in range(n_requests):
        t += rng.exponential(1.0 / rate_per_s)
        out.append((t, random_molecule(rng, max_atoms, families, axis_points)))
    return out


def clf_tz(spec=(26, 20, 8, 4, 3), seed_index=1) -> Job:
    """ClF-shaped diatomic (bond 1.628 A) with triple-zeta-sized bases (25 + 25 functions, 75 + 75
    auxiliary): the two-centre molecule of the paper's grid-convergence study (Figs. 3-4)."""
    rng = rng_for(seed_index)
    Z = np.array([17.0, 9.0])
    xyz = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 1.628 * BOHR_PER_ANGSTROM]])
    basis, aux = build_basis(rng, Z.astype(int), "TZ", "auxTZ", n_max=4)
    return Job("ClF_TZ", xyz, Z, basis, aux, GridSpec(*spec))


def of2_tz(spec=(26, 20, 8, 4, 3), long_bond=False, seed_index=1) -> Job:
    """OF2-shaped triatomic (O-F 1.405 A, F-O-F 103.1 deg) with triple-zeta-sized bases: the
    three-centre molecule of Figs. 3-5.  long_bond moves one F out to 41.41 A along its bond (the
    stretched geometry of Fig. S1)."""
    rng = rng_for(seed_index)
    Z = np.array([8.0, 9.0, 9.0])
    r = 1.405 * BOHR_PER_ANGSTROM
    h = math.radians(103.1) / 2.0
    u1 = np.array([math.sin(h), 0.0, math.cos(h)])
    u2 = np.array([-math.sin(h), 0.0, math.cos(h)])
    r1 = 41.41 * BOHR_PER_ANGSTROM if long_bond else r
    xyz = np.array([[0.0, 0.0, 0.0], r1 * u1, r * u2])
    basis, aux = build_basis(rng, Z.astype(int), "TZ", "auxTZ", n_max=4)
    return Job("OF2_TZ_long" if long_bond else "OF2_TZ", xyz, Z, basis, aux, GridSpec(*spec))


WORKLOADS = {
    "diatomic_small": diatomic_small,
    "triatomic_qz": triatomic_qz,
    "triatomic_5z": triatomic_5z,
    "hydrocarbon9": hydrocarbon9,
}


def scaled_triatomic(points_per_axis, family="QZ", aux_family="auxQZ", seed_index=1, n_max=4,
                     precision="fp64") -> Job:
    """The triatomic shape at another grid size or basis (used for small parity cases)."""
    rng = rng_for(seed_index)
    Z = np.array([8.0, 1.0, 1.0])
    basis, aux = build_basis(rng, Z.astype(int), family, aux_family, n_max=n_max)
    g = GridSpec(points_per_axis[0] // 4, points_per_axis[1] // 4, points_per_axis[2] // 4, 4, 3)
    return Job(f"triatomic_{family}_{points_per_axis[0]}x{points_per_axis[1]}x{points_per_axis[2]}",
               triatomic_geometry(), Z, basis, aux, g, precision=precision)
