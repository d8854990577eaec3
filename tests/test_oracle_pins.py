"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix (no GPU).

Each test names the passage of the paper (arXiv 2510.15204) whose definition it pins.  The reference
values never come from the oracle itself: they are closed forms, library routines (numpy/scipy), an
independent adaptive 2-D quadrature in elliptic coordinates (tests/axial_reference.py), or brute
force.
"""
import math

import numpy as np
import pytest
from scipy import integrate, special

import oracle as O
from axial_reference import Fn, integral as ref_integral
from conftest import MiniJob, Spec

PI = math.pi


# ---------------------------------------------------------------------------------------------
# Gauss-Legendre rule (Section 2.1: GL quadrature per cell and axis)
# ---------------------------------------------------------------------------------------------

@pytest.mark.parametrize("q", list(range(1, 17)))
def test_gauss_legendre_matches_numpy(q):
    x, w = O.gauss_legendre(q)
    xr, wr = np.polynomial.legendre.leggauss(q)
    assert np.max(np.abs(x - xr)) < 1e-14
    assert np.max(np.abs(w - wr)) < 1e-14


# ---------------------------------------------------------------------------------------------
# Grid: point count, volume, polynomial exactness, third-centre moves (eqs. 2-7, 10-12, 17, Alg. 1-2)
# ---------------------------------------------------------------------------------------------

TRI = np.array([[0.0, 0.0, 0.0], [1.4186, 0.0, 1.1082], [-1.4186, 0.0, 1.1082]])


def _local_coords(xyz, A, B, info, x, y, z):
    """(mu, nu, phi) of global points, recovered from the focus distances and the frame."""
    a = info["a"]
    RA, RB = xyz[A], xyz[B]
    rA = np.sqrt((x - RA[0]) ** 2 + (y - RA[1]) ** 2 + (z - RA[2]) ** 2)
    rB = np.sqrt((x - RB[0]) ** 2 + (y - RB[1]) ** 2 + (z - RB[2]) ** 2)
    mu = np.arccosh(np.maximum((rA + rB) / (2 * a), 1.0))
    nu = np.arccos(np.clip((rB - rA) / (2 * a), -1, 1))
    d = np.stack([x - info["M"][0], y - info["M"][1], z - info["M"][2]], axis=1)
    lx, ly = d @ info["ex"], d @ info["ey"]
    phi = np.mod(np.arctan2(ly, lx), 2 * PI)
    return mu, nu, phi


@pytest.mark.parametrize("A,B,C,nsp", [(1, 2, -1, 3), (1, 2, 0, 1), (1, 2, 0, 2), (1, 2, 0, 3), (0, 1, 2, 4)])
def test_point_count_formula(A, B, C, nsp):
    spec = (7, 6, 5, 3, nsp, 2.3, 0.25)
    info = O.grid_info(TRI, A, B, C, spec)
    split = info["split"]
    assert split == (C >= 0 and nsp >= 2)
    expect = (7 * 6 * 5 + (8 * (nsp ** 3 - 1) if split else 0)) * 27
    assert info["n_points"] == expect
    x, y, z, w = O.grid_points(TRI, A, B, C, spec)
    assert x.size == expect and np.all(w > 0)


@pytest.mark.parametrize("C", [-1, 0])
def test_weights_sum_to_spheroid_volume(C):
    # sum of weights = volume enclosed by mu <= mu_max = (4 pi / 3) a^3 cosh(M) sinh^2(M)
    spec = (24, 16, 6, 8, 3, 2.3, 0.25)
    info = O.grid_info(TRI, 1, 2, C, spec)
    x, y, z, w = O.grid_points(TRI, 1, 2, C, spec)
    a, M = info["a"], info["mu"][-1]
    vol = 4 * PI / 3 * a ** 3 * math.cosh(M) * math.sinh(M) ** 2
    assert abs(w.sum() / vol - 1) < 1e-12


@pytest.mark.parametrize("C,nsp,q", [(-1, 3, 3), (0, 3, 3), (0, 2, 4)])
def test_polynomial_exactness_per_axis(C, nsp, q):
    """sum_g (w_g / J_g) p(mu,nu,phi) is exact for degree <= 2Q-1 per axis over the coordinate box."""
    spec = (6, 5, 4, q, nsp, 2.3, 0.25)
    info = O.grid_info(TRI, 1, 2, C, spec)
    x, y, z, w = O.grid_points(TRI, 1, 2, C, spec)
    mu, nu, phi = _local_coords(TRI, 1, 2, info, x, y, z)
    a = info["a"]
    J = a ** 3 * np.sinh(mu) * np.sin(nu) * (np.sinh(mu) ** 2 + np.sin(nu) ** 2)
    base = w / J
    Mx = info["mu"][-1]
    for (p1, p2, p3) in [(0, 0, 0), (2 * q - 1, 0, 0), (0, 2 * q - 1, 1), (1, 2, 2 * q - 1),
                         (2 * q - 1, 2 * q - 1, 2 * q - 1)]:
        num = np.sum(base * mu ** p1 * nu ** p2 * phi ** p3)
        exact = Mx ** (p1 + 1) / (p1 + 1) * PI ** (p2 + 1) / (p2 + 1) * (2 * PI) ** (p3 + 1) / (p3 + 1)
        assert abs(num / exact - 1) < 1e-9, (p1, p2, p3)


def test_third_centre_lies_on_moved_lines():
    spec = (12, 10, 8, 4, 3, 2.3, 0.25)
    for (A, B, C) in [(0, 1, 2), (1, 2, 0), (0, 2, 1)]:
        info = O.grid_info(TRI, A, B, C, spec)
        a = info["a"]
        dp = np.linalg.norm(TRI[C] - TRI[A])
        dm = np.linalg.norm(TRI[C] - TRI[B])
        muC = math.acosh((dp + dm) / (2 * a))
        nuC = math.acos((dm - dp) / (2 * a))
        assert info["moved_mu"] and info["moved_nu"] and info["split"]
        assert abs(info["mu"][info["istar"]] - muC) < 1e-14
        assert abs(info["nu"][info["jstar"]] - nuC) < 1e-14
        assert np.all(np.diff(info["mu"]) > 0) and np.all(np.diff(info["nu"]) > 0)
        d = TRI[C] - info["M"]
        assert d @ info["ex"] > 0 and abs(d @ info["ey"]) < 1e-14  # C at phi = 0
        # A at local +a on the axis
        assert np.allclose((TRI[A] - info["M"]) @ info["ez"], a, atol=1e-14)


def test_third_centre_beyond_grid_is_not_moved():
    xyz = np.array([[0, 0, 0.7], [0, 0, -0.7], [0, 0, 80.0]])
    info = O.grid_info(xyz, 0, 1, 2, (8, 8, 4, 4, 3, 2.3, 0.25))
    assert not info["moved_mu"] and not info["moved_nu"] and not info["split"]


def test_translation_and_swap_invariance():
    xyz = np.array([[0.1, -0.2, 0.3], [0.9, 0.5, -0.4]])
    basis = [[0, 2, 1, 1, 1.3], [1, 3, 2, -1, 0.9], [0, 1, 0, 0, 2.0]]
    aux = [[0, 2, 1, -1, 1.8], [1, 1, 0, 0, 2.5]]
    spec = Spec(6, 6, 4)
    j1 = MiniJob(xyz, [1, 3], basis, aux, spec)
    j2 = MiniJob(xyz + np.array([3.0, -1.0, 2.0]), [1, 3], basis, aux, spec)
    sw = [[1 - b[0]] + b[1:] for b in basis]
    swa = [[1 - b[0]] + b[1:] for b in aux]
    j3 = MiniJob(xyz[::-1].copy(), [3, 1], sw, swa, spec)
    r1, r2, r3 = (O.compute_full(j) for j in (j1, j2, j3))
    for key in ("S", "T", "V", "PQ", "abP"):
        assert np.max(np.abs(r1[key] - r2[key])) < 1e-12, key
        assert np.max(np.abs(r1[key] - r3[key])) < 1e-12, key


# ---------------------------------------------------------------------------------------------
# STO values (eq. 1) and real spherical harmonics
# ---------------------------------------------------------------------------------------------

def test_real_ylm_matches_scipy():
    rng = np.random.default_rng(1)
    v = rng.normal(size=(50, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    th = np.arccos(v[:, 2])
    ph = np.arctan2(v[:, 1], v[:, 0])
    for l in range(0, 7):
        for m in range(-l, l + 1):
            am = abs(m)
            Yc = special.sph_harm_y(l, am, th, ph)  # complex, Condon-Shortley phase
            if m == 0:
                ref = Yc.real
            elif m > 0:
                ref = math.sqrt(2) * (-1) ** am * Yc.real
            else:
                ref = math.sqrt(2) * (-1) ** am * Yc.imag
            got = O.eval_fn("ylm", [0, l + 1, l, m, 1.0], [0, 0, 0], v[:, 0], v[:, 1], v[:, 2])
            assert np.max(np.abs(got - ref)) < 1e-13, (l, m)


def test_unsold_theorem():
    rng = np.random.default_rng(2)
    v = rng.normal(size=(20, 3))
    for l in range(0, 7):
        s = np.zeros(20)
        for m in range(-l, l + 1):
            s += O.eval_fn("ylm", [0, l + 1, l, m, 1.0], [0, 0, 0], v[:, 0], v[:, 1], v[:, 2]) ** 2
        assert np.max(np.abs(s - (2 * l + 1) / (4 * PI))) < 1e-13


def test_sto_value_closed_form():
    # 2p_z: N r e^{-z r} sqrt(3/4pi) cos(theta) = N sqrt(3/4pi) z e^{-zeta r}
    zeta = 1.7
    N = (2 * zeta) ** 2.5 / math.sqrt(24)
    p = np.array([[0.3, -0.2, 0.5], [1.0, 1.0, -1.0]])
    got = O.eval_fn("chi", [0, 2, 1, 0, zeta], [0, 0, 0], p[:, 0], p[:, 1], p[:, 2])
    r = np.linalg.norm(p, axis=1)
    ref = N * math.sqrt(3 / (4 * PI)) * p[:, 2] * np.exp(-zeta * r)
    assert np.max(np.abs(got - ref)) < 1e-15


def test_kinetic_factor_by_finite_differences():
    rng = np.random.default_rng(3)
    h = 1e-3
    for (n, l, m, zeta) in [(1, 0, 0, 1.3), (3, 1, -1, 0.8), (4, 3, 2, 1.1), (5, 2, 0, 2.0)]:
        fn = [0, n, l, m, zeta]
        for _ in range(3):
            p = rng.normal(size=3)
            lap = 0.0
            for d in range(3):
                e = np.zeros(3)
                e[d] = h
                vals = [O.eval_fn("chi", fn, [0, 0, 0], *(p + k * e)[:, None]) [0] for k in (-2, -1, 0, 1, 2)]
                lap += (-vals[0] + 16 * vals[1] - 30 * vals[2] + 16 * vals[3] - vals[4]) / (12 * h * h)
            got = O.eval_fn("kin", fn, [0, 0, 0], *p[:, None])[0]
            assert abs(got - (-0.5 * lap)) < 1e-6 * (1 + abs(got))


# ---------------------------------------------------------------------------------------------
# Coulomb potential of an auxiliary STO (eqs. 15-16)
# ---------------------------------------------------------------------------------------------

@pytest.mark.parametrize("k", [1, 2, 3, 5, 8, 12])
def test_incomplete_gamma_matches_scipy(k):
    for x in [1e-6, 1e-3, 0.1, 0.7, 2.0, k + 0.5, k + 1.5, 10.0, 40.0]:
        lo = O.lower_gamma(k, x)
        up = O.upper_gamma(k, x)
        ref_lo = special.gamma(k) * special.gammainc(k, x)
        ref_up = special.gamma(k) * special.gammaincc(k, x)
        assert abs(lo - ref_lo) <= 1e-13 * abs(ref_lo) + 1e-300
        assert abs(up - ref_up) <= 1e-13 * abs(ref_up) + 1e-300


def test_potential_of_1s_closed_form():
    zeta = 1.9
    r = np.array([1e-4, 0.01, 0.3, 1.0, 4.0, 20.0])
    x = zeta * r
    # charge 8 sqrt(pi) zeta^-3/2 spread as a normalised exponential: V = q/r [1 - (1 + x/2) e^-x]
    # (evaluated in 50-digit arithmetic: the closed form cancels badly for small x)
    import mpmath as mp
    mp.mp.dps = 50
    ref = np.array([float(4 * mp.sqrt(mp.pi) * mp.mpf(zeta) ** -0.5
                          * (2 / mp.mpf(xx) - (2 / mp.mpf(xx) + 1) * mp.exp(-mp.mpf(xx)))) for xx in x])
    got = O.eval_fn("pot", [0, 1, 0, 0, zeta], [0, 0, 0], 0 * r, 0 * r, r)
    assert np.max(np.abs(got / ref - 1)) < 1e-13


@pytest.mark.parametrize("n,l,m,zeta", [(1, 0, 0, 0.8), (2, 1, 1, 1.5), (3, 2, -2, 2.4), (4, 3, 0, 1.1),
                                        (5, 4, -3, 3.0), (7, 6, 5, 2.2), (3, 0, 0, 0.9)])
def test_potential_by_radial_quadrature(n, l, m, zeta):
    """V(r) = 4pi/(2l+1) Y_lm [r^{-l-1} int_0^r R s^{l+2} ds + r^l int_r^inf R s^{1-l} ds]."""
    Nn = (2 * zeta) ** (n + 0.5) / math.sqrt(math.factorial(2 * n))
    R = lambda s: Nn * s ** (n - 1) * math.exp(-zeta * s)
    rng = np.random.default_rng(n * 10 + l)
    for _ in range(4):
        d = rng.normal(size=3)
        d *= rng.uniform(0.05, 8.0) / np.linalg.norm(d)
        r = np.linalg.norm(d)
        inner = integrate.quad(lambda s: R(s) * s ** (l + 2), 0, r, epsabs=0, epsrel=2e-14, limit=200)[0]
        outer = integrate.quad(lambda s: R(s) * s ** (1 - l), r, np.inf, epsabs=0, epsrel=2e-14, limit=200)[0]
        Y = O.eval_fn("ylm", [0, n, l, m, zeta], [0, 0, 0], *d[:, None])[0]
        ref = 4 * PI / (2 * l + 1) * Y * (r ** (-l - 1) * inner + r ** l * outer)
        got = O.eval_fn("pot", [0, n, l, m, zeta], [0, 0, 0], *d[:, None])[0]
        assert abs(got - ref) <= 1e-11 * abs(ref) + 1e-14


@pytest.mark.parametrize("n,l,m,zeta", [(1, 0, 0, 1.0), (2, 1, -1, 1.4), (3, 2, 1, 1.9), (5, 4, 2, 2.5)])
def test_potential_satisfies_poisson(n, l, m, zeta):
    """lap V_P = -4 pi chi_P, by a 4th-order finite-difference stencil."""
    fn = [0, n, l, m, zeta]
    rng = np.random.default_rng(7)
    h = 2e-2
    for _ in range(3):
        p = rng.normal(size=3) * 1.2
        lap = 0.0
        for d in range(3):
            e = np.zeros(3)
            e[d] = h
            vals = [O.eval_fn("pot", fn, [0, 0, 0], *(p + k * e)[:, None])[0] for k in (-2, -1, 0, 1, 2)]
            lap += (-vals[0] + 16 * vals[1] - 30 * vals[2] + 16 * vals[3] - vals[4]) / (12 * h * h)
        chi = O.eval_fn("chi", fn, [0, 0, 0], *p[:, None])[0]
        assert abs(lap + 4 * PI * chi) < 2e-6 * (1 + abs(4 * PI * chi))


def test_potential_far_field_multipole():
    for (n, l, m, zeta) in [(2, 1, 0, 1.5), (4, 3, -2, 2.0), (7, 6, 6, 3.0)]:
        d = np.array([0.3, -0.4, 0.8])
        d *= 90.0 / zeta / np.linalg.norm(d)
        r = np.linalg.norm(d)
        Nn = (2 * zeta) ** (n + 0.5) / math.sqrt(math.factorial(2 * n))
        Y = O.eval_fn("ylm", [0, n, l, m, zeta], [0, 0, 0], *d[:, None])[0]
        ref = 4 * PI / (2 * l + 1) * Nn * math.factorial(n + l + 1) * zeta ** (-(n + l + 2)) * Y / r ** (l + 1)
        got = O.eval_fn("pot", [0, n, l, m, zeta], [0, 0, 0], *d[:, None])[0]
        assert abs(got / ref - 1) < 1e-13


# ---------------------------------------------------------------------------------------------
# Integrals: closed forms, one-centre identities, independent 2-D quadrature
# ---------------------------------------------------------------------------------------------

H2 = np.array([[0.0, 0.0, 0.7], [0.0, 0.0, -0.7]])
BIG = Spec(40, 40, 16)


def test_1s1s_closed_forms():
    z = 1.2
    R = 1.4
    p = z * R
    j = MiniJob(H2, [1, 1], [[0, 1, 0, 0, z], [1, 1, 0, 0, z]], [[0, 1, 0, 0, 2.0]], BIG)
    r = O.compute_full(j, want=("S", "T", "V"))
    assert abs(r["S"][0, 1] - math.exp(-p) * (1 + p + p * p / 3)) < 1e-10
    assert abs(r["S"][0, 0] - 1) < 1e-10
    assert abs(r["T"][0, 1] - z * z / 2 * math.exp(-p) * (1 + p - p * p / 3)) < 1e-10
    assert abs(r["T"][0, 0] - z * z / 2) < 1e-10
    VAA = -z - (1 / R - (z + 1 / R) * math.exp(-2 * z * R))
    VAB = -2 * z * (1 + p) * math.exp(-p)
    assert abs(r["V"][0, 0] - VAA) < 1e-10
    assert abs(r["V"][0, 1] - VAB) < 1e-10


@pytest.mark.parametrize("n,l,zeta", [(1, 0, 1.5), (2, 1, 1.2), (3, 2, 2.0), (4, 3, 1.6), (3, 0, 1.4)])
def test_one_centre_identities(n, l, zeta):
    """<chi|chi> = 1, <1/r> = zeta/n, T_aa = zeta^2/2 [1 - 2(n(n-1)-l(l+1))/(n(2n-1))] (Z_B = 0)."""
    basis = [[0, n, l, m, zeta] for m in range(-l, l + 1)]
    j = MiniJob(H2, [1, 0], basis, [[0, 1, 0, 0, 2.0]], BIG)
    r = O.compute_full(j, want=("S", "T", "V"))
    nb = len(basis)
    # tolerances: the (40,40,16)-cell grid's own quadrature error for these exponents (~1e-10)
    assert np.max(np.abs(r["S"] - np.eye(nb))) < 2e-9
    T_ref = zeta ** 2 / 2 * (1 - 2 * (n * (n - 1) - l * (l + 1)) / (n * (2 * n - 1)))
    assert np.max(np.abs(r["T"] - T_ref * np.eye(nb))) < 1e-8
    assert np.max(np.abs(r["V"] + zeta / n * np.eye(nb))) < 2e-9


def test_one_centre_coulomb_of_1s():
    zeta = 2.5
    j = MiniJob(H2, [1, 1], [[0, 1, 0, 0, 1.0]], [[0, 1, 0, 0, zeta]], BIG)
    r = O.compute_full(j, want=("PQ",))
    assert abs(r["PQ"][0, 0] - 20 * PI / zeta ** 2) < 1e-9


def test_one_centre_metric_by_radial_integral():
    """(P|Q) for same (l,m) on one centre = int chi_Q(r) v_P(r) r^2 dr (angular parts orthonormal)."""
    P = (3, 2, 1, 2.2)
    Q = (3, 2, 1, 3.1)
    j = MiniJob(H2, [1, 1], [[0, 1, 0, 0, 1.0]], [[0, *P], [0, *Q]], BIG)
    r = O.compute_full(j, want=("PQ",))

    def radial(nlz, s, pot):
        n, l, _, z = nlz
        Nn = (2 * z) ** (n + 0.5) / math.sqrt(math.factorial(2 * n))
        if not pot:
            return Nn * s ** (n - 1) * math.exp(-z * s)
        x = z * s
        lo = special.gamma(n + l + 2) * special.gammainc(n + l + 2, x)
        up = special.gamma(n - l + 1) * special.gammaincc(n - l + 1, x)
        return 4 * PI / (2 * l + 1) * Nn * z ** (-(n + 1)) * (x ** (-l - 1) * lo + x ** l * up)

    ref = integrate.quad(lambda s: radial(Q, s, False) * radial(P, s, True) * s * s, 0, np.inf,
                         epsabs=0, epsrel=2e-14, limit=400)[0]
    assert abs(r["PQ"][0, 1] - ref) < 1e-9


AXIAL_CASES = [
    # (fa, fb) basis functions on A, B as (centre, n, l, m, zeta)
    (("A", 2, 1, 0, 1.5), ("B", 3, 2, 0, 0.9)),
    (("A", 2, 1, 1, 1.3), ("B", 3, 2, 1, 1.1)),
    (("A", 3, 2, -2, 1.7), ("B", 4, 2, -2, 1.2)),
    (("A", 1, 0, 0, 2.3), ("B", 4, 3, 0, 1.0)),
]


@pytest.mark.parametrize("fa,fb", AXIAL_CASES)
def test_two_centre_S_T_V_vs_2d_quadrature(fa, fb):
    a = 0.9
    xyz = np.array([[0, 0, a], [0, 0, -a]])
    Z = [1.3, 0.7]
    basis = [[0, *fa[1:]], [1, *fb[1:]]]
    j = MiniJob(xyz, Z, basis, [[0, 1, 0, 0, 2.0]], BIG)
    r = O.compute_full(j, want=("S", "T", "V"))
    A_, B_ = Fn(*fa), Fn(*fb)
    S_ref = ref_integral([A_, B_], a)
    T_ref = 0.5 * (ref_integral([A_, Fn(*fb, kind="kin")], a) + ref_integral([Fn(*fa, kind="kin"), B_], a))
    V_ref = -Z[0] * ref_integral([A_, B_, Fn("A", 1, 0, 0, 1.0, "rinv")], a) \
            - Z[1] * ref_integral([A_, B_, Fn("B", 1, 0, 0, 1.0, "rinv")], a)
    assert abs(r["S"][0, 1] - S_ref) < 1e-10
    assert abs(r["T"][0, 1] - T_ref) < 1e-9
    assert abs(r["V"][0, 1] - V_ref) < 1e-9


@pytest.mark.parametrize("fa,fb", AXIAL_CASES[:3])
def test_two_centre_abP_and_metric_vs_2d_quadrature(fa, fb):
    a = 0.9
    xyz = np.array([[0, 0, a], [0, 0, -a]])
    aux = [[0, 2, 1, 0, 2.6], [1, 3, 2, fb[3], 2.1], [1, 1, 0, 0, 3.0]]
    basis = [[0, *fa[1:]], [1, *fb[1:]]]
    j = MiniJob(xyz, [1, 1], basis, aux, BIG)
    r = O.compute_full(j, want=("PQ", "abP"))
    A_, B_ = Fn(*fa), Fn(*fb)
    for P, auxfn in enumerate(aux):
        cen = "A" if auxfn[0] == 0 else "B"
        ref = ref_integral([A_, B_, Fn(cen, *auxfn[1:], kind="pot")], a)
        assert abs(r["abP"][P, 0, 1] - ref) < 1e-9, P
        assert abs(r["abP"][P, 1, 0] - ref) < 1e-9, P
    # metric between aux 0 (A) and aux 1 (B): 1/2 (int V_0 chi_1 + int V_1 chi_0)
    f0 = Fn("A", *aux[0][1:])
    f1 = Fn("B", *aux[1][1:])
    ref = 0.5 * (ref_integral([Fn("A", *aux[0][1:], kind="pot"), f1], a)
                 + ref_integral([Fn("B", *aux[1][1:], kind="pot"), f0], a))
    assert abs(r["PQ"][0, 1] - ref) < 1e-9


def test_three_centre_grid_moved_singularity():
    """int rho_A / r_C and int rho_A V_{P@C} on G(A,B|C): closed form / independent 2-D quadrature
    with foci A and C.  Agreement is at the grid-error level, as the paper reports for 3-centre terms."""
    xyz = TRI
    zeta_a = 1.3
    fa = [0, 1, 0, 0, zeta_a]
    spec = (24, 24, 12, 4, 3, 2.3, 0.25)
    A, B, C = 0, 1, 2
    x, y, z, w = O.grid_points(xyz, A, B, C, spec)
    chi = O.eval_fn("chi", fa, xyz[A], x, y, z)
    rC = np.sqrt((x - xyz[C, 0]) ** 2 + (y - xyz[C, 1]) ** 2 + (z - xyz[C, 2]) ** 2)
    R = np.linalg.norm(xyz[A] - xyz[C])
    exact = 1 / R - (zeta_a + 1 / R) * math.exp(-2 * zeta_a * R)
    got = np.sum(w * chi * chi / rC)
    assert abs(got - exact) < 2e-6
    # without the third-centre refinement the error is larger (Section 2.2)
    x0, y0, z0, w0 = O.grid_points(xyz, A, B, -1, spec)
    chi0 = O.eval_fn("chi", fa, xyz[A], x0, y0, z0)
    rC0 = np.sqrt((x0 - xyz[C, 0]) ** 2 + (y0 - xyz[C, 1]) ** 2 + (z0 - xyz[C, 2]) ** 2)
    assert abs(np.sum(w0 * chi0 * chi0 / rC0) - exact) > 5 * abs(got - exact)
    # aux potential on C: axial about the A-C axis -> 2-D reference with foci A, C
    fP = [C, 2, 1, 0, 1.7]  # m = 0 about the global z axis is not axial about A-C: use s function
    fP = [C, 2, 0, 0, 1.7]
    vP = O.eval_fn("pot", fP, xyz[C], x, y, z)
    got = np.sum(w * chi * chi * vP)
    aC = R / 2
    ref = ref_integral([Fn("A", 1, 0, 0, zeta_a), Fn("A", 1, 0, 0, zeta_a), Fn("B", 2, 0, 0, 1.7, "pot")], aC)
    assert abs(got - ref) < 2e-6 * abs(ref)


def test_grid_convergence_rmse_decreases():
    """RMSE (eq. 13) of S, T and (ab|P) against a larger grid shrinks along a grid ladder."""
    xyz = np.array([[0, 0, 0.8], [0, 0, -0.8]])
    basis = [[0, 1, 0, 0, 1.4], [0, 2, 1, 1, 1.1], [1, 2, 1, 1, 0.9], [1, 3, 2, 0, 1.3]]
    aux = [[0, 1, 0, 0, 2.0], [1, 2, 1, 1, 1.8]]
    ref = O.compute_full(MiniJob(xyz, [1, 1], basis, aux, Spec(36, 36, 12)), want=("S", "T", "abP"))
    errs = []
    for s in [(8, 8, 4), (14, 14, 6), (22, 22, 8)]:
        r = O.compute_full(MiniJob(xyz, [1, 1], basis, aux, Spec(*s)), want=("S", "T", "abP"))
        errs.append([math.sqrt(np.mean((r[k] - ref[k]) ** 2)) for k in ("S", "T", "abP")])
    errs = np.array(errs)
    assert np.all(np.diff(errs, axis=0) < 0)
    assert np.all(errs[-1] < 1e-7)


# ---------------------------------------------------------------------------------------------
# Routing, symmetry, assembly and Cholesky
# ---------------------------------------------------------------------------------------------

def test_grid_list_counts():
    for n in (2, 3, 4, 5):
        xyz = np.array([[1.9 * k, 0.3 * k * k, 0.0] for k in range(n)])
        j = MiniJob(xyz, [1] * n, [[0, 1, 0, 0, 1.0]], [[0, 1, 0, 0, 1.0]], Spec(4, 4, 4))
        g = O.grid_list(j)
        assert len(g) == (1 if n == 2 else n * (n - 1) * (n - 2) // 2)
        assert len(set(g)) == len(g)


def test_outputs_symmetric_and_metric_positive_definite():
    xyz = TRI
    basis = [[0, 1, 0, 0, 3.0], [0, 2, 1, 1, 1.2], [1, 1, 0, 0, 1.1], [2, 2, 1, -1, 0.9], [2, 1, 0, 0, 1.0]]
    aux = [[0, 1, 0, 0, 4.0], [0, 2, 1, 0, 2.5], [1, 1, 0, 0, 2.0], [2, 1, 0, 0, 2.2]]
    r = O.compute_full(MiniJob(xyz, [8, 1, 1], basis, aux, Spec(8, 8, 6)))
    assert r["status"] == 0
    for k in ("S", "T", "V", "PQ"):
        assert np.allclose(r[k], r[k].T, atol=0, rtol=0)
    assert np.allclose(r["abP"], r["abP"].transpose(0, 2, 1), atol=0, rtol=0)
    assert np.all(np.linalg.eigvalsh(r["S"]) > 0)
    L = r["PQ_chol"]
    assert np.allclose(L, np.tril(L))
    assert np.max(np.abs(L @ L.T - r["PQ"])) < 1e-12 * np.max(np.abs(r["PQ"]))
    assert np.max(np.abs(L - np.linalg.cholesky(r["PQ"]))) < 1e-12 * np.max(np.abs(L))


def test_cholesky_matches_numpy_and_flags_non_pd():
    rng = np.random.default_rng(5)
    X = rng.normal(size=(30, 30))
    A = X @ X.T + 30 * np.eye(30)
    L, rc = O.cholesky(A)
    assert rc == 0 and np.max(np.abs(L - np.linalg.cholesky(A))) < 1e-12
    B = A.copy()
    B[3, 3] = -1.0
    _, rc = O.cholesky(B)
    assert rc == -5


def test_duplicated_aux_makes_metric_not_pd():
    aux = [[0, 1, 0, 0, 2.0], [0, 1, 0, 0, 2.0]]
    r = O.compute_full(MiniJob(H2, [1, 1], [[0, 1, 0, 0, 1.0]], aux, Spec(6, 6, 4)))
    assert r["status"] == -5


def test_contraction_equals_einsum_on_evaluated_columns():
    """Diatomic: S, V and (ab|P) from the oracle equal numpy einsum over the grid's columns."""
    xyz = np.array([[0.2, 0.1, 0.6], [-0.3, 0.4, -0.5]])
    Z = [1.0, 2.0]
    basis = [[0, 1, 0, 0, 1.5], [0, 2, 1, -1, 1.1], [1, 2, 1, 0, 0.8], [1, 3, 2, 2, 1.2]]
    aux = [[0, 1, 0, 0, 2.4], [1, 2, 1, 1, 1.9], [1, 3, 2, -1, 2.2]]
    spec = Spec(6, 5, 4)
    r = O.compute_full(MiniJob(xyz, Z, basis, aux, spec))
    x, y, z, w = O.grid_points(xyz, 0, 1, -1, spec.as_tuple())
    Phi = np.array([O.eval_fn("chi", f, xyz[int(f[0])], x, y, z) for f in basis])
    Vp = np.array([O.eval_fn("pot", f, xyz[int(f[0])], x, y, z) for f in aux])
    pot = -sum(Z[c] / np.sqrt((x - xyz[c, 0]) ** 2 + (y - xyz[c, 1]) ** 2 + (z - xyz[c, 2]) ** 2)
               for c in range(2))
    assert np.max(np.abs(r["S"] - np.einsum("ag,bg,g->ab", Phi, Phi, w))) < 1e-13
    assert np.max(np.abs(r["V"] - np.einsum("ag,bg,g->ab", Phi, Phi, w * pot))) < 1e-12
    assert np.max(np.abs(r["abP"] - np.einsum("ag,bg,pg,g->pab", Phi, Phi, Vp, w))) < 1e-12


def test_pair_point_count():
    j = MiniJob(H2, [1, 1], [[0, 1, 0, 0, 1.0], [1, 1, 0, 0, 1.0]], [[0, 1, 0, 0, 1.0]], Spec(4, 4, 4))
    np_ = 4 * 4 * 4 * 64
    _, wpp = O.compute_elements(j, [O.S, O.ABP], [0, 0], [1, 1], [0, 0])
    assert wpp == 2 * np_


def test_paper_grid_sizes_golden():
    """Q points per axis per cell (reading of Section 3): the paper's Table 1 PS grid must be about
    the ~700,000 points it was chosen to match (the BP grid of 5810 x 120 points per atom)."""
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "paper_grids.json")
    gold = json.load(open(path))
    bp = gold["bp_grid_points_per_atom"]
    for g in gold["grids"]:
        spec = (g["n_mu"], g["n_nu"], g["n_phi"], g["q"], g["n_sp"], 2.3, 0.25)
        info = O.grid_info(TRI, 1, 2, 0, spec)
        expect = (g["n_mu"] * g["n_nu"] * g["n_phi"] + 8 * (g["n_sp"] ** 3 - 1)) * g["q"] ** 3
        assert info["n_points"] == expect
        if "approx_points" in g:
            assert abs(info["n_points"] / g["approx_points"] - 1) < g["rel_tol"]
            assert abs(info["n_points"] / (bp["angular"] * bp["radial"]) - 1) < g["rel_tol"]
