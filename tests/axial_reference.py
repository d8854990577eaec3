"""Independent reference integrals for centres on the z axis (test helper, no oracle code).

For centres A = (0,0,+a) and B = (0,0,-a), every function of the form R(r) Y_lm(theta, phi) about A or
B separates into F(xi, eta) * trig(|m| phi) in elliptic coordinates xi = cosh(mu), eta = cos(nu),
because the azimuth about either centre is the same phi.  The same holds for a function about any
other point (0,0,z_c) of the axis; such a centre sits on the boundary of the (mu, eta) rectangle
(at eta = +-1 beyond the foci, at mu = 0 between them), where its cusp or 1/r singularity is handled
by a break point of the nested adaptive quadrature.  An integral over all space of a product of
such functions is therefore (integral over phi of the trig factors) times a 2-D integral over
(xi, eta) with volume element a^3 (xi^2 - eta^2).  Here the 2-D integral is done by adaptive
scipy quadrature in (mu, eta) and the phi integral by an exact trapezoid sum, which shares nothing
with the prolate-spheroidal cell/Gauss-Legendre scheme under test.

Functions come from library routines: scipy.special.lpmv (associated Legendre, with the
Condon-Shortley phase removed) and scipy.special.gammainc/gammaincc (regularised incomplete gamma).
"""
import math

import numpy as np
from scipy import integrate, special


def ylm_norm(l, m):
    am = abs(m)
    n = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - am) / math.factorial(l + am))
    return n if m == 0 else math.sqrt(2.0) * n


def legendre_no_cs(l, m, x):
    am = abs(m)
    return ((-1) ** am) * special.lpmv(am, l, x)


def sto_norm(n, zeta):
    return (2 * zeta) ** (n + 0.5) / math.sqrt(math.factorial(2 * n))


def radial_chi(n, zeta, r):
    return sto_norm(n, zeta) * r ** (n - 1) * np.exp(-zeta * r)


def radial_pot(n, l, zeta, r):
    """Radial factor of the Coulomb potential of N r^(n-1) e^(-zeta r) Y_lm (times Y_lm gives V)."""
    x = zeta * r
    k1, k2 = n + l + 2, n - l + 1
    lower = special.gamma(k1) * special.gammainc(k1, x)
    upper = special.gamma(k2) * special.gammaincc(k2, x)
    return (4 * math.pi / (2 * l + 1)) * sto_norm(n, zeta) * zeta ** (-(n + 1)) * (
        x ** (-l - 1) * lower + x ** l * upper)


def radial_kin(n, l, zeta, r):
    """-1/2 lap of the radial-angular function divided by the angular part."""
    f = zeta * zeta - 2 * zeta * n / r + (n * (n - 1) - l * (l + 1)) / (r * r)
    return -0.5 * f * radial_chi(n, zeta, r)


class Fn:
    """One factor of an integrand: a function about centre 'A' (z=+a), 'B' (z=-a), or about the
    on-axis point (0, 0, centre) when centre is a number."""

    def __init__(self, centre, n, l, m, zeta, kind="chi"):
        self.centre, self.n, self.l, self.m, self.zeta, self.kind = centre, n, l, m, zeta, kind

    def zc(self, a):
        if self.centre == "A":
            return a
        if self.centre == "B":
            return -a
        return float(self.centre)

    def f2d(self, a, xi, eta):
        rho = a * math.sqrt(max((xi * xi - 1) * (1 - eta * eta), 0.0))
        z = a * xi * eta - self.zc(a)
        r = math.hypot(rho, z)
        ct = z / r
        ang = ylm_norm(self.l, self.m) * legendre_no_cs(self.l, self.m, ct)
        if self.kind == "chi":
            rad = radial_chi(self.n, self.zeta, r)
        elif self.kind == "pot":
            rad = radial_pot(self.n, self.l, self.zeta, r)
        elif self.kind == "kin":
            rad = radial_kin(self.n, self.l, self.zeta, r)
        elif self.kind == "rinv":
            return 1.0 / r
        else:
            raise ValueError(self.kind)
        return rad * ang

    def trig(self, phi):
        if self.kind == "rinv" or self.m == 0:
            return np.ones_like(phi)
        am = abs(self.m)
        return np.cos(am * phi) if self.m > 0 else np.sin(am * phi)


def phi_integral(fns, n=64):
    phi = 2 * math.pi * np.arange(n) / n
    prod = np.ones(n)
    for f in fns:
        prod = prod * f.trig(phi)
    return 2 * math.pi * prod.mean()


def integral(fns, a, mu_max=9.0, eps=1e-13):
    """Integral over all space of the product of the factors (foci at z = +a and -a)."""
    pf = phi_integral(fns)
    if abs(pf) < 1e-14:
        return 0.0
    mu_breaks, eta_breaks = set(), set()
    for f in fns:
        zc = f.zc(a)
        if abs(abs(zc) - a) <= 1e-14 * a:
            continue
        if abs(zc) > a:
            mu_breaks.add(math.acosh(abs(zc) / a))
        else:
            eta_breaks.add(zc / a)
    if mu_breaks or eta_breaks:
        return pf * _nested(fns, a, mu_max, sorted(mu_breaks), sorted(eta_breaks), eps)

    def g(eta, mu):
        xi = math.cosh(mu)
        v = a ** 3 * (xi * xi - eta * eta) * math.sinh(mu)
        for f in fns:
            v *= f.f2d(a, xi, eta)
        return v

    val, err = integrate.dblquad(g, 0.0, mu_max, -1.0, 1.0, epsabs=eps, epsrel=1e-12)
    return pf * val


def _nested(fns, a, mu_max, mu_breaks, eta_breaks, eps):
    """Nested adaptive quadrature in (mu, eta) with break points at the off-focus centres."""

    def inner(mu):
        xi = math.cosh(mu)
        sh = math.sinh(mu)

        def g(eta):
            v = a ** 3 * (xi * xi - eta * eta) * sh
            for f in fns:
                v *= f.f2d(a, xi, eta)
            return v

        return integrate.quad(g, -1.0, 1.0, points=eta_breaks or None, epsabs=0.1 * eps, epsrel=1e-12,
                              limit=400)[0]

    return integrate.quad(inner, 0.0, mu_max, points=mu_breaks or None, epsabs=eps, epsrel=1e-12,
                          limit=400)[0]
