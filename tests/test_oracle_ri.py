"""Pins of the oracle's RI assembly (eq. 14) against closed forms (no GPU).

When the auxiliary set contains the product density of a basis pair, the Coulomb-metric fit of that
density is exact, so the RI integral equals the exact Coulomb integral.  Products of two 1s Slater
functions on one centre are 1s-type densities e^{-(za+zb) r}, whose Coulomb integrals have closed
forms; so do two 1s(zeta=1) densities on different centres.
"""
import math

import numpy as np
import pytest
from scipy import linalg

import oracle as O
from conftest import MiniJob, Spec


def test_forward_substitution_matches_lapack():
    rng = np.random.default_rng(3)
    n, m = 37, 11
    L = np.tril(rng.normal(size=(n, n))) + n * np.eye(n)
    A = rng.normal(size=(n, m))
    X = O.forward_substitution(L, A)
    assert np.max(np.abs(X - linalg.solve_triangular(L, A, lower=True))) < 1e-13


def test_pair_index_is_a_bijection():
    nb = 9
    seen = sorted(O.pair_index(a, b) for a in range(nb) for b in range(a + 1))
    assert seen == list(range(nb * (nb + 1) // 2))
    assert all(O.pair_index(a, b) == O.pair_index(b, a) for a in range(nb) for b in range(nb))


def _j_same_centre(p, q):
    """Coulomb energy of two normalised densities p^3/(8 pi) e^{-p r} and q^3/(8 pi) e^{-q r} on one
    centre: the potential of the second is 1/r - e^{-q r} (1/r + q/2)."""
    return p / 2 - p ** 3 / (2 * (p + q) ** 2) - p ** 3 * q / (2 * (p + q) ** 3)


def _j_two_centre(R):
    """Coulomb energy of two 1s(zeta = 1) densities e^{-2r}/pi a distance R apart."""
    return 1 / R - math.exp(-2 * R) * (1 / R + 11 / 8 + 3 * R / 4 + R * R / 6)


def test_self_repulsion_of_1s_density():
    """(1s1s|1s1s) for zeta = 1 is 5/8 (J(2, 2) of the formula above, a textbook value)."""
    assert abs(_j_same_centre(2.0, 2.0) - 0.625) < 1e-15
    assert abs(_j_same_centre(2.0, 3.0) - _j_same_centre(3.0, 2.0)) < 1e-15


def test_ri_exact_for_one_centre_1s_products():
    """Basis {1s(z1), 1s(z2)} on atom 0; auxiliary set = their three product densities there (plus a
    function on atom 1).  Every (ab|cd) equals S_ab S_cd J(za + zb, zc + zd)."""
    z = [1.0, 1.5]
    xyz = [[0.0, 0.0, 0.0], [0.0, 0.0, 1.4]]
    basis = [[0, 1, 0, 0, z[0]], [0, 1, 0, 0, z[1]]]
    aux = [[0, 1, 0, 0, 2 * z[0]], [0, 1, 0, 0, z[0] + z[1]], [0, 1, 0, 0, 2 * z[1]], [1, 1, 0, 0, 2.0]]
    job = MiniJob(xyz, [1.0, 1.0], basis, aux, Spec(30, 30, 10, 4, 3))
    ref = O.compute_full(job)
    assert ref["status"] == 0
    B, eri = O.ri_assemble(ref["abP"], ref["PQ_chol"])
    assert B.shape == (4, 3) and eri.shape == (3, 3)
    pairs = [(a, b) for a in range(2) for b in range(a + 1)]
    for (a, b) in pairs:
        for (c, d) in pairs:
            pab, pcd = z[a] + z[b], z[c] + z[d]
            sab = (2 * math.sqrt(z[a] * z[b]) / pab) ** 3
            scd = (2 * math.sqrt(z[c] * z[d]) / pcd) ** 3
            exact = sab * scd * _j_same_centre(pab, pcd)
            got = eri[O.pair_index(a, b), O.pair_index(c, d)]
            assert abs(got - exact) < 1e-8, ((a, b), (c, d), got, exact)


@pytest.mark.parametrize("R", [1.4, 2.5])
def test_ri_exact_for_two_centre_1s_densities(R):
    """1s(zeta = 1) on each of two atoms, auxiliary 1s(2) on each: (aa|aa) = 5/8 and (aa|bb) = J(R)."""
    xyz = [[0.0, 0.0, 0.0], [0.0, 0.0, R]]
    basis = [[0, 1, 0, 0, 1.0], [1, 1, 0, 0, 1.0]]
    aux = [[0, 1, 0, 0, 2.0], [1, 1, 0, 0, 2.0]]
    job = MiniJob(xyz, [1.0, 1.0], basis, aux, Spec(30, 30, 10, 4, 3))
    ref = O.compute_full(job)
    B, eri = O.ri_assemble(ref["abP"], ref["PQ_chol"])
    aa, bb = O.pair_index(0, 0), O.pair_index(1, 1)
    assert abs(eri[aa, aa] - 0.625) < 1e-8
    assert abs(eri[bb, bb] - 0.625) < 1e-8
    assert abs(eri[aa, bb] - _j_two_centre(R)) < 1e-8
    assert np.allclose(eri, eri.T, rtol=0, atol=1e-15)
