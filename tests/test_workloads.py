"""The seeded synthetic workloads have the sizes the benchmark configurations state (no GPU)."""
import numpy as np

from paper_2510_15204_amd import workloads as W


def _count(arr, atom):
    return int(np.sum(arr[:, 0] == atom))


def test_diatomic_small():
    j = W.diatomic_small()
    assert j.n_atoms == 2 and j.n_bf == 10 and j.n_aux == 24
    assert np.allclose(np.linalg.norm(j.xyz[0] - j.xyz[1]), 1.4)
    assert sorted(set(j.basis[:, 2].astype(int))) == [0, 1]
    assert np.all((j.basis[:, 4] >= 0.5) & (j.basis[:, 4] <= 3.0))
    assert np.all((j.aux[:, 4] >= 0.8) & (j.aux[:, 4] <= 6.0)) and j.aux[:, 2].max() == 2
    assert (j.grid.n_mu * 4, j.grid.n_nu * 4, j.grid.n_phi * 4) == (40, 40, 16)


def test_triatomic_qz():
    j = W.triatomic_qz()
    assert [_count(j.basis, a) for a in range(3)] == [55, 30, 30]
    assert [_count(j.aux, a) for a in range(3)] == [165, 90, 90]
    assert j.basis[:, 2].max() == 3 and j.aux[:, 2].max() == 4 and j.basis[:, 1].max() <= 4
    assert (j.grid.n_mu, j.grid.n_nu, j.grid.n_phi, j.grid.q, j.grid.n_sp) == (24, 24, 12, 4, 3)
    d = [np.linalg.norm(j.xyz[k] - j.xyz[0]) for k in (1, 2)]
    assert np.allclose(d, 1.8)
    v1, v2 = j.xyz[1] - j.xyz[0], j.xyz[2] - j.xyz[0]
    assert abs(np.degrees(np.arccos(v1 @ v2 / 1.8 ** 2)) - 104.0) < 1e-9


def test_triatomic_5z():
    j = W.triatomic_5z()
    assert [_count(j.basis, a) for a in range(3)] == [91, 55, 55]
    assert [_count(j.aux, a) for a in range(3)] == [273, 165, 165]
    assert j.basis[:, 2].max() == 4 and j.aux[:, 2].max() == 6


def test_hydrocarbon9():
    j = W.hydrocarbon9()
    Z = j.Z.astype(int)
    assert list(Z) == [6, 6, 6, 1, 1, 1, 1, 1, 1]
    assert j.n_bf == 3 * 55 + 6 * 30 and j.n_aux == 3 * 165 + 6 * 90
    assert len(j.pair_grids) == 36
    for s in j.pair_grids.values():
        for n in (s.n_mu, s.n_nu, s.n_phi):
            assert 16 <= n <= 32
    cc = np.linalg.norm(j.xyz[0] - j.xyz[1])
    assert abs(cc - 2.9) < 0.2


def test_seeded_and_reproducible():
    a, b = W.triatomic_qz(), W.triatomic_qz()
    assert np.array_equal(a.basis, b.basis) and np.array_equal(a.aux, b.aux)


def test_serving_stream_shapes():
    s = W.serving_stream(n_requests=30)
    t = [x[0] for x in s]
    assert all(np.diff(t) > 0)
    for _, j in s:
        assert 2 <= j.n_atoms <= 12
        assert set(j.Z.astype(int)) <= {1, 6, 7, 8}
        d = np.linalg.norm(j.xyz[:, None] - j.xyz[None], axis=-1) + 10 * np.eye(j.n_atoms)
        assert d.min() >= 1.8 - 1e-12
