"""GPU: RI assembly (eq. 14) through the C ABI against the oracle's forward substitution and product."""
import math
import sys

import numpy as np
import pytest

import oracle as O
from conftest import MiniJob, Spec
from paper_2510_15204_amd import psint
from paper_2510_15204_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = psint.Context(0)
    yield c
    c.close()


def _pd_job(n_max_basis=4):
    """Triatomic with a triple-zeta-sized basis (43 functions, 946 pairs: 14 full 64-pair tiles and a
    ragged one) and 75 well-separated auxiliary functions ((P|Q) condition number about 2e4; 75 = two
    32-row blocks plus a ragged 11)."""
    rng = W.rng_for(1)
    Z = np.array([8.0, 1.0, 1.0])
    basis, _ = W.build_basis(rng, Z.astype(int), "TZ", "auxTZ", n_max=n_max_basis)
    aux = []
    for a in range(3):
        aux += [[a, 1, 0, 0, z] for z in (9.0, 3.0, 1.0)]
        aux += [[a, 2, 1, m, z] for z in (4.0, 1.5) for m in (-1, 0, 1)]
        aux += [[a, 3, 2, m, 2.5] for m in range(-2, 3)]
        aux += [[a, 4, 3, m, 2.2] for m in range(-3, 4)]
    aux += [[0, 3, 2, m, 1.2] for m in range(-2, 3)] + [[1, 4, 3, m, 1.4] for m in range(-3, 4)]
    return MiniJob(W.triatomic_geometry(), Z, basis, aux, Spec(10, 10, 8, 4, 3))


@pytest.fixture(scope="module")
def oracle_inputs():
    job = _pd_job()
    ref = O.compute_full(job)
    assert ref["status"] == 0
    B, eri = O.ri_assemble(ref["abP"], ref["PQ_chol"])
    return job, ref, B, eri


def test_ri_matches_oracle_on_oracle_inputs(ctx, oracle_inputs):
    """Same (ab|P) and L on both sides (the oracle's): B and eri agree to rounding (relative 1e-11;
    the solve amplifies rounding by at most the factor's condition number, about 1e2 here)."""
    job, ref, Bo, erio = oracle_inputs
    B, eri, ms = ctx.ri_assemble(ref["abP"], ref["PQ_chol"])
    nb = len(job.basis)
    assert B.shape == (75, nb * (nb + 1) // 2) and eri.shape == (B.shape[1], B.shape[1])
    eb = np.max(np.abs(B - Bo)) / np.max(np.abs(Bo))
    ee = np.max(np.abs(eri - erio)) / np.max(np.abs(erio))
    _say(f"ri: B rel err {eb:.2e}, eri rel err {ee:.2e}, {ms:.3f} ms")
    assert eb < 1e-11 and ee < 1e-11
    assert np.array_equal(eri, eri.T)


def test_ri_device_path_equals_host_path(ctx, oracle_inputs):
    import torch
    job, ref, _, _ = oracle_inputs
    Bh, eh, _ = ctx.ri_assemble(ref["abP"], ref["PQ_chol"])
    dev = torch.device("cuda:0")
    Bd, ed, _ = ctx.ri_assemble(torch.from_numpy(ref["abP"]).to(dev), torch.from_numpy(ref["PQ_chol"]).to(dev))
    assert np.array_equal(Bd.cpu().numpy(), Bh) and np.array_equal(ed.cpu().numpy(), eh)
    # only one of the outputs
    _, e2, _ = ctx.ri_assemble(ref["abP"], ref["PQ_chol"], want_B=False)
    assert np.array_equal(e2, eh)
    B3, e3, _ = ctx.ri_assemble(ref["abP"], ref["PQ_chol"], want_eri=False)
    assert e3 is None and np.array_equal(B3, Bh)


def test_ri_scratch_shares_the_context_budget(ctx, oracle_inputs):
    """RI scratch comes from the context's device memory.  With a budget that holds the job's arena
    or the scratch of an RI call but not both, the RI call takes back the arena ps_compute keeps for a
    repeat of its last job (so the repeat is planned again rather than replayed); the job's results
    match the oracle, and RI equals RI on a context without the limit."""
    job, ref, _, _ = oracle_inputs
    gran = 2 << 20  # the device pool's allocation granularity
    up = lambda b: (b + gran - 1) // gran * gran  # noqa: E731
    # RI inputs of their own size (88 basis functions, 3916 pairs, 75 auxiliaries): scratch ~130 MB
    rng = np.random.default_rng(5)
    nb, na = 88, len(job.aux)
    abP = rng.standard_normal((na, nb, nb))
    L = np.tril(rng.uniform(0.1, 0.2, (na, na)), -1) + np.diag(rng.uniform(1.0, 2.0, na))
    npair = nb * (nb + 1) // 2
    ntile = (npair + 127) // 128
    ri_bytes = 0
    for b in (na * nb * nb * 8, na * na * 8, na * npair * 8, na * npair * 8, na * na * 8,
              ntile * (ntile + 1) // 2 * 8, npair * npair * 8):  # host staging, X, B, G, tiles, eri
        ri_bytes += (b + 255) // 256 * 256
    ri_bytes = up(ri_bytes)
    arena = up(ctx.plan_work(job)["device_bytes"])
    budget = up(ri_bytes + arena // 2)
    c = psint.Context(0, budget_bytes=budget)
    try:
        a2 = up(c.plan_work(job)["device_bytes"])
        _say(f"arena {a2 / 1e6:.1f} MB, RI scratch {ri_bytes / 1e6:.1f} MB, budget {budget / 1e6:.1f} MB")
        assert a2 + ri_bytes > budget >= max(a2, ri_bytes)
        out, _, rc = c.compute(job)
        assert rc == psint.PS_OK
        B1, e1, _ = c.ri_assemble(abP, L)
        out2, st2, _ = c.compute(job)
        B2, e2, _ = c.ri_assemble(abP, L)
    finally:
        c.close()
    assert st2["graph_replay"] == 0
    for k in ("S", "T", "V", "PQ", "abP"):
        assert np.max(np.abs(out[k] - ref[k])) < 1e-10
    for k in ("S", "T", "V", "PQ", "PQ_chol", "abP"):
        assert np.array_equal(out2[k], out[k])
    B0, e0, _ = ctx.ri_assemble(abP, L)
    for x, y in ((B1, B0), (e1, e0), (B2, B0), (e2, e0)):
        assert np.array_equal(x, y)


def test_ri_between_repeats_keeps_the_replay(oracle_inputs):
    """With memory to spare, an RI call between two runs of the same job leaves the job's arena,
    plan and captured graphs alone: the third run is a graph replay and all results are unchanged."""
    job, ref, _, _ = oracle_inputs
    c = psint.Context(0)
    try:
        out1, st1, _ = c.compute(job)
        out2, st2, _ = c.compute(job)
        B, eri, _ = c.ri_assemble(out2["abP"], out2["PQ_chol"])
        out3, st3, _ = c.compute(job)
        B2, eri2, _ = c.ri_assemble(out3["abP"], out3["PQ_chol"])
    finally:
        c.close()
    assert st1["graph_replay"] == 0 and st2["graph_replay"] == 1 and st3["graph_replay"] == 1
    for k in ("S", "T", "V", "PQ", "PQ_chol", "abP"):
        assert np.array_equal(out2[k], out1[k]) and np.array_equal(out3[k], out1[k])
    assert np.array_equal(B2, B) and np.array_equal(eri2, eri)
    assert np.max(np.abs(out1["abP"] - ref["abP"])) < 1e-10


def test_ri_end_to_end_closed_forms(ctx):
    """GPU quadrature + GPU Cholesky + GPU RI on 1s(zeta = 1) atoms with 1s(2) auxiliaries: the
    densities lie in the auxiliary span, so (aa|aa) = 5/8 and (aa|bb) = J(R) exactly (up to the grid)."""
    R = 1.4
    job = MiniJob([[0.0, 0.0, 0.0], [0.0, 0.0, R]], [1.0, 1.0], [[0, 1, 0, 0, 1.0], [1, 1, 0, 0, 1.0]],
                  [[0, 1, 0, 0, 2.0], [1, 1, 0, 0, 2.0]], Spec(30, 30, 10, 4, 3))
    out, _, rc = ctx.compute(job)
    assert rc == psint.PS_OK
    _, eri, _ = ctx.ri_assemble(out["abP"], out["PQ_chol"])
    J = 1 / R - math.exp(-2 * R) * (1 / R + 11 / 8 + 3 * R / 4 + R * R / 6)
    aa, bb = O.pair_index(0, 0), O.pair_index(1, 1)
    _say(f"(aa|aa) - 5/8 = {eri[aa, aa] - 0.625:.2e}, (aa|bb) - J = {eri[aa, bb] - J:.2e}")
    assert abs(eri[aa, aa] - 0.625) < 1e-8 and abs(eri[bb, bb] - 0.625) < 1e-8
    assert abs(eri[aa, bb] - J) < 1e-8


@pytest.mark.parametrize("nb,na", [(1, 1), (2, 33), (11, 64), (12, 65), (20, 97), (5, 1024), (5, 1025), (65, 33),
                                   (130, 40)])
def test_ri_edge_sizes(ctx, nb, na):
    """Single pair / single auxiliary function, one-past-a-block sizes, several 16-pair strips, the
    largest n_aux the one-launch substitution holds in LDS (1024) and the first beyond it (one launch
    per block step), and n_bf 65 and 130, whose rows a >= 64 take the gather's second lap of 64 lanes
    (one wave per row of (ab|P)): random SPD factor and random (ab|P) symmetric in a, b, compared
    with the oracle."""
    rng = np.random.default_rng(nb * 100 + na)
    M = rng.normal(size=(na, na))
    L = np.linalg.cholesky(M @ M.T + na * np.eye(na))
    abP = rng.normal(size=(na, nb, nb))
    abP = 0.5 * (abP + abP.transpose(0, 2, 1))
    Bo, eo = O.ri_assemble(abP, L)
    B, e, _ = ctx.ri_assemble(abP, np.tril(L) + np.triu(rng.normal(size=(na, na)), 1))  # upper part ignored
    assert np.max(np.abs(B - Bo)) <= 1e-12 * max(1.0, np.max(np.abs(Bo)))
    assert np.max(np.abs(e - eo)) <= 1e-12 * max(1.0, np.max(np.abs(eo)))


def test_ri_rejects_bad_arguments(ctx):
    with pytest.raises(psint.PsError) as e:
        ctx.ri_assemble(np.zeros((0, 3, 3)), np.zeros((0, 0)))
    assert e.value.status == psint.PS_E_INVALID
