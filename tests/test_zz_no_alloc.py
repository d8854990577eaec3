"""GPU: the allocation-free RI entry point (ps_ri_assemble_noalloc) against ps_ri_assemble.

Both run the same kernels in the same order, so on the same inputs their outputs must be identical
bit for bit.  Two calls in a row, the second smaller, check that a call never reads what the previous
one left in the shared static scratch; a size beyond the scratch is rejected on the host."""
import sys

import numpy as np
import pytest

from paper_2510_15204_amd import psint

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _inputs(nb, na, seed):
    """Random (ab|P), symmetric in a and b, and a well-conditioned lower factor."""
    rng = np.random.default_rng(seed)
    abP = rng.normal(size=(na, nb, nb))
    abP = 0.5 * (abP + abP.transpose(0, 2, 1))
    L = np.tril(rng.normal(size=(na, na)) * 0.1) + np.diag(1.0 + rng.uniform(size=na))
    return abP, L


def _noalloc(ctx, abP, L, want_B):
    import torch
    dev = torch.device("cuda:0")
    na, nb = abP.shape[0], abP.shape[1]
    npair = nb * (nb + 1) // 2
    a, l = torch.from_numpy(abP).to(dev), torch.from_numpy(L).to(dev)
    B = torch.full((na, npair), np.nan, dtype=torch.float64, device=dev) if want_B else None
    eri = torch.full((npair, npair), np.nan, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    ctx.ri_assemble_noalloc(a, l, B=B, eri=eri)
    torch.cuda.synchronize()
    return (B.cpu().numpy() if want_B else None), eri.cpu().numpy()


@pytest.mark.parametrize("sizes", [((60, 130), (20, 40)), ((30, 1100), (12, 33))])
def test_noalloc_matches_ri_assemble_on_two_calls(sizes):
    """(n_bf, n_aux) pairs: the first runs the one-launch substitution (130 <= 1024 auxiliary
    functions) or the per-step one (1100), the second is smaller; each output equals ps_ri_assemble's."""
    ctx = psint.Context(0)
    try:
        for k, (nb, na) in enumerate(sizes):
            abP, L = _inputs(nb, na, 100 + k)
            _say(f"no-alloc RI: n_bf={nb} n_aux={na}")
            Bref, eref, _ = ctx.ri_assemble(abP, L)
            for want_B in (True, False):
                B, eri = _noalloc(ctx, abP, L, want_B)
                assert np.array_equal(eri, eref), (nb, na, want_B)
                if want_B:
                    assert np.array_equal(B, Bref), (nb, na)
    finally:
        ctx.close()


def test_noalloc_rejects_sizes_beyond_its_scratch():
    import torch
    ctx = psint.Context(0)
    try:
        nb, na = 200, 500  # gathered rows alone: 500 x 20100 doubles = 80 MB > 64 MiB
        dev = torch.device("cuda:0")
        abP = torch.zeros((na, nb, nb), dtype=torch.float64, device=dev)
        L = torch.eye(na, dtype=torch.float64, device=dev)
        eri = torch.empty((nb * (nb + 1) // 2,) * 2, dtype=torch.float64, device=dev)
        with pytest.raises(psint.PsError) as e:
            ctx.ri_assemble_noalloc(abP, L, eri=eri)
        assert e.value.status == psint.PS_E_NOMEM and "static scratch" in str(e.value)
    finally:
        ctx.close()
