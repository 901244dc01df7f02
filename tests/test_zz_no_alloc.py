"""The allocation-free contraction entry point (mitnc_contract_noalloc)
against mitnc_contract with a caller-provided work buffer.

Both run the same kernels with the same K split, so the outputs must agree
bit for bit; both are also held to the Eq. (3) bound against the FP64
oracle.  Two calls in a row, the second on a smaller problem, check that the
fixed scratch keeps no state a later call depends on.
"""
import numpy as np
import pytest

import synth
from helpers import gamma, ref_contract, require_gpu

pytestmark = pytest.mark.gpu

SPLITK, TILE = 4, 2


def _operands(mb, nb, kb, seed):
    rng = np.random.default_rng(seed)
    M = [1000 + i for i in range(mb)]
    N = [2000 + i for i in range(nb)]
    K = [3000 + i for i in range(kb)]
    la = [int(x) for x in rng.permutation(M + K)]
    lb = [int(x) for x in rng.permutation(K + N)]
    lc = [int(x) for x in rng.permutation(M + N)]
    a = synth.complex_normal(1 << len(la), seed=seed + 1).astype(np.complex64)
    b = synth.complex_normal(1 << len(lb), seed=seed + 2).astype(np.complex64)
    return la, lb, lc, a, b


@pytest.mark.parametrize("cases", [
    [(3, 3, 18, SPLITK), (2, 1, 12, SPLITK)],     # register-only split-K, then a smaller one
    [(4, 4, 16, SPLITK), (3, 2, 10, SPLITK)],
    [(7, 6, 15, TILE), (6, 5, 12, TILE)],         # split-K over LDS tiles
    [(6, 6, 4, TILE), (5, 5, 3, TILE)],           # no split: no scratch used
])
def test_noalloc_matches_contract(cases):
    require_gpu()
    import torch
    from paper_2504_09186_amd import tnc
    for mb, nb, kb, kernel in cases:
        seed = 5000 + 100 * mb + 10 * nb + kb
        la, lb, lc, a, b = _operands(mb, nb, kb, seed)
        print(f"noalloc case m{mb} n{nb} k{kb} kernel {kernel} seed {seed}", flush=True)
        ta, tb = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
        ref_c = tnc.contract(ta, la, tb, lb, lc, kernel=kernel)
        out = torch.full((1 << len(lc),), complex(float("nan"), 0), dtype=torch.complex64, device=ta.device)
        got = tnc.contract(ta, la, tb, lb, lc, kernel=kernel, out=out, noalloc=True)
        torch.cuda.synchronize()
        g, r = got.cpu().numpy(), ref_c.cpu().numpy()
        assert np.array_equal(g.view(np.uint32), r.view(np.uint32))
        exact = ref_contract(a, la, b, lb, lc)
        bound = ref_contract(a, la, b, lb, lc, absval=True).real * gamma((1 << kb) + 4) * 6.0
        assert np.all(np.abs(g.astype(np.complex128) - exact) <= bound + 1e-30)


def test_split_rule_fits_scratch():
    """Host-side check: with the library's split rule (the K split stops once
    output tiles x splits reach the class's workgroup target), no single
    contraction needs more partials than the fixed 32 MiB scratch; the
    largest, a complex64 LDS-tiled split with 128 x 64 output tiles (2^9
    workgroups), needs exactly 32 MiB."""
    from paper_2504_09186_amd import tnc
    worst = 0
    for mb, nb, kb, kernel in [(7, 6, 15, TILE), (9, 8, 20, TILE), (12, 10, 16, TILE), (4, 4, 24, SPLITK),
                               (6, 6, 22, SPLITK), (2, 2, 27, SPLITK), (8, 2, 18, 3)]:
        la, lb, lc, _, _ = _operands(mb, nb, 0, 1)
        K = [3000 + i for i in range(kb)]
        need = tnc.contract_work_bytes(la + K, K + lb, lc, kernel=kernel)
        worst = max(worst, need)
    assert 0 < worst <= (32 << 20)
