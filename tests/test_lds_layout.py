"""Host checks of the tile kernels' LDS layouts chosen by the planner
(reported by the step introspection).  No GPU needed.

FP16/BF16 tile kernels: the LDS word address of a tile entry is the XOR of
one vector per set tile bit.  The map must be a bijection of the tile onto
words inside the stage (A: TM rows of TK words, expanded B: 2 TN rows), keep
4-word groups whole (16-byte fragment reads), and give the fragment reads of
8 (16) consecutive rows distinct 4-word blocks modulo 32 (64) four-byte banks.
Complex64 tile kernels: row k of a stage stores column c at c ^ H(k) with
H(k) inside the row."""
import numpy as np
import pytest

import synth
from paper_2504_09186_amd import tnc

TB_M, TB_K, TB_N = 0, 1, 2
# template tile bits (rows m, columns n, k) of the TILE, TALL and SPLITK kernels
GEOM = {0: {2: (7, 6, 3), 3: (7, 4, 4), 4: (4, 4, 6)}, 1: {2: (7, 6, 5), 3: (7, 4, 5), 4: (4, 4, 7)}}


def _plan(precision, force_kernel=-1):
    c = synth.lattice_circuit(4, 5, 12, seed=71)
    spec = synth.output_spec(20, list(range(16, 20)), seed=72)
    net = tnc.Network(c, spec)
    net.path_search(seed=73, trials=4, max_log2=20, min_sliced=2, max_sliced=30)
    return tnc.Plan(net, precision=precision, force_kernel=force_kernel)


def _tile_steps(plan):
    out = []
    for i, r in enumerate(plan.steps()):
        if int(r[0]) in (2, 3, 4):
            out.append((int(r[0]), plan.step_info(i)))
    return out


def _xor_rank(vs):
    piv = {}
    r = 0
    for v in vs:
        x = int(v)
        while x:
            h = x.bit_length() - 1
            if h in piv:
                x ^= piv[h]
            else:
                piv[h] = x
                r += 1
                break
    return r


def _addr(vecs, e):
    a = 0
    for b, v in enumerate(vecs):
        if (e >> b) & 1:
            a ^= v
    return a


@pytest.mark.parametrize("kernel", [2, 3, 4])
def test_half_tile_layout_is_a_conflict_free_bijection(kernel):
    plan = _plan(1, kernel)
    steps = _tile_steps(plan)
    assert steps, "no MFMA-class steps in the plan"
    for cls, si in steps:
        tmb, tnb, tkb = GEOM[1][cls]
        TM, TN, TK = 1 << tmb, 1 << tnb, 1 << tkb
        arow, brow, kcol = si["lds_a_row"], si["lds_b_row"], si["lds_k_col"]
        tm, tn, tk = si["tm"], si["tn"], si["tk"]
        assert len(set(kcol[:tk])) == tk and all(c < tkb for c in kcol[:tk])
        def vec(code, rows, row_cls, row_off):
            c, i = code >> 5, code & 31
            return rows[i + row_off] if c == row_cls else 1 << kcol[i]
        va = [vec(c, arow, TB_M, 0) for c in si["a_tile"][:tm + tk]]
        vb = [vec(c, brow, TB_N, 1) for c in si["b_tile"][:tk + tn]]
        # bijection onto words of the stage
        wa = {_addr(va, e) for e in range(1 << (tm + tk))}
        assert len(wa) == 1 << (tm + tk) and max(wa) < TM * TK
        wb = {_addr(vb, e) ^ (brow[0] * c) for e in range(1 << (tk + tn)) for c in (0, 1)}
        assert len(wb) == 2 << (tk + tn) and max(wb) < 2 * TN * TK
        # row vectors keep 4-word groups whole; all template rows are distinct
        for rows, nrows in ((arow, tmb), (brow, tnb + 1)):
            assert all(r % 4 == 0 for r in rows[:nrows])
            assert _xor_rank(rows[:nrows]) == nrows
            # fragment reads: rows 0-7 distinct 4-word blocks mod 32 banks, rows 0-15 mod 64
            blocks32 = [(r >> 2) & 7 for r in rows[:3]]
            blocks64 = [(r >> 2) & 15 for r in rows[:4]]
            assert _xor_rank(blocks32) == 3 and _xor_rank(blocks64) == 4
        assert si["vec_a"] in (1, 4) and si["vec_b"] in (1, 4)


@pytest.mark.parametrize("kernel", [2, 3, 4])
def test_complex64_tile_swizzle_stays_in_rows(kernel):
    plan = _plan(0, kernel)
    steps = _tile_steps(plan)
    assert steps
    for cls, si in steps:
        tmb, tnb, tkb = GEOM[0][cls]
        assert all(g < (1 << tmb) for g in si["lds_a_swz"])
        assert all(g < (1 << tnb) for g in si["lds_b_swz"])
        assert si["lds_a_row"] == [0] * 8 and si["lds_b_row"] == [0] * 8


def test_complex64_swizzle_spreads_staging_writes():
    """Lanes 0-15 of a staging write take consecutive tile entries (address
    order); with the chosen row masks their float2 slots are distinct mod 16
    (32 banks) whenever the lowest tile bits allow it (rows and columns
    below the 5th address bit)."""
    plan = _plan(0, 2)
    n_checked = 0
    for cls, si in _tile_steps(plan):
        tmb, tnb, tkb = GEOM[0][cls]
        for op, tile, ntile, swz, cols in (("A", si["a_tile"], si["tm"] + si["tk"], si["lds_a_swz"], 1 << tmb),
                                           ("B", si["b_tile"], si["tk"] + si["tn"], si["lds_b_swz"], 1 << tnb)):
            codes = tile[:min(4, ntile)]
            if any((c >> 5) != TB_K and (c & 31) >= 4 for c in codes):
                continue  # a column bit above 2^4 among the lanes: no row mask can help
            slots = set()
            for e in range(1 << len(codes)):
                k = col = 0
                for b, c in enumerate(codes):
                    if (e >> b) & 1:
                        if (c >> 5) == TB_K:
                            k |= 1 << (c & 31)
                        else:
                            col |= 1 << (c & 31)
                h = 0
                for j in range(8):
                    if (k >> j) & 1:
                        h ^= swz[j]
                slots.add((k * cols + (col ^ h)) % 16)
            assert len(slots) == 1 << len(codes), (op, codes, swz)
            n_checked += 1
    assert n_checked > 0
