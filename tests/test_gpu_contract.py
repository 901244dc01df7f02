"""Single pairwise contractions on the GPU against the FP64 oracle.

Each kernel class gets random bit layouts (the permutation is fused into the
loads), ragged tiles, batch bits and degenerate ranks.  Bound: the elementwise
GEMM error bound of Eq. (3), |C^ - C| <= gamma_K |A||B|, applied to the
complex arithmetic the kernels use, on the complex64 inputs actually fed to
them.  The MFMA kernels use the 3M split: Re C = T1 - T2, Im C = T3 - T1 - T2
with T1 = Ar Br, T2 = Ai Bi, T3 = (Ar + Ai)(Br + Bi); each real product has
error <= gamma_{K+2} times its absolute product, |Ar||Br| + |Ai||Bi| <= |a||b|
and (|Ar| + |Ai|)(|Br| + |Bi|) <= 2|a||b|, so |C^ - C| <= 6 gamma_{K+4} |A||B|
covers them and the direct 4-multiply form of the other kernels.
"""
import numpy as np
import pytest

import synth
from helpers import gamma, ref_contract, require_gpu

pytestmark = pytest.mark.gpu

SMALL, STEM, TILE, TALL, SPLITK, STREAM = 0, 1, 2, 3, 4, 5


def _case(mb, nb, kb, bb, seed, in_place=False, rows_ordered=False):
    """Random layouts; with in_place, C takes A's layout with the k bits
    replaced by n bits (the planner's output policy).  With rows_ordered, the
    row indices past the four lowest of A keep A's relative order in C (what
    the stream kernel requires); the rest of C stays random."""
    rng = np.random.default_rng(seed)
    M = [1000 + i for i in range(mb)]
    N = [2000 + i for i in range(nb)]
    K = [3000 + i for i in range(kb)]
    Bt = [-1 - i for i in range(bb)]
    la = list(rng.permutation(M + K + Bt)) if (mb + kb + bb) else []
    lb = list(rng.permutation(K + N + Bt)) if (kb + nb + bb) else []
    lc = list(rng.permutation(M + N + Bt)) if (mb + nb + bb) else []
    if rows_ordered and mb > 5:
        by_a = sorted(M, key=la.index)
        high = set(by_a[4:])
        slots = sorted(i for i, x in enumerate(lc) if x in high)
        for i, x in zip(slots, by_a[4:]):
            lc[i] = x
    if in_place:
        nit = iter(N)
        lc = [x for x in (next(nit, None) if x in K else x for x in la) if x is not None] + list(nit)
    a = synth.complex_normal(1 << len(la), seed=seed + 1).astype(np.complex64)
    b = synth.complex_normal(1 << len(lb), seed=seed + 2).astype(np.complex64)
    return [int(x) for x in la], [int(x) for x in lb], [int(x) for x in lc], a, b


def _run(mb, nb, kb, bb, kernel, seed, in_place=False):
    require_gpu()
    import torch
    from paper_2504_09186_amd import tnc
    la, lb, lc, a, b = _case(mb, nb, kb, bb, seed, in_place, rows_ordered=kernel == STREAM)
    print(f"contract case m{mb} n{nb} k{kb} b{bb} kernel {kernel} seed {seed}", flush=True)
    ta = torch.from_numpy(a).cuda()
    tb = torch.from_numpy(b).cuda()
    c = tnc.contract(ta, la, tb, lb, lc, kernel=kernel)
    torch.cuda.synchronize()
    got = c.cpu().numpy().astype(np.complex128)
    ref = ref_contract(a, la, b, lb, lc)
    bound = ref_contract(a, la, b, lb, lc, absval=True).real * gamma((1 << kb) + 4) * 6.0
    err = np.abs(got - ref)
    assert np.all(err <= bound + 1e-30), f"max err/bound {np.max(err / (bound + 1e-30))}"
    rel = np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300)
    assert rel < 1e-5
    return rel


@pytest.mark.parametrize("mb,nb,kb,bb", [(0, 0, 0, 0), (3, 2, 2, 0), (4, 4, 6, 0), (2, 3, 5, 2),
                                         (0, 5, 3, 0), (6, 0, 1, 1)])
def test_small(mb, nb, kb, bb):
    _run(mb, nb, kb, bb, SMALL, seed=10 * mb + nb + 100 * kb)


@pytest.mark.parametrize("mb,nb,kb,bb", [(12, 2, 2, 0), (14, 1, 1, 0), (10, 2, 4, 0), (9, 0, 3, 0),
                                         (5, 2, 2, 0), (11, 1, 3, 2), (0, 2, 2, 0), (13, 2, 0, 0)])
def test_stem(mb, nb, kb, bb):
    _run(mb, nb, kb, bb, STEM, seed=7 + mb + 10 * nb + 100 * kb)


@pytest.mark.parametrize("mb,nb,kb,bb", [(7, 7, 6, 0), (8, 6, 9, 0), (6, 6, 4, 0), (9, 7, 5, 1),
                                         (3, 2, 0, 0), (5, 3, 3, 0), (7, 8, 12, 0), (0, 0, 4, 0)])
def test_tile(mb, nb, kb, bb):
    _run(mb, nb, kb, bb, TILE, seed=3 + mb + 10 * nb + 100 * kb)


@pytest.mark.parametrize("mb,nb,kb,bb", [(9, 3, 5, 0), (10, 4, 8, 0), (7, 2, 4, 1), (12, 1, 2, 0),
                                         (8, 4, 13, 0)])
def test_tall(mb, nb, kb, bb):
    _run(mb, nb, kb, bb, TALL, seed=5 + mb + 10 * nb + 100 * kb)


@pytest.mark.parametrize("mb,nb,kb,bb", [(3, 3, 16, 0), (4, 4, 14, 0), (2, 1, 12, 0), (0, 0, 10, 0),
                                         (3, 3, 9, 1), (4, 3, 18, 0), (1, 2, 3, 0)])
def test_splitk(mb, nb, kb, bb):
    _run(mb, nb, kb, bb, SPLITK, seed=9 + mb + 10 * nb + 100 * kb)


# Every (k steps, column blocks) instantiation, K < 4 and N < 16 padding, and
# runs long enough for several iterations per wave (m20 n2 k2, m18 n4 k6,
# m16 n5 k5, m15 n5 k5 b2).
@pytest.mark.parametrize("mb,nb,kb,bb", [(12, 0, 0, 0), (12, 1, 1, 0), (13, 2, 2, 0), (14, 5, 5, 0),
                                         (12, 4, 6, 0), (12, 6, 4, 0), (15, 3, 3, 0), (12, 5, 3, 0),
                                         (16, 4, 5, 0), (12, 6, 2, 0), (12, 5, 4, 0), (12, 6, 3, 0),
                                         (20, 2, 2, 0), (18, 4, 6, 0), (8, 0, 0, 0), (8, 2, 2, 0), (9, 5, 5, 0),
                                         (10, 4, 6, 0), (8, 6, 4, 0), (11, 3, 3, 0), (10, 2, 2, 2), (12, 5, 5, 3),
                                         (9, 4, 6, 1), (8, 3, 3, 4), (8, 1, 2, 8), (16, 5, 5, 0), (15, 5, 5, 2)])
@pytest.mark.parametrize("in_place", [False, True])
def test_stream(mb, nb, kb, bb, in_place):
    """Random C layouts (row indices past the lane bits in A's order, the lane
    bits, column and batch indices anywhere) and the planner's in-place
    layout; batch indices split the waves' row runs."""
    _run(mb, nb, kb, bb, STREAM, seed=13 + mb + 10 * nb + 100 * kb, in_place=in_place)


@pytest.mark.parametrize("mb,nb,kb,bb", [(10, 10, 8, 0), (3, 3, 17, 0), (16, 2, 2, 0), (4, 4, 4, 0),
                                         (11, 4, 6, 0)])
def test_auto(mb, nb, kb, bb):
    _run(mb, nb, kb, bb, -1, seed=11 + mb + 10 * nb + 100 * kb)


# Skinny split-K (M N <= 16, K >= 2^8): batch indices, splits from many down
# to none (direct store), every (M, N) register shape class.
@pytest.mark.parametrize("mb,nb,kb,bb", [(2, 1, 17, 3), (2, 2, 12, 2), (0, 4, 10, 0), (4, 0, 9, 1), (1, 3, 8, 0),
                                         (3, 1, 14, 5), (1, 1, 8, 10), (2, 1, 13, 8), (0, 0, 8, 0)])
def test_splitk_skinny(mb, nb, kb, bb):
    _run(mb, nb, kb, bb, SPLITK, seed=21 + mb + 10 * nb + 100 * kb + 1000 * bb)


# TALL steps with N <= 4 and long K (batch bits, split K).
@pytest.mark.parametrize("mb,nb,kb,bb", [(9, 2, 10, 1), (12, 1, 8, 0), (7, 0, 13, 0), (6, 2, 12, 2), (8, 1, 9, 3),
                                         (5, 0, 8, 0)])
def test_tall_long_k(mb, nb, kb, bb):
    _run(mb, nb, kb, bb, TALL, seed=31 + mb + 10 * nb + 100 * kb + 1000 * bb)


def test_splitk_long_k_accuracy():
    """K = 2^22: the blocked (split-K + FP64) summation keeps the error far
    below a single FP32 chain over K."""
    rel = _run(3, 3, 22, 0, SPLITK, seed=4242)
    assert rel < 2e-6



def test_splitk_k27_elementwise():
    """The narrow-factor GEPDOT of the split-common evaluation: two rank-29 /
    rank-28 operands sharing 27 indices (M = 4, N = 2, K = 2^27; 4 GiB and
    2 GiB of complex64), elementwise against FP64 sums.  K is split over
    2^12 waves; a wave's lanes run FP32 chains of K / (2^12 * 64) = 512
    products (4-multiply complex form), a 64-lane shuffle tree adds them, and
    the splits are summed in FP64 in a fixed order (Eq. 3 with blocked
    summation).  Bound per entry: 6 gamma_{2^10} sum_k |a_k||b_k| (covers the
    chain, the tree and FP64) plus the final complex64 rounding 2^-23 |C|.
    An unblocked FP32 chain over 2^27 terms has an expected error of about
    u sqrt(K) sum_k |a_k||b_k| ~ 7e-4 of it, above this bound."""
    require_gpu()
    import torch
    from paper_2504_09186_amd import tnc
    kb, mb, nb = 27, 2, 1
    K = [3000 + i for i in range(kb)]
    la = K + [1000, 1001]        # A[m][k]: k on the low 27 address bits
    lb = K + [2000]              # B[n][k]
    lc = [1000, 1001, 2000]      # C[n][m]
    print("split-K case m2 n1 k27 (seed 4270)", flush=True)
    a = synth.complex_normal_c64(1 << (kb + mb), seed=4270)
    b = synth.complex_normal_c64(1 << (kb + nb), seed=4271)
    ta = torch.from_numpy(a).cuda()
    tb = torch.from_numpy(b).cuda()
    c = tnc.contract(ta, la, tb, lb, lc, kernel=SPLITK)
    torch.cuda.synchronize()
    got = c.cpu().numpy().astype(np.complex128)
    del ta, tb
    A2, B2 = a.reshape(1 << mb, 1 << kb), b.reshape(1 << nb, 1 << kb)
    ref = np.zeros((1 << nb, 1 << mb), dtype=np.complex128)
    absab = np.zeros((1 << nb, 1 << mb))
    step = 1 << 23
    for k0 in range(0, 1 << kb, step):
        ac = A2[:, k0:k0 + step].astype(np.complex128)
        bc = B2[:, k0:k0 + step].astype(np.complex128)
        ref += bc @ ac.T
        absab += np.abs(bc) @ np.abs(ac).T
    ref, absab = ref.reshape(-1), absab.reshape(-1)
    bound = 6.0 * gamma(1 << 10) * absab + 2.0 ** -23 * np.abs(ref)
    err = np.abs(got - ref)
    print(f"max err / bound {np.max(err / bound):.3e}, max err / sum|a||b| {np.max(err / absab):.3e}")
    assert np.all(err <= bound)

@pytest.mark.parametrize("prec", [1, 2])
def test_half_splitk_rank30_exact(prec):
    """The split-K GEPDOT on FP16 / BF16 storage at the narrow-factor shape of
    the split-common evaluation with a rank-30 operand: A[m][k] (M = 4, K =
    2^28, 4 GiB of 16-bit pairs) times B[n][k] (N = 2, 2 GiB).  Entries are
    Gaussian integers (A sparse with parts in {-1, 0, 1}, B = +-1 +-i), so
    every product and every partial sum, in the FP32 MFMA chains and the FP64
    reduction alike, is an exact small integer: the stored result must equal
    C 2^-s_C bit for bit (|C| < 2^8 is exact in both 16-bit formats).  Any k
    range read twice, skipped or read from the wrong address changes C."""
    require_gpu()
    import torch
    from paper_2504_09186_amd import tnc
    kb, mb, nb = 28, 2, 1
    K = [3000 + i for i in range(kb)]
    la = K + [1000, 1001]        # A index = k + 2^28 m
    lb = K + [2000]              # B index = k + 2^28 n
    lc = [1000, 1001, 2000]      # C index = m + 4 n
    one, neg = (0x3C00, 0xBC00) if prec == 1 else (0x3F80, 0xBF80)
    rng = np.random.default_rng(4300 + prec)
    idx = np.unique(rng.integers(0, 1 << (kb + mb), size=1 << 12, dtype=np.int64))
    parts = rng.integers(-1, 2, size=(idx.size, 2))
    enc = lambda v: np.where(v > 0, one, np.where(v < 0, neg, 0)).astype(np.uint32)
    wa = np.zeros(1 << (kb + mb), dtype=np.uint32)
    wa[idx] = enc(parts[:, 0]) | (enc(parts[:, 1]) << 16)
    br = rng.integers(0, 2, size=1 << (kb + nb), dtype=np.uint8)
    bi = rng.integers(0, 2, size=1 << (kb + nb), dtype=np.uint8)
    wb = np.where(br == 1, np.uint32(neg), np.uint32(one)) | (np.where(bi == 1, np.uint32(neg), np.uint32(one)) << 16)
    # exact reference: only the nonzero entries of A contribute
    ref = np.zeros(1 << (mb + nb), dtype=np.complex128)
    k, m = idx & ((1 << kb) - 1), idx >> kb
    a = parts[:, 0] + 1j * parts[:, 1]
    for n in range(1 << nb):
        bv = (1 - 2.0 * br[k + (n << kb)]) + 1j * (1 - 2.0 * bi[k + (n << kb)])
        np.add.at(ref, m + (n << mb), a * bv)
    mx = max(np.max(np.abs(ref.real)), np.max(np.abs(ref.imag)))
    assert 0 < mx < 256
    s_c = int(np.frexp(mx)[1] - 1) - 13       # max |C| 2^-s_C in [2^13, 2^14)
    print(f"half split-K rank 30: m{mb} n{nb} k{kb} prec {prec} (seed {4300 + prec}) s_C {s_c}", flush=True)
    ta = torch.from_numpy(wa.view(np.int32)).cuda()
    tb = torch.from_numpy(wb.view(np.int32)).cuda()
    del wa, wb
    c = tnc.contract(ta, la, tb, lb, lc, kernel=SPLITK, precision=prec, out_scale=2.0 ** -s_c)
    torch.cuda.synchronize()
    del ta, tb
    got = _from_half_words(c, prec) * 2.0 ** s_c
    assert np.array_equal(got, ref), f"got {got} want {ref}"


# ---------------------------------------------------------------- FP16 / BF16 storage
def _to_half_words(x, prec):
    """complex entries -> int32 words of two 16-bit halves (re low)."""
    import torch
    re = torch.from_numpy(np.ascontiguousarray(x.real.astype(np.float32)))
    im = torch.from_numpy(np.ascontiguousarray(x.imag.astype(np.float32)))
    dt = torch.float16 if prec == 1 else torch.bfloat16
    h = torch.stack([re.to(dt), im.to(dt)], dim=1).contiguous()  # rounding to nearest even
    back = h.float().numpy()
    return h.view(torch.int32).reshape(-1).clone(), back[:, 0] + 1j * back[:, 1]


def _from_half_words(w, prec):
    import torch
    dt = torch.float16 if prec == 1 else torch.bfloat16
    h = w.cpu().view(dt).reshape(-1, 2).float().numpy()
    return h[:, 0] + 1j * h[:, 1]


@pytest.mark.parametrize("prec", [1, 2])
@pytest.mark.parametrize("mb,nb,kb,bb,kernel", [
    (8, 8, 7, 0, TILE), (9, 3, 6, 0, TALL), (3, 3, 14, 0, SPLITK), (10, 2, 2, 0, STEM), (3, 2, 4, 1, SMALL),
    (7, 6, 9, 1, TILE), (0, 0, 9, 0, SPLITK), (5, 5, 0, 0, TILE), (13, 5, 5, 0, STREAM), (12, 2, 1, 0, STREAM),
    (12, 4, 6, 0, STREAM), (8, 3, 2, 0, STREAM), (9, 6, 4, 0, STREAM), (10, 5, 5, 2, STREAM)])
def test_half_storage(prec, mb, nb, kb, bb, kernel):
    """16-bit storage, FP32 accumulate, values far below the 16-bit range.
    The true operands are x = X 2^-30 and y = Y 2^-20 (X, Y complex normal
    rounded to 16 bits: |x| ~ 2^-30 is below FP16's smallest subnormal, so
    only the mantissa plus exponent form can carry it).  The kernel gets the
    mantissas X, Y and out_scale = 2^-s_C with s_C chosen so that the largest
    stored |Re|, |Im| falls in [2^13, 2^14); the value is read back as
    stored * 2^(e_A + e_B + s_C) and compared elementwise with the FP64
    contraction of the true tiny operands.  Bound: FP32 accumulation error
    6 gamma_{K+4} |x||y| plus one rounding of the output (2^-11 FP16, 2^-8
    BF16 relative)."""
    la, lb, lc, a, b = _case(mb, nb, kb, bb, 77 + mb + 10 * nb + 100 * kb + prec, rows_ordered=kernel == STREAM)
    _half_check(prec, la, lb, lc, a, b, kernel)


def _half_check(prec, la, lb, lc, a, b, kernel):
    require_gpu()
    import torch
    from paper_2504_09186_amd import tnc
    kb = len(set(la) & set(lb)) - len([x for x in la if x < 0])
    mb, nb, bb = len(la) - kb, len(lb) - kb, len([x for x in la if x < 0])
    mb -= bb
    nb -= bb
    ea, eb = -30, -20
    wa, xr = _to_half_words(a.astype(np.complex128), prec)  # mantissas X
    wb, yr = _to_half_words(b.astype(np.complex128), prec)
    x_true, y_true = np.ldexp(xr.real, ea) + 1j * np.ldexp(xr.imag, ea), np.ldexp(yr.real, eb) + 1j * np.ldexp(yr.imag, eb)
    ref = ref_contract(x_true, la, y_true, lb, lc)
    absab = ref_contract(x_true, la, y_true, lb, lc, absval=True).real
    # output exponent from the true result's largest component
    mx = max(np.max(np.abs(ref.real)), np.max(np.abs(ref.imag)))
    s_c = int(np.frexp(mx)[1] - 1) - 13 - (ea + eb)
    scale = 2.0 ** -s_c
    print(f"half contract m{mb} n{nb} k{kb} b{bb} kernel {kernel} prec {prec} s_C {s_c}", flush=True)
    c = tnc.contract(wa.cuda(), la, wb.cuda(), lb, lc, kernel=kernel, precision=prec, out_scale=scale)
    torch.cuda.synchronize()
    stored = _from_half_words(c, prec)
    smax = max(np.max(np.abs(stored.real)), np.max(np.abs(stored.imag)))
    assert 2.0 ** 13 * (1 - 2 ** -8) <= smax < 2.0 ** 14 * (1 + 2 ** -8)
    e_c = ea + eb + s_c
    got = np.ldexp(stored.real, e_c) + 1j * np.ldexp(stored.imag, e_c)
    u_out = 2.0 ** -11 if prec == 1 else 2.0 ** -8
    bound = absab * gamma((1 << kb) + 4) * 6.0 + np.abs(ref) * u_out * 1.01 + 1e-300
    err = np.abs(got - ref)
    assert np.all(err <= bound), f"max err/bound {np.max(err / bound)}"


def _case_low_bits(mb, nb, kb, a_low, b_low, seed):
    """Layouts whose lowest address bits are chosen: a_low / b_low list the
    classes ('m', 'k', 'n') of A's / B's lowest bits (in order); the other
    bits are random.  This steers the FP16/BF16 tile kernels onto their
    16-byte load paths (the two lowest tile bits at address bits 0 and 1),
    with the four words of a load landing on one LDS row (k bits) or on
    different rows (m or n bits)."""
    rng = np.random.default_rng(seed)
    M = [1000 + i for i in range(mb)]
    N = [2000 + i for i in range(nb)]
    K = [3000 + i for i in range(kb)]
    def layout(low, pools):
        pools = {c: list(rng.permutation(v)) for c, v in pools.items()}
        head = [int(pools[c].pop()) for c in low]
        rest = [int(x) for v in pools.values() for x in v]
        return head + [int(x) for x in rng.permutation(rest)] if rest else head
    la = layout(a_low, {"m": M, "k": K})
    lb = layout(b_low, {"k": K, "n": N})
    lc = [int(x) for x in rng.permutation(M + N)]
    a = synth.complex_normal(1 << len(la), seed=seed + 1).astype(np.complex64)
    b = synth.complex_normal(1 << len(lb), seed=seed + 2).astype(np.complex64)
    return la, lb, lc, a, b


@pytest.mark.parametrize("prec", [1, 2])
@pytest.mark.parametrize("mb,nb,kb,a_low,b_low,kernel", [
    (9, 7, 8, "kk", "kk", TILE), (9, 7, 8, "kk", "kn", TILE), (9, 7, 8, "mk", "kk", TILE),
    (8, 8, 7, "mm", "nn", TILE), (9, 4, 7, "kk", "kk", TALL), (9, 4, 7, "mm", "kn", TALL),
    (4, 4, 10, "kk", "kk", SPLITK), (3, 3, 11, "km", "nk", SPLITK)])
def test_half_tile_load_paths(prec, mb, nb, kb, a_low, b_low, kernel):
    """FP16/BF16 tile kernels on layouts that take the 16-byte load paths of
    A and B (the lowest two bits of an operand are both tile bits); same
    bound as test_half_storage."""
    la, lb, lc, a, b = _case_low_bits(mb, nb, kb, a_low, b_low, 500 + mb + 10 * nb + 100 * kb + prec)
    print(f"half tile load paths m{mb} n{nb} k{kb} A low {a_low} B low {b_low} kernel {kernel} prec {prec}",
          flush=True)
    _half_check(prec, la, lb, lc, a, b, kernel)
