"""Host-side pins of the LDS index algebra the FFT kernels rely on.

The kernels pad LDS arrays of complex values by one element per 2^s (s =
kLdsPadShift in llg_internal.hpp): lp(a) = a + (a >> s).  They address every
access as lp(base) plus a block-uniform offset lp(x), which is exact when base
and x share no set bit (the shift of a bitwise union is the union of the
shifts).  These tests rebuild the index maps of a Stockham pass, of the
column kernel's first and last passes and its component planes, and of the
row kernels' components, check that premise for every pass shape, and check
the split itself; a plane-size slip (2 lp(P) for lp(2P)) fails them.
"""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def pad_shift():
    txt = open(os.path.join(ROOT, "paper_2411_19109_amd", "csrc", "llg_internal.hpp")).read()
    return int(re.search(r"constexpr int kLdsPadShift = (\d+);", txt).group(1))


S = pad_shift()


def lp(a):
    return a + (a >> S)


def test_pad_period_fills_the_banks_once():
    # 2^s complex values of 8 bytes = 64 four-byte banks
    assert S == 5


def test_split_needs_disjoint_bits():
    # the identity holds for disjoint bits and fails in general
    assert lp(96 + 7) == lp(96) + lp(7)
    assert lp(16 + 16) != lp(16) + lp(16)
    assert lp(2 * 16) != 2 * lp(16)  # the plane-offset slip the kernels must avoid


def stockham_maps(l0, lL, extra, R, lNs, nsig):
    """(a0, k, b0, ko) per work item of one pass: its R inputs at a0 + r 2^k,
    outputs at b0 + r 2^ko (signals 2^ls1 apart, 2^l0 of them interleaved)."""
    LR = R.bit_length() - 1
    ls1 = l0 + lL + extra
    lnbf = lL - LR
    k, ko = l0 + lnbf, lNs + l0
    for it in range(nsig << lnbf):
        a0 = ((it >> k) << ls1) + (it & ((1 << k) - 1))
        j = (it >> l0) & ((1 << lnbf) - 1)
        jm = j & ((1 << lNs) - 1)
        b0 = ((it >> k) << ls1) + (it & ((1 << l0) - 1)) + ((((j - jm) << LR) + jm) << l0)
        yield a0, k, b0, ko


@pytest.mark.parametrize("R", [2, 4, 8, 16])
def test_stockham_pass_offsets_split(R):
    LR = R.bit_length() - 1
    n = 0
    for l0 in range(0, 5):
        for lL in range(LR, 10):
            for extra in (0, 2):
                for lNs in range(0, lL - LR + 1):
                    seen = set()
                    for a0, k, b0, ko in stockham_maps(l0, lL, extra, R, lNs, 3 << l0):
                        for r in range(R):
                            assert a0 & (r << k) == 0 and b0 & (r << ko) == 0
                            assert lp(a0 + (r << k)) == lp(a0) + lp(r << k)
                            assert lp(b0 + (r << ko)) == lp(b0) + lp(r << ko)
                            seen.add(b0 + (r << ko))
                            n += 1
                    # the outputs of a pass cover every element of every signal once
                    assert len(seen) == (3 << l0) << lL
    assert n > 10000


def test_column_first_last_and_planes_split():
    for lL in range(1, 10):
        for ltk in range(0, 5):
            for LMR in (1, 2, 3, 4):
                LR = min(lL, LMR)
                lnb = lL - LR
                for it in range(3 << (ltk + lnb)):
                    tk = it & ((1 << ltk) - 1)
                    j = (it >> ltk) & ((1 << lnb) - 1)
                    c = it >> (ltk + lnb)
                    first = (c << (lL + ltk)) + ((j << LR) << ltk) + tk
                    last = (c << (lL + ltk)) + (j << ltk) + tk
                    for r in range(1 << LR):
                        assert lp(first + (r << ltk)) == lp(first) + lp(r << ltk)
                        assert lp(last + (r << (lnb + ltk))) == lp(last) + lp(r << (lnb + ltk))
            # component planes of the tensor multiply (plane = Py TK, a power of two)
            plane = 1 << (lL + ltk)
            for e in range(plane):
                for cc in range(3):
                    assert lp(cc * plane + e) == lp(e) + lp(cc * plane)


def test_row_components_split():
    for lP in range(0, 12):
        P = 1 << lP
        for x in range(P):
            for s_ in range(3):
                assert lp(s_ * P + x) == lp(x) + lp(s_ * P)
