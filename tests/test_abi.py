"""Host-side checks of the C ABI (no GPU): the library loads and exports every
entry point of include/kkt.h, and the plan's partition and layout are right."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import partition

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _kkt():
    from paper_2511_00946_amd import kkt
    return kkt


def test_header_symbols_exported():
    kkt = _kkt()
    hdr = open(os.path.join(ROOT, "include", "kkt.h")).read()
    decl = set(re.findall(r"^\s*(?:int|int64_t|const char \*)\s*(kkt_\w+)\s*\(", hdr, re.M))
    assert decl == set(kkt.EXPORTED), decl ^ set(kkt.EXPORTED)
    lib = ctypes.CDLL(kkt.LIB_PATH)
    for name in decl:
        assert hasattr(lib, name), name


def test_status_strings():
    lib = _kkt().lib()
    for rc in (0, -1, -2, -3, -4, -5, -6):
        assert lib.kkt_status_string(rc).decode() not in ("", "unknown status")


@pytest.mark.parametrize("N,p", [(128, 4), (128, 8), (128, 16), (128, 32), (2048, 64), (64, 4), (16, 2),
                                 (16, 8), (7, 4), (200, 12), (2356, 12)])
def test_plan_partition_matches_eq13(N, p):
    kkt = _kkt()
    plan = kkt.Plan([(N, 6, 2, p)])
    n1, nk = partition.segment_lengths(N, p)
    assert plan.segment_lengths(0) == [n1] + [nk] * (p - 1)


def test_plan_rejects_bad_dims():
    kkt = _kkt()
    for d in [(0, 4, 0, 1), (5, 0, 0, 1), (5, 33, 0, 1), (5, 4, 17, 1), (5, 4, 0, 4), (10, 4, 0, 3, 5)]:
        with pytest.raises(kkt.KKTError):
            kkt.Plan([d])
    with pytest.raises(kkt.KKTError):
        kkt.Plan([(5, 4, 0, 1)], nrhs=9)


def test_explicit_first_segment_length():
    kkt = _kkt()
    plan = kkt.Plan([(20, 4, 1, 3, 8)])
    assert plan.segment_lengths(0) == [8, 5, 5]


def test_pool_layout_is_packed_system_after_system():
    kkt = _kkt()
    dims = [(5, 3, 2, 1), (7, 4, 0, 2), (9, 2, 1, 3)]
    plan = kkt.Plan(dims, nrhs=2)
    offD = offC = offB = offR = offRHS = 0
    for s, (N, b, ng, p) in enumerate(dims):
        lay = plan.layouts[s]
        assert (lay.off_D, lay.off_C, lay.off_B, lay.off_corner, lay.off_rhs) == (offD, offC, offB, offR, offRHS)
        offD += N * b * b
        offC += (N - 1) * b * b
        offB += N * ng * b
        offR += ng * ng
        offRHS += (N * b + ng) * 2
    pl = plan.pool_lengths()
    assert (pl["D"], pl["C"], pl["B"], pl["corner"], pl["rhs"]) == (offD, offC, offB, offR, offRHS)
    assert plan.info.workspace_bytes % 256 == 0 and plan.factor_offset % 256 == 0


def test_factor_words_count_fill():
    kkt = _kkt()
    N, b, p = 40, 5, 4
    plan = kkt.Plan([(N, b, 0, p)])
    n1, nk = partition.segment_lengths(N, p)
    k_words = N * b * b + (N - 1) * b * b
    fill = (p - 1) * (nk - 1) * b * b + (p - 2) * b * b
    assert plan.info.input_words == k_words
    assert plan.info.factor_words == k_words + fill
