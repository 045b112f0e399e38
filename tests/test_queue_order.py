"""The contour queue's dispersed order (paper_2501_03322_amd/csrc/twk_queue.h:
the golden-ratio stride, its modular inverse and the position map the
kernels use), compiled for the CPU by the emulation harness (tests/emu) and
checked against independent integer arithmetic.  CPU only.

The order is a scheduling choice of this implementation (the paper's
dispatch takes sources as queued, Sec. 3): every task must still run
exactly once, a limb-darkened epoch's annulus contours must stay together,
and any run of consecutive queue positions should sample the whole queue
evenly."""
import ctypes as C
import math

import numpy as np
import pytest

INV_PHI = 0.6180339887498949


@pytest.fixture(scope="module")
def q():
    from emu import build_emu
    lib = C.CDLL(build_emu.build())
    ll = C.c_longlong
    lib.emu_golden_stride.argtypes = [ll, C.POINTER(ll), C.POINTER(ll)]
    lib.emu_golden_stride.restype = None
    lib.emu_dispersed_task.argtypes = [ll, C.c_ulonglong, ll, ll]
    lib.emu_dispersed_task.restype = ll

    def stride(n):
        g, gi = ll(), ll()
        lib.emu_golden_stride(n, C.byref(g), C.byref(gi))
        return g.value, gi.value

    return dict(stride=stride, task=lib.emu_dispersed_task)


def _reference_stride(n):
    """First s >= floor(n / phi) (wrapping to 1) with gcd(s, n) = 1."""
    if n <= 2:
        return 1
    s = int(n * INV_PHI)
    while math.gcd(s, n) != 1:
        s = s + 1 if s + 1 < n else 1
    return s


SIZES = list(range(1, 1200)) + [2 ** 20, 2 ** 26, 2 ** 28, 2 ** 28 - 1, 720720, 3603600,
                                 11801776, 23602353, 1000003, 999983 * 2]


def test_stride_is_the_coprime_next_to_n_over_phi_and_inverts(q):
    for n in SIZES:
        g, gi = q["stride"](n)
        assert g == _reference_stride(n), n
        assert math.gcd(g, n) == 1 and 0 <= gi < max(n, 2), n
        assert (g * gi) % n == 1 % n, n
        if n > 2:
            assert abs(g - n * INV_PHI) < 64, n  # coprimes are dense near n / phi


@pytest.mark.parametrize("n,grp", [(1, 1), (7, 1), (64, 1), (1000, 1), (100003, 1), (10, 10),
                                   (70, 10), (12340, 10), (3 * 4099, 3), (64 * 64, 64)])
def test_position_map_is_a_permutation_keeping_groups(q, n, grp):
    ng = n // grp
    g, _ = q["stride"](ng)
    t = np.array([q["task"](p, g, grp, ng) for p in range(n)])
    assert np.array_equal(np.sort(t), np.arange(n))
    # the tasks of a group stay together, in order, at the group's positions
    tg = t.reshape(ng, grp)
    assert np.all(tg % grp == np.arange(grp)) and np.all(tg // grp == tg[:, :1] // grp)
    # consecutive positions visit groups g apart
    assert np.all((tg[1:, 0] // grp - tg[:-1, 0] // grp) % ng == g % ng)


def test_placement_inverse_gives_the_same_visiting_order(q):
    """The learned placement puts class rank r at r * ginv mod N; position p
    then holds rank p * g mod N, the order the plain path's pops take."""
    for n in (1, 2, 3, 97, 1000, 65536, 123457):
        g, gi = q["stride"](n)
        r = np.arange(n, dtype=np.int64)
        pos = (r * gi) % n
        assert np.array_equal(np.sort(pos), r)
        assert np.array_equal((pos * g) % n, r)


def test_windows_sample_the_queue_evenly(q):
    """Any window of W consecutive positions (W about the persistent grid)
    visits groups spread over the whole queue: the largest gap between the
    visited group indices stays within a small multiple of N / W (the
    golden-ratio stride's three-gap bound), where source order would visit
    one block of W adjacent groups."""
    for n in (118017, 1180177, 2 ** 20 + 7):
        g, _ = q["stride"](n)
        for w in (256, 1792):
            for start in (0, n // 3, n - w):
                idx = np.sort((np.arange(start, start + w, dtype=np.int64) * g) % n)
                gaps = np.diff(np.concatenate([idx, [idx[0] + n]]))
                assert gaps.max() <= 3.0 * n / w, (n, w, start, gaps.max())


@pytest.fixture(scope="module")
def merged():
    from emu import build_emu
    lib = C.CDLL(build_emu.build())
    ll = C.c_longlong
    lib.emu_merged_place.argtypes = [C.c_int, ll, ll, ll]
    lib.emu_merged_place.restype = ll
    return lambda long_row, q, n0, n1: lib.emu_merged_place(1 if long_row else 0, q, n0, n1)


@pytest.mark.parametrize("n0,n1", [(0, 5), (5, 0), (1, 1), (10, 3), (1000, 37), (7, 100),
                                   (123457, 999), (50, 50), (3, 1000), (2 ** 20, 3001)])
def test_merged_places_spread_the_long_class(merged, n0, n1):
    """The learned order's merge of the two classes: the places form a
    permutation of 0 .. n0+n1-1, each class keeps its dispersed order, and
    the long rows lie evenly in the first half (the k-th long row after
    about k n0 / (2 n1) other rows), checked against the keys' definition
    with exact fractions."""
    from fractions import Fraction
    pl = np.array([merged(True, q, n0, n1) for q in range(n1)], dtype=np.int64)
    po = np.array([merged(False, b, n0, n1) for b in range(n0)], dtype=np.int64)
    assert np.array_equal(np.sort(np.concatenate([pl, po])), np.arange(n0 + n1))
    assert np.all(np.diff(pl) > 0) and np.all(np.diff(po) > 0)
    if n0 < 3000:  # brute force over the other class's keys
        for q in range(0, n1, max(1, n1 // 50)):
            key = Fraction(2 * q + 1, 4 * n1)
            before = sum(1 for b in range(n0) if Fraction(2 * b + 1, 2 * n0) < key)
            assert pl[q] == q + before, (q, pl[q], before)
    if n1 and n0 > n1:
        assert pl.max() <= n1 + n0 // 2 + 1
