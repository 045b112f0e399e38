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
