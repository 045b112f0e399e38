"""The device contour engine, compiled for the CPU with an emulated 64-lane
wavefront (tests/emu), against the FP64 oracle.  Runs without a GPU and
catches logic errors of the engine before any GPU run."""
import ctypes as C
import os

import numpy as np
import pytest

GATE = 1e-4


@pytest.fixture(scope="module")
def emu():
    from emu import build_emu
    lib = C.CDLL(build_emu.build())
    dp = C.POINTER(C.c_double)
    lib.emu_finite_mag.argtypes = [C.c_double] * 6 + [C.c_int, dp, dp, C.POINTER(C.c_int),
                                                      C.POINTER(C.c_uint), dp]
    lib.emu_point.argtypes = [C.c_double] * 4 + [dp, C.POINTER(C.c_int), C.POINTER(C.c_uint), dp]

    def finite(s, q, x, y, rho, tol, mixed=0):
        m, e, n, f = C.c_double(), C.c_double(), C.c_int(), C.c_uint()
        sw = (C.c_double * 3)()
        lib.emu_finite_mag(s, q, x, y, rho, tol, mixed, C.byref(m), C.byref(e), C.byref(n),
                           C.byref(f), sw)
        return m.value, e.value, n.value, f.value

    def point(s, q, x, y):
        m, n, f = C.c_double(), C.c_int(), C.c_uint()
        img = (C.c_double * 10)()
        lib.emu_point(s, q, x, y, C.byref(m), C.byref(n), C.byref(f), img)
        return m.value, n.value, f.value

    return dict(finite=finite, point=point)


CASES = [
    (1.0, 0.1, 0.2 + 0.2j, 0.1),
    (1.0, 1e-2, 0.02 + 0.01j, 0.02),
    (0.8, 5e-3, -0.45 + 0.12j, 0.03),
    (1.0, 1e-3, 0.05 + 0.01j, 1e-3),
    (0.5, 1e-6, -1.49981640625 + 0.0035j, 1e-4),
    (3.0, 1e-4, 2.666 + 0.0005j, 1e-4),
    (1.0, 1e-4, 0.0 + 0.0j, 1e-3),
    (2.0, 1e-9, 1.5 + 0.01j, 1e-3),
]


@pytest.mark.parametrize("mixed", [0, 1])
def test_engine_cases_against_oracle(emu, oracle, mixed):
    for (s, q, z, rho) in CASES:
        m, e, n, f = emu["finite"](s, q, z.real, z.imag, rho, 1e-4, mixed)
        r = oracle.finite_mag(s, q, [z.real], [z.imag], rho, oracle.JUDGE_TOL, oracle.judge_cfg())[0][0]
        assert abs(m / r - 1) <= GATE, (s, q, z, rho, m, r)
        assert 64 <= n <= 4096


def test_engine_near_caustics_against_oracle(emu, oracle):
    import pins
    rng = np.random.default_rng(21)
    for s, q, rho in [(1.0, 1e-3, 1e-3), (0.6, 1e-5, 2e-4), (1.6, 2e-2, 3e-3)]:
        ca = pins.caustic(s, q, 1024)
        z = ca[rng.integers(0, ca.size, 12)] + rho * rng.uniform(0, 2, 12) * np.exp(
            2j * np.pi * rng.uniform(0, 1, 12))
        for zz in z:
            m, e, n, f = emu["finite"](s, q, zz.real, zz.imag, rho, 1e-4, 0)
            r = oracle.finite_mag(s, q, [zz.real], [zz.imag], rho, oracle.JUDGE_TOL,
                                  oracle.judge_cfg())[0][0]
            assert abs(m / r - 1) <= GATE, (s, q, zz, rho, m, r)


def test_engine_follows_serial_sampler(emu, oracle):
    """Same schedule as the oracle's serial run of the paper's sampler at half
    the stated tolerance: equal magnification to rounding on most sources and
    mostly the same number of samples."""
    import pins
    rng = np.random.default_rng(5)
    s, q, rho = 1.0, 1e-3, 1e-3
    ca = pins.caustic(s, q, 1024)
    z = ca[rng.integers(0, ca.size, 24)] + rho * rng.uniform(0, 2, 24) * np.exp(
        2j * np.pi * rng.uniform(0, 1, 24))
    same_n = 0
    rels = []
    for zz in z:
        m, e, n, f = emu["finite"](s, q, zz.real, zz.imag, rho, 1e-4, 0)
        rm, re_, rn, rf = oracle.finite_mag(s, q, [zz.real], [zz.imag], rho, 5e-5)
        rels.append(abs(m / rm[0] - 1))
        same_n += n == rn[0]
    print("median rel", np.median(rels), "same sample count", same_n, "of", len(z))
    assert np.median(rels) < 1e-8
    assert same_n >= 0.75 * len(z)


def test_point_classification_against_oracle(emu, oracle):
    rng = np.random.default_rng(8)
    for _ in range(300):
        s = 10 ** rng.uniform(-0.5, 0.5)
        q = 10 ** rng.uniform(-6, -1)
        x, y = rng.uniform(-1.5, 1.5, 2)
        m, n, f = emu["point"](s, q, x, y)
        rm, rn, rf = oracle.point_mag(s, q, [x], [y])
        if (f | rf[0]) & 32:
            continue
        assert n == rn[0]
        assert abs(m / rm[0] - 1) < 1e-10
