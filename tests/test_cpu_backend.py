"""The multi-core CPU backend of the method (paper_2501_03322_amd/cpu,
include/twk_cpu.h; the CPU version of the paper's Sec. 4.5) against the FP64
oracle at its tight tolerance: the single light curve (every epoch), the
paper's worked sources, sources near caustics, and subsamples of the
uniform and the limb-darkened light-curve batches (the epochs with the
largest error estimate and random ones).  CPU only."""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

GATE = 1e-4


@pytest.fixture(scope="module")
def cpu():
    from paper_2501_03322_amd import build, cpu as backend
    import os
    if not os.path.exists(backend.LIB_PATH):
        build.build_cpu()
    backend.load()
    return backend


def _tight(oracle, s, q, z, rho):
    return oracle.finite_mag(s, q, [z.real], [z.imag], rho, oracle.TIGHT_TOL, oracle.tight_cfg())[0][0]


def test_single_curve_every_epoch(cpu, oracle):
    from paper_2501_03322_amd import inputs
    c = inputs.single_curve()
    mag, err, ns, fl = cpu.lightcurves(c.s, c.q, c.u0, c.alpha, c.rho, c.tau, 1e-4, threads=4)
    zx, zy = oracle.trajectory(c.u0[0], c.alpha[0], c.tau)
    rm = oracle.finite_mag(c.s[0], c.q[0], zx, zy, c.rho[0], oracle.TIGHT_TOL, oracle.tight_cfg())[0]
    assert np.abs(mag / rm - 1).max() <= GATE
    ok = np.array([oracle.ps_adequate(c.s[0], c.q[0], complex(x, y), c.rho[0], 1e-4)[0]
                   for x, y in zip(zx, zy)])
    assert np.array_equal(ok, (fl & 1) != 0)
    assert np.all(ns[(fl & 1) == 0] >= 64) and np.all(ns[(fl & 1) != 0] == 0)


def test_paper_sources_and_near_caustics(cpu, oracle):
    import pins
    cases = [(1.0, 0.1, 0.2 + 0.2j, 0.1), (0.8, 5e-3, -0.45 + 0.12j, 0.03),
             (0.5, 1e-6, -1.49981640625 + 0.0035j, 1e-4), (3.0, 1e-4, 2.666 + 0.0005j, 1e-4),
             (0.5, 1e-6, -1.49998960 - 0.0035j, 1e-4), (0.5, 1e-6, -1.49993410 - 0.0035j, 1e-4),
             (2.0, 1e-9, 1.5 + 0.01j, 1e-3)]
    for (s, q, z, rho) in cases:
        m = cpu.finite_mag(s, q, [z.real], [z.imag], rho, GATE, all_fs=True)[0][0]
        assert abs(m / _tight(oracle, s, q, z, rho) - 1) <= GATE, (s, q, z, rho)
    rng = np.random.default_rng(4)
    for (s, q, rho) in [(1.0, 1e-3, 1e-3), (0.7, 1e-4, 3e-4), (1.3, 3e-2, 5e-3)]:
        ca = pins.caustic(s, q, 1024)
        z = ca[rng.integers(0, ca.size, 48)] + rho * rng.uniform(0, 2, 48) * np.exp(
            2j * np.pi * rng.uniform(0, 1, 48))
        m = cpu.finite_mag(s, q, z.real, z.imag, rho, GATE, all_fs=True, threads=4)[0]
        with ThreadPoolExecutor(8) as ex:
            r = np.array(list(ex.map(lambda zz: _tight(oracle, s, q, zz, rho), z)))
        assert np.abs(m / r - 1).max() <= GATE, (s, q, rho)


@pytest.mark.parametrize("batch", ["uniform", "limb_darkened"])
def test_batch_subsample(cpu, oracle, batch):
    from paper_2501_03322_amd import inputs
    c = inputs.batched_curves() if batch == "uniform" else inputs.large_ld_curves()
    sub = c.subset(np.random.default_rng(1).choice(c.nsets, 4 if batch == "uniform" else 2, replace=False))
    mag, err, ns, fl = cpu.lightcurves(sub.s, sub.q, sub.u0, sub.alpha, sub.rho, sub.tau, sub.tol,
                                       gamma=sub.gamma, n_annuli=sub.n_annuli, threads=4)
    assert np.all(np.isfinite(mag))
    fs = np.nonzero((fl & 1) == 0)[0]
    pick = np.concatenate([fs[np.argsort(err[fs] / mag[fs])[-16:]],
                           np.random.default_rng(2).choice(mag.size, 16, replace=False)])

    def one(i):
        k, j = divmod(int(i), sub.nepochs)
        zx, zy = oracle.trajectory(sub.u0[k], sub.alpha[k], sub.tau[j:j + 1])
        z = complex(zx[0], zy[0])
        if sub.gamma is None:
            return _tight(oracle, sub.s[k], sub.q[k], z, sub.rho[k])
        mk = [_tight(oracle, sub.s[k], sub.q[k], z, sub.rho[k] * np.sqrt(a / sub.n_annuli))
              for a in range(1, sub.n_annuli + 1)]
        return oracle.ld_combine(sub.gamma[k], np.array(mk))
    with ThreadPoolExecutor(8) as ex:
        r = np.array(list(ex.map(one, pick)))
    assert np.abs(mag[pick] / r - 1).max() <= GATE


def test_bad_arguments(cpu):
    with pytest.raises(ValueError):
        cpu.finite_mag(-1.0, 1e-3, [0.1], [0.0], 1e-3, 1e-4)
    with pytest.raises(ValueError):
        cpu.lightcurves([1.0], [1e-3], [0.0], [0.0], [1e-3], [0.0], 1e-4, gamma=None, n_annuli=3)
    m = cpu.finite_mag(1.0, 1e-3, [np.nan], [0.0], 1e-3, 1e-4)
    assert np.isnan(m[0][0]) and m[3][0] == 16
