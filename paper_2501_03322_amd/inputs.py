"""Seeded synthetic workloads shared by the tests, the benchmark and the
oracle runs.  This module only draws parameters; it holds none of the
method's arithmetic (source positions along trajectories are computed by the
GPU path and by the oracle separately).

Draw order per configuration is fixed: numpy's PCG64 generator seeded as
stated, one vectorised draw per parameter in the order listed.
"""
from dataclasses import dataclass
from typing import Optional

import numpy as np


@dataclass
class LightCurveSet:
    s: np.ndarray
    q: np.ndarray
    u0: np.ndarray
    alpha: np.ndarray
    rho: np.ndarray
    tau: np.ndarray
    gamma: Optional[np.ndarray] = None
    n_annuli: int = 1
    tol: float = 1e-4

    @property
    def nsets(self):
        return self.s.size

    @property
    def nepochs(self):
        return self.tau.size

    def subset(self, idx):
        idx = np.asarray(idx)
        g = None if self.gamma is None else self.gamma[idx]
        return LightCurveSet(self.s[idx], self.q[idx], self.u0[idx], self.alpha[idx], self.rho[idx],
                             self.tau, g, self.n_annuli, self.tol)


def single_curve():
    """One lens (s=1, q=1e-3), uniform source rho=1e-3, u0=0.01, alpha=0.5 rad,
    1000 epochs evenly spaced over tau in [-2, 2], tol 1e-4."""
    one = lambda v: np.array([v], dtype=np.float64)
    return LightCurveSet(one(1.0), one(1e-3), one(0.01), one(0.5), one(1e-3),
                         np.linspace(-2.0, 2.0, 1000))


def batched_curves(nsets=1024, nepochs=2000, seed=1):
    """Fit-style batch: log10 s ~ U[-0.5,0.5], log10 q ~ U[-5,-1],
    alpha ~ U[0,2pi), u0 ~ U[-0.1,0.1], log10 rho ~ U[-4,-2]; tau over
    [-1.5, 1.5]; uniform source; tol 1e-4."""
    rng = np.random.default_rng(seed)
    s = 10.0 ** rng.uniform(-0.5, 0.5, nsets)
    q = 10.0 ** rng.uniform(-5.0, -1.0, nsets)
    alpha = rng.uniform(0.0, 2.0 * np.pi, nsets)
    u0 = rng.uniform(-0.1, 0.1, nsets)
    rho = 10.0 ** rng.uniform(-4.0, -2.0, nsets)
    return LightCurveSet(s, q, u0, alpha, rho, np.linspace(-1.5, 1.5, nepochs))


def training_curves(nsets=1000, nepochs=2000, seed=2):
    """Training sample for the learned budget predictor: drawn as the batch."""
    return batched_curves(nsets, nepochs, seed)


def evaluation_curves(nsets=1024, nepochs=4000, seed=3):
    """Held-out evaluation batch for the learned predictor."""
    return batched_curves(nsets, nepochs, seed)


def large_ld_curves(nsets=16384, nepochs=8000, seed=4, n_annuli=10):
    """High-cadence large batch with linear limb darkening: s, q, alpha, u0,
    rho, Gamma drawn in that order with log10 q ~ U[-6,-1], log10 rho ~
    U[-4,-2.5], Gamma ~ U[0.3,0.6] and s, alpha, u0 as in the batch."""
    rng = np.random.default_rng(seed)
    s = 10.0 ** rng.uniform(-0.5, 0.5, nsets)
    q = 10.0 ** rng.uniform(-6.0, -1.0, nsets)
    alpha = rng.uniform(0.0, 2.0 * np.pi, nsets)
    u0 = rng.uniform(-0.1, 0.1, nsets)
    rho = 10.0 ** rng.uniform(-4.0, -2.5, nsets)
    gamma = rng.uniform(0.3, 0.6, nsets)
    return LightCurveSet(s, q, u0, alpha, rho, np.linspace(-1.5, 1.5, nepochs), gamma, n_annuli)


def wide_training_curves(nsets=1000, nepochs=2000, seed=5):
    """Training batch over the high-cadence batch's parameter ranges: s, q,
    alpha, u0, rho drawn in that order with log10 q ~ U[-6,-1], log10 rho ~
    U[-4,-2.5] and s, alpha, u0 as in the batch; uniform source (the learned
    features of a limb-darkened epoch are those of its outer disk)."""
    rng = np.random.default_rng(seed)
    s = 10.0 ** rng.uniform(-0.5, 0.5, nsets)
    q = 10.0 ** rng.uniform(-6.0, -1.0, nsets)
    alpha = rng.uniform(0.0, 2.0 * np.pi, nsets)
    u0 = rng.uniform(-0.1, 0.1, nsets)
    rho = 10.0 ** rng.uniform(-4.0, -2.5, nsets)
    return LightCurveSet(s, q, u0, alpha, rho, np.linspace(-1.5, 1.5, nepochs))


# Magnification map: s=0.9, q=1e-4, rho=1e-3 on a 2048 x 2048 grid over a
# 0.2 x 0.2 box centred on the central caustic.  The centre is the midpoint
# of the central caustic's x-extent in the centre-of-mass frame, computed
# once from the caustic of this lens and recorded here.
MAP_S, MAP_Q, MAP_RHO = 0.9, 1e-4, 1e-3
MAP_CENTRE = (3.5013e-3, 0.0)
MAP_WIDTH = 0.2


def map_pixels(n=2048, centre=MAP_CENTRE, width=MAP_WIDTH):
    """Pixel-centre coordinates (x, y) of an n x n map."""
    cx, cy = centre
    x = cx - width / 2 + (np.arange(n) + 0.5) * width / n
    y = cy - width / 2 + (np.arange(n) + 0.5) * width / n
    return x, y


def random_sources(n, seed, box=1.6, logq=(-6.0, -1.0), logs=(-0.5, 0.5), logrho=(-4.0, -2.0)):
    """Independent random (s, q, zeta, rho) draws for parity tests."""
    rng = np.random.default_rng(seed)
    s = 10.0 ** rng.uniform(*logs, n)
    q = 10.0 ** rng.uniform(*logq, n)
    zx = rng.uniform(-box, box, n)
    zy = rng.uniform(-box, box, n)
    rho = 10.0 ** rng.uniform(*logrho, n)
    return s, q, zx, zy, rho
