"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Gate (stated by the project): relative magnification error <= 1e-4 against
the oracle run at a tight tolerance, image counts equal exactly except where
either side flags a near-degenerate ghost/real decision.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

GATE = 1e-4


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2501_03322_amd import twk
    c = twk.Context(0)
    yield c
    c.close()


def _np(t):
    return t.cpu().numpy()


def _log(msg):
    print(msg, flush=True)


FS_CASES = [
    # (s, q, zeta, rho)  caustic crossings, cusps, planetary and central caustics
    (1.0, 0.1, 0.2 + 0.2j, 0.1),
    (1.0, 1e-2, 0.02 + 0.01j, 0.02),
    (0.8, 5e-3, -0.45 + 0.12j, 0.03),
    (1.0, 1e-3, 0.05 + 0.01j, 1e-3),
    (0.5, 1e-6, -1.49981640625 + 0.0035j, 1e-4),
    (3.0, 1e-4, 2.666 + 0.0005j, 1e-4),
    (0.5, 1e-4, -1.5 + 0.035j, 5e-5),
    (1.0, 1e-4, 0.0 + 0.0j, 1e-3),
    (0.5, 1e-6, -1.49998960 - 0.0035j, 1e-4),
    (0.5, 1e-6, -1.49993410 - 0.0035j, 1e-4),
    (2.0, 1e-9, 1.5 + 0.01j, 1e-3),
]


def test_point_mag_parity(ctx, oracle):
    rng = np.random.default_rng(7)
    for trial in range(6):
        s = 10 ** rng.uniform(-0.5, 0.5)
        q = 10 ** rng.uniform(-6, -1)
        zx = rng.uniform(-1.5, 1.5, 4000)
        zy = rng.uniform(-1.5, 1.5, 4000)
        _log(f"point_mag s={s:.4g} q={q:.3g}")
        mag, nimg, fl = ctx.point_mag(s, q, zx, zy)
        rmag, rn, rfl = oracle.point_mag(s, q, zx, zy)
        mag, nimg, fl = _np(mag), _np(nimg), _np(fl)
        ok = ((fl & 32) == 0) & ((rfl & 32) == 0)
        assert np.array_equal(nimg[ok], rn[ok])
        np.testing.assert_allclose(mag[ok], rmag[ok], rtol=1e-10)


def test_point_mag_above_one_launch(ctx):
    """More point sources than one launch of a one-lane-per-source kernel
    takes (2^30 + 4000): the call splits into launches, and the tail of the
    second launch equals the same sources in a call of their own."""
    import torch
    n = (1 << 30) + 4000
    _log(f"point mag, n = {n}")
    dev = torch.device("cuda", 0)
    zx = torch.remainder(torch.arange(n, dtype=torch.float64, device=dev), 997.0) * 1e-3 - 0.5
    zy = torch.full((n,), 0.013, dtype=torch.float64, device=dev)
    mag, nimg, fl = ctx.point_mag(1.0, 1e-2, zx, zy)
    torch.cuda.synchronize()
    for lo in (0, (1 << 30) - 2000, n - 3000):
        m2, n2, f2 = ctx.point_mag(1.0, 1e-2, zx[lo:lo + 3000].clone(), zy[lo:lo + 3000].clone())
        assert torch.equal(mag[lo:lo + 3000], m2) and torch.equal(nimg[lo:lo + 3000], n2), lo
    assert bool(torch.all(mag >= 1.0 - 1e-12))
    del zx, zy, mag, nimg, fl
    torch.cuda.empty_cache()


@pytest.mark.parametrize("mode", [0, 1])
def test_finite_mag_cases(ctx, oracle, mode):
    for (s, q, z, rho) in FS_CASES:
        _log(f"finite case s={s} q={q} z={z} rho={rho} mode={mode}")
        mag, err, ns, fl = ctx.finite_mag(s, q, [z.real], [z.imag], rho, 1e-4, mode | 8)
        rm, re_, rn, rf = oracle.finite_mag(s, q, [z.real], [z.imag], rho, oracle.TIGHT_TOL,
                                            oracle.tight_cfg())
        m = _np(mag)[0]
        assert abs(m / rm[0] - 1) <= GATE, (s, q, z, rho, m, rm[0])
        assert _np(ns)[0] >= 64


def _near_caustic_sources(s, q, rho, n, seed):
    import pins
    rng = np.random.default_rng(seed)
    ca = pins.caustic(s, q, 2048)
    pick = ca[rng.integers(0, ca.size, n)]
    off = rho * rng.uniform(0, 2.0, n) * np.exp(2j * np.pi * rng.uniform(0, 1, n))
    z = pick + off
    return z.real.copy(), z.imag.copy()


@pytest.mark.parametrize("lens", [(1.0, 1e-3, 1e-3), (0.7, 1e-4, 3e-4), (1.3, 3e-2, 5e-3),
                                  (0.5, 1e-6, 1e-4), (2.5, 1e-5, 2e-4)])
def test_finite_mag_near_caustics(ctx, oracle, lens):
    s, q, rho = lens
    zx, zy = _near_caustic_sources(s, q, rho, 96, seed=int(1e6 * q) % 1000 + 11)
    for mode in (0, 1):
        _log(f"near caustic s={s} q={q} rho={rho} mode={mode}")
        mag, err, ns, fl = ctx.finite_mag(s, q, zx, zy, rho, 1e-4, mode | 8)
        rm, re_, rn, rf = oracle.finite_mag(s, q, zx, zy, rho, oracle.TIGHT_TOL, oracle.tight_cfg())
        rel = np.abs(_np(mag) / rm - 1)
        assert rel.max() <= GATE, (lens, mode, rel.max(), int(rel.argmax()))


def test_sample_cap(ctx, oracle):
    """A tolerance that 4096 samples cannot meet: the refinement ends at the
    cap, the result carries the cap flag, its sample count and a finite error
    estimate above the requested one, and the capped value still agrees with
    the oracle's tight value.  The oracle's serial run of the same sampler
    ends at the cap as well."""
    from paper_2501_03322_amd import twk
    s, q, rho, tol = 1.0, 1e-3, 1e-3, 1e-12
    zx, zy = _near_caustic_sources(s, q, rho, 8, seed=21)
    rm = oracle.finite_mag(s, q, zx, zy, rho, oracle.TIGHT_TOL, oracle.tight_cfg())[0]
    om, oe, on, of = oracle.finite_mag(s, q, zx, zy, rho, tol)
    assert np.all(of & oracle.FLAG_CAP) and np.all(on <= 4096) and np.all(on > 4096 - 64)
    for mode in (twk.MODE_FP64, twk.MODE_MIXED):
        _log(f"sample cap mode={mode}")
        mag, err, ns, fl = [_np(t) for t in ctx.finite_mag(s, q, zx, zy, rho, tol,
                                                           mode | twk.MODE_ALL_FS)]
        assert np.all(fl & twk.FLAG_CAP), (mode, fl)
        assert np.all(ns <= 4096) and np.all(ns > 4096 - 64), (mode, ns)
        assert np.all(np.isfinite(err)) and np.all(err > tol * mag), (mode, err / mag)
        rel = np.abs(mag / rm - 1)
        assert rel.max() <= GATE, (mode, rel.max())
        if mode == twk.MODE_FP64:  # the same sampler, stopped at the same cap
            assert np.abs(mag / om - 1).max() <= 1e-6


def test_finite_mag_each_time_varying_lens(ctx, oracle):
    """Per-element lenses: a binary in orbital motion (separation and axis
    angle changing linearly in time) crossing its caustic, every epoch
    against the oracle run with that epoch's lens; the same call with one
    lens for all elements equals twk_finite_mag bit for bit; an element with
    an invalid lens is flagged non-finite without disturbing the others."""
    import torch
    from paper_2501_03322_amd import twk
    tau = np.linspace(-1.2, 1.2, 240)
    s = 1.0 + 0.05 * tau           # ds/dt
    alpha = 0.6 + 0.3 * tau        # d(alpha)/dt: the binary axis rotates
    q = np.full_like(tau, 2e-3)
    rho = np.full_like(tau, 3e-3)
    u0 = 0.02
    z = np.array([complex(*[v[0] for v in oracle.trajectory(u0, a, [t])]) for a, t in zip(alpha, tau)])
    zx, zy = z.real.copy(), z.imag.copy()
    rm = np.array([oracle.finite_mag(s[i], q[i], [zx[i]], [zy[i]], rho[i], oracle.TIGHT_TOL,
                                     oracle.tight_cfg())[0][0] for i in range(tau.size)])
    for mode in (twk.MODE_FP64, twk.MODE_MIXED, twk.MODE_MIXED | twk.MODE_ALL_FS):
        _log(f"time-varying lens, mode={mode}")
        mag, err, ns, fl = [_np(t) for t in ctx.finite_mag_each(s, q, zx, zy, rho, 1e-4, mode)]
        rel = np.abs(mag / rm - 1)
        assert rel.max() <= GATE, (mode, rel.max(), int(rel.argmax()))
        assert np.any((fl & twk.FLAG_POINT) == 0)  # contours were needed
        if not mode & twk.MODE_ALL_FS:
            assert np.any((fl & twk.FLAG_POINT) != 0)  # and point values sufficed elsewhere
    # one lens for all: identical to the scalar entry point
    one = np.full_like(tau, 1.0)
    a = [_np(t).copy() for t in ctx.finite_mag_each(one, q, zx, zy, rho, 1e-4, twk.MODE_MIXED)]
    b = [_np(t).copy() for t in ctx.finite_mag(1.0, 2e-3, zx, zy, 3e-3, 1e-4, twk.MODE_MIXED)]
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    # invalid elements
    s_bad = s.copy()
    s_bad[5] = -1.0
    rho_bad = rho.copy()
    rho_bad[9] = np.nan
    mag, err, ns, fl = [_np(t) for t in ctx.finite_mag_each(s_bad, q, zx, zy, rho_bad, 1e-4,
                                                            twk.MODE_MIXED)]
    for i in (5, 9):
        assert np.isnan(mag[i]) and (fl[i] & twk.FLAG_NONFINITE)
    ok = np.ones(tau.size, bool)
    ok[[5, 9]] = False
    assert np.abs(mag[ok] / rm[ok] - 1).max() <= GATE
    with pytest.raises(ValueError):
        ctx.finite_mag_each(s[:10], q, zx, zy, rho, 1e-4)
    torch.cuda.synchronize()


def test_fp64_engine_follows_paper_sampler(ctx, oracle):
    """The FP64 engine and the oracle's serial run of the same sampler
    (64 initial, 64 per round, cap 4096) agree closely, and mostly use the
    same number of samples.  The engine stops at the stated tolerance, halved
    once a contour crosses a caustic; the oracle runs with the same rule."""
    s, q, rho = 1.0, 1e-3, 1e-3
    zx, zy = _near_caustic_sources(s, q, rho, 128, seed=5)
    mag, err, ns, fl = ctx.finite_mag(s, q, zx, zy, rho, 1e-4, 8)
    rm, re_, rn, rf = oracle.finite_mag(s, q, zx, zy, rho, 1e-4, oracle.cfg(1e-4, cross_tol=0.5))
    rel = np.abs(_np(mag) / rm - 1)
    assert np.median(rel) < 1e-8
    assert np.mean(_np(ns) == rn) > 0.75


def test_lightcurve_single(ctx, oracle):
    """One lens, 1000 epochs (s=1, q=1e-3, rho=1e-3, u0=0.01, alpha=0.5): the
    full path (point-source test + contour) on every epoch."""
    from paper_2501_03322_amd import inputs
    c = inputs.single_curve()
    zx, zy = oracle.trajectory(c.u0[0], c.alpha[0], c.tau)
    rm, re_, rn, rf = oracle.finite_mag(c.s[0], c.q[0], zx, zy, c.rho[0], oracle.TIGHT_TOL,
                                        oracle.tight_cfg())
    for mode in (0, 1):
        _log(f"single light curve mode={mode}")
        mag, err, ns, fl = ctx.lightcurves(c.s, c.q, c.u0, c.alpha, c.rho, c.tau, 1e-4, mode)
        rel = np.abs(_np(mag) / rm - 1)
        assert rel.max() <= GATE, (mode, rel.max(), int(rel.argmax()))
        ps = (_np(fl) & 1) != 0
        dec = np.array([oracle.ps_adequate(c.s[0], c.q[0], complex(x, y), c.rho[0], 1e-4)[0]
                        for x, y in zip(zx, zy)])
        assert np.array_equal(ps, dec)


@pytest.mark.parametrize("nepochs", [1, 3, 6, 101])
def test_lightcurve_ragged_runs(ctx, oracle, nepochs):
    """Epoch counts that are not a multiple of the point-source pass's run of
    consecutive epochs (and shorter than one run): every epoch against the
    oracle, and the point-source decisions equal to the oracle's."""
    from paper_2501_03322_amd import inputs
    c = inputs.batched_curves(nsets=3, nepochs=nepochs, seed=7)
    for mode in (0, 1):
        _log(f"ragged light curves: 3 x {nepochs}, mode={mode}")
        mag, err, ns, fl = [_np(t) for t in ctx.lightcurves(c.s, c.q, c.u0, c.alpha, c.rho, c.tau,
                                                            1e-4, mode)]
        assert mag.shape == (3 * nepochs,)
        for k in range(3):
            zx, zy = oracle.trajectory(c.u0[k], c.alpha[k], c.tau)
            rm = oracle.finite_mag(c.s[k], c.q[k], zx, zy, c.rho[k], oracle.TIGHT_TOL,
                                   oracle.tight_cfg())[0]
            got = mag[k * nepochs:(k + 1) * nepochs]
            rel = np.abs(got / rm - 1)
            assert rel.max() <= GATE, (mode, k, rel.max(), int(rel.argmax()))
            ps = (fl[k * nepochs:(k + 1) * nepochs] & 1) != 0
            dec = np.array([oracle.ps_adequate(c.s[k], c.q[k], complex(x, y), c.rho[k], 1e-4)[0]
                            for x, y in zip(zx, zy)])
            assert np.array_equal(ps, dec), (mode, k)


def test_lightcurve_batch_sampled(ctx, oracle):
    """The full fit-style batch (1024 sets x 2000 epochs) in one call, checked
    on a stratified sample of epochs against the oracle one by one."""
    from paper_2501_03322_amd import inputs
    c = inputs.batched_curves()
    _log("batch: 1024 x 2000")
    mag, err, ns, fl = ctx.lightcurves(c.s, c.q, c.u0, c.alpha, c.rho, c.tau, 1e-4, 1)
    mag, ns, fl = _np(mag), _np(ns), _np(fl)
    assert np.all(np.isfinite(mag)) and np.all(mag >= 1.0 - 1e-9)
    fs = np.nonzero((fl & 1) == 0)[0]
    pt = np.nonzero((fl & 1) != 0)[0]
    rng = np.random.default_rng(3)
    pick = np.concatenate([rng.choice(fs, min(240, fs.size), replace=False),
                           rng.choice(pt, min(160, pt.size), replace=False)])
    worst = 0.0
    for i in pick:
        k, j = divmod(int(i), c.nepochs)
        zx, zy = oracle.trajectory(c.u0[k], c.alpha[k], c.tau[j:j + 1])
        rm, _, _, _ = oracle.finite_mag(c.s[k], c.q[k], zx, zy, c.rho[k], oracle.TIGHT_TOL,
                                        oracle.tight_cfg())
        worst = max(worst, abs(mag[i] / rm[0] - 1))
        assert abs(mag[i] / rm[0] - 1) <= GATE, (i, k, j, mag[i], rm[0])
    _log(f"batch sampled worst rel {worst:.3g} fs={fs.size}")


def test_edge_cases(ctx, oracle):
    import torch
    from paper_2501_03322_amd import twk
    # empty input
    out = ctx.finite_mag(1.0, 1e-3, [], [], 1e-3, 1e-4)
    assert out[0].numel() == 0
    # non-finite inputs are flagged and return NaN
    mag, err, ns, fl = ctx.finite_mag(1.0, 1e-3, [np.nan, 0.1], [0.0, 0.0], 1e-3, 1e-4)
    mag, fl = _np(mag), _np(fl)
    assert np.isnan(mag[0]) and (fl[0] & twk.FLAG_NONFINITE)
    assert np.isfinite(mag[1])
    # invalid arguments
    for bad in [dict(s=-1.0), dict(q=0.0), dict(rho=0.0), dict(tol=-1.0)]:
        a = dict(s=1.0, q=1e-3, rho=1e-3, tol=1e-4)
        a.update(bad)
        with pytest.raises(twk.TwkError):
            ctx.finite_mag(a["s"], a["q"], [0.1], [0.0], a["rho"], a["tol"])
    with pytest.raises(twk.TwkError):
        ctx.finite_mag(1.0, 1e-3, [0.1], [0.0], 1e-3, 1e-4, mode=1 << 20)
    # extreme lenses of the robust domain (0.1 <= s <= 10, q >= 1e-9)
    for (s, q, z, rho) in [(0.1, 1e-9, 0.01 + 0.001j, 1e-3), (10.0, 1e-9, 9.9 + 0.0j, 1e-3),
                           (0.1, 0.5, 0.0 + 0.0j, 1e-2), (10.0, 1.0, 4.9 + 0.01j, 1e-2)]:
        mag, err, ns, fl = ctx.finite_mag(s, q, [z.real], [z.imag], rho, 1e-4, 8)
        rm = oracle.finite_mag(s, q, [z.real], [z.imag], rho, oracle.TIGHT_TOL, oracle.tight_cfg())[0]
        assert abs(_np(mag)[0] / rm[0] - 1) <= GATE, (s, q, z)
    torch.cuda.synchronize()


def test_deterministic(ctx):
    s, q, rho = 1.0, 1e-3, 1e-3
    zx, zy = _near_caustic_sources(s, q, rho, 64, seed=9)
    a = [_np(t).copy() for t in ctx.finite_mag(s, q, zx, zy, rho, 1e-4, 9)]
    b = [_np(t).copy() for t in ctx.finite_mag(s, q, zx, zy, rho, 1e-4, 9)]
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_limb_darkened_lightcurves(ctx, oracle):
    """Linear limb darkening over 10 equal-area annuli (large limb-darkened
    batch's parameter ranges): sampled epochs against the oracle's annulus
    combination of tight-tolerance uniform-disk values."""
    from paper_2501_03322_amd import inputs
    c = inputs.large_ld_curves(nsets=48, nepochs=400, seed=4)
    _log("limb darkened: 48 x 400, 10 annuli")
    mag, err, ns, fl = ctx.lightcurves(c.s, c.q, c.u0, c.alpha, c.rho, c.tau, 1e-4, 1,
                                       gamma=c.gamma, n_annuli=10)
    mag, fl = _np(mag), _np(fl)
    assert np.all(np.isfinite(mag))
    fs = np.nonzero((fl & 1) == 0)[0]
    pt = np.nonzero((fl & 1) != 0)[0]
    rng = np.random.default_rng(4)
    pick = np.concatenate([rng.choice(fs, min(40, fs.size), replace=False),
                           rng.choice(pt, min(20, pt.size), replace=False)])
    for i in pick:
        k, j = divmod(int(i), c.nepochs)
        zx, zy = oracle.trajectory(c.u0[k], c.alpha[k], c.tau[j:j + 1])
        mu_k = [oracle.finite_mag(c.s[k], c.q[k], zx, zy, c.rho[k] * np.sqrt(a / 10), oracle.TIGHT_TOL,
                                  oracle.tight_cfg())[0][0] for a in range(1, 11)]
        ref = oracle.ld_combine(c.gamma[k], mu_k)
        assert abs(mag[i] / ref - 1) <= GATE, (i, k, j, mag[i], ref)


def test_magnification_map(ctx, oracle):
    """Magnification map of the central caustic (s=0.9, q=1e-4, rho=1e-3):
    a 64 x 64 map checked pixel by pixel on a sample, and the full 2048 x
    2048 map in the launch configuration of a map run, checked on sampled
    pixels."""
    from paper_2501_03322_amd import inputs
    s, q, rho = inputs.MAP_S, inputs.MAP_Q, inputs.MAP_RHO
    for n, nsample in [(64, 60), (2048, 60)]:
        _log(f"map {n} x {n}")
        mag, err, ns, fl = ctx.mag_map(s, q, rho, inputs.MAP_CENTRE, inputs.MAP_WIDTH,
                                       inputs.MAP_WIDTH, n, n, 1e-4, 1)
        mag, fl = _np(mag), _np(fl)
        assert np.all(np.isfinite(mag))
        x, y = inputs.map_pixels(n)
        rng = np.random.default_rng(n)
        fs = np.nonzero((fl & 1) == 0)[0]
        pick = np.concatenate([rng.choice(fs, min(nsample, fs.size), replace=False),
                               rng.choice(mag.size, nsample // 2, replace=False)])
        for p in pick:
            iy, ix = divmod(int(p), n)
            rm = oracle.finite_mag(s, q, [x[ix]], [y[iy]], rho, oracle.TIGHT_TOL, oracle.tight_cfg())[0][0]
            assert abs(mag[p] / rm - 1) <= GATE, (n, ix, iy, mag[p], rm)


def test_large_limb_darkened_batch_full_size(ctx, oracle):
    """The high-cadence limb-darkened batch at its full size (16384 sets x
    8000 epochs, 10 annuli) in one call on the headline path (learned budget
    + mixed precision, the committed weights when present) at the launch
    tuning the benchmark's autotuner picks on this chip (LDS capacity 128,
    the most resident waves, budget shift 0): every value finite, and
    sampled epochs against the oracle's annulus combination."""
    import os
    import time
    from paper_2501_03322_amd import inputs, twk
    c = inputs.large_ld_curves()
    n = c.nsets * c.nepochs
    mode = twk.MODE_MIXED
    wpath = os.path.join(os.path.dirname(twk.__file__), "weights", "mlp_budget.bin")
    if os.path.exists(wpath):
        ctx.mlp_load(wpath)
        mode |= twk.MODE_MLP
    saved = ctx.get_tuning()
    mx = 1
    for w in range(2, 33):
        try:
            ctx.set_tuning(lds_cap=128, waves_per_cu=w, budget_shift=0.0)
            mx = w
        except twk.TwkError:
            break
    ctx.set_tuning(lds_cap=128, waves_per_cu=mx, budget_shift=0.0)
    try:
        _log(f"limb darkened full size: {c.nsets} x {c.nepochs} x 10 annuli, mode {mode}")
        t0 = time.perf_counter()
        mag, err, ns, fl = ctx.lightcurves(c.s, c.q, c.u0, c.alpha, c.rho, c.tau, 1e-4, mode,
                                           gamma=c.gamma, n_annuli=10)
        ctx.sync()
        _log(f"  call done in {time.perf_counter() - t0:.1f} s; stats {ctx.stats()}")
        mag, fl = _np(mag), _np(fl)
        del err, ns
    finally:
        ctx.set_tuning(**saved.as_dict())
    assert mag.shape == (n,) and np.all(np.isfinite(mag))
    fs = np.nonzero((fl & 1) == 0)[0]
    pt = np.nonzero((fl & 1) != 0)[0]
    _log(f"  contour epochs {fs.size} of {n}")
    rng = np.random.default_rng(16384)
    pick = np.concatenate([rng.choice(fs, min(12, fs.size), replace=False),
                           rng.choice(pt, min(6, pt.size), replace=False)])
    for i in pick:
        k, j = divmod(int(i), c.nepochs)
        zx, zy = oracle.trajectory(c.u0[k], c.alpha[k], c.tau[j:j + 1])
        mu_k = [oracle.finite_mag(c.s[k], c.q[k], zx, zy, c.rho[k] * np.sqrt(a / 10), oracle.TIGHT_TOL,
                                  oracle.tight_cfg())[0][0] for a in range(1, 11)]
        ref = oracle.ld_combine(c.gamma[k], mu_k)
        assert abs(mag[i] / ref - 1) <= GATE, (i, k, j, mag[i], ref)


def test_magnification_map_mixed_vs_fp64(ctx):
    """The 2048 x 2048 central-caustic map on the mixed path against the FP64
    path, pixel by pixel: both meet the tolerance against the exact value, so
    they differ by at most twice it; the same pixels take the point value;
    the distribution of the difference is reported."""
    from paper_2501_03322_amd import inputs
    s, q, rho = inputs.MAP_S, inputs.MAP_Q, inputs.MAP_RHO
    n = 2048
    res = {}
    for mode in (0, 1):
        mag, err, ns, fl = ctx.mag_map(s, q, rho, inputs.MAP_CENTRE, inputs.MAP_WIDTH,
                                       inputs.MAP_WIDTH, n, n, 1e-4, mode)
        res[mode] = (_np(mag), _np(fl))
    m64, f64 = res[0]
    m32, f32 = res[1]
    assert np.all(np.isfinite(m32)) and np.all(np.isfinite(m64))
    assert np.array_equal(f64 & 1, f32 & 1)
    rel = np.abs(m32 / m64 - 1)
    fs = (f64 & 1) == 0
    _log(f"map mixed vs FP64: contour pixels {int(fs.sum())}, rel. difference median "
         f"{np.median(rel[fs]):.2e}, 99.9% {np.quantile(rel[fs], 0.999):.2e}, max {rel.max():.2e}")
    assert rel.max() <= 2 * GATE
