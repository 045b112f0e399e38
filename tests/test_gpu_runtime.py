"""Launch runtime on the GPU: graph capture and replay, launch tuning and
the autotuner.  None of them may change a result: replays, persistent grid
sizes and LDS capacities give bit-identical magnifications."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2501_03322_amd import inputs
    c = inputs.batched_curves()
    k = slice(0, 96)
    dev = torch.device("cuda", 0)
    args = [torch.as_tensor(a[k] if a.size == c.nsets else a, device=dev)
            for a in (c.s, c.q, c.u0, c.alpha, c.rho, c.tau)]
    return c, args


def _log(msg):
    print(msg, flush=True)


def _run(ctx, args, mode, tol=1e-4, out=None):
    if out is None:
        out = ctx.alloc_out(args[0].numel() * args[5].numel())
    ctx.lightcurves(*args, tol, mode=mode, out=out)
    ctx.sync()
    return out


def test_graph_replay_bitwise(lc):
    """Graph replays of the full launch sequence (counter reset, point pass,
    contour kernel) reproduce the eager result bit for bit, replay after
    replay, with eager work and synchronisations in between."""
    import torch
    from paper_2501_03322_amd import twk
    c, args = lc
    st = torch.cuda.Stream()
    ctx = twk.Context(0, stream=st)
    with torch.cuda.stream(st):
        for mode in (twk.MODE_MIXED, twk.MODE_FP64):
            ctx.set_tuning(graphs=0)
            ref = [t.clone() for t in _run(ctx, args, mode)]
            ctx.set_tuning(graphs=1)
            out = ctx.alloc_out(ref[0].numel())
            for rep in range(4):
                for t in out:
                    t.zero_()
                _run(ctx, args, mode, out=out)
                for a, b in zip(out, ref):
                    assert torch.equal(a, b), (mode, rep)
                # eager work between the replays
                torch.cuda.synchronize()
                _ = (ref[0] * 2.0).sum().item()
            # a new tolerance is a new call: captured afresh, still equal to eager
            ctx.set_tuning(graphs=0)
            ref2 = _run(ctx, args, mode, tol=3e-4)
            ctx.set_tuning(graphs=1)
            got = _run(ctx, args, mode, tol=3e-4)
            assert torch.equal(got[0], ref2[0])
            stats = ctx.stats()
            assert stats["fs_tasks"] == int(((ref2[3] & 1) == 0).sum().item())
        # per-element lenses replay the same way
        rng = np.random.default_rng(4)
        n = 3000
        el = [torch.as_tensor(a, device=args[0].device) for a in (
            10.0 ** rng.uniform(-0.3, 0.3, n), 10.0 ** rng.uniform(-4, -1, n),
            rng.uniform(-1.0, 1.0, n), rng.uniform(-0.3, 0.3, n), 10.0 ** rng.uniform(-3, -2, n))]
        ctx.set_tuning(graphs=0)
        ref = [t.clone() for t in ctx.finite_mag_each(*el, 1e-4, twk.MODE_MIXED)]
        ctx.set_tuning(graphs=1)
        out = ctx.alloc_out(n)
        for rep in range(3):
            for t in out:
                t.zero_()
            ctx.finite_mag_each(*el, 1e-4, twk.MODE_MIXED, out=out)
            ctx.sync()
            for a, b in zip(out, ref):
                assert torch.equal(a, b), ("each", rep)
            torch.cuda.synchronize()
        # timing a replayed call: whole-call time only
        ctx.enable_timing(True)
        _run(ctx, args, twk.MODE_MIXED, tol=3e-4)
        kt = ctx.kernel_times()
        assert kt["total_ms"] > 0
        assert kt["ps_ms"] < 0.05 * kt["total_ms"] and kt["mlp_ms"] < 0.05 * kt["total_ms"]
        assert kt["fs_ms"] < 0.05 * kt["total_ms"] and kt["rest_ms"] > 0.95 * kt["total_ms"]
        ctx.enable_timing(False)
    ctx.close()


@pytest.mark.parametrize("cap", [64, 128, 256])
def test_tuning_does_not_change_results(lc, cap):
    import torch
    from paper_2501_03322_amd import twk
    c, args = lc
    ctx = twk.Context(0)
    for mode in (twk.MODE_MIXED, twk.MODE_FP64):
        ctx.set_tuning(lds_cap=128, waves_per_cu=1)
        ref = [t.clone() for t in _run(ctx, args, mode)]
        for frac in (0.25, 1.0):
            ctx.set_tuning(lds_cap=cap, waves_per_cu=1)
            mx = 1
            # largest accepted grid for this capacity
            for w in range(2, 33):
                try:
                    ctx.set_tuning(lds_cap=cap, waves_per_cu=w)
                    mx = w
                except twk.TwkError:
                    break
            w = max(1, int(mx * frac))
            ctx.set_tuning(lds_cap=cap, waves_per_cu=w)
            _log(f"mode {mode}, cap {cap}: waves per CU {w} of {mx}")
            got = _run(ctx, args, mode)
            for a, b in zip(got, ref):
                assert torch.equal(a, b), (mode, cap, w)
    ctx.close()


def test_long_contours_across_capacities(oracle):
    """Sources near caustics at a tight tolerance (hundreds to thousands of
    limb samples: nearly every contour outgrows the LDS copy and is finished
    in global memory by the persistent kernel's second phase): identical
    results at LDS capacities 64, 128 and 256, in both precisions, and
    within 1e-4 of the oracle on a sample of them."""
    import torch
    from paper_2501_03322_amd import twk
    import pins
    rng = np.random.default_rng(9)
    s, q, rho = 1.0, 1e-3, 1e-3
    ca = pins.caustic(s, q, 2048)
    z = ca[rng.integers(0, ca.size, 3000)] + rho * rng.uniform(0, 1.5, 3000) * np.exp(
        2j * np.pi * rng.uniform(0, 1, 3000))
    dev = torch.device("cuda", 0)
    zx = torch.as_tensor(z.real, device=dev)
    zy = torch.as_tensor(z.imag, device=dev)
    ctx = twk.Context(0)
    for mode in (twk.MODE_MIXED, twk.MODE_FP64):
        ref = None
        for cap in (64, 128, 256):
            ctx.set_tuning(lds_cap=cap, waves_per_cu=1)
            out = ctx.finite_mag(s, q, zx, zy, rho, 1e-6, mode | twk.MODE_ALL_FS)
            ctx.sync()
            st = ctx.stats()
            _log(f"mode {mode}, cap {cap}: {st['fs_tasks']} contours, {st['spilled']} finished in "
                 f"global memory, {st['samples']} samples")
            if cap == 64:
                assert st["spilled"] > 0.9 * st["fs_tasks"]
            if ref is None:
                ref = [t.clone() for t in out]
            else:
                for a, b in zip(out, ref):
                    assert torch.equal(a, b), (mode, cap)
        pick = rng.choice(z.size, 12, replace=False)
        mag = ref[0].cpu().numpy()[pick]
        rm = oracle.finite_mag(s, q, z.real[pick], z.imag[pick], rho, oracle.TIGHT_TOL,
                               oracle.tight_cfg())[0]
        assert np.abs(mag / rm - 1).max() <= 1e-4, (mode, np.abs(mag / rm - 1).max())
    ctx.close()


def test_tuning_rejects_bad_values():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2501_03322_amd import twk
    ctx = twk.Context(0, stream=torch.cuda.Stream())
    for kw in ({"lds_cap": 300}, {"waves_per_cu": 0}, {"waves_per_cu": 1000},
               {"budget_shift": 9.0}, {"graphs": 2}):
        with pytest.raises(twk.TwkError):
            ctx.set_tuning(**kw)
    ctx.close()


def test_autotune(lc, oracle):
    """The autotuner returns a valid tuning, leaves it in the context, and
    the tuned call still meets the gate (learned path, random weights)."""
    import torch
    from oracle import mlp_ref as M
    from paper_2501_03322_amd import twk
    c, args = lc
    ctx = twk.Context(0)
    p = M.init(3, [1.2, -3.0, 0.0, 0.0, -3.0, 0.3, 0.5, -2.0], [0.6, 1.2, 0.8, 0.8, 0.6, 0.4, 1.5, 1.5])
    p["b3"][0] = 7.0
    ctx.mlp_set(M.flatten(p))
    small = [a[:32] if a.numel() == 96 else a for a in args]
    best = ctx.autotune(*small, 1e-4, mode=twk.MODE_MLP | twk.MODE_MIXED, trials=1)
    _log(f"autotuned: {best.as_dict()}")
    assert best.lds_cap in (64, 128, 256) and best.waves_per_cu >= 1
    assert ctx.get_tuning().as_dict() == best.as_dict()
    mag, err, ns, fl = _run(ctx, args, twk.MODE_MLP | twk.MODE_MIXED)
    mag, fl = mag.cpu().numpy(), fl.cpu().numpy()
    rng = np.random.default_rng(4)
    fs = np.nonzero((fl & 1) == 0)[0]
    for i in rng.choice(fs, min(40, fs.size), replace=False):
        k, j = divmod(int(i), c.nepochs)
        zx, zy = oracle.trajectory(c.u0[k], c.alpha[k], c.tau[j:j + 1])
        rm = oracle.finite_mag(c.s[k], c.q[k], zx, zy, c.rho[k], oracle.TIGHT_TOL,
                               oracle.tight_cfg())[0][0]
        assert abs(mag[i] / rm - 1) <= 1e-4
    ctx.close()


def test_batch_size_limits():
    """Element counts whose product would overflow (or exceed 2^48) are
    refused before any device work; an empty batch is a no-op."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2501_03322_amd import twk
    ctx = twk.Context(0, stream=torch.cuda.Stream())
    f = ctx.lib.twk_lightcurves

    def call(nsets, nepochs, na=1):
        return f(ctx.h, nsets, None, None, None, None, None, None, nepochs, None, na, 1e-4, 0,
                 None, None, None, None)
    assert call(1 << 40, 1 << 30) == twk.EINVAL
    assert call(1 << 62, 4) == twk.EINVAL
    assert call(1 << 28, 1 << 20, 1) == twk.EINVAL  # 2^48 elements: allowed size, NULL arrays
    assert call(-1, 10) == twk.EINVAL
    assert call(0, 10) == twk.OK and call(10, 0) == twk.OK
    assert call(1, (1 << 30) + 1) == twk.EINVAL  # epochs of one set exceed one launch
    assert ctx.lib.twk_point_mag(ctx.h, 1.0, 1e-3, (1 << 48) + 1, None, None, None, None,
                                 None) == twk.EINVAL
    ctx.close()
