"""twk_finite_mag_noalloc (the entry point that allocates nothing; its
scratch is a fixed device array) against twk_finite_mag through the C ABI:
two calls in a row, the second with fewer sources (the array keeps the
first call's contents), both precisions; results bit-identical; sizes above
the limit and the learned mode refused."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

GATE = 1e-4


def _sources(n, seed):
    rng = np.random.default_rng(seed)
    # around the resonant caustic of s = 1, q = 1e-3: many contour tasks,
    # caustic crossings and point-source epochs
    return rng.uniform(-0.08, 0.16, n), rng.uniform(-0.06, 0.06, n)


def test_noalloc_matches_finite_mag(oracle):
    import torch
    from paper_2501_03322_amd import twk
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = twk.Context(0)
    for mode in (twk.MODE_MIXED, twk.MODE_FP64):
        for n, seed in ((20000, 1), (3000, 2)):
            zx, zy = _sources(n, seed)
            print(f"noalloc mode={mode} n={n}", flush=True)
            ref = [t.clone() for t in ctx.finite_mag(1.0, 1e-3, zx, zy, 2e-3, GATE, mode)]
            got = ctx.finite_mag_noalloc(1.0, 1e-3, zx, zy, 2e-3, GATE, mode)
            ctx.sync()
            for a, b in zip(got, ref):
                assert torch.equal(a, b), (mode, n)
            fl = ref[3].cpu().numpy()
            assert np.sum((fl & 1) == 0) > n // 20  # contour work was done
        # a few against the oracle
        m = got[0].cpu().numpy()
        for i in (0, 7, 1500):
            r = oracle.finite_mag(1.0, 1e-3, zx[i:i + 1], zy[i:i + 1], 2e-3, oracle.TIGHT_TOL,
                                  oracle.tight_cfg())[0][0]
            assert abs(m[i] / r - 1) <= GATE
    # all sources by contour
    zx, zy = _sources(500, 3)
    ref = ctx.finite_mag(1.0, 1e-3, zx, zy, 2e-3, GATE, twk.MODE_MIXED | twk.MODE_ALL_FS)
    got = ctx.finite_mag_noalloc(1.0, 1e-3, zx, zy, 2e-3, GATE, twk.MODE_MIXED | twk.MODE_ALL_FS)
    ctx.sync()
    assert all(torch.equal(a, b) for a, b in zip(got, ref))
    # limits
    with pytest.raises(twk.TwkError) as e:
        ctx.finite_mag_noalloc(1.0, 1e-3, np.zeros(65537), np.zeros(65537), 2e-3, GATE)
    assert e.value.status == twk.EINVAL
    with pytest.raises(twk.TwkError) as e:
        ctx.finite_mag_noalloc(1.0, 1e-3, zx, zy, 2e-3, GATE, twk.MODE_MIXED | twk.MODE_MLP)
    assert e.value.status == twk.EINVAL
    ctx.close()
