"""The paper's dispatch of the contour work on the GPU (TWK_MODE_ROUNDS:
one launch per refinement round over the list of unfinished sources,
records in global memory between launches), through the C ABI.  It runs
the same rounds as the persistent kernel, so its results are bit-identical
to the persistent path's, and it meets the gate against the oracle."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

GATE = 1e-4


def _log(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2501_03322_amd import twk
    c = twk.Context(0)
    yield c
    c.close()


def _equal(a, b):
    import torch
    return all(torch.equal(x, y) for x, y in zip(a, b))


@pytest.mark.parametrize("mixed", [0, 1])
def test_rounds_match_persistent_on_light_curves(ctx, mixed):
    """96 parameter sets x 2000 epochs of the fit-style batch (uniform
    source) and 24 limb-darkened sets of the high-cadence batch (10
    annuli): the round-by-round dispatch equals the persistent kernel bit
    for bit (magnification, error, samples, flags)."""
    from paper_2501_03322_amd import inputs, twk
    for name, c, k in (("uniform", inputs.batched_curves(), 96),
                       ("limb-darkened", inputs.large_ld_curves(), 24)):
        c = c.subset(np.arange(k))
        _log(f"rounds vs persistent: {name} {c.nsets} x {c.nepochs}, mixed={mixed}")
        outs = []
        for extra in (0, twk.MODE_ROUNDS):
            out = ctx.lightcurves(c.s, c.q, c.u0, c.alpha, c.rho, c.tau, c.tol, mode=mixed | extra,
                                  gamma=c.gamma, n_annuli=c.n_annuli)
            ctx.sync()
            outs.append([t.clone() for t in out])
            st = ctx.stats()
            _log(f"  mode {mixed | extra}: {st['fs_tasks']} contour tasks, {st['samples']} samples")
        assert _equal(outs[0], outs[1]), name


def test_rounds_against_oracle(ctx, oracle):
    """Caustic crossings, cusps, planetary and central caustics (every source
    by contour): FP64 round-by-round dispatch within the gate of the tight
    oracle."""
    from paper_2501_03322_amd import twk
    from test_gpu_parity import FS_CASES
    for (s, q, z, rho) in FS_CASES:
        _log(f"rounds case s={s} q={q} z={z} rho={rho}")
        mag, err, ns, fl = ctx.finite_mag(s, q, [z.real], [z.imag], rho, GATE,
                                          twk.MODE_FP64 | twk.MODE_ROUNDS | twk.MODE_ALL_FS)
        m = mag.cpu().numpy()[0]
        r = oracle.finite_mag(s, q, [z.real], [z.imag], rho, oracle.TIGHT_TOL, oracle.tight_cfg())[0][0]
        assert abs(m / r - 1) <= GATE, (s, q, z, rho, m, r)


def test_rounds_several_batches_and_graph_setting(oracle):
    """More contour tasks than one batch of the dispatch holds (40,000 > 32,768
    sources near a caustic): equal to the persistent kernel bit for bit, also
    with graph replay switched on (the dispatch then runs uncaptured)."""
    import torch
    from paper_2501_03322_amd import twk
    st = torch.cuda.Stream()
    ctx = twk.Context(0, stream=st)
    rng = np.random.default_rng(5)
    n = 40000
    zx = rng.uniform(-0.06, 0.12, n)
    zy = rng.uniform(-0.05, 0.05, n)
    with torch.cuda.stream(st):
        ref = [t.clone() for t in ctx.finite_mag(1.0, 1e-3, zx, zy, 2e-3, GATE,
                                                 twk.MODE_MIXED | twk.MODE_ALL_FS)]
        ctx.sync()
        for graphs in (0, 1):
            ctx.set_tuning(graphs=graphs)
            _log(f"rounds, {n} sources, graphs={graphs}")
            out = ctx.finite_mag(1.0, 1e-3, zx, zy, 2e-3, GATE,
                                 twk.MODE_MIXED | twk.MODE_ALL_FS | twk.MODE_ROUNDS)
            ctx.sync()
            assert _equal(out, ref), graphs
        assert ctx.stats()["fs_tasks"] == n
    ctx.close()
    # a few of them against the oracle
    m = ref[0].cpu().numpy()
    for i in rng.choice(n, 12, replace=False):
        r = oracle.finite_mag(1.0, 1e-3, zx[i:i + 1], zy[i:i + 1], 2e-3, oracle.TIGHT_TOL,
                              oracle.tight_cfg())[0][0]
        assert abs(m[i] / r - 1) <= GATE, (i, m[i], r)
