"""Train the learned sample budget on the GPU and write its weights.

Training set: the seed-2 light-curve batch (1000 parameter sets x 2000
epochs, drawn like the fit-style batch) and the seed-5 batch over the
high-cadence batch's ranges (1000 x 2000, log10 q down to -6).  Inputs: the
eight point-source
features of every epoch (twk_features).  Labels from the plain FP64 path
with the point-source test switched off, so that every epoch gets a
contour: log2 of the limb samples it used, and whether the point value
misses the tolerance (|mu_ps / mu_FS - 1| > tol).  Training: minibatch
Adam on the device (twk_mlp_train).  Evaluation on 128 sets of the seed-3
batch and 128 sets of a seed-6 batch over the high-cadence ranges,
including how often the contours that need 256 samples or more are
predicted so.  Writes weights/mlp_budget.bin and a JSON record beside
it.

    python -m paper_2501_03322_amd.train_mlp [--epochs 8] [--out PATH]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

DEFAULT_OUT = os.path.join(HERE, "weights", "mlp_budget.bin")
TOL = 1e-4


def labelled(ctx, c, tol=TOL):
    """Features and labels of every epoch of a light-curve set."""
    import torch
    from paper_2501_03322_amd import twk
    feat, mu, _ = ctx.features(c.s, c.q, c.u0, c.alpha, c.rho, c.tau, tol)
    mag, _, ns, _ = ctx.lightcurves(c.s, c.q, c.u0, c.alpha, c.rho, c.tau, tol,
                                    twk.MODE_FP64 | twk.MODE_ALL_FS)
    yb = torch.log2(ns.to(torch.float32))
    yf = ((mu / mag - 1.0).abs() > tol).to(torch.float32)
    keep = torch.isfinite(feat).all(dim=1) & torch.isfinite(mag)
    return feat[keep].contiguous(), yb[keep].contiguous(), yf[keep].contiguous()


def evaluate(ctx, c):
    import torch
    feat, yb, yf = labelled(ctx, c)
    out = ctx.mlp_infer(feat)
    p = out[:, 0].double()
    y = yb.double()
    fs = yf > 0.5
    res = {"rows": int(y.numel()),
           "corr_log2N": float(torch.corrcoef(torch.stack([p, y]))[0, 1]),
           "mae_log2N": float((p - y).abs().mean()),
           "mae_log2N_fs_needed": float((p - y)[fs].abs().mean()) if fs.any() else None,
           "fs_head_accuracy": float(((out[:, 1] > 0) == fs).double().mean()),
           "long_class_accuracy": float(((p >= 8.0) == (y >= 8.0)).double().mean()),
           "long_fraction": float((y >= 8.0).double().mean()),
           "long_recall": float(((p >= 8.0) & (y >= 8.0)).double().sum() / max(float((y >= 8.0).double().sum()), 1.0)),
           "fs_needed_fraction": float(fs.double().mean())}
    return res


def train(out_path=DEFAULT_OUT, epochs=8, batch=4096, lr=2e-3, lr_end=1e-4, seed=1, log=print):
    import torch
    from paper_2501_03322_amd import inputs, twk
    ctx = twk.Context(0)
    t0 = time.perf_counter()
    parts = [labelled(ctx, inputs.training_curves()), labelled(ctx, inputs.wide_training_curves())]
    feat, yb, yf = (torch.cat([p[i] for p in parts]).contiguous() for i in range(3))
    torch.cuda.synchronize()
    log(f"training rows {feat.shape[0]}: labels in {time.perf_counter() - t0:.1f} s, "
        f"mean log2 N {float(yb.mean()):.3f}, FS-needed fraction {float(yf.mean()):.4f}")
    t1 = time.perf_counter()
    hist = ctx.mlp_train(feat, yb, yf, epochs=epochs, batch=batch, lr=lr, lr_end=lr_end, seed=seed)
    log(f"trained {epochs} epochs in {time.perf_counter() - t1:.1f} s; loss per epoch "
        + " ".join(f"{v:.4f}" for v in hist))
    os.makedirs(os.path.dirname(out_path), exist_ok=True)
    ctx.mlp_save(out_path)
    ev = inputs.evaluation_curves()
    res = evaluate(ctx, ev.subset(np.arange(128)))
    log("evaluation (seed 3, 128 sets x 4000 epochs): " + json.dumps(res))
    res_wide = evaluate(ctx, inputs.wide_training_curves(nsets=128, nepochs=4000, seed=6))
    log("evaluation (seed 6, high-cadence ranges, 128 sets x 4000 epochs): " + json.dumps(res_wide))
    rec = {"weights": os.path.basename(out_path),
           "training_set": "seed 2 and seed 5 (high-cadence ranges), 1000 x 2000 epochs each",
           "labels": "plain FP64 path, point-source test off, tol 1e-4",
           "epochs": epochs, "batch": batch, "lr": lr, "lr_end": lr_end, "seed": seed,
           "loss_per_epoch": [float(v) for v in hist], "evaluation": res,
           "evaluation_high_cadence_ranges": res_wide}
    with open(os.path.splitext(out_path)[0] + ".json", "w") as f:
        json.dump(rec, f, indent=1)
    ctx.close()
    return rec


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--out", default=DEFAULT_OUT)
    a = ap.parse_args()
    train(a.out, a.epochs, a.batch, a.lr, log=lambda m: print(m, flush=True))


if __name__ == "__main__":
    main()
