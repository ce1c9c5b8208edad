"""Generate MPM training data, train the surrogate, evaluate it on held-out
solves and serve a query stream through the router.

  python -m paper_2301_08343_amd.surrogate_pipeline --train 16384 --heldout 512 \
      --epochs 20 --queries 10000 --out DIR

Seeds: training samples 0 .. train-1, held-out 50000 .., queries 100000 ..;
all contacts are GelSight-sized draws solved at the data spacing. Writes
DIR/surrogate.safetensors (FP32 weights and router calibration) and
DIR/report.json; progress goes to stdout.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import torch

from . import dataset as D
from . import router as RT
from . import training as TR
from .surrogate import Net, forward_flops

HELDOUT_SEED0 = 50_000
QUERY_SEED0 = 100_000


def log(msg):
    print(msg, flush=True)


def save(path, net: Net, train_feats, threshold, meta):
    from safetensors.torch import save_file
    save_file({"flat": net.flat.detach().cpu(), "train_features": train_feats.detach().cpu()}, path,
              metadata={k: json.dumps(v) for k, v in dict(meta, threshold=threshold).items()})


def load(path, batch=512):
    from safetensors import safe_open
    with safe_open(path, framework="pt") as f:
        meta = {k: json.loads(v) for k, v in f.metadata().items()}
        flat = f.get_tensor("flat")
        feats = f.get_tensor("train_features")
    net = Net(batch=batch, res=meta["res"], enc=tuple(meta["enc"]), mid=meta["mid"])
    net.flat.copy_(flat)
    net.repack()
    return net, feats.cuda(), meta


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=16384)
    ap.add_argument("--heldout", type=int, default=512)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--queries", type=int, default=10000)
    ap.add_argument("--plain-sample", type=int, default=512)
    ap.add_argument("--h", type=float, default=D.H_DATA)
    ap.add_argument("--gen-batch", type=int, default=256)
    ap.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    os.makedirs(a.out, exist_ok=True)
    rep = {"args": vars(a)}

    t = time.perf_counter()
    xtr, ytr = D.generate(range(a.train), h=a.h, batch=a.gen_batch, log=log)
    xte, yte = D.generate(range(HELDOUT_SEED0, HELDOUT_SEED0 + a.heldout), h=a.h, batch=a.gen_batch, log=log)
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t
    c0 = D.contacts_for([0], a.h)[0]
    ps = (a.train + a.heldout) * c0["particles"] * c0["steps"]
    rep["data"] = {"samples": a.train + a.heldout, "seconds": gen_s, "particle_substeps": ps,
                   "particle_substeps_per_s": ps / gen_s, "particles_per_contact": c0["particles"],
                   "substeps_per_contact": c0["steps"], "h_m": a.h}
    log(f"data: {json.dumps(rep['data'])}")

    net = Net(batch=a.batch, seed=0)
    hist = TR.train(net, xtr, ytr, epochs=a.epochs, batch=a.batch, lr=a.lr, log=log)
    tsec = sum(h[2] for h in hist)
    steps = a.epochs * (a.train // a.batch)
    flops = 3 * forward_flops() * steps * a.batch
    rep["train"] = {"epochs": a.epochs, "seconds": tsec, "samples_per_s": steps * a.batch / tsec,
                    "tflops": flops / tsec / 1e12, "final_loss": hist[-1][1],
                    "loss_curve": [h[1] for h in hist]}
    rep["heldout"] = TR.evaluate(net, xte, yte)
    rep["train_fit"] = TR.evaluate(net, xtr[:a.heldout], ytr[:a.heldout])
    log(f"held-out: {json.dumps(rep['heldout'])}")

    ftr = RT.features(xtr)
    thr = RT.Router.calibrate(ftr, RT.features(xte))
    meta = {"res": net.res, "enc": list(net.enc), "mid": net.mid, "h_m": a.h, "train_samples": a.train,
            "y_unit_m": D.Y_UNIT, "x_unit_m": D.X_UNIT, "gap_clip_m": D.GAP_CLIP}
    save(os.path.join(a.out, "surrogate.safetensors"), net, ftr, thr, meta)
    rep["router_threshold"] = thr

    if a.queries > 0:
        del xtr, ytr
        torch.cuda.empty_cache()
        qs = D.contacts_for(range(QUERY_SEED0, QUERY_SEED0 + a.queries), a.h)
        serve_net = Net(batch=512, seed=0)
        serve_net.flat.copy_(net.flat)
        serve_net.repack()
        r = RT.Router(serve_net, ftr, thr)
        ans, rrep = r.serve(qs, log=log)
        rep["router"] = rrep
        log(f"router: {json.dumps(rrep)}")
        k = min(a.plain_sample, a.queries)
        ymp, prep = RT.plain_mpm(qs[:k], log=log)
        rep["plain_mpm"] = dict(prep, note=f"first {k} queries; frames/s extrapolates to the stream")
        served = TR.per_sample_rmse(ans[:k], ymp, 2) * D.Y_UNIT * 1e6
        rep["served_vs_mpm_height_rmse_um"] = float((served ** 2).mean().sqrt())
        rep["speedup_frames_per_s"] = rrep["frames_per_s"] / prep["frames_per_s"]
        log(f"plain MPM: {json.dumps(prep)}; served answers vs MPM: "
            f"{rep['served_vs_mpm_height_rmse_um']:.2f} um; speedup {rep['speedup_frames_per_s']:.1f}x")

    with open(os.path.join(a.out, "report.json"), "w") as f:
        json.dump(rep, f, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
