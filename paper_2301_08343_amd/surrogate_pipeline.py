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

import numpy as np
import torch

from . import dataset as D
from . import router as RT
from . import training as TR
from .surrogate import Net, forward_flops

HELDOUT_SEED0 = 50_000
QUERY_SEED0 = 100_000
# the router's classes split each indenter family at these press depths:
# three equal bins of the drawn depth range, 0.2 .. 1.5 mm
DEPTH_EDGES_M = (0.2e-3 + 1.3e-3 / 3, 0.2e-3 + 2.6e-3 / 3)


def heldout_report(net, x, y, seeds, h):
    """Held-out errors by indenter family, plus the per-class statistics
    (family and depth bin, the router's classes) its error budget starts
    from, and the class definition."""
    rep = TR.evaluate(net, x, y, groups=[s % 5 for s in seeds])
    cs = D.contacts_for(seeds, h, full=False)
    by_class = TR.evaluate(net, x, y, groups=[RT.query_class(c, DEPTH_EDGES_M) for c in cs])
    rep["height_ms_um2_stats_by_class"] = by_class["height_ms_um2_stats_by_group"]
    rep["height_rmse_um_by_class"] = by_class["height_rmse_um_by_group"]
    rep["router_depth_edges_m"] = list(DEPTH_EDGES_M)
    return rep


def log(msg):
    print(msg, flush=True)


def save(path, net: Net, train_feats, threshold, meta):
    from safetensors.torch import save_file
    save_file({"flat": net.flat.detach().cpu(), "train_features": train_feats.detach().cpu()}, path,
              metadata={k: json.dumps(v) for k, v in dict(meta, threshold=threshold).items()})


def save_compact(path, net: Net, threshold, meta):
    """Weights as bfloat16 (exactly what the kernels use) and biases as FP32:
    a model loaded from it predicts bit for bit as the one saved."""
    from safetensors.torch import save_file
    ws, bs = [], []
    for name, ci, co, t in net.specs:
        w, b = net.param(name)
        ws.append(w.detach().reshape(-1))
        bs.append(b.detach())
    save_file({"weights_bf16": torch.cat(ws).to(torch.bfloat16).cpu(), "biases": torch.cat(bs).cpu()}, path,
              metadata={k: json.dumps(v) for k, v in dict(meta, threshold=threshold).items()})


def load_compact(path, batch=512):
    from safetensors import safe_open
    with safe_open(path, framework="pt") as f:
        meta = {k: json.loads(v) for k, v in f.metadata().items()}
        wb = f.get_tensor("weights_bf16").float()
        bb = f.get_tensor("biases")
    net = Net(batch=batch, res=meta["res"], enc=tuple(meta["enc"]), mid=meta["mid"],
              contact_residual=meta.get("contact_residual", 0.0))
    ow = ob = 0
    for name, ci, co, t in net.specs:
        w, b = net.param(name)
        w.copy_(wb[ow:ow + w.numel()].view_as(w))
        b.copy_(bb[ob:ob + co])
        ow += w.numel()
        ob += co
    net.repack()
    return net, meta


def load(path, batch=512):
    from safetensors import safe_open
    with safe_open(path, framework="pt") as f:
        meta = {k: json.loads(v) for k, v in f.metadata().items()}
        flat = f.get_tensor("flat")
        feats = f.get_tensor("train_features")
    net = Net(batch=batch, res=meta["res"], enc=tuple(meta["enc"]), mid=meta["mid"],
              contact_residual=meta.get("contact_residual", 0.0))
    net.flat.copy_(flat)
    net.repack()
    return net, feats.cuda(), meta


def train_features(n, h, chunk=2048):
    """Router features of training seeds 0 .. n-1 (gap fields only, no solve)."""
    out = []
    for k in range(0, n, chunk):
        out.append(RT.features(D.inputs(D.contacts_for(range(k, min(n, k + chunk)), h, full=False))))
    return torch.cat(out)


def served_sample(n, k, seed=11):
    """About k query indices spread over a stream of n: query i is in the
    sample when the i-th SplitMix64 output of `seed` is below (k / n) 2^64."""
    from .workloads import SplitMix64
    rng = SplitMix64(seed)
    lim = int(min(1.0, k / n) * 2.0 ** 64)
    return [i for i in range(n) if rng.next_u64() < lim]


def serve_benchmark(net, ftr, thr, h, queries, plain_sample, prior_rmse_um=None, prior_stats=None, depth_edges=None,
                    log=log):
    """The query stream through the router, and plain batched MPM on a seeded
    sample of about `plain_sample` queries spread over the whole stream: its
    rate is the plain MPM's frames/s, and its answers measure the error of
    the answers the router served for those queries (per family too). With
    prior_stats (per family: count, mean and sd of the held-out height mean
    squared error) the router runs its error-budget policy, else per-family
    breakers started from prior_rmse_um."""
    rep = {}
    qs = D.contacts_for(range(QUERY_SEED0, QUERY_SEED0 + queries), h, full=False)
    if prior_stats:
        r = RT.Router(net, ftr, thr, policy="budget", prior_stats=prior_stats, depth_edges=depth_edges)
    else:
        r = RT.Router(net, ftr, thr, prior_rmse_um=prior_rmse_um)
    ans, rrep, route = r.serve(qs, log=log)
    rep["router"] = rrep
    log(f"router: {json.dumps(rrep)}")
    pick = served_sample(queries, plain_sample)
    ymp, prep = RT.plain_mpm([qs[i] for i in pick], log=log)
    rep["plain_mpm"] = dict(prep, note=f"{len(pick)} queries sampled over the stream; frames/s is per query")
    served = (TR.per_sample_rmse(ans[torch.tensor(pick, device=ans.device)], ymp, 2) * D.Y_UNIT * 1e6).cpu()
    fam = torch.tensor([qs[i]["cfg"]["shape"] for i in pick])
    by_route = torch.tensor(route[pick].astype(np.int64))
    rep["served_vs_mpm_height_rmse_um"] = float((served ** 2).mean().sqrt())
    rep["served_sample"] = {
        "queries": len(pick), "first_index": pick[0], "last_index": pick[-1], "seed": 11,
        "height_rmse_um_by_family": {str(int(k)): float((served[fam == k] ** 2).mean().sqrt())
                                     for k in torch.unique(fam)},
        "surrogate_answers": int((by_route == RT.Router.SURROGATE).sum()),
        "height_rmse_um_of_surrogate_answers": (
            float((served[by_route == RT.Router.SURROGATE] ** 2).mean().sqrt())
            if bool((by_route == RT.Router.SURROGATE).any()) else None)}
    rep["speedup_frames_per_s"] = rrep["frames_per_s"] / prep["frames_per_s"]
    log(f"plain MPM: {json.dumps(prep)}; served answers vs MPM: "
        f"{rep['served_vs_mpm_height_rmse_um']:.2f} um; speedup {rep['speedup_frames_per_s']:.1f}x")
    return rep


def resolution_check(weights, n, h_full=0.1e-3, gen_batch=64, log=log):
    """The data spacing's own error: the held-out contacts 50000 .. 50000+n-1
    solved at the surrogate's data spacing and again at h_full (the 0.1 mm
    lattice of the benchmark press: 1.6M particles, 2000 substeps), both
    resampled to the same top-surface cells. Reports the height RMSE between
    the two solves (the resolution error of the training data), and the
    surrogate's error against each."""
    net, meta = load_compact(weights, batch=256)
    h = meta["h_m"]
    seeds = list(range(HELDOUT_SEED0, HELDOUT_SEED0 + n))
    groups = [s % 5 for s in seeds]
    t = time.perf_counter()
    x, y_c = D.generate(seeds, h=h, batch=256, log=log)
    torch.cuda.synchronize()
    t_c = time.perf_counter() - t
    t = time.perf_counter()
    x_f, y_f = D.generate(seeds, h=h_full, batch=gen_batch, log=log)
    torch.cuda.synchronize()
    t_f = time.perf_counter() - t
    cf = D.contacts_for([seeds[0]], h_full, full=False)[0]
    um = D.Y_UNIT * 1e6
    dz = TR.per_sample_rmse(y_c, y_f, 2).cpu() * um
    g = torch.as_tensor(groups)
    rep = {
        "samples": n, "h_data_m": h, "h_full_m": h_full,
        "full_particles_per_contact": cf["particles"], "full_substeps": cf["steps"],
        "full_solve_seconds": t_f, "data_solve_seconds": t_c,
        "full_particle_substeps_per_s": n * cf["particles"] * cf["steps"] / t_f,
        # the inputs do not depend on the lattice spacing: the same indenter
        # pose over the same top face
        "input_max_abs_diff_mm": float((x - x_f).abs().max()),
        "data_vs_full_height_rmse_um": float((dz ** 2).mean().sqrt()),
        "data_vs_full_height_rmse_um_by_group": {
            str(int(k)): float((dz[g == k] ** 2).mean().sqrt()) for k in torch.unique(g)},
        "surrogate_vs_data": TR.evaluate(net, x, y_c, groups=groups),
        "surrogate_vs_full": TR.evaluate(net, x, y_f, groups=groups),
    }
    log(f"resolution: {json.dumps(rep)}")
    return rep


def evaluate_weights(a, rep):
    """Held-out evaluation of committed weights (--evaluate): the held-out
    contacts are solved again (the same seeds and spacing as in training), the
    model's errors replace the `heldout` entry of its metadata, and the query
    stream is served with them."""
    net, meta = load_compact(a.weights, batch=512)
    h = meta["h_m"]
    xte, yte = D.generate(range(HELDOUT_SEED0, HELDOUT_SEED0 + a.heldout), h=h, batch=a.gen_batch, log=log)
    rep["heldout"] = heldout_report(net, xte, yte, list(range(HELDOUT_SEED0, HELDOUT_SEED0 + a.heldout)), h)
    log(f"held-out: {json.dumps(rep['heldout'])}")
    thr = meta.pop("threshold")
    meta["heldout"] = rep["heldout"]
    save_compact(os.path.join(a.out, "surrogate_compact.safetensors"), net, thr, meta)
    if a.queries > 0:
        ftr = train_features(meta["train_samples"], h)
        rep.update(serve_benchmark(net, ftr, thr, h, a.queries, a.plain_sample,
                                   prior_rmse_um=rep["heldout"].get("height_rmse_um_by_group"),
                                   prior_stats=rep["heldout"].get("height_ms_um2_stats_by_class"),
                                   depth_edges=rep["heldout"].get("router_depth_edges_m")))
    with open(os.path.join(a.out, "report.json"), "w") as f:
        json.dump(rep, f, indent=1)
    return 0


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
    ap.add_argument("--no-symmetry", action="store_true", help="train without the mirror/transpose copies")
    ap.add_argument("--no-residual", action="store_true", help="no FP32 contact term on the output")
    ap.add_argument("--resolution-check", type=int, default=0, metavar="N",
                    help="only compare N held-out solves at the data spacing with 0.1 mm solves "
                         "(and the --weights model against both)")
    ap.add_argument("--weights", default=None, help="compact weights for --resolution-check or --evaluate")
    ap.add_argument("--evaluate", action="store_true",
                    help="no training: evaluate the --weights model on the held-out solves, write it again with "
                         "those errors in its metadata (DIR/surrogate_compact.safetensors), then serve the queries")
    ap.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    os.makedirs(a.out, exist_ok=True)
    rep = {"args": vars(a)}
    if a.resolution_check > 0:
        if not a.weights:
            ap.error("--resolution-check needs --weights")
        rep["resolution"] = resolution_check(a.weights, a.resolution_check, gen_batch=min(a.gen_batch, 64))
        with open(os.path.join(a.out, "resolution.json"), "w") as f:
            json.dump(rep, f, indent=1)
        return 0

    if a.evaluate:
        if not a.weights:
            ap.error("--evaluate needs --weights")
        return evaluate_weights(a, rep)

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

    net = Net(batch=a.batch, seed=0, contact_residual=0.0 if a.no_residual else D.X_UNIT / D.Y_UNIT)
    hist = TR.train(net, xtr, ytr, epochs=a.epochs, batch=a.batch, lr=a.lr, symmetry=not a.no_symmetry, log=log)
    tsec = sum(h[2] for h in hist)
    steps = a.epochs * (a.train // a.batch)
    flops = 3 * forward_flops() * steps * a.batch
    rep["train"] = {"epochs": a.epochs, "seconds": tsec, "samples_per_s": steps * a.batch / tsec,
                    "tflops": flops / tsec / 1e12, "final_loss": hist[-1][1],
                    "loss_curve": [h[1] for h in hist]}
    rep["heldout"] = heldout_report(net, xte, yte, list(range(HELDOUT_SEED0, HELDOUT_SEED0 + a.heldout)), a.h)
    rep["train_fit"] = TR.evaluate(net, xtr[:a.heldout], ytr[:a.heldout], groups=[s % 5 for s in range(a.heldout)])
    log(f"held-out: {json.dumps(rep['heldout'])}")

    ftr = RT.features(xtr)
    thr = RT.Router.calibrate(ftr, RT.features(xte))
    meta = {"res": net.res, "enc": list(net.enc), "mid": net.mid, "h_m": a.h, "train_samples": a.train,
            "contact_residual": net.contact_residual,
            "y_unit_m": D.Y_UNIT, "x_unit_m": D.X_UNIT, "gap_clip_m": D.GAP_CLIP}
    save(os.path.join(a.out, "surrogate.safetensors"), net, ftr, thr, meta)
    save_compact(os.path.join(a.out, "surrogate_compact.safetensors"), net, thr,
                 dict(meta, heldout=rep["heldout"]))
    rep["router_threshold"] = thr

    if a.queries > 0:
        del xtr, ytr
        torch.cuda.empty_cache()
        serve_net = Net(batch=512, seed=0, contact_residual=net.contact_residual)
        serve_net.flat.copy_(net.flat)
        serve_net.repack()
        rep.update(serve_benchmark(serve_net, ftr, thr, a.h, a.queries, a.plain_sample,
                                   prior_rmse_um=rep["heldout"].get("height_rmse_um_by_group"),
                                   prior_stats=rep["heldout"].get("height_ms_um2_stats_by_class"),
                                   depth_edges=rep["heldout"].get("router_depth_edges_m")))

    with open(os.path.join(a.out, "report.json"), "w") as f:
        json.dump(rep, f, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
