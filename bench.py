"""Benchmark of the tactile MLS-MPM hot path on one MI355X.

One step = one tactile frame of the GelSight-sized press: S explicit MLS-MPM
substeps of the 1.6M-particle block (block sort, P2G, grid update with the
rigid-indenter contact, G2P with the neo-Hookean update), then the 200 x 200
depth map and the 480 x 640 Phong image. The metric is particle-substeps/s
over the timed frames. Inputs are synthetic and resident on the GPU before
the timed region starts.

Prints ONE JSON line. With --gpus above 1 it exits: the library runs on one
GPU (independent contacts would shard one process per GPU; one large block
would split into slabs of grid blocks that exchange their tile halos each
substep).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E nameplate, GB/s

# Algorithmic bytes (FP32) of one substep, per particle and per active grid
# node (a node inside some particle's 3x3x3 stencil): what each kernel must
# read and write once, whatever its tiling
#   P2G:  bin entry 4 + u 12 + v 12 + A 36 read per particle; mass + momentum
#         16 written per active node
#   grid: mass + momentum 16 read, velocity 12 written and the next
#         accumulation buffer 16 cleared per active node
#   G2P:  bin entry 4 + u 12 + H 36 read, u 12 + v 12 + H 36 + A 36 written per
#         particle; velocity 12 read per active node
BYTES_PER_PARTICLE = {"p2g": 64, "grid": 0, "g2p": 148}
BYTES_PER_ACTIVE_NODE = {"p2g": 16, "grid": 44, "g2p": 12}
TIMED_KERNELS = ("p2g", "grid", "g2p")
TIMING_EVERY = 5  # frames between frames whose kernels carry HIP events


def design_bytes(kernel, particles, active_blocks, B):
    """What this design moves besides the algorithmic bytes: P2G stores each
    live block's whole (B+3)^3 tile of mass and momentum (16 B per node) and
    the grid update gathers them back; G2P also writes the next substep's bin
    entry (4 B) and stages a (B+3)^3 tile of 16-byte velocities per live
    block. Reported beside the algorithmic figure, never as the roofline."""
    tile = (B + 3) ** 3 * active_blocks
    if kernel == "p2g":
        return 64 * particles + 16 * tile
    if kernel == "grid":
        return 16 * tile + 16 * B ** 3 * active_blocks
    return 152 * particles + 16 * tile

# Counter-measured HBM bytes per launch (rocprofv3 FETCH_SIZE and WRITE_SIZE,
# scaled by what they read for a plain device copy) live in the committed
# profile summary together with the hash of the kernel sources they were
# taken on; they are reported only while the sources still match.
PROFILE = os.path.join(ROOT, "profiles", "mpm_gelsight_1.6M_fp32.md")
KERNEL_SOURCES = ("paper_2301_08343_amd/csrc/sim_kernels.hpp", "paper_2301_08343_amd/csrc/device_common.hpp",
                  "paper_2301_08343_amd/csrc/tacchi.hip")


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def committed_profile(kernel, field="bytes_per_launch"):
    """A per-launch counter figure of `kernel` from the committed profile
    summary (HBM bytes or VALU instructions), or None when the kernel sources
    have changed since it was taken."""
    try:
        with open(PROFILE) as fh:
            text = fh.read()
    except OSError:
        return None
    m = re.search(r"<!-- traffic (\{.*?\}) -->", text)
    if not m:
        return None
    d = json.loads(m.group(1))
    if d.get("source_sha256") != kernel_source_hash():
        return None
    return d.get(field, {}).get(kernel)


def committed_traffic(kernel):
    return committed_profile(kernel, "bytes_per_launch")


# VALU issue: one wave instruction holds its SIMD 4 cycles (16 lanes per
# cycle, no packed FP32 here): 1024 SIMDs x 2.4 GHz / 4 wave instructions/s
VALU_ISSUE_PER_S = 1024 * 2.4e9 / 4


def valu_issue_frac(kernel, launch_ms):
    n = committed_profile(kernel, "valu_instr_per_launch")
    return None if n is None else n / VALU_ISSUE_PER_S / (launch_ms * 1e-3)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40, help="timed frames (40 x 50 = the whole 2000-substep press)")
    ap.add_argument("--warmup", type=int, default=2, help="untimed frames, on a separate instance")
    ap.add_argument("--substeps", type=int, default=50, help="MPM substeps per frame")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="first run one plain device copy of this size (for HBM counter calibration)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--tile", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--surrogate", default=os.path.join(ROOT, "paper_2301_08343_amd", "weights",
                                                        "surrogate_h0.2mm.safetensors"),
                    help="trained surrogate; its query-stream leg runs when the file exists")
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--no-streaming", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--surrogate-steps", type=int, default=0,
                    help="only time N surrogate training steps and N forward passes (batch 256, random data)")
    ap.add_argument("--queries", type=int, default=10000)
    ap.add_argument("--plain-sample", type=int, default=512)
    ap.add_argument("--no-families", action="store_true")
    ap.add_argument("--cpu-worker", type=int, default=-1, help=argparse.SUPPRESS)
    return ap.parse_args()


def surrogate_leg(args):
    """Contact-query stream through the trained surrogate and its router vs
    plain batched MPM (run after the timed MPM frames)."""
    import torch
    from paper_2301_08343_amd import surrogate_pipeline as SP
    from paper_2301_08343_amd.surrogate import forward_flops

    def log(m):
        print(m, file=sys.stderr, flush=True)

    net, meta = SP.load_compact(args.surrogate, batch=512)
    x = torch.zeros(512, meta["res"], meta["res"], 2, dtype=torch.float32, device="cuda")
    net.forward(x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = 20
    for _ in range(reps):
        net.forward(x)
    torch.cuda.synchronize()
    inf_s = (time.perf_counter() - t0) / reps
    ftr = SP.train_features(meta["train_samples"], meta["h_m"])
    held = meta.get("heldout", {})
    prior = held.get("height_rmse_um_by_group")
    # the error budget over (family, depth bin) classes when the weights carry
    # their statistics, else over families
    edges = held.get("router_depth_edges_m")
    stats = held.get("height_ms_um2_stats_by_class") if edges else held.get("height_ms_um2_stats_by_group")
    rep = SP.serve_benchmark(net, ftr, meta["threshold"], meta["h_m"], args.queries, args.plain_sample,
                             prior_rmse_um=prior, prior_stats=stats, depth_edges=edges, log=log)
    r, p = rep["router"], rep["plain_mpm"]
    return {"metric": "tactile frames/s, surrogate + MPM fallback vs plain batched MPM",
            "frames_per_s": r["frames_per_s"], "plain_mpm_frames_per_s": p["frames_per_s"],
            "speedup": rep["speedup_frames_per_s"],
            "latency_p50_ms": r["latency_p50_ms"], "latency_p99_ms": r["latency_p99_ms"],
            "plain_mpm_latency_p50_ms": p["latency_p50_ms"], "plain_mpm_latency_p99_ms": p["latency_p99_ms"],
            "audited_height_rmse_um": r["audited_height_rmse_um"],
            "served_vs_mpm_height_rmse_um": rep["served_vs_mpm_height_rmse_um"],
            "heldout_height_rmse_um": meta.get("heldout", {}).get("height_rmse_um"),
            "queries": r["queries"], "mpm_fallbacks": r["mpm_fallbacks"], "ood": r["ood"],
            "audited": r["audited"], "breaker_tripped_families": r["breaker_tripped"],
            "served_by_surrogate": r["served_by_surrogate"],
            "served_sample": rep["served_sample"],
            "served_within_limit": rep["served_vs_mpm_height_rmse_um"] <= 5.0,
            "breaker_tripped_at_start": r["breaker_tripped_at_start"],
            "breaker_rerouted_in_batch": r["breaker_rerouted_in_batch"],
            "per_family": r["per_class"],
            "router_policy": r["policy"], "router_budget": r.get("budget"),
            "inference_frames_per_s": 512 / inf_s,
            "inference_tflops": 512 * forward_flops(meta["res"]) / inf_s / 1e12,
            "plain_mpm_sample": p["queries"], "data_h_m": meta["h_m"], "train_samples": meta["train_samples"],
            "heldout_height_rmse_um_by_family": prior,
            "dtype": "bf16 storage, fp32 accumulation"}


def streaming_leg(n=200):
    """Per-substep wall time of the robot-simulator loop (Sec. III-C) through
    the binding: one tacchi_step call per substep, one tacchi_run call for n
    substeps, and tacchi_run_until_force (a device-side force test after every
    substep, limit never reached); on the GelSight press (1.6M particles,
    FP32) and on the 18,432-particle sphere press (FP64, launch-bound)."""
    import math
    import numpy as np
    import torch
    from paper_2301_08343_amd import workloads as W
    from paper_2301_08343_amd.sim import Sim
    out = {}
    for name, wl, prec in (("gelsight_1.6M_fp32", W.gelsight_contact(seed=0, steps=2000), "f32"),
                           ("sphere_18k_fp64", W.small_sphere_contact(seed=0, steps=1000), "f64"),
                           ("sphere_18k_fp32", W.small_sphere_contact(seed=0, steps=1000), "f32")):
        poses, dt = wl["poses"], wl["dt"]
        sim = Sim(wl["cfg"], poses[0], precision=prec)
        sim.run(poses[1:21], dt)
        sim.sync()
        res = {}
        k = 21
        for mode in ("step_per_call", "run", "run_until_force"):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if mode == "step_per_call":
                for j in range(n):
                    sim.step(poses[k + j], dt)
            elif mode == "run":
                sim.run(poses[k:k + n], dt)
            else:
                assert sim.run_until_force(poses[k:k + n], dt, math.inf) == n
            sim.sync()
            res[mode + "_us_per_substep"] = (time.perf_counter() - t0) / n * 1e6
            k += n
        if name.startswith("gelsight"):
            # the grid update (where the contact model acts) under no-slip and
            # Coulomb contact, mid-press, from the library's HIP events
            for model, label in ((Sim.STICKY, "sticky"), (Sim.COULOMB, "coulomb")):
                sim.set_contact(model, 0.3)
                sim.timing_enable(("grid",))
                sim.timing_read(reset=True)
                sim.run(poses[k:k + n], dt)
                sim.sync()
                g = sim.timing_read(reset=True)["grid"]
                res[f"grid_ms_{label}"] = g[0] / max(1, g[1])
                k += n
            sim.timing_enable(())
            sim.set_contact(Sim.STICKY)
            # the indenter as 1e4 / 1e5 / 1e6 points (the paper's three point
            # cloud densities), 0.5 mm shell of the press's sphere
            m = wl["cfg"]["rho"] * (wl["cfg"]["block_size"][0] / wl["cfg"]["n"][0]) ** 3
            for npts in (10_000, 100_000, 1_000_000):
                sim.set_indenter_points(W.sphere_points(wl["cfg"]["sp"][0], npts, 0.5e-3, 0), 10 * m)
                sim.sync()
                sim.timing_enable(("grid",))
                sim.timing_read(reset=True)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                sim.run(poses[k:k + n], dt)
                sim.sync()
                res[f"points_{npts}_us_per_substep"] = (time.perf_counter() - t0) / n * 1e6
                g = sim.timing_read(reset=True)["grid"]
                # clear + scatter + grid update
                res[f"grid_ms_points_{npts}"] = g[0] / max(1, g[1])
                k += n
            sim.timing_enable(())
            sim.set_indenter_points(np.zeros((0, 3)), 0.0)
        res["particles"] = sim.N
        sim.close()
        out[name] = res
    return out


def batch_leg(n=256, substeps=2000):
    """The uneven batch: n contacts (particle counts log-uniform in 2e4-4e5,
    corotated material, tilted indenters; seeds 0 .. n-1) advanced together
    through their whole presses by graph-captured batched launches. Creation
    runs the tuner (a fresh cache: every (material, size class) is timed over
    all its settings) and is reported apart; the timed region is the run."""
    import collections
    import tempfile
    import torch
    from paper_2301_08343_amd import workloads as W
    from paper_2301_08343_amd.batch import Batch
    contacts = [W.batch_contact(seed, steps=substeps) for seed in range(n)]
    with tempfile.TemporaryDirectory() as d:
        cache = os.path.join(d, "tune.json")
        t0 = time.perf_counter()
        b = Batch(contacts, substeps, tune_cache=cache, tune=True)
        b.sync()
        setup = time.perf_counter() - t0
        with open(cache) as fh:
            table = json.load(fh)["entries"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.run(substeps)
    b.sync()
    el = time.perf_counter() - t0
    total = sum(c["particles"] for c in contacts)
    tuning = b.tuning()
    us_tuned, us_default = b.tuning_check()
    choices = collections.Counter(f"B{t}_wg{w}_ipw{q}" for t, w, q, _ in tuning)
    fallbacks = sum(b.contact(i).polar_fallbacks() for i in range(n))
    b.close()
    classes = collections.Counter(int(math.floor(math.log2(W.lattice_count(c["cfg"])))) for c in contacts)
    tuner = [{"model": e["model"], "log2n": e["log2n"], "contacts": classes.get(e["log2n"], 0),
              "chosen": f"B{e['tile']}_wg{e['wg']}_ipw{e['ipw']}", "us_per_substep": e["us_per_substep"],
              "candidates_us": {f"B{c[0]}_wg{c[1]}_ipw{c[2]}": c[3] for c in e["candidates"]}}
             for e in sorted(table, key=lambda e: (e["model"], e["log2n"]))]
    return {"contacts": n, "particles": total, "substeps": substeps,
            "particle_substeps_per_s": total * substeps / el, "seconds": el, "setup_seconds_with_tuning": setup,
            "polar_fp64_fallbacks": fallbacks, "tuner_choices": dict(choices), "tuner_table": tuner,
            "tuner_batch_check_us_per_substep": {"tuned": us_tuned, "default_everywhere": us_default,
                                                 "kept": "tuned" if us_tuned <= us_default else "default"}}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_worker(seed, budget_s):
    """One oracle process on one uneven-batch contact (corotated, tilted
    indenter) for about budget_s seconds; prints its rate as JSON."""
    import oracle
    from paper_2301_08343_amd import workloads as W
    wl = W.batch_contact(seed, steps=2000)
    sim = oracle.OracleSim(wl["cfg"], wl["poses"][0])
    t0 = time.perf_counter()
    k = 0
    while time.perf_counter() - t0 < budget_s and k + 1 < len(wl["poses"]):
        st = sim.step(wl["poses"][k + 1], wl["dt"])
        if st != 0:
            raise RuntimeError(f"oracle failed with status {st}")
        k += 1
    el = time.perf_counter() - t0
    print(json.dumps({"seed": seed, "particles": int(sim.N), "substeps": k, "seconds": el}), flush=True)


def cpu_all_cores(budget_s):
    """The oracle on every host core at once: one process per core, each on
    its own contact of the uneven batch (independent contacts, the way the
    CPU would serve a batch); the aggregate of their rates."""
    import subprocess
    nproc = os.cpu_count() or 1
    procs = min(16, nproc)  # the host share one GPU's job may use
    env = dict(os.environ, OMP_NUM_THREADS="1")
    runs = [subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-worker", str(seed),
                              "--cpu-seconds", str(budget_s)], stdout=subprocess.PIPE, text=True, env=env)
            for seed in range(procs)]
    rates, parts = [], []
    for r in runs:
        out, _ = r.communicate()
        if r.returncode != 0:
            raise RuntimeError(f"oracle worker failed with status {r.returncode}")
        d = json.loads(out.strip().splitlines()[-1])
        rates.append(d["particles"] * d["substeps"] / d["seconds"])
        parts.append(d["particles"])
    return {"value": sum(rates), "unit": "particle-substeps/s", "processes": procs, "nproc": nproc,
            "sample": f"{procs} uneven-batch contacts (seeds 0-{procs - 1}, {min(parts)}-{max(parts)} particles, "
                      f"corotated), one oracle process each, ~{budget_s:.0f} s"}


def cpu_baseline(wl, budget_s):
    """The FP64 oracle (single thread) on the same workload for as many
    substeps as fit in about `budget_s` seconds; then the same oracle on all
    host cores at once (independent contacts)."""
    import oracle
    oracle.build(force=False)
    sim = oracle.OracleSim(wl["cfg"], wl["poses"][0])
    n = int(sim.N)
    t0 = time.perf_counter()
    k = 0
    while True:
        st = sim.step(wl["poses"][k + 1], wl["dt"])
        if st != 0:
            raise RuntimeError(f"oracle failed with status {st}")
        k += 1
        if time.perf_counter() - t0 > budget_s or k + 1 >= len(wl["poses"]):
            break
    el = time.perf_counter() - t0
    del sim
    # and the 18,432-particle sphere press (the FP64 parity workload), 200 substeps
    from paper_2301_08343_amd import workloads as W
    sw = W.small_sphere_contact(seed=0, steps=1000)
    small = oracle.OracleSim(sw["cfg"], sw["poses"][0])
    t1 = time.perf_counter()
    small.run(sw["poses"], sw["dt"], 0, 200)
    el_small = time.perf_counter() - t1
    return {"value": n * k / el, "unit": "particle-substeps/s", "cores": 1, "kind": "oracle",
            "sample": f"first {k} substeps of the same {n}-particle press, FP64, one thread",
            "nproc": os.cpu_count(), "cpu_model": cpu_model(),
            "sphere_18k_fp64_value": int(small.N) * 200 / el_small,
            "all_cores": cpu_all_cores(budget_s)}


def family_presses(tile, substeps=50, frames=40):
    """The whole 2000-substep GelSight press of each other indenter family
    (seeds 1-4: flat punch, cone, edge, textured plate), frames of 50
    substeps with the depth map and the image, one timed run each."""
    import torch
    from paper_2301_08343_amd import workloads as W
    from paper_2301_08343_amd.sim import Sim
    out = {}
    for seed in (1, 2, 3, 4):
        wl = W.gelsight_contact(seed=seed, steps=substeps * frames)
        sim = Sim(wl["cfg"], wl["poses"][0], precision="f32", tile=tile)
        sim.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for f in range(frames):
            sim.run(wl["poses"][f * substeps + 1:(f + 1) * substeps + 1], wl["dt"])
            sim.heightmap()
            sim.render(wl["render"])
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out[W.SHAPE_NAMES[wl["cfg"]["shape"]]] = {
            "particle_substeps_per_s": sim.N * substeps * frames / el, "ms_per_step": el * 1e3 / frames,
            "depth_m": wl["depth"], "polar_fp64_fallbacks": sim.polar_fallbacks()}
        sim.close()
    return out


def active_nodes(x, cfg):
    """Grid nodes inside some particle's 3 x 3 x 3 stencil (x: [N][3] m)."""
    import numpy as np
    g0, g1, g2 = cfg["gn"]
    base = np.floor((x - np.array(cfg["grid_origin"])) / cfg["dx"] - 0.5).astype(np.int64)
    mark = np.zeros(g0 * g1 * g2, dtype=bool)
    for a in range(3):
        for b in range(3):
            for c in range(3):
                mark[((base[:, 2] + c) * g1 + base[:, 1] + b) * g0 + base[:, 0] + a] = True
    return int(mark.sum())


def surrogate_steps(n):
    """The surrogate's own kernels alone: n training steps (forward, backward,
    AdamW) and n forward passes at batch 256 on random data."""
    import torch
    from paper_2301_08343_amd.surrogate import Net, forward_flops
    torch.cuda.set_device(0)
    net = Net(batch=256, seed=0)
    g = torch.Generator(device="cuda").manual_seed(0)
    x = torch.randn(256, 64, 64, 2, device="cuda", generator=g)
    y = torch.randn(256, 64, 64, 3, device="cuda", generator=g)
    for _ in range(3):
        net.train_step(x, y, 1e-3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(n):
        net.train_step(x, y, 1e-3)
    torch.cuda.synchronize()
    ts = (time.perf_counter() - t0) / n
    t0 = time.perf_counter()
    for _ in range(n):
        net.forward(x)
    torch.cuda.synchronize()
    tf = (time.perf_counter() - t0) / n
    f = forward_flops()
    # per forward convolution: HIP events on the launching stream around each
    # layer of one extra forward pass (median of 5 passes)
    runs = []
    for _ in range(5):
        net.layer_timer = []
        net.forward(x)
        torch.cuda.synchronize()
        runs.append(net.layer_timer)
    net.layer_timer = None
    peak_tf, peak_gbs = 2500.0, HBM_PEAK_GBS
    layers = []
    for k, (name, _, nb, r, cin_p, co, taps, z, _, _) in enumerate(runs[0]):
        ms = sorted(run[k][8].elapsed_time(run[k][9]) for run in runs)[2]
        ci = next(c for nm, c, _, _ in net.specs if nm == name)
        flops = 2.0 * nb * r * r * co * taps * ci
        # input read once, output (and the stored pre-activation) written once, weights once
        nbytes = 2.0 * nb * r * r * (cin_p + co * (2 if z else 1)) + 2.0 * co * taps * cin_p
        ai = flops / nbytes
        bound = "mfma" if ai > peak_tf * 1e12 / (peak_gbs * 1e9) else "hbm"
        tfs, gbs = flops / (ms * 1e-3) / 1e12, nbytes / (ms * 1e-3) / 1e9
        layers.append({"layer": name, "pixels": r * r, "cin": ci, "cout": co, "us": ms * 1e3, "tflops": tfs,
                       "GBps": gbs, "flop_per_byte": ai, "bound": bound,
                       "frac": tfs / peak_tf if bound == "mfma" else gbs / peak_gbs})
    return {"metric": "surrogate training samples/s", "value": 256 / ts, "unit": "samples/s",
            "train_step_ms": ts * 1e3, "train_tflops": 3 * f * 256 / ts / 1e12,
            "forward_ms": tf * 1e3, "forward_tflops": f * 256 / tf / 1e12, "batch": 256, "steps": n,
            "peak_tflops_bf16_dense": peak_tf, "dtype": "bf16 storage, fp32 accumulation", "layers": layers}


def main():
    args = parse()
    if args.cpu_worker >= 0:
        cpu_worker(args.cpu_worker, args.cpu_seconds)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "multi-GPU sharding is not built", file=sys.stderr)
        sys.exit(2)
    if args.surrogate_steps > 0:
        print(json.dumps(surrogate_steps(args.surrogate_steps)), flush=True)
        return
    import numpy as np
    import torch
    from paper_2301_08343_amd import workloads as W
    from paper_2301_08343_amd.sim import Sim

    S = args.substeps
    # the press reaches its drawn depth after 2000 substeps; longer runs hold it
    wl = W.gelsight_contact(seed=args.seed, steps=2000)
    cfg, dt, rp = wl["cfg"], wl["dt"], wl["render"]
    need = max(args.warmup, args.steps) * S + 1
    poses = np.concatenate([wl["poses"], np.repeat(wl["poses"][-1:], max(0, need - len(wl["poses"])), 0)])
    torch.cuda.set_device(0)
    if args.calibrate_copy_mib:
        n = args.calibrate_copy_mib << 18
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def frame(sim, f):
        sim.run(poses[f * S + 1:(f + 1) * S + 1], dt)
        sim.heightmap()
        return sim.render(rp)

    warm = Sim(cfg, poses[0], precision="f32", tile=args.tile)
    for f in range(args.warmup):
        frame(warm, f)
    warm.sync()
    warm.close()
    del warm
    sim = Sim(cfg, poses[0], precision="f32", tile=args.tile)
    N = sim.N
    sim.sync()
    sim.timing_read(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for f in range(args.steps):
        # kernel events on every TIMING_EVERY-th frame: events around every
        # launch of every frame cost the frame 7 % (measured), every fifth 1 %
        sim.timing_enable(TIMED_KERNELS if f % TIMING_EVERY == 0 else ())
        img = frame(sim, f)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    timing = sim.timing_read(reset=True)
    sim.timing_enable(())
    sim.sync()
    # active grid nodes and blocks of the final state (outside the timed region)
    x, _, _, _ = sim.read_particles()
    xs = x.double().cpu().numpy().T
    nodes = active_nodes(xs, cfg)
    cell = np.floor((xs - np.array(cfg["grid_origin"])) / cfg["dx"]).astype(np.int64) // args.tile
    active = len(np.unique(cell[:, 0] + 4096 * (cell[:, 1] + 4096 * cell[:, 2])))
    assert bool(torch.isfinite(img).all())

    value = N * S * args.steps / el
    k_ms = {k: timing[k][0] / max(1, timing[k][1]) for k in TIMED_KERNELS}
    dom = max(k_ms, key=lambda k: timing[k][0])
    per_kernel = {}
    for k in TIMED_KERNELS:
        b = BYTES_PER_PARTICLE[k] * N + BYTES_PER_ACTIVE_NODE[k] * nodes
        per_kernel[k] = {"algorithmic_bytes_per_launch": b, "avg_launch_ms": k_ms[k],
                         "achieved": b / (k_ms[k] * 1e-3) / 1e9, "launches": timing[k][1],
                         "traffic": committed_traffic(k), "valu_issue_frac": valu_issue_frac(k, k_ms[k]),
                         "design_bytes_per_launch": design_bytes(k, N, active, args.tile)}
    algo_bytes = per_kernel[dom]["algorithmic_bytes_per_launch"]
    achieved = per_kernel[dom]["achieved"]
    # a plain device copy of 1 GiB (read + write) as the measured bandwidth
    # ceiling beside the 8 TB/s nameplate (after the timed region; left out
    # of counter-calibration runs, whose only large copy is the calibration)
    copy_gbs = None
    if not args.calibrate_copy_mib:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(2):
            dst.copy_(src)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            dst.copy_(src)
        e1.record()
        e1.synchronize()
        copy_gbs = 2 * src.numel() * 4 * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e9
        del src, dst
    for k in per_kernel:
        per_kernel[k]["frac"] = per_kernel[k]["achieved"] / HBM_PEAK_GBS
        per_kernel[k]["frac_of_copy"] = per_kernel[k]["achieved"] / copy_gbs if copy_gbs else None
    out = {
        "metric": "MPM particle-substeps/s",
        "value": value,
        "unit": "particle-substeps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"gelsight_press_{W.SHAPE_NAMES[cfg['shape']]}_1.6M_fp32",
                   "particles": N, "lattice": list(cfg["n"]), "grid": list(cfg["gn"]),
                   "substeps_per_step": S, "dt": dt, "depth_m": wl["depth"],
                   "heightmap": [cfg["n"][1], cfg["n"][0]], "image": [rp["h"], rp["w"]],
                   "tile": args.tile},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": committed_traffic(dom),
                     "avg_launch_ms": k_ms[dom], "algorithmic_bytes_per_launch": algo_bytes,
                     "bytes_per_particle": BYTES_PER_PARTICLE, "bytes_per_active_node": BYTES_PER_ACTIVE_NODE,
                     "particles": N, "active_nodes": nodes, "active_blocks": active,
                     "copy_GBps": copy_gbs, "frac_of_copy": achieved / copy_gbs if copy_gbs else None,
                     "substep_GBps": sum(per_kernel[k]["algorithmic_bytes_per_launch"] for k in TIMED_KERNELS)
                     * value / N / 1e9,
                     "kernels": per_kernel},
        "kernel_ms": {k: v[0] / max(1, v[1]) for k, v in timing.items() if v[1]},
        "kernel_timing_every_nth_frame": TIMING_EVERY,
    }
    if not args.no_cpu_baseline:
        wl_cpu = W.gelsight_contact(seed=args.seed, steps=2000)
        out["cpu_baseline"] = cpu_baseline(wl_cpu, args.cpu_seconds)
    else:
        out["cpu_baseline"] = None
    del sim
    torch.cuda.empty_cache()
    out["families"] = None if args.no_families else family_presses(args.tile, S)
    out["streaming"] = None if args.no_streaming else streaming_leg()
    out["batch"] = None if args.no_batch else batch_leg()
    if not args.no_surrogate and os.path.exists(args.surrogate):
        out["surrogate"] = surrogate_leg(args)
    if not args.no_surrogate:
        # the surrogate's training step on its own (batch 256, random data);
        # the per-layer table is printed by --surrogate-steps
        tr = surrogate_steps(10)
        out["surrogate_training"] = {k: v for k, v in tr.items() if k != "layers"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
