"""Throughput of the EC PIC/MCC hot path on one MI355X.

A step is one pass of the whole hot path over the discharge: EC gather, push,
electrode absorption, null-collision MCC, int64 deposit and the FP64 field
solve of every case, plus the periodic compaction/cell sort.  Inputs are
synthetic and already resident in HBM when the timed region starts.

Prints one JSON line.  Default workload: the production-size explicit RF
discharge (2048 cells, 1e7 electrons + 1e7 ions, 30 mTorr, 300 V at
13.56 MHz, dt = 1/(2000 f)).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
# Algorithmic bytes of the particle pass (k_step) per particle-step: read the
# cell word, offset and vx, write them back (4 B each); the implicit pass also
# reads and writes abar.  Per listed collision candidate: slot and v (8 B; the
# implicit list also carries abar, 4 B).
PASS_BYTES = {0: 24, 1: 32}
LIST_BYTES = {0: 8, 1: 12}
# Algorithmic bytes of the collision kernel (k_collide) per candidate: the
# list entry, the cell word, offset, id, vy, vz of the slot (24 B) and the
# velocity and cell word written back (8 B).
COLLIDE_BYTES = {0: 40, 1: 52}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_workload(name, scale):
    import workloads as W
    if name == "ccp2048_explicit":
        return [W.c4(np_per_species=int(10_000_000 * scale))]
    if name == "ccp64_explicit":
        return [W.c1()]
    if name == "ccp256_implicit":
        return [W.c3()]
    if name == "sweep64":
        return W.c5(np_scale=scale)
    raise SystemExit(f"unknown workload {name}")


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("pic_kernels.hip", "pic_common.hpp", "pic_device.hpp"):
        with open(os.path.join(ROOT, "paper_1310_5284_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE scaled by the copy calibration), or None when
    the summary is for another workload or the kernel sources changed since."""
    name = kernel.split("<")[0]
    path = os.path.join(ROOT, "profiles", f"{name}_{workload}_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel") != kernel or kv.get("source_hash") != kernel_source_hash():
        return None
    try:
        return int(float(kv["bytes_per_launch"]))
    except (KeyError, ValueError):
        return None


def cpu_baseline(wl, steps_budget_s=12.0, frac=0.05):
    """The FP64 oracle (single thread) on a particle sample of the workload."""
    import numpy as np

    import oracle
    import workloads as W
    case, sps, procs = W.to_oracle(wl)
    rng = np.random.default_rng(1)
    sub = []
    for sp in sps:
        n = sp["xi"].size
        k = max(1, int(n * frac))
        idx = np.sort(rng.choice(n, size=k, replace=False)) if n else np.zeros(0, int)
        d = dict(sp)
        for key in ("xi", "vx", "vy", "vz", "id"):
            d[key] = sp[key][idx]
        d["abar"] = None
        d["w"] = sp["w"] / frac          # same densities with fewer particles
        sub.append(d)
    sim = oracle.Sim(case, sub, procs)
    sim.step(2)
    n_ps = 0
    steps = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < steps_budget_s:
        n_ps += sim.count(0) + sim.count(1)
        sim.step(1)
        steps += 1
    dt = time.perf_counter() - t0
    return dict(value=n_ps / dt, unit="particle-steps/s", cores=1, kind="oracle",
                sample=f"{frac:g} of the particles of the same discharge (weights scaled "
                       f"to keep the densities), {steps} steps, FP64, single thread")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="ccp2048_explicit")
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--tile", type=int, default=0, help="particles per workgroup (default 16384)")
    ap.add_argument("--sort-every", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--fp64-steps", type=int, default=20,
                    help="steps of the plain FP64 GPU form timed for comparison (0: skip)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run the streaming copy kernel of BYTES and print its rate")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(multi-GPU sharding is described in DESIGN.md but not built)", file=sys.stderr)
        sys.exit(2)

    import paper_1310_5284_amd as P

    if args.copy_calibration:
        ms = P.copy_calibration(args.copy_calibration, reps=10)
        print(json.dumps(dict(calibration="copy", bytes_read=args.copy_calibration,
                              bytes_written=args.copy_calibration, ms_per_copy=ms,
                              GBps=2 * args.copy_calibration / (ms * 1e-3) / 1e9)), flush=True)
        return

    log(f"[bench] building inputs: {args.workload} scale {args.scale}")
    wls = make_workload(args.workload, args.scale)
    log("[bench] pic_init")
    ctx = P.PicContext(wls)
    tile = args.tile or 16384
    sort_every = args.sort_every or 64
    ctx.set_schedule(sort_every=sort_every, diag_every=0, tile=tile)
    implicit = all(w["case"]["scheme"] == 1 for w in wls)
    stepper = ctx.step

    def live():
        return sum(sum(ctx.counts(k)["n"]) for k in range(len(wls)))

    log(f"[bench] warmup {args.warmup} steps")
    done = 0
    while done < args.warmup:
        k = min(50, args.warmup - done)
        stepper(k)
        done += k
        log(f"[bench] warmup {done}/{args.warmup}")
    n_before = live()
    ctx.sync()
    log(f"[bench] timing {args.steps} steps, {n_before} particles")
    t0 = time.perf_counter()
    stepper(args.steps)
    ctx.sync()
    t1 = time.perf_counter()
    kern_ms, launches = ctx.last_timing()
    coll_ms, coll_launches = ctx.last_timing_collide()
    n_after = live()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    particles = 0.5 * (n_before + n_after)
    value = particles * args.steps / (t1 - t0)

    # candidates of the last step (ledger), as the per-step count
    sch = 1 if implicit else 0
    cands = sum(int(sum(ctx.ledger(k)["n_candidates"])) for k in range(len(wls)))
    avg_launch_s = kern_ms / 1e3 / max(launches, 1)
    launches_per_step = launches / args.steps
    alg_bytes = (PASS_BYTES[sch] * particles + LIST_BYTES[sch] * cands) / launches_per_step
    achieved = alg_bytes / avg_launch_s / 1e9
    roof = dict(bound="hbm", achieved=round(achieved, 1), peak=PEAK_HBM_GBS, unit="GB/s",
                frac=round(achieved / PEAK_HBM_GBS, 4), traffic=None,
                kernel="k_step<%d,false>" % sch,
                avg_launch_ms=round(avg_launch_s * 1e3, 4),
                alg_bytes_per_launch=int(alg_bytes),
                alg_bytes_rule="%d B per particle + %d B per listed candidate"
                               % (PASS_BYTES[sch], LIST_BYTES[sch]))
    coll_avg_s = coll_ms / 1e3 / max(coll_launches, 1)
    coll_bytes = COLLIDE_BYTES[sch] * cands / max(coll_launches / args.steps, 1e-9)
    collide = dict(kernel="k_collide<%d,false>" % sch, avg_launch_ms=round(coll_avg_s * 1e3, 4),
                   candidates_per_step=cands,
                   achieved_GBps=round(coll_bytes / max(coll_avg_s, 1e-12) / 1e9, 1),
                   alg_bytes_rule="%d B per candidate" % COLLIDE_BYTES[sch])
    roof["traffic"] = measured_traffic(args.workload, roof["kernel"])

    out = dict(metric="particle-steps/sec (push+deposit+MCC) vs plain FP64 GPU form at "
                      "matched EEDF",
               value=value, unit="particle-steps/s", n_gpus=1, steps=args.steps,
               warmup=args.warmup, ms_per_step=ms_per_step, higher_is_better=True,
               scaling="weak", vs_baseline=None, dtype="f32",
               data="synthetic",
               config=dict(workload=args.workload, cases=len(wls),
                           cells=[w["case"]["n_cells"] for w in wls][:4],
                           particles=int(particles), tile=tile, sort_every=sort_every,
                           scheme="implicit" if implicit else "explicit"),
               roofline=roof, collide=collide)
    if args.fp64_steps > 0 and not implicit:
        # the plain FP64 GPU form of the same method, from the same state
        log(f"[bench] plain FP64 GPU form: {args.fp64_steps} steps")
        ctx.fp64_init()
        ctx.fp64_step(2)
        n64 = live()
        t0 = time.perf_counter()
        ctx.fp64_step(args.fp64_steps)
        t1 = time.perf_counter()
        v64 = n64 * args.fp64_steps / (t1 - t0)
        out["fp64_gpu_form"] = dict(value=v64, unit="particle-steps/s",
                                    ms_per_step=(t1 - t0) * 1e3 / args.fp64_steps,
                                    steps=args.fp64_steps)
        out["speedup_vs_fp64_form"] = value / v64
    if not args.no_cpu:
        log("[bench] cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(wls[0], args.cpu_seconds)
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
