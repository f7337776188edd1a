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
# reads and writes abar.  Per listed collision candidate: slot, v and the cell
# word of x_{n+1} (12 B); the implicit list also carries abar and the offset.
PASS_BYTES = {0: 24, 1: 32}
LIST_BYTES = {0: 12, 1: 20}
# Algorithmic bytes of the collision kernel (k_collide) per candidate: read the
# list entry and the 16-byte record (id, vy, vz), write the cell word back
# (explicit: 12 + 16 + 4; implicit: 20 + 16 + cell word, offset, vx, abar).
# Per real collision the new velocity is written: vx, vy, vz explicit (the
# implicit pass rewrites vx anyway, so vy, vz only).
COLLIDE_BYTES = {0: 32, 1: 52}
COLLISION_BYTES = {0: 12, 1: 8}
# Bytes per particle-step of a plain streaming form of the method that reads
# every particle's whole state each step (the whole-step comparison figure).
STREAM_BYTES = {0: 40, 1: 48}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_workload(name, scale):
    import workloads as W
    if name == "ccp2048_explicit":
        return [W.c4(np_per_species=int(10_000_000 * scale))]
    if name == "ccp2048_mc":
        # the same discharge with the momentum-conserving gather (scheme (1))
        wl = W.c4(np_per_species=int(10_000_000 * scale))
        wl["case"]["gather"] = 1
        return [wl]
    if name == "ccp2048_mc_implicit":
        # the D1 implicit discharge with the momentum-conserving gather
        wl = W.c4(np_per_species=int(10_000_000 * scale), scheme=1)
        wl["case"]["gather"] = 1
        return [wl]
    if name == "ccp2048_ec2":
        # the same discharge with m = 2 weighting (quadratic deposit)
        wl = W.c4(np_per_species=int(10_000_000 * scale))
        wl["case"]["gather"] = 2
        return [wl]
    if name == "ccp2048_implicit":
        # the same discharge stepped by the D1 implicit scheme
        return [W.c4(np_per_species=int(10_000_000 * scale), scheme=1)]
    if name == "ccp2048_ec2_implicit":
        # D1 implicit with m = 2 weighting (quadratic deposit, susceptibility
        # of the dual grid)
        wl = W.c4(np_per_species=int(10_000_000 * scale), scheme=1)
        wl["case"]["gather"] = 2
        return [wl]
    if name == "ccp2048_nonuniform":
        # the same discharge on a sheath-refined grid (cells about 4x narrower
        # within 15 % of the gap from either electrode)
        return [W.c4(np_per_species=int(10_000_000 * scale),
                     cell_dx=W.sheath_refined_widths(2048, 0.025))]
    if name == "ccp2048_nonuniform_ec2_implicit":
        # D1 implicit with m = 2 weighting on the sheath-refined grid
        wl = W.c4(np_per_species=int(10_000_000 * scale), scheme=1,
                  cell_dx=W.sheath_refined_widths(2048, 0.025))
        wl["case"]["gather"] = 2
        return [wl]
    if name == "ccp2048_subcycle8":
        # the same discharge with the ions pushed every 8th step with 8 dt
        wl = W.c4(np_per_species=int(10_000_000 * scale))
        wl["case"]["ion_subcycle"] = 8
        return [wl]
    if name == "ccp2048_implicit_subcycle8":
        # the D1 implicit discharge with the ions pushed every 8th step with 8 dt
        wl = W.c4(np_per_species=int(10_000_000 * scale), scheme=1)
        wl["case"]["ion_subcycle"] = 8
        return [wl]
    if name == "ccp64_explicit":
        return [W.c1()]
    if name == "ccp256_implicit":
        # omega_p dt = 2: at 5 the D1 discharge heats and ionizes without bound
        wl = W.c3(wdt=2.0)
        for sp in wl["species"]:
            sp["capacity"] = 2 * sp["cell"].size
        return [wl]
    if name == "sweep64":
        # room for the ionization growth of the high-pressure cases over the
        # autotuning, warm-up and timed steps
        wls = W.c5(np_scale=scale)
        for wl in wls:
            for sp in wl["species"]:
                sp["capacity"] = 3 * max(sp["cell"].size, 16) + 64
        return wls
    raise SystemExit(f"unknown workload {name}")


def kernel_source_hash():
    """sha256 (first 16 hex) of the sources of the particle kernels (k_step,
    k_collide and the helpers they include) with comments and blank space
    removed: a comment edit does not change the kernels."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in ("pic_step.hip", "pic_weights.hpp", "pic_common.hpp", "pic_device.hpp"):
        with open(os.path.join(ROOT, "paper_1310_5284_amd", "csrc", f)) as fh:
            t = fh.read()
        t = re.sub(r"/\*.*?\*/", " ", t, flags=re.S)
        t = re.sub(r"//[^\n]*", " ", t)
        h.update(" ".join(t.split()).encode())
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


def _oracle_sample(wl, frac):
    """A particle sample of the workload in the oracle's form (same densities)."""
    import numpy as np

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
    return case, sub, procs


def _oracle_rate(case, sub, procs, budget_s):
    """Particle-steps per second of the FP64 oracle (one thread) on a sample."""
    import oracle
    sim = oracle.Sim(case, sub, procs)
    sim.step(2)
    n_ps = steps = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        n_ps += sim.count(0) + sim.count(1)
        sim.step(1)
        steps += 1
    return n_ps / (time.perf_counter() - t0), steps


def cpu_baseline(wl, steps_budget_s=12.0, frac=0.05, where="the same discharge", max_procs=16):
    """The FP64 oracle on a particle sample of the workload, as it stands (one
    thread per process): one process per usable host core (at most
    max_procs), each stepping the same sample; value = their summed rate."""
    import multiprocessing as mp
    case, sub, procs = _oracle_sample(wl, frac)
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:
        ncpu = os.cpu_count() or 1
    n = max(1, min(ncpu, max_procs))
    try:
        with mp.get_context("spawn").Pool(n) as pool:
            job = pool.starmap_async(_oracle_rate, [(case, sub, procs, steps_budget_s)] * n)
            res = job.get(timeout=steps_budget_s + 120.0)   # a worker that died raises here
    except Exception as e:   # no child processes here: one thread in this one
        log(f"[bench] oracle processes failed ({e}); timing one thread")
        n = 1
        res = [_oracle_rate(case, sub, procs, steps_budget_s)]
    rates = [r for r, _ in res]
    return dict(value=sum(rates), unit="particle-steps/s", cores=n, kind="oracle",
                per_core_value=sum(rates) / n,
                sample=f"{frac:g} of the particles of {where} (weights scaled "
                       f"to keep the densities), FP64, {n} single-thread processes "
                       f"stepping it for {steps_budget_s:g} s each "
                       f"({min(s for _, s in res)}-{max(s for _, s in res)} steps); "
                       f"{ncpu} usable host cores")


def drift_table(P, steps, fp64_steps=0):
    """Total-energy drift of the periodic thermal plasma (512 cells, 1000
    electrons per cell on a fixed neutralising background) on the GPU path,
    EC (m = 1 and m = 2) and MC weightings, dx / lambda_D = 0.5, 5, 20 at omega_p dt = 0.2, and at
    dx = 5 lambda_D also omega_p dt = 0.1 and 0.05 over the same time.  The
    energy at integer steps is the mean of the kinetic energies of the two
    half steps plus the field energy; drift = slope of E / E_0 per step
    (least squares over about 200 samples), err = max |E / E_0 - 1|.  With
    fp64_steps > 0 the plain FP64 GPU form runs the EC and MC rows too, from
    the same initial state, over fp64_steps steps at omega_p dt = 0.2 (the
    same time at the smaller steps)."""
    import numpy as np

    import workloads as W
    rows = []
    for ratio in (0.5, 5.0, 20.0):
        for gather in (0, 1, 2):
            for wdt in ((0.2, 0.1, 0.05) if ratio == 5.0 else (0.2,)):
                n = int(round(steps * 0.2 / wdt))
                every = max(1, n // 200)
                wl = W.c2(ratio=ratio, gather=gather, ppc=1000, n_cells=512, wdt=wdt)
                ctx = P.PicContext([wl])
                ctx.set_schedule(sort_every=64, diag_every=0, tile=4096)
                ctx.set_launch(graph=0, timing_every=0)
                t0 = time.perf_counter()
                xs, es = [], []
                done = 0
                while done < n:
                    k = min(every, n - done)
                    ctx.step(k)
                    done += k
                    L = ctx.ledger()
                    xs.append(done)
                    es.append(0.5 * (L["K_before"][0] + L["K_after"][0]) + L["WE"])
                dt_s = time.perf_counter() - t0
                e = np.array(es) / es[0]
                row = dict(dx_over_lambda_D=ratio, gather=("EC", "MC", "EC2")[gather],
                           omega_p_dt=wdt, steps=n,
                           drift_per_step=float(np.polyfit(xs, e, 1)[0]),
                           max_rel_err=float(np.abs(e - 1.0).max()),
                           steps_per_s=n / dt_s)
                if gather != 2 and fp64_steps > 0:
                    # the plain FP64 GPU form from the same initial state
                    ctx.close()
                    ctx = P.PicContext([wl])
                    ctx.fp64_init()
                    n64 = int(round(fp64_steps * 0.2 / wdt))
                    ev64 = max(1, n64 // 200)
                    xs64, es64 = [], []
                    done = 0
                    t0 = time.perf_counter()
                    while done < n64:
                        k = min(ev64, n64 - done)
                        ctx.fp64_step(k)
                        done += k
                        L = ctx.fp64_ledger()
                        xs64.append(done)
                        es64.append(0.5 * (L["K_before"][0] + L["K_after"][0]) + L["WE"])
                    t64 = time.perf_counter() - t0
                    e64 = np.array(es64) / es64[0]
                    row["fp64"] = dict(steps=n64, drift_per_step=float(np.polyfit(xs64, e64, 1)[0]),
                                       max_rel_err=float(np.abs(e64 - 1.0).max()),
                                       steps_per_s=n64 / t64)
                ctx.close()
                rows.append(row)
                log(f"[bench] drift {rows[-1]}")
    return dict(measurement="energy drift, periodic thermal plasma, GPU path", rows=rows)


def batch_record(P, steps=256, seq_steps=64):
    """The 64-case batch (sweep64: 128-1024 cells, 1e4-2e6 particles per
    species, explicit and implicit mixed) stepped by one context, against the
    same cases stepped one context after another (the sequential per-case
    baseline).  Both at tile 16384 and sort period 128, timed over whole sort
    periods after a warm-up; the batch with the collision kernel's store
    policy that the autotuner picks for it (the sequential contexts keep the
    default); returns the sub-record of the JSON line."""
    wls = make_workload("sweep64", 1.0)
    schemes = [int(w["case"]["scheme"]) for w in wls]

    policy = [None]

    def run(ctx_wls, n, warm, tune=False):
        ctx = P.PicContext(ctx_wls)
        ctx.set_schedule(sort_every=1, diag_every=0, tile=16384)
        ctx.set_launch(graph=0, timing_every=0)
        ctx.step(warm)
        if tune:
            # one tile and one period: the trials that count are the store policies
            _, _, ms = ctx.autotune(tiles=[16384], sorts=[128], steps_per_trial=128)
            policy[0] = dict(chosen=("cached", "nontemporal")[int(ms[3] < ms[2])],
                             ms_per_step={"cached": round(ms[2], 4),
                                          "nontemporal": round(ms[3], 4)})
        ctx.set_schedule(sort_every=128 if n % 128 == 0 else n, diag_every=0, tile=16384)
        live = lambda: [sum(ctx.counts(k)["n"]) for k in range(len(ctx_wls))]
        a = live()
        ctx.sync()
        t0 = time.perf_counter()
        ctx.step(n)
        ctx.sync()
        t = time.perf_counter() - t0
        b = live()
        ctx.close()
        return [0.5 * (x + y) for x, y in zip(a, b)], t

    log("[bench] batch: 64 cases in one context")
    per, t = run(wls, steps, 64, tune=True)
    value = sum(per) * steps / t
    stream = sum((48.0 if schemes[k] else 40.0) * per[k] for k in range(len(wls))) / sum(per)
    log("[bench] batch: the same cases one context after another")
    seq_ps = seq_t = 0.0
    for k, wl in enumerate(wls):
        pk, tk = run([wl], seq_steps, 16)
        seq_ps += pk[0] * seq_steps
        seq_t += tk
    seq = seq_ps / seq_t
    return dict(workload="sweep64", cases=len(wls), particles=int(sum(per)),
                implicit_cases=int(sum(schemes)), tile=16384, sort_every=128, steps=steps,
                store_policy=policy[0],
                ms_per_step=t * 1e3 / steps, value=value, unit="particle-steps/s",
                step_equivalent=dict(bytes_per_particle_step=round(stream, 2),
                                     GBps=round(value * stream / 1e9, 1),
                                     frac=round(value * stream / 1e9 / PEAK_HBM_GBS, 4)),
                sequential=dict(value=seq, steps_per_case=seq_steps,
                                note="each case alone in its own context, one after another"),
                speedup_vs_sequential=value / seq)


def param_study(P, periods, window=10, ppc=400, scale=1.0):
    """The paper's parameter study (Sec. III, Table 1 workload), qualitatively:
    a 1D capacitive discharge in argon-like gas at 50 mTorr, 4 cm gap, 200 V at
    27 MHz, no secondary emission, initial density 2e16 m^-3 (Te 2 eV, Ti
    0.026 eV), dt = 1.5e-11 s (2458 steps per RF period), ppc particles per
    cell and species, on grids of 800, 400, 200, 100 and 64 cells, with the
    four schemes (momentum- or energy-conserving gather x leap-frog or D1
    implicit): 20 cases in one batched context.  The synthetic cross sections
    stand in for the argon data, and the run covers `periods` RF periods
    instead of the paper's 16-22 thousand, so only the direction of the
    paper's findings can be checked: growth of the macro-particle count and
    heating of the electrons where the momentum-conserving gather meets
    dx > 3 lambda_D, the energy-conserving cases staying bounded, and the
    trends of the density and of the heating peak with dx.  Returns the
    per-case histories (per RF period) and window averages."""
    import numpy as np

    import workloads as W
    freq, volts, gap, p_mtorr, n0, dt = 27.12e6, 200.0, 0.04, 50.0, 2e16, 1.5e-11
    per = int(round(1.0 / (freq * dt)))
    grids = (800, 400, 200, 100, 64)
    schemes = [("MC", "explicit", 1, 0), ("EC", "explicit", 0, 0),
               ("MC", "implicit", 1, 1), ("EC", "implicit", 0, 1)]
    wls, tags = [], []
    k = 0
    for gname, sname, gather, scheme in schemes:
        for N in grids:
            wl = W.ccp_workload(f"table1_{gname}_{sname}_{N}", n_cells=N,
                                np_per_species=int(ppc * N * scale), gap_m=gap, volts=volts,
                                freq=freq, dt=dt, p_mtorr=p_mtorr, n0=n0, Te=2.0,
                                scheme=scheme, gather=gather, seed=0x7AB1E + k,
                                # the coarse grids may diverge (MC): room to
                                # grow, so that the batch runs its periods
                                capacity_factor=40.0 if N <= 100 else 4.0)
            wls.append(wl)
            tags.append(dict(gather=gname, scheme=sname, cells=N))
            k += 1
    lam = math.sqrt(8.8541878128e-12 * 2.0 / (n0 * 1.602176634e-19))
    ctx = P.PicContext(wls)
    ctx.set_schedule(sort_every=64, diag_every=0, tile=16384)
    ctx.set_launch(graph=0, timing_every=0)
    hist = [dict(n_e=[], n_i=[], K_e=[]) for _ in wls]
    t0 = time.perf_counter()
    for p_ in range(periods):
        if p_ == periods - window:
            ctx.reset_accumulators()
            ctx.set_schedule(sort_every=64, diag_every=1, tile=16384)
        try:
            ctx.step(per)
        except Exception as e:   # a case that outgrew its capacity ends the study
            log(f"[bench] study stopped after {p_} periods: {e}")
            break
        for c in range(len(wls)):
            cnt = ctx.counts(c)
            L = ctx.ledger(c)
            hist[c]["n_e"].append(int(cnt["n"][0]))
            hist[c]["n_i"].append(int(cnt["n"][1]))
            hist[c]["K_e"].append(float(L["K_after"][0]))
        log(f"[bench] study period {p_ + 1}/{periods} ({time.perf_counter() - t0:.0f} s): "
            + " ".join(str(h["n_e"][-1]) for h in hist))
    rows = []
    for c, tag in enumerate(tags):
        N = tag["cells"]
        dx = gap / N
        dens, ns = ctx.density(c)
        heat = ctx.heating(c)
        eedf, bin_eV, es = ctx.eedf(c)
        ne = hist[c]["n_e"]
        row = dict(tag, dx_over_lambda_D0=round(dx / lam, 2), history=hist[c])
        if ns > 0:
            de = np.asarray(dens[0])
            he = np.asarray(heat[0]) / max(ns * dt, 1e-300)   # W/m^2 per cell
            x = (np.arange(N) + 0.5) * dx
            half = N // 2
            peak = int(np.argmax(he[:half]))
            pe = eedf.reshape(-1, 2).sum(1).astype(np.float64)
            pe /= max(pe.sum(), 1.0)
            row.update(window_periods=window, n_e_peak=float(de.max()),
                       n_e_centre=float(de[N // 2]),
                       heating_peak_x_mm=float(x[peak] * 1e3),
                       absorbed_power_W_m2=float(sum(np.asarray(h).sum() for h in heat)
                                                 / max(ns * dt, 1e-300)),
                       mean_electron_eV=float((pe * (np.arange(pe.size) + 0.5) * 2 * bin_eV).sum()))
        row["growth_e"] = (ne[-1] / ne[0]) if ne and ne[0] else None
        rows.append(row)
    ctx.close()
    return dict(study="Table 1 workload, qualitative (synthetic cross sections)",
                rf_periods=periods, window_periods=window, steps_per_period=per,
                lambda_D0_m=lam, ppc=int(ppc * scale), cases=rows,
                wall_s=time.perf_counter() - t0)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # about 2000 steps (autotuning trials included) before the timed window
    ap.add_argument("--steps", type=int, default=2048)
    ap.add_argument("--warmup", type=int, default=1500)
    ap.add_argument("--workload", default="ccp2048_explicit")
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--tile", type=int, default=0, help="particles per workgroup (default 16384)")
    ap.add_argument("--sort-every", type=int, default=0)
    ap.add_argument("--autotune", type=int, default=32, metavar="STEPS",
                    help="steps per autotuning trial of tile and sort period (0: off; "
                         "off when --tile or --sort-every is given)")
    ap.add_argument("--graph", type=int, default=0, choices=(0, 1),
                    help="replay whole sort periods from a captured HIP graph")
    ap.add_argument("--timing-every", type=int, default=0,
                    help="HIP events around the kernels of every n-th step of the timed "
                         "window (they cost about 4 us each; default 0: none there, the "
                         "kernel durations come from the sample after the window)")
    ap.add_argument("--sample-steps", type=int, default=64,
                    help="untimed steps after the timed window with HIP events around "
                         "every particle and collision kernel (the roofline's durations)")
    ap.add_argument("--batch", type=int, default=1, choices=(0, 1),
                    help="also run the 64-case batch (sweep64) and its sequential "
                         "per-case baseline (default workload only)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--fp64-steps", type=int, default=20,
                    help="steps of the plain FP64 GPU form timed for comparison (0: skip)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run the streaming copy kernel of BYTES and print its rate")
    ap.add_argument("--drift", type=int, default=0, metavar="STEPS",
                    help="only measure the energy drift of the periodic thermal plasma "
                         "(512 cells, 1000 electrons per cell) over STEPS steps at "
                         "omega_p dt = 0.2 (the same time at 0.1 and 0.05)")
    ap.add_argument("--study", type=int, default=0, metavar="PERIODS",
                    help="only run the paper's parameter study (Table 1 workload, grids "
                         "800-64 x four schemes) for PERIODS RF periods")
    ap.add_argument("--drift-fp64", type=int, default=0, metavar="STEPS",
                    help="with --drift: also the plain FP64 GPU form over STEPS steps")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: one GPU only; --gpus {args.gpus} is not supported "
              "(sharding over several GPUs is designed but not built)", file=sys.stderr)
        sys.exit(2)

    import paper_1310_5284_amd as P

    if args.copy_calibration:
        ms = P.copy_calibration(args.copy_calibration, reps=10)
        print(json.dumps(dict(calibration="copy", bytes_read=args.copy_calibration,
                              bytes_written=args.copy_calibration, ms_per_copy=ms,
                              GBps=2 * args.copy_calibration / (ms * 1e-3) / 1e9)), flush=True)
        return

    if args.drift:
        print(json.dumps(drift_table(P, args.drift, args.drift_fp64)), flush=True)
        return

    if args.study:
        print(json.dumps(param_study(P, args.study, scale=args.scale)), flush=True)
        return

    log(f"[bench] building inputs: {args.workload} scale {args.scale}")
    wls = make_workload(args.workload, args.scale)
    cpu = None
    if not args.no_cpu:
        # before this process touches the GPU: the oracle runs in fresh
        # child interpreters
        log("[bench] cpu baseline (oracle)")
        cpu = cpu_baseline(wls[0], args.cpu_seconds,
                           where="the same discharge" if len(wls) == 1 else "case 0 of the batch")
    log("[bench] pic_init")
    ctx = P.PicContext(wls)
    tile = args.tile or 16384
    sort_every = args.sort_every or 64
    ctx.set_schedule(sort_every=sort_every, diag_every=0, tile=tile)
    tuned = None
    if args.autotune and not (args.tile or args.sort_every):
        # the autotuner's trials are real steps before the warm-up
        tile, sort_every, ms = ctx.autotune(steps_per_trial=args.autotune)
        tiles, sorts = (1024, 2048, 4096, 8192, 16384, 32512), (16, 32, 64, 128)
        policy = int(ms[11] < ms[10])
        tuned = dict(steps_per_trial=args.autotune,
                     tile_ms_per_step={str(t): round(m, 4) for t, m in zip(tiles, ms[:6])},
                     sort_ms_per_step={str(t): round(m, 4) for t, m in zip(sorts, ms[6:10])},
                     store_policy_ms_per_step={"cached": round(ms[10], 4),
                                               "nontemporal": round(ms[11], 4)},
                     store_policy=("cached", "nontemporal")[policy])
        log(f"[bench] autotune: tile {tile}, sort every {sort_every}, "
            f"{tuned['store_policy']} collision stores")
    schemes = [int(w["case"]["scheme"]) for w in wls]
    implicit = all(sc == 1 for sc in schemes)
    groups = len(set(schemes))          # one k_step and one k_collide launch per group
    stepper = ctx.step

    def live_per_case():
        # particle-steps per step: subcycled ions count in their push steps
        # only (1/K of them per step on average)
        out = []
        for k, w in enumerate(wls):
            n = ctx.counts(k)["n"]
            ksub = max(1, int(w["case"].get("ion_subcycle", 0)))
            out.append(n[0] + n[1] / ksub)
        return out

    def coprime(every):
        # event samples every `every`-th step: with subcycled ions that
        # period is made coprime to K, so that the samples visit every phase
        ks = [max(1, int(w["case"].get("ion_subcycle", 0))) for w in wls]
        while every > 1 and any(math.gcd(every, k) > 1 for k in ks):
            every += 1
        return every

    # The timed window runs at the tuned sort period; the default K (2048, a
    # multiple of every period the autotuner tries) makes it whole periods,
    # so that it carries its share of the compaction.
    period = sort_every
    steps = args.steps
    ctx.set_launch(graph=args.graph, timing_every=0)
    log(f"[bench] warmup {args.warmup} steps")
    done = 0
    while done < args.warmup:
        k = min(50, args.warmup - done)
        stepper(k)
        done += k
        log(f"[bench] warmup {done}/{args.warmup}")
    # start the window right after a compaction: one step with a period of 1
    ctx.set_schedule(sort_every=1, diag_every=0, tile=tile)
    stepper(1)
    ctx.set_schedule(sort_every=period, diag_every=0, tile=tile)
    ctx.set_launch(graph=args.graph, timing_every=coprime(args.timing_every))
    n_before = live_per_case()
    ctx.sync()
    log(f"[bench] timing {steps} steps ({steps // period} sort periods of "
        f"{period}), {sum(n_before)} particles")
    t0 = time.perf_counter()
    stepper(steps)
    ctx.sync()
    t1 = time.perf_counter()
    n_after = live_per_case()
    ms_per_step = (t1 - t0) * 1e3 / steps
    per_case = [0.5 * (a + b) for a, b in zip(n_before, n_after)]
    particles = sum(per_case)
    value = particles * steps / (t1 - t0)
    # kernel durations: HIP events around every particle and collision kernel
    # of an untimed sample after the window (the events cost ~4 us each, so
    # they stay out of the window)
    ctx.set_schedule(sort_every=sort_every, diag_every=0, tile=tile)
    ctx.set_launch(graph=0, timing_every=1)
    stepper(args.sample_steps)
    kern_ms, launches = ctx.last_timing()
    coll_ms, coll_launches = ctx.last_timing_collide()

    # algorithmic bytes of one step from the particles and the candidates and
    # collisions of the last step (ledger); per launch = per step / groups
    step_bytes = coll_step_bytes = 0.0
    cands = real = 0
    for k, w in enumerate(wls):
        sc = schemes[k]
        L = ctx.ledger(k)
        ck, rk = int(sum(L["n_candidates"])), int(L["n_coll"].sum())
        cands += ck
        real += rk
        step_bytes += PASS_BYTES[sc] * per_case[k] + LIST_BYTES[sc] * ck
        coll_step_bytes += COLLIDE_BYTES[sc] * ck + COLLISION_BYTES[sc] * rk
    if launches == 0:
        log("[bench] no timed launch in the sample (see --sample-steps)")
    avg_launch_s = kern_ms / 1e3 / max(launches, 1)
    alg_bytes = step_bytes / groups
    achieved = alg_bytes / avg_launch_s / 1e9 if avg_launch_s > 0 else 0.0
    kname = "k_step<%d,false>" % schemes[0] if groups == 1 else "k_step<0|1,false>"
    rule = " and ".join("%s: %d B per particle + %d B per listed candidate"
                        % (("explicit", "implicit")[sc], PASS_BYTES[sc], LIST_BYTES[sc])
                        for sc in sorted(set(schemes)))
    roof = dict(bound="hbm", achieved=round(achieved, 1), peak=PEAK_HBM_GBS, unit="GB/s",
                frac=round(achieved / PEAK_HBM_GBS, 4), traffic=None,
                kernel=kname, avg_launch_ms=round(avg_launch_s * 1e3, 4),
                timed_launches=launches,
                timed_in="untimed sample of %d steps after the window, events around "
                         "every launch" % args.sample_steps,
                alg_bytes_per_launch=int(alg_bytes),
                alg_bytes_rule=rule)
    coll_avg_s = coll_ms / 1e3 / max(coll_launches, 1)
    coll_bytes = coll_step_bytes / groups
    collide = dict(kernel=kname.replace("k_step", "k_collide"),
                   avg_launch_ms=round(coll_avg_s * 1e3, 4),
                   candidates_per_step=cands, collisions_per_step=real,
                   achieved_GBps=round(coll_bytes / max(coll_avg_s, 1e-12) / 1e9, 1),
                   alg_bytes_rule=" and ".join(
                       "%s: %d B per candidate + %d B per real collision"
                       % (("explicit", "implicit")[sc], COLLIDE_BYTES[sc], COLLISION_BYTES[sc])
                       for sc in sorted(set(schemes))))
    roof["traffic"] = measured_traffic(args.workload, roof["kernel"])
    if roof["traffic"] and avg_launch_s > 0:
        roof["traffic_GBps"] = round(roof["traffic"] / avg_launch_s / 1e9, 1)
    # the whole step priced at the bytes a plain streaming form of the method
    # moves per particle-step (explicit: read cell, off, vx, vy, vz, id and
    # write cell, off, vx = 40 B; implicit: + abar read and written = 48 B)
    plain = sum(STREAM_BYTES[sc] * per_case[k] for k, sc in enumerate(schemes)) / particles
    roof["step_equivalent"] = dict(bytes_per_particle_step=round(plain, 2),
                                   GBps=round(value * plain / 1e9, 1),
                                   frac=round(value * plain / 1e9 / PEAK_HBM_GBS, 4))
    collide["traffic"] = measured_traffic(args.workload, collide["kernel"])

    out = dict(metric="particle-steps/sec (push+deposit+MCC) vs plain FP64 GPU form at "
                      "matched EEDF",
               value=value, unit="particle-steps/s", n_gpus=1, steps=args.steps,
               warmup=args.warmup, ms_per_step=ms_per_step, higher_is_better=True,
               scaling="weak", vs_baseline=None, dtype="f32",
               data="synthetic",
               config=dict(workload=args.workload, cases=len(wls),
                           cells=[w["case"]["n_cells"] for w in wls][:4],
                           particles=int(particles), tile=tile, sort_every=sort_every,
                           scheme=("explicit", "implicit", "mixed")[
                               2 if groups == 2 else schemes[0]],
                           graph=args.graph, timing_every=args.timing_every,
                           window_sort_every=period,
                           window_sort_periods=round(steps / period, 3)),
               roofline=roof, collide=collide)
    if tuned:
        out["autotune"] = tuned
    if args.fp64_steps > 0 and \
            all(w["case"].get("gather", 0) != 2 and w["case"].get("cell_dx") is None and
                w["case"].get("ion_subcycle", 0) <= 1 for w in wls):
        # the plain FP64 GPU form of the same method, from the same state
        log(f"[bench] plain FP64 GPU form: {args.fp64_steps} steps")
        ctx.fp64_init()
        ctx.fp64_step(2)
        n64 = sum(live_per_case())
        t0 = time.perf_counter()
        ctx.fp64_step(args.fp64_steps)
        t1 = time.perf_counter()
        v64 = n64 * args.fp64_steps / (t1 - t0)
        out["fp64_gpu_form"] = dict(value=v64, unit="particle-steps/s",
                                    ms_per_step=(t1 - t0) * 1e3 / args.fp64_steps,
                                    steps=args.fp64_steps)
        out["speedup_vs_fp64_form"] = value / v64
    ctx.close()
    if args.batch and args.workload == "ccp2048_explicit" and args.scale == 1.0:
        out["batched"] = batch_record(P)
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
