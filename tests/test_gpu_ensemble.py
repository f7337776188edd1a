"""Statistical parity over seed ensembles (Sec. III discharges): the HIP path
and the FP64 oracle each run the same discharge from 5 seeds (the particle
load and the Philox key both change with the seed), free-running, and their
seed means are compared over the last periods of the run:

  * time-averaged node densities of both species (relative L2),
  * the electron energy distribution on 1 eV bins (L1 of the normalised
    distributions) and the mean electron energy,
  * the energy the field gives the particles over the window (absorbed
    power).

Each metric must agree to 2 % and to within 3 times the combined
seed-to-seed standard error of the two means (for a profile: the norm of the
difference against 3 times the norm of the per-bin standard errors).

Discharges: the 64-cell explicit discharge (10 RF periods, last 4 averaged),
and the 256-cell D1 implicit discharge at omega_p dt = 2 (6 RF periods,
last 3), which is also compared with the explicit scheme on its own inputs
at omega_p dt = 0.2 (same physical time), and with itself at 0.2.  The paper
gives no numbers for these synthetic discharges: parity is with the oracle;
the implicit and explicit runs are compared for convergence at the same
step and for the direction of the large-step result."""
import math
import multiprocessing
import os
from concurrent.futures import ProcessPoolExecutor

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

E = 1.602176634e-19
ME = 9.1093837015e-31
SEEDS = [0xE1, 0xE2, 0xE3, 0xE4, 0xE5]
TOL = 0.02
EEDF_BIN_EV = 0.5
EEDF_BINS = 256


def workload(kind, seed):
    if kind == "ccp64":
        return W.c1(collisions=1, np_per_species=16384, seed=seed), 400, 6, 4
    wdt = {"ccp256_implicit": 2.0, "ccp256_implicit_dt0.1": 0.1}.get(kind, 0.2)
    scheme = 0 if kind == "ccp256_explicit" else 1
    wl = W.c3(ppc=200, wdt=wdt, scheme=scheme, seed=seed)
    for sp in wl["species"]:
        sp["capacity"] = 2 * sp["cell"].size
    per = int(round(1.0 / (wl["case"]["rf_freq_hz"] * wl["case"]["dt_s"])))
    return wl, per, 3, 3


def node_volume(N):
    return np.concatenate([[0.5], np.ones(N - 1), [0.5]])


def metrics(dens, eedf, absorbed):
    p = eedf.reshape(-1, 2).sum(1)
    p = p / p.sum()
    c = (np.arange(p.size) + 0.5) * 2 * EEDF_BIN_EV
    return dict(dens=dens, eedf=p, mean_eV=float((p * c).sum()), absorbed=float(absorbed))


def gpu_run(kind, seed):
    import paper_1310_5284_amd as P
    wl, per, p0, pw = workload(kind, seed)
    ctx = P.PicContext([wl])
    ctx.set_schedule(sort_every=64, diag_every=0, tile=4096)
    ctx.step(p0 * per)
    ctx.reset_accumulators()
    ctx.set_schedule(sort_every=64, diag_every=1, tile=4096)
    ctx.step(pw * per)
    dens, n = ctx.density()
    heat = ctx.heating()
    eedf, bin_eV, _ = ctx.eedf()
    ctx.close()
    assert n == pw * per and abs(bin_eV - EEDF_BIN_EV) < 1e-12
    return metrics(np.concatenate(dens), eedf.astype(np.float64), sum(h.sum() for h in heat))


def oracle_run(kind, seed, every=4):
    import oracle
    wl, per, p0, pw = workload(kind, seed)
    case, sps, procs = W.to_oracle(wl)
    sim = oracle.Sim(case, sps, procs)
    N = case["n_cells"]
    sim.step(p0 * per)
    h0 = sim.heating()
    vol = node_volume(N) * (case["gap_m"] / N)
    dens = [np.zeros(N + 1), np.zeros(N + 1)]
    eedf = np.zeros(EEDF_BINS)
    ns = 0
    done = 0
    while done < pw * per:
        k = min(every, pw * per - done)
        sim.step(k)
        done += k
        ns += 1
        for s in range(2):
            sp = sim.species(s)
            dens[s] += oracle.deposit_linear(N, sp["xi"]) * sim.w[s] / vol
            if s == 0:
                # v_{n+1/2}, as the GPU samples it (an implicit state holds
                # v~ = v_{n+1/2} + dt abar / 2)
                vx = sp["vx"] - 0.5 * case["dt_s"] * sp["abar"] if case["scheme"] == 1 \
                    else sp["vx"]
                eps = 0.5 * ME * (vx ** 2 + sp["vy"] ** 2 + sp["vz"] ** 2) / E
                b = np.minimum(np.floor(eps / EEDF_BIN_EV).astype(np.int64), EEDF_BINS - 1)
                eedf += np.bincount(b, minlength=EEDF_BINS)
    h1 = sim.heating()
    absorbed = sum((h1[s] - h0[s]).sum() for s in range(2))
    return metrics(np.concatenate([d / ns for d in dens]), eedf, absorbed)


def ensemble(runs):
    out = {}
    for key in ("dens", "eedf", "mean_eV", "absorbed"):
        a = np.array([np.asarray(r[key], dtype=np.float64) for r in runs])
        out[key] = (a.mean(0), a.std(0, ddof=1) / math.sqrt(len(runs)))
    return out


def compare(g, o, tol, name):
    rep = {}
    for key in ("dens", "eedf"):
        (mg, sg), (mo, so) = g[key], o[key]
        diff = np.linalg.norm(mg - mo)
        rel = diff / np.linalg.norm(mo) if key == "dens" else np.abs(mg - mo).sum()
        se = 3.0 * math.sqrt(float((sg ** 2 + so ** 2).sum()))
        rep[key] = (rel, diff, se)
        print(f"{name} {key}: relative {rel:.4f}, |diff| {diff:.4g}, 3 SE {se:.4g}")
        assert rel < tol, (name, key, rel)
        assert diff <= se, (name, key, diff, se)
    for key in ("mean_eV", "absorbed"):
        (mg, sg), (mo, so) = g[key], o[key]
        rel = abs(mg - mo) / abs(mo)
        se = 3.0 * math.sqrt(sg ** 2 + so ** 2)
        rep[key] = (rel, abs(mg - mo), se)
        print(f"{name} {key}: {mg:.5g} / {mo:.5g}, relative {rel:.4f}, 3 SE {se:.4g}")
        assert rel < tol, (name, key, rel)
        assert abs(mg - mo) <= se, (name, key, mg, mo, se)
    return rep


@pytest.mark.parametrize("kind", ["ccp64", "ccp256_implicit"])
def test_seed_ensemble_matches_oracle(kind):
    # the oracle runs in fresh interpreters (one per seed) while the GPU runs
    n = min(len(SEEDS), max(1, (os.cpu_count() or 1)))
    with ProcessPoolExecutor(n, mp_context=multiprocessing.get_context("spawn")) as ex:
        jobs = [ex.submit(oracle_run, kind, s) for s in SEEDS]
        g = ensemble([gpu_run(kind, s) for s in SEEDS])
        o = ensemble([j.result(timeout=600) for j in jobs])
    compare(g, o, TOL, kind)


def test_implicit_discharge_converges_to_the_explicit_one():
    # D1 against leap-frog on the same inputs (3 seeds each, the same
    # physical time).  D1 damps the plasma oscillation at every step size
    # (|lambda| of its cold-plasma map: 0.9999519 per step at omega_p dt =
    # 0.1, 0.9993 at 0.2, 0.707 at 2), which drains field energy and leaves
    # the electrons colder than leap-frog; the gap closes as dt shrinks.
    # Checked: the densities agree to 10 % at every step size, the electrons
    # never come out hotter, and the mean-energy gap to leap-frog falls
    # monotonically from omega_p dt = 2 to 0.2 to 0.1
    ge = ensemble([gpu_run("ccp256_explicit", s) for s in SEEDS[:3]])
    rows = []
    for kind, wdt in (("ccp256_implicit", 2.0), ("ccp256_implicit_dt0.2", 0.2),
                      ("ccp256_implicit_dt0.1", 0.1)):
        gi = ensemble([gpu_run(kind, s) for s in SEEDS[:3]])
        dd = np.linalg.norm(gi["dens"][0] - ge["dens"][0]) / np.linalg.norm(ge["dens"][0])
        l1 = np.abs(gi["eedf"][0] - ge["eedf"][0]).sum()
        gap = (ge["mean_eV"][0] - gi["mean_eV"][0]) / ge["mean_eV"][0]
        print(f"D1 at omega_p dt {wdt} vs leap-frog at 0.2: density L2 {dd:.4f}, EEDF L1 "
              f"{l1:.4f}, mean energy {gi['mean_eV'][0]:.4f} / {ge['mean_eV'][0]:.4f} eV")
        rows.append((wdt, dd, gap))
    for wdt, dd, gap in rows:
        assert dd < 0.10, (wdt, dd)
        assert gap > -0.03, (wdt, gap)
    gaps = [g for _, _, g in rows]
    assert gaps[0] > gaps[1] > gaps[2], gaps
