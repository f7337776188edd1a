"""Parity at the benchmark sizes, in the launch configuration the benchmark
times (tile and sort period as the autotuner picks them for each workload).

The oracle cannot step 2e7 particles per step in a test, so a step is
checked in two parts: every field of the full state (deposits, cell counts,
rho, phi, E) against the oracle's deposit and solve of that state, and the
particle step on a random sample of each species, which the oracle advances
with the GPU's field (a sample's own charge would not reproduce it).  The
sampled particles must match to the same tolerances as the small
teacher-forced runs; children of sampled parents are compared too."""
import numpy as np
import pytest

import oracle
import workloads as W
from parity import (FIELD_TOL, POS_TOL, VEL_TOL, check_children, compare_fields,
                    compare_particles, to_oracle_species)

pytestmark = pytest.mark.gpu


def P():
    import paper_1310_5284_amd as P
    return P


def full_fields(ctx, wl, k):
    """Fields of case k's current state: GPU against the oracle's solve."""
    st = ctx.state(k)
    sim = oracle.Sim(dict(wl["case"], step0=st["step"]), to_oracle_species(st, wl),
                     wl["processes"], startup=False)
    sim.compute_fields()
    return compare_fields(ctx.fields(k), sim.fields(), wl["case"].get("scheme", 0) == 1,
                          gather=wl["case"].get("gather", 0))


def sampled_step(ctx, wls, cases, n_sample, seed):
    """One step of the whole batch; the listed cases are checked on samples."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sims, picked = {}, {}
    for k in cases:
        wl = wls[k]
        st = ctx.state(k)
        E = ctx.fields(k)["E"]
        sps = to_oracle_species(st, wl)
        sub, ids = [], []
        for sp in sps:
            n = sp["xi"].size
            idx = np.sort(rng.choice(n, size=min(n, n_sample), replace=False))
            sub.append({key: (v[idx] if isinstance(v, np.ndarray) else v)
                        for key, v in sp.items()})
            ids.append(sp["id"][idx])
        sim = oracle.Sim(dict(wl["case"], step0=st["step"]), sub, wl["processes"],
                         startup=False)
        sim.step_with_field(E)
        sims[k], picked[k] = sim, ids
    ctx.step(1)
    rep = dict(pos=0.0, vel=0.0, abar=0.0, mismatches=0, n=0)
    for k in cases:
        wl = wls[k]
        c = wl["case"]
        g2 = to_oracle_species(ctx.state(k), wl)
        errs = [None, None]
        for s in range(2):
            o = sims[k].species(s)
            keep = np.isin(g2[s]["id"], np.concatenate([picked[k][s], o["id"]]))
            g = {key: (v[keep] if isinstance(v, np.ndarray) else v) for key, v in g2[s].items()}
            vr = float(np.sqrt(np.mean(o["vx"] ** 2 + o["vy"] ** 2 + o["vz"] ** 2))) \
                if o["vx"].size else 0.0
            err, mism = compare_particles(g, o, c["n_cells"], c.get("bc", 0) == 1, vr,
                                          prev_ids=picked[k][s],
                                          implicit=c.get("scheme", 0) == 1)
            errs[s] = err
            rep["pos"] = max(rep["pos"], err["pos"])
            rep["vel"] = max(rep["vel"], err["vel"])
            rep["abar"] = max(rep["abar"], err.get("abar", 0.0))
            rep["mismatches"] += mism
            rep["n"] += err["n"]
        check_children(errs)
    return rep


def check(rep, n_allow=2):
    assert rep["pos"] <= POS_TOL, rep
    assert rep["vel"] <= VEL_TOL, rep
    assert rep["abar"] <= 1e-5, rep
    assert rep["mismatches"] <= n_allow, rep


def test_ccp2048_full_size():
    # 1e7 electrons + 1e7 ions, tile 16384, sort every 64 (the benchmark's)
    wls = [W.c4(np_per_species=10_000_000)]
    ctx = P().PicContext(wls)
    ctx.set_schedule(sort_every=64, diag_every=0, tile=16384)
    ctx.step(65)                       # past the first compaction and sort
    rep = sampled_step(ctx, wls, [0], 8192, seed=41)
    print(rep)
    check(rep)
    fe = full_fields(ctx, wls[0], 0)
    print(fe)
    assert max(fe.values()) <= FIELD_TOL, fe
    ctx.close()


@pytest.mark.parametrize("name", ["ccp2048_mc", "ccp2048_mc_implicit", "ccp2048_ec2_implicit",
                                  "ccp2048_nonuniform", "ccp2048_nonuniform_ec2_implicit",
                                  "ccp2048_subcycle8", "ccp2048_implicit_subcycle8"])
def test_widened_workloads_full_size(name):
    # the benchmark's other 2048-cell discharges (the MC gather with either
    # scheme, m = 2 implicit, the sheath-refined grid with EC explicit and
    # with m = 2 implicit, ions subcycled at K = 8 with either scheme) at
    # tile 16384, sort 64;
    # the subcycled one is sampled in a step where the ions stand (65) and in
    # one where they move (72)
    import bench
    wls = bench.make_workload(name, 1.0)
    ctx = P().PicContext(wls)
    ctx.set_schedule(sort_every=64, diag_every=0, tile=16384)
    ctx.step(65)
    rep = sampled_step(ctx, wls, [0], 8192, seed=43)
    print(name, rep)
    check(rep)
    if name.endswith("subcycle8"):
        ctx.step(6)
        assert ctx.state()["step"] % 8 == 0
        rep = sampled_step(ctx, wls, [0], 8192, seed=44)
        print(name, rep)
        check(rep)
    fe = full_fields(ctx, wls[0], 0)
    print(name, fe)
    assert max(fe.values()) <= FIELD_TOL, fe
    ctx.close()


def test_sweep64_full_size():
    # the 64-case batch (explicit and implicit mixed), tile 4096, sort every 128
    wls = W.c5()
    ctx = P().PicContext(wls)
    ctx.set_schedule(sort_every=128, diag_every=0, tile=4096)
    ctx.step(130)
    schemes = [w["case"]["scheme"] for w in wls]
    sizes = [w["species"][0]["cell"].size for w in wls]
    # the largest and the smallest case of each scheme
    cases = []
    for sc in (0, 1):
        ks = [k for k in range(len(wls)) if schemes[k] == sc]
        cases += [max(ks, key=lambda k: sizes[k]), min(ks, key=lambda k: sizes[k])]
    rep = sampled_step(ctx, wls, cases, 2048, seed=42)
    print(cases, rep)
    check(rep)
    for k in cases:
        fe = full_fields(ctx, wls[k], k)
        print(k, fe)
        assert max(fe.values()) <= FIELD_TOL, (k, fe)
    ctx.close()


def test_ccp256_implicit_full_size_teacher_forced():
    # 200 particles per cell and species, omega_p dt = 2, tile 1024, sort 128
    from parity import assert_report, teacher_forced
    wl = W.c3(wdt=2.0)
    for sp in wl["species"]:
        sp["capacity"] = 2 * sp["cell"].size
    ctx = P().PicContext([wl])
    ctx.set_schedule(sort_every=128, diag_every=0, tile=1024)
    ctx.step(127)                      # the next steps cross the first sort
    rep = teacher_forced(ctx, wl, 4)
    print(rep)
    assert_report(rep)
    ctx.close()
