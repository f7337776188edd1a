"""The plain FP64 GPU form of the method (the throughput comparison point),
explicit and D1 implicit with the EC and MC gathers, against the FP64
oracle, free-running from the same state; and its energy ledger against the
oracle's.

Both sides compute in float64 with the same Philox draws, so trajectories
agree to rounding (summation order of the deposit) amplified by the chaotic
dynamics over the run; a particle may differ only where a float64 decision
(cell edge, electrode, collision process) fell within rounding of its
threshold.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from parity import to_oracle_species

pytestmark = pytest.mark.gpu

TOL = 1e-9


def P():
    import paper_1310_5284_amd as P
    return P


def run_pair(wl, steps, warm=5):
    """The FP64 form and the oracle from the same state of the mixed path."""
    ctx = P().PicContext([wl])
    ctx.set_schedule(sort_every=16, diag_every=0, tile=1024)
    ctx.step(warm)
    st = ctx.state()
    sim = oracle.Sim(dict(wl["case"], step0=st["step"]), to_oracle_species(st, wl),
                     wl["processes"], startup=False)
    ctx.fp64_init()
    ctx.fp64_step(steps)
    sim.step(steps)
    return ctx, sim, st["vel_unit"]


def compare_states(ctx, sim, vu):
    mism = 0
    for s in range(2):
        g = ctx.fp64_state(0, s)
        o = sim.species(s)
        gi = {int(x): k for k, x in enumerate(g["id"])}
        oi = {int(x): k for k, x in enumerate(o["id"])}
        common = sorted(set(gi) & set(oi))
        mism += len(set(gi) ^ set(oi))
        assert len(common) > 0.9 * len(oi)
        ig = np.array([gi[p] for p in common])
        io = np.array([oi[p] for p in common])
        dx = np.abs(g["xi"][ig] - o["xi"][io])
        vg = np.stack([g[k][ig] * vu for k in ("vx", "vy", "vz")])
        vo = np.stack([o[k][io] for k in ("vx", "vy", "vz")])
        vs = np.linalg.norm(vo, axis=0) + np.sqrt(np.mean(vo ** 2) * 3)
        dv = np.abs(vg - vo).max(axis=0) / vs
        bad = (dx > TOL) | (dv > TOL)
        if bad.any() or set(gi) ^ set(oi):
            only_g = sorted(set(gi) - set(oi))[:3]
            only_o = sorted(set(oi) - set(gi))[:3]
            print(f"species {s}: n_gpu {len(gi)} n_oracle {len(oi)} common {len(common)} "
                  f"bad {int(bad.sum())} only_gpu {len(set(gi) - set(oi))} {only_g} "
                  f"only_oracle {len(set(oi) - set(gi))} {only_o}")
            for k in np.nonzero(bad)[0][:4]:
                print("  id", common[k], "xi", g["xi"][ig[k]], o["xi"][io[k]],
                      "v_gpu", vg[:, k], "v_oracle", vo[:, k])
        mism += int(bad.sum())
        ok = ~bad
        assert dx[ok].max(initial=0) <= TOL and dv[ok].max(initial=0) <= TOL
    return mism


def compare_ledgers(gl, ol, mism):
    # energies relative to the species' kinetic energy; counts exact unless a
    # float64 decision fell within rounding of its threshold (then the step's
    # energies carry that particle's share too)
    for s in range(2):
        K = max(abs(ol["K_before"][s]), abs(ol["K_after"][s]), 1e-300)
        for key in ("K_before", "K_after", "work", "coll_dK"):
            tol = 1e-9 if mism == 0 else 1e-3
            assert abs(gl[key][s] - ol[key][s]) <= tol * K, (key, s, gl[key][s], ol[key][s])
        np.testing.assert_allclose(gl["absorbed_K"][s], ol["absorbed_K"][s], rtol=0,
                                   atol=(1e-9 if mism == 0 else 1e-3) * K)
        if mism == 0:
            assert np.array_equal(gl["absorbed_n"][s], ol["absorbed_n"][s])
            assert np.array_equal(gl["n_coll"][s], ol["n_coll"][s])
            assert gl["n_candidates"][s] == ol["n_candidates"][s]
            assert gl["n_created"][s] == ol["n_created"][s]
    assert abs(gl["WE"] - ol["WE"]) <= 1e-9 * abs(ol["WE"])


@pytest.mark.parametrize("collisions", [0, 1])
def test_fp64_form_follows_oracle(collisions):
    wl = W.c1(collisions=collisions, np_per_species=4096)
    ctx, sim, vu = run_pair(wl, 30)
    mism = compare_states(ctx, sim, vu)
    assert mism <= 2, mism
    compare_ledgers(ctx.fp64_ledger(), sim.ledger(), mism)
    if collisions:
        assert sim.ledger()["n_candidates"][0] > 0


@pytest.mark.parametrize("gather", [0, 1])
def test_fp64_form_implicit_follows_oracle(gather):
    # the D1 scheme on the 256-cell discharge at omega_p dt = 2 (EC and MC)
    wl = W.c3(ppc=24, wdt=2.0)
    wl["case"]["gather"] = gather
    for sp in wl["species"]:
        sp["capacity"] = 2 * sp["cell"].size
    ctx, sim, vu = run_pair(wl, 30)
    mism = compare_states(ctx, sim, vu)
    assert mism <= 2, mism
    compare_ledgers(ctx.fp64_ledger(), sim.ledger(), mism)
    assert sim.ledger()["n_candidates"][0] > 0


def test_fp64_form_ledger_closes():
    # K_after = K_before + work - absorbed + collisional change, every step,
    # and the next step starts from the last one's K_after
    wl = W.c1(collisions=1, np_per_species=8192)
    wl["case"]["gas_density_m3"] = W.gas_density(300.0)
    ctx = P().PicContext([wl])
    ctx.fp64_init()
    prev = None
    colls = 0
    for _ in range(12):
        ctx.fp64_step(1)
        L = ctx.fp64_ledger()
        colls += int(L["n_coll"].sum())
        for s in range(2):
            rhs = L["K_before"][s] + L["work"][s] - L["absorbed_K"][s].sum() + L["coll_dK"][s]
            assert abs(L["K_after"][s] - rhs) <= 1e-12 * max(L["K_after"][s], 1e-300)
            if prev is not None:
                assert abs(L["K_before"][s] - prev["K_after"][s]) <= 1e-15 * prev["K_after"][s]
        prev = L
    assert colls > 0
