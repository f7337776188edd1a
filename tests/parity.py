"""Teacher-forced parity of the GPU library against the FP64 oracle.

At every step the GPU state (int32 cell + float offset, velocities in cells
per step) is loaded exactly into the oracle (xi = cell + off, v = v_hat dx/dt
in float64); the oracle computes the fields of that state and takes one FP64
step, and both are compared with what the GPU computed.  PIC is chaotic, so a
free-running comparison is not gated; teacher forcing bounds the error of a
single step.

Decisions taken by floating point on the GPU in float32 (which cell a moved
particle lands in, absorption at an electrode, which collision process wins)
can differ from the FP64 decision when the oracle's value lies within float32
rounding of the threshold.  Such particles are counted, not compared:
  * a particle alive on one side only must sit within POS_MARGIN cells of an
    electrode on the side that kept it;
  * a particle whose velocity disagrees is accepted only if it collided on at
    least one side (process choice near u1 = cumulative probability);
and the count must stay within the allowance (1 per 1e6 particle-steps, at
least 2).  Candidacy (u0 < P_null) is an exact integer decision and must agree.
"""
from __future__ import annotations

import numpy as np

import oracle
import workloads as W

FIELD_TOL = 1e-5       # normwise relative, per field
POS_TOL = 1e-5         # relative to the step's move: cells x max(1, |v| dt/dx)
VEL_TOL = 1e-5         # relative to |v| + v_rms
POS_MARGIN = 1e-5      # cells: decision band at electrodes and cell edges
LEDGER_TOL = 1e-5      # relative to the species' kinetic energy


def to_oracle_species(st, wl):
    vu, au = st["vel_unit"], st["acc_unit"]
    out = []
    for s, sp in enumerate(st["species"]):
        src = wl["species"][s]
        out.append(dict(q=src["q"], m=src["m"], w=src["w"], vel_unit=vu,
                        xi=sp["cell"].astype(np.float64) + sp["off"].astype(np.float64),
                        vx=sp["vx"].astype(np.float64) * vu, vy=sp["vy"].astype(np.float64) * vu,
                        vz=sp["vz"].astype(np.float64) * vu,
                        abar=sp["abar"].astype(np.float64) * au, id=sp["id"],
                        wait=sp["mcc_wait"]))
    return out


def normwise(a, b):
    den = np.abs(b).max()
    return float(np.abs(a - b).max() / den) if den > 0 else float(np.abs(a - b).max())


def compare_fields(gf, of, implicit, case=None, gather=0):
    err = {}
    for k in ("rho", "phi", "E"):
        err[k] = normwise(gf[k], of[k])
    if implicit:
        err["chi"] = normwise(gf["chi"], of["chi"])
    for s, key in enumerate(("Qe", "Qi")):
        q = gf["qfix"][s].astype(np.float64) / 2 ** 24
        cnt = np.concatenate([of["cnt_e" if s == 0 else "cnt_i"], [0]])
        if gather == 2:
            # quadratic weights: a node takes the particles of cells g-2..g+1,
            # each weight computed in float32 and rounded to 2^-24
            near = cnt + np.roll(cnt, 1) + np.roll(cnt, 2) + np.roll(cnt, -1)
            bound = 3.0 * (near + 1) * 2.0 ** -24 + 1e-9 * np.abs(of[key]).max()
        else:
            # each particle's two weights are rounded to 2^-25 at most
            bound = (cnt + np.roll(cnt, 1) + 1) * 2.0 ** -24 + 1e-9 * np.abs(of[key]).max()
        assert np.all(np.abs(q - of[key]) <= bound), f"fixed-point deposit {key}"
        cg = gf["cell_count"][s].astype(np.float64)
        assert np.array_equal(cg, of["cnt_e" if s == 0 else "cnt_i"]), "cell counts"
    return err


def compare_particles(g, o, N, periodic, vrms):
    """g, o: dicts of arrays (oracle units).  Returns (errors, mismatches)."""
    gi = {int(x): k for k, x in enumerate(g["id"])}
    oi = {int(x): k for k, x in enumerate(o["id"])}
    common = sorted(set(gi) & set(oi))
    # alive on one side only: an absorption decision at an electrode or a
    # child of a collision decided differently; both are counted
    mism = len(set(gi) ^ set(oi))
    if not common:
        return dict(pos=0.0, vel=0.0, n=0), mism
    ig = np.array([gi[p] for p in common])
    io = np.array([oi[p] for p in common])
    dxi = g["xi"][ig] - o["xi"][io]
    if periodic:
        dxi = (dxi + N / 2) % N - N / 2
    vg = np.stack([g["vx"][ig], g["vy"][ig], g["vz"][ig]])
    vo = np.stack([o["vx"][io], o["vy"][io], o["vz"][io]])
    scale = np.linalg.norm(vo, axis=0) + vrms
    dv = np.abs(vg - vo).max(axis=0) / scale
    bad_v = dv > VEL_TOL
    # a position moved by |v| dt/dx cells in float32 carries ~6e-8 of that move
    move = np.maximum(1.0, np.abs(vo[0]) / g.get("vel_unit", 1.0))
    relx = np.abs(dxi) / move
    bad_x = relx > POS_TOL
    # a velocity or position off by more than the tolerance is a collision-
    # process decision if the particle's transverse velocity changed on
    # either side (only collisions change vy, vz)
    vy_changed = (np.abs(vg[1] - vo[1]) > VEL_TOL * scale)
    dec = (bad_v | bad_x) & vy_changed
    # the next waiting time of a candidate is an integer drawn in float64
    # (floor of ln u / ln(1 - P_null)) on both sides: equal unless the quotient
    # lies within rounding of an integer
    if "wait" in g and "wait" in o:
        dec |= g["wait"][ig] != o["wait"][io]
    mism += int(dec.sum())
    ok = ~dec
    err = dict(pos=float(relx[ok].max(initial=0.0)),
               vel=float(dv[ok].max(initial=0.0)), n=len(common))
    if "abar" in g:
        da = np.abs(g["abar"][ig] - o["abar"][io])
        sa = np.abs(o["abar"][io]).max(initial=0.0) + 1e-300
        err["abar"] = float(da[ok].max(initial=0.0) / sa)
    return err, mism


def teacher_forced(ctx, wl, steps, case=0, check_ledger=True, verbose=False):
    """Run `steps` teacher-forced steps; returns a report of the worst errors."""
    c = wl["case"]
    N = c["n_cells"]
    periodic = c.get("bc", 0) == 1
    implicit = c.get("scheme", 0) == 1
    rep = dict(fields={}, pos=0.0, vel=0.0, abar=0.0, mismatches=0, particle_steps=0,
               ledger=0.0, steps=0)
    for n in range(steps):
        st = ctx.state(case)
        gf = ctx.fields(case)
        sps = to_oracle_species(st, wl)
        case_o = dict(c, step0=st["step"])
        sim = oracle.Sim(case_o, sps, wl["processes"], startup=False)
        sim.compute_fields()
        of = sim.fields()
        fe = compare_fields(gf, of, implicit, gather=c.get("gather", 0))
        for k, v in fe.items():
            rep["fields"][k] = max(rep["fields"].get(k, 0.0), v)
        sim.step(1)
        ctx.step(1)
        st2 = ctx.state(case)
        g2 = to_oracle_species(st2, wl)
        mism_step = 0
        for s in range(2):
            o = sim.species(s)
            if o["id"].size == 0 and g2[s]["id"].size == 0:
                continue
            vr = float(np.sqrt(np.mean(o["vx"] ** 2 + o["vy"] ** 2 + o["vz"] ** 2))) \
                if o["vx"].size else 0.0
            err, mism = compare_particles(g2[s], o, N, periodic, vr)
            rep["pos"] = max(rep["pos"], err["pos"])
            rep["vel"] = max(rep["vel"], err["vel"])
            if implicit and "abar" in err:
                rep["abar"] = max(rep["abar"], err["abar"])
            mism_step += mism
            rep["particle_steps"] += err["n"]
        rep["mismatches"] += mism_step
        if check_ledger:
            gl = ctx.ledger(case)
            ol = sim.ledger()
            assert gl["step"] == st["step"]
            Ktot = max(float(ol["K_before"].sum() + ol["K_after"].sum()), 1e-300)
            for s in range(2):
                # relative to the species' energy; a species that starts empty
                # is judged against the energy of both
                K = max(ol["K_before"][s], ol["K_after"][s]) or Ktot
                e = abs(gl["K_before"][s] - ol["K_before"][s]) / K
                if mism_step == 0:
                    for key in ("work", "coll_dK"):
                        e = max(e, abs(gl[key][s] - ol[key][s]) / K)
                    e = max(e, np.abs(gl["absorbed_K"][s] - ol["absorbed_K"][s]).max() / K)
                    assert np.array_equal(gl["absorbed_n"][s], ol["absorbed_n"][s]), "absorbed"
                    assert np.array_equal(gl["n_coll"][s], ol["n_coll"][s]), "collisions"
                    assert gl["n_created"][s] == ol["n_created"][s], "created"
                assert gl["n_candidates"][s] == ol["n_candidates"][s], "candidacy is exact"
                rep["ledger"] = max(rep["ledger"], e)
            we = ol["WE"]
            if we > 0:
                rep["ledger"] = max(rep["ledger"], abs(gl["WE"] - we) / we)
        rep["steps"] += 1
        if verbose:
            print(n, rep, flush=True)
    return rep


def assert_report(rep, field_tol=FIELD_TOL):
    for k, v in rep["fields"].items():
        assert v <= field_tol, (k, v, rep)
    assert rep["pos"] <= POS_TOL, rep
    assert rep["vel"] <= VEL_TOL, rep
    assert rep["abar"] <= 1e-5, rep
    assert rep["ledger"] <= LEDGER_TOL, rep
    allow = max(2, int(1e-6 * rep["particle_steps"]))
    assert rep["mismatches"] <= allow, rep
