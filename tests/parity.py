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
rounding of the threshold.  Such particles are counted, not compared, and
each must be explained:
  * a particle alive on one side only must sit, on the side that kept it,
    within POS_MARGIN x max(1, |v| dt/dx) cells of an electrode (plus its
    predicted move for the implicit scheme, whose state holds x~), or be a
    child born in this step while a parent's collision process was decided
    differently (at most one child per species per such parent);
  * a particle whose velocity disagrees is accepted only if it collided on at
    least one side (process choice near u1 = cumulative probability);
and the count must stay within the allowance (1 per 1e6 particle-steps, at
least 2).

Candidacy is by waiting time: a particle's count of non-candidate steps is
decremented each step and the particle is a candidate when it is zero; the
next wait W = floor(ln u0 / ln(1 - P_null)) is an integer drawn in float64 on
both sides.  The oracle holds W uncapped; the GPU packs it into a 17-bit
count, storing a larger W as the largest count with a capped flag and
drawing the trial afresh when such a count runs out.  So: an uncapped GPU
wait must equal the oracle's (a quotient within rounding of an integer is a
counted decision); a capped GPU wait must be below the oracle's; the number
of candidates per step is exact, except for particles loaded with a capped
count at zero (an open trial, decided differently by construction), which
are left out of the comparison and reported.
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
# the GPU's waiting-time word: count (17 bits) | capped flag
WAIT_MAX = 0x1FFFF
WAIT_CAPPED = 0x20000


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
                        wait=(sp["mcc_wait"] & WAIT_MAX).astype(np.int64),
                        wait_capped=(sp["mcc_wait"] & WAIT_CAPPED) != 0))
    return out


def open_trials(sp):
    """ids of particles loaded with a capped count at zero (open trials)."""
    if "wait_capped" not in sp:
        return np.zeros(0, np.uint64)
    return sp["id"][sp["wait_capped"] & (sp["wait"] == 0)]


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


def compare_particles(g, o, N, periodic, vrms, prev_ids=None, implicit=False, exclude=None):
    """g, o: dicts of arrays (oracle units) after one step.  prev_ids: the ids
    present before the step (children born in the step are those not in
    it); exclude: ids left out (open trials).  Returns (errors, mismatches);
    errors["decisions"] counts collision-process decisions and
    errors["children"] the one-sided children born in the step, which the
    caller checks against the decisions of the parent species.  A particle
    alive on one side only that is neither near an electrode nor such a
    child fails the comparison."""
    vu = g.get("vel_unit", 1.0)
    gi = {int(x): k for k, x in enumerate(g["id"])}
    oi = {int(x): k for k, x in enumerate(o["id"])}
    excl = set() if exclude is None else {int(x) for x in exclude}
    prev = None if prev_ids is None else {int(x) for x in prev_ids}
    one_sided = (set(gi) ^ set(oi)) - excl
    children = 0
    for p in sorted(one_sided):
        side, k = (g, gi[p]) if p in gi else (o, oi[p])
        xi = float(side["xi"][k])
        v = abs(float(side["vx"][k])) / vu          # cells per step
        reach = POS_MARGIN * max(1.0, v) + (v if implicit else 0.0)
        near = (not periodic) and (xi <= reach or N - xi <= reach)
        if near:
            continue
        if prev is not None and p not in prev and (p >> 63) == 1:
            children += 1
            continue
        raise AssertionError(
            f"particle {p} alive only on the {'GPU' if side is g else 'oracle'} side "
            f"at xi = {xi:.9g} of {N} cells (|v| = {v:.3g} cells/step): neither an "
            f"absorption decision at an electrode nor a child of a collision decision")
    mism = len(one_sided)
    common = sorted((set(gi) & set(oi)) - excl)
    if not common:
        return dict(pos=0.0, vel=0.0, n=0, decisions=0, children=children,
                    open=len(excl)), mism
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
    move = np.maximum(1.0, np.abs(vo[0]) / vu)
    relx = np.abs(dxi) / move
    bad_x = relx > POS_TOL
    # a velocity or position off by more than the tolerance is a collision-
    # process decision if the particle's transverse velocity changed on
    # either side (only collisions change vy, vz)
    vy_changed = (np.abs(vg[1] - vo[1]) > VEL_TOL * scale)
    dec = (bad_v | bad_x) & vy_changed
    decisions = int(dec.sum())
    # the next waiting time of a candidate is an integer drawn in float64 on
    # both sides: equal unless the quotient lies within rounding of an
    # integer; a capped GPU count only bounds the oracle's wait from below
    if "wait" in g and "wait" in o:
        gw = g["wait"][ig].astype(np.int64)
        ow = o["wait"][io].astype(np.int64)
        capped = g["wait_capped"][ig] if "wait_capped" in g else np.zeros(gw.size, bool)
        wait_ok = np.where(capped, ow > gw, ow == gw)
        dec |= ~wait_ok
    mism += int(dec.sum())
    ok = ~dec
    err = dict(pos=float(relx[ok].max(initial=0.0)),
               vel=float(dv[ok].max(initial=0.0)), n=len(common), decisions=decisions,
               children=children, open=len(excl))
    if "abar" in g:
        da = np.abs(g["abar"][ig] - o["abar"][io])
        sa = np.abs(o["abar"][io]).max(initial=0.0) + 1e-300
        err["abar"] = float(da[ok].max(initial=0.0) / sa)
    return err, mism


def check_children(errs):
    """One-sided children of a step: at most one per species for each
    collision-process decision of the electrons (their only parents)."""
    dec_e = errs[0]["decisions"] if errs[0] is not None else 0
    for s, e in enumerate(errs):
        if e is not None:
            assert e["children"] <= dec_e, (
                f"species {s}: {e['children']} children alive on one side only, "
                f"but {dec_e} electron collision decisions differ")


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
        opened = [open_trials(sp) for sp in sps]
        errs = [None, None]
        for s in range(2):
            o = sim.species(s)
            if o["id"].size == 0 and g2[s]["id"].size == 0:
                continue
            vr = float(np.sqrt(np.mean(o["vx"] ** 2 + o["vy"] ** 2 + o["vz"] ** 2))) \
                if o["vx"].size else 0.0
            err, mism = compare_particles(g2[s], o, N, periodic, vr, prev_ids=sps[s]["id"],
                                          implicit=implicit, exclude=opened[s])
            errs[s] = err
            rep["pos"] = max(rep["pos"], err["pos"])
            rep["vel"] = max(rep["vel"], err["vel"])
            if implicit and "abar" in err:
                rep["abar"] = max(rep["abar"], err["abar"])
            mism_step += mism
            rep["particle_steps"] += err["n"]
        check_children(errs)
        n_open = [int(x.size) for x in opened]
        rep["open_trials"] = rep.get("open_trials", 0) + sum(n_open)
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
                if mism_step == 0 and sum(n_open) == 0:
                    for key in ("work", "coll_dK"):
                        e = max(e, abs(gl[key][s] - ol[key][s]) / K)
                    e = max(e, np.abs(gl["absorbed_K"][s] - ol["absorbed_K"][s]).max() / K)
                    assert np.array_equal(gl["absorbed_n"][s], ol["absorbed_n"][s]), "absorbed"
                    assert np.array_equal(gl["n_coll"][s], ol["n_coll"][s]), "collisions"
                    assert gl["n_created"][s] == ol["n_created"][s], "created"
                # exact, but for open trials of capped GPU waits
                assert abs(int(gl["n_candidates"][s]) - int(ol["n_candidates"][s])) <= n_open[s], \
                    ("candidacy is exact", s, gl["n_candidates"][s], ol["n_candidates"][s])
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
