"""GPU edge cases, determinism, resume and closed-form checks through the C-ABI."""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from parity import assert_report, teacher_forced

pytestmark = pytest.mark.gpu

E = 1.602176634e-19
ME = 9.1093837015e-31
EPS0 = 8.8541878128e-12


def P():
    import paper_1310_5284_amd as P
    return P


def ctx_for(wl, tile=1024, sort_every=16, **kw):
    ctx = P().PicContext([wl], **kw)
    ctx.set_schedule(sort_every=sort_every, diag_every=0, tile=tile)
    return ctx


def sorted_state(ctx, case=0):
    st = ctx.state(case)
    out = []
    for sp in st["species"]:
        o = np.argsort(sp["id"])
        out.append({k: v[o] for k, v in sp.items()})
    return out


def test_cold_plasma_exact_omega_p_on_gpu():
    # EC cold plasma: each cell oscillates at exactly omega_p (see the oracle
    # pin); the GPU's float32 state must follow A cos(n theta) to 1e-5 cells
    N, ppc, wdt, A = 32, 16, 0.3, 0.1
    n0 = 1e15
    wp = math.sqrt(n0 * E * E / (EPS0 * ME))
    dt, dx = wdt / wp, 1e-3
    offs = (0.25 + 0.5 * (np.arange(ppc) + 0.5) / ppc)
    j = np.repeat(np.arange(N), ppc)
    amp = A * np.sin(2 * np.pi * 3 * j / N)
    xi = j + np.tile(offs, N) + amp
    v = amp * (0.5 * wdt ** 2) * dx / dt
    n = xi.size
    cell = np.floor(xi).astype(np.int32)
    e = dict(q=-E, m=ME, w=n0 * dx / ppc, cell=cell, off=(xi - cell).astype(np.float32),
             vx=v.astype(np.float32), vy=np.zeros(n, np.float32), vz=np.zeros(n, np.float32),
             id=np.arange(n, dtype=np.uint64), capacity=n)
    wl = dict(case=dict(n_cells=N, gap_m=N * dx, bc=1, dt_s=dt, background_rho=n0 * E),
              species=[e, W.empty_species(E, W.M_AR)], processes=[])
    ctx = ctx_for(wl, tile=256)
    theta = math.acos(1 - 0.5 * wdt ** 2)
    base = j + np.tile(offs, N)
    for step in range(1, 101):
        ctx.step(1)
        s = sorted_state(ctx)[0]
        x = s["cell"].astype(np.float64) + s["off"]
        err = np.abs(x - (base + amp * math.cos(step * theta))).max()
        assert err < 1e-5, (step, err)


def test_empty_ion_species_and_two_cells():
    wl = W.c1(collisions=1, np_per_species=2000)
    wl["case"]["n_cells"] = 2
    for sp in wl["species"]:
        sp["cell"] = (sp["cell"] % 2).astype(np.int32)
    # two 1.25 cm cells: electrons fall through the whole RF voltage and ionize
    wl["species"][0]["capacity"] = 16000
    wl["species"][1] = W.empty_species(E, W.M_AR, w=wl["species"][0]["w"], capacity=16000)
    ctx = ctx_for(wl, tile=256)
    rep = teacher_forced(ctx, wl, 20)
    assert_report(rep)


def test_particles_on_cell_edges_and_ragged_tail():
    wl = W.c1(collisions=0, np_per_species=777)
    for sp in wl["species"]:
        sp["off"][::3] = 0.0                         # exactly on a node
        sp["off"][1::7] = np.nextafter(np.float32(1.0), np.float32(0.0))
    ctx = ctx_for(wl, tile=256)
    rep = teacher_forced(ctx, wl, 30)
    assert_report(rep)


def test_determinism_of_state_and_fields():
    wl = W.c1(collisions=1, np_per_species=8192)
    outs = []
    for _ in range(2):
        ctx = ctx_for(wl, tile=512, sort_every=7)
        ctx.step(60)
        outs.append((sorted_state(ctx), ctx.fields()))
        ctx.close()
    (s1, f1), (s2, f2) = outs
    for a, b in zip(s1, s2):
        for k in a:
            assert np.array_equal(a[k], b[k]), k
    for k in ("rho", "phi", "E"):
        assert np.array_equal(f1[k], f2[k]), k


def _variant(name, np_per_species=4096):
    # the 64-cell discharge as is, implicit, with ions subcycled (K = 3;
    # explicit or implicit), on a sheath-refined grid (implicit), or m = 2
    # implicit
    if name in ("nonuniform_implicit", "nonuniform_ec2_implicit"):
        return W.ccp_workload("ccp64_nonuniform", n_cells=64, np_per_species=np_per_species,
                              volts=100.0, p_mtorr=50.0, scheme=1, seed=0x65,
                              cell_dx=W.sheath_refined_widths(64, 0.025),
                              gather=2 if "ec2" in name else 0)
    wl = W.c1(collisions=1, np_per_species=np_per_species,
              scheme=1 if "implicit" in name else 0)
    if "subcycle3" in name:
        wl["case"]["ion_subcycle"] = 3
    if name == "ec2_implicit":
        wl["case"]["gather"] = 2
    return wl


@pytest.mark.parametrize("variant", ["explicit", "implicit", "subcycle3", "implicit_subcycle3",
                                     "nonuniform_implicit"])
def test_resume_equals_uninterrupted(variant):
    # 40 steps: a subcycled run resumes between two ion pushes
    wl = _variant(variant)
    a = ctx_for(wl, sort_every=1000)
    a.step(40)
    st = a.state()
    b_wl = dict(wl)
    b_wl["case"] = dict(wl["case"], step0=st["step"])
    b_wl["species"] = [dict(wl["species"][s], **st["species"][s]) for s in range(2)]
    b = ctx_for(b_wl, sort_every=1000, flags=P().FLAG_INTERNAL_UNITS)
    a.step(30)
    b.step(30)
    for x, y in zip(sorted_state(a), sorted_state(b)):
        for k in x:
            assert np.array_equal(x[k], y[k]), k
    fa, fb = a.fields(), b.fields()
    for k in ("rho", "E"):
        np.testing.assert_array_equal(fa[k], fb[k])


def test_capacity_overflow_is_reported():
    wl = W.c1(collisions=1, np_per_species=3000)
    wl["case"]["gas_density_m3"] = W.gas_density(3000.0)
    for sp in wl["species"]:
        sp["capacity"] = sp["cell"].size + 2
        sp["vx"] = sp["vx"] * (10.0 if sp["m"] < 1e-27 else 1.0)
    ctx = ctx_for(wl, tile=256)
    with pytest.raises(P().PicError) as ei:
        ctx.step(50)
    assert ei.value.code == P().PIC_E_CAPACITY


def test_unstable_explicit_case_is_rejected():
    wl = W.c1(collisions=0, np_per_species=2000)
    wl["case"]["dt_s"] = 2.5 / 1.784e9 * 8   # omega_p dt >> 2 at the load density
    with pytest.raises(P().PicError) as ei:
        P().PicContext([wl])
    assert ei.value.code == P().PIC_E_UNSTABLE
    P().PicContext([wl], flags=P().FLAG_ALLOW_UNSTABLE).close()


def test_invalid_inputs_are_rejected():
    wl = W.c1(collisions=0, np_per_species=100)
    wl["species"][0]["cell"][5] = 64          # outside [0, N)
    with pytest.raises(P().PicError) as ei:
        P().PicContext([wl])
    assert ei.value.code == P().PIC_E_INVAL
    wl = W.c1(collisions=0, np_per_species=100)
    wl["species"][1]["off"][0] = 1.0          # offset must be < 1
    with pytest.raises(P().PicError):
        P().PicContext([wl])
    wl = W.c1(collisions=0, np_per_species=100)
    ctx = P().PicContext([wl])
    with pytest.raises(P().PicError) as ei:
        ctx.step_implicit(1)                  # explicit case
    assert ei.value.code == P().PIC_E_INVAL


@pytest.mark.parametrize("timing_every", [0, 1, 3])
def test_graph_replay_equals_host_launches(timing_every):
    # a mixed batch (explicit + implicit case) stepped with every kernel
    # launched from the host, and again with whole sort periods replayed from
    # a captured graph; calls that start and end inside a period mix both
    wls = [W.c1(collisions=1, np_per_species=6144, scheme=0),
           W.c1(collisions=1, np_per_species=4096, scheme=1)]
    outs = []
    for graph in (0, 1):
        ctx = P().PicContext(wls)
        ctx.set_schedule(sort_every=7, diag_every=0, tile=1024)
        ctx.set_launch(graph=graph, timing_every=timing_every)
        for n in (3, 25, 2, 30):
            ctx.step(n)
            ms, launches = ctx.last_timing()
            assert (launches > 0) == (timing_every > 0)
            assert ms >= 0.0
        outs.append([(sorted_state(ctx, k), ctx.fields(k)) for k in range(2)])
        ctx.close()
    for (s1, f1), (s2, f2) in zip(*outs):
        for a, b in zip(s1, s2):
            for k in a:
                assert np.array_equal(a[k], b[k]), k
        for k in ("rho", "phi", "E"):
            assert np.array_equal(f1[k], f2[k]), k


def test_graph_replay_with_every_grid_variant():
    # one batch of subcycled (explicit and implicit), sheath-refined (EC and
    # m = 2 implicit; the implicit launch then reads every case's grid tables
    # from global memory) and m = 2 implicit cases:
    # the subcycling phase is read on the device, so replays of a captured
    # sort period step exactly as host launches do
    wls = [_variant("subcycle3", 3000), _variant("nonuniform_implicit", 3000),
           _variant("ec2_implicit", 3000), _variant("implicit_subcycle3", 3000),
           _variant("nonuniform_ec2_implicit", 3000)]
    outs = []
    for graph in (0, 1):
        ctx = P().PicContext(wls)
        ctx.set_schedule(sort_every=5, diag_every=0, tile=1024)
        ctx.set_launch(graph=graph, timing_every=0)
        for n in (4, 13, 7):
            ctx.step(n)
        outs.append([(sorted_state(ctx, k), ctx.fields(k)) for k in range(len(wls))])
        ctx.close()
    for (s1, f1), (s2, f2) in zip(*outs):
        for a, b in zip(s1, s2):
            for k in a:
                assert np.array_equal(a[k], b[k]), k
        for k in ("rho", "phi", "E", "chi"):
            assert np.array_equal(f1[k], f2[k]), k


@pytest.mark.parametrize("graph", [0, 1])
def test_store_policies_step_identically(graph):
    # the collision kernel's store policy changes only the cache behaviour:
    # a mixed batch (both schemes, collisions, ionization) steps to the same
    # state and fields with either, also when the policy changes between
    # calls (a captured graph holds the policy it was captured with)
    wls = [W.c1(collisions=1, np_per_species=6144, scheme=0),
           W.c1(collisions=1, np_per_species=4096, scheme=1)]
    outs = []
    for pol in ((0, 0, 0), (1, 1, 1), (1, 0, 1)):
        ctx = P().PicContext(wls)
        ctx.set_schedule(sort_every=7, diag_every=0, tile=1024)
        ctx.set_launch(graph=graph, timing_every=0)
        for p, n in zip(pol, (9, 23, 12)):
            ctx.set_store_policy(p)
            ctx.step(n)
        outs.append([(sorted_state(ctx, k), ctx.fields(k)) for k in range(2)])
        ctx.close()
    for other in outs[1:]:
        for (s1, f1), (s2, f2) in zip(outs[0], other):
            for a, b in zip(s1, s2):
                for k in a:
                    assert np.array_equal(a[k], b[k]), k
            for k in ("rho", "phi", "E"):
                assert np.array_equal(f1[k], f2[k]), k
    ctx = P().PicContext(wls[:1])
    for bad in (-1, 2):
        with pytest.raises(P().PicError) as ei:
            ctx.set_store_policy(bad)
        assert ei.value.code == P().PIC_E_INVAL
    ctx.close()


def test_launch_mode_rejects_bad_values():
    ctx = ctx_for(W.c1(collisions=0, np_per_species=1024))
    for g, t in ((2, 1), (-1, 1), (0, -1)):
        with pytest.raises(P().PicError):
            ctx.set_launch(graph=g, timing_every=t)
    ctx.close()


def test_autotune_picks_a_candidate_and_steps_like_pic_step():
    wl = W.c1(collisions=1, np_per_species=8192 + 5)
    ctx = ctx_for(wl, tile=1024, sort_every=16)
    ctx.step(3)
    tile, sort, ms = ctx.autotune(tiles=[256, 1024, 4096], sorts=[5, 16], steps_per_trial=6)
    assert tile in (256, 1024, 4096) and sort in (5, 16)
    assert len(ms) == 7 and all(m > 0.0 for m in ms)
    assert ms[[256, 1024, 4096].index(tile)] == min(ms[:3])
    assert ms[3 + [5, 16].index(sort)] == min(ms[3:5])   # then the two store policies
    ctx.step(4)
    n = ctx.state()["step"] - wl["case"].get("step0", 0)
    # the same number of plain steps at another schedule gives the same state
    ref = ctx_for(wl, tile=2048, sort_every=7)
    ref.step(n)
    for a, b in zip(sorted_state(ctx), sorted_state(ref)):
        for k in a:
            assert np.array_equal(a[k], b[k]), k
    fa, fb = ctx.fields(), ref.fields()
    for k in ("rho", "phi", "E"):
        assert np.array_equal(fa[k], fb[k]), k
    with pytest.raises(P().PicError):
        ctx.autotune(tiles=[300], sorts=[8], steps_per_trial=2)
    ctx.close()
    ref.close()


def test_batch_with_the_dual_grid_equals_separate_runs():
    # an m = 1 and an m = 2 implicit case in one launch: the launch's shared
    # memory holds the susceptibility words of the dual grid, and each case
    # lays it out by its own weighting; both step as they do alone
    wls = [W.c1(collisions=1, np_per_species=4096, scheme=1),
           W.c1(collisions=1, np_per_species=6144 + 3, scheme=1, seed=0xD2)]
    wls[1]["case"]["gather"] = 2
    batch = P().PicContext(wls)
    batch.set_schedule(sort_every=7, diag_every=0, tile=1024)
    batch.step(30)
    for k, wl in enumerate(wls):
        alone = ctx_for(wl, sort_every=7)
        alone.step(30)
        for a, b in zip(sorted_state(batch, k), sorted_state(alone)):
            for key in a:
                assert np.array_equal(a[key], b[key]), (k, key)
        fb, fa = batch.fields(k), alone.fields()
        for key in ("rho", "phi", "E", "chi"):
            assert np.array_equal(fb[key], fa[key]), (k, key)
        alone.close()
    batch.close()
