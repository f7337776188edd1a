"""GPU parity: the HIP path through the C-ABI against the FP64 oracle,
teacher-forced one step at a time (see tests/parity.py for the protocol).

Sizes span several workgroups and a ragged tail: the tile is set small so a
species of a few thousand particles runs on many workgroups."""
import math

import numpy as np
import pytest

import workloads as W
from parity import assert_report, teacher_forced

pytestmark = pytest.mark.gpu


def ctx_for(wl, tile=1024, sort_every=16, **kw):
    import paper_1310_5284_amd as P
    ctx = P.PicContext([wl], **kw)
    ctx.set_schedule(sort_every=sort_every, diag_every=0, tile=tile)
    return ctx


@pytest.mark.parametrize("collisions", [0, 1])
def test_ccp64_explicit_teacher_forced(collisions):
    wl = W.c1(collisions=collisions, np_per_species=16384 + 77)
    ctx = ctx_for(wl)
    rep = teacher_forced(ctx, wl, 100)
    print(rep)
    assert_report(rep)


@pytest.mark.parametrize("gather", [0, 1, 2])
def test_periodic_thermal_teacher_forced(gather):
    wl = W.c2(ratio=5.0, gather=gather, ppc=100, n_cells=32)
    ctx = ctx_for(wl)
    rep = teacher_forced(ctx, wl, 100)
    print(rep)
    assert_report(rep)


@pytest.mark.parametrize("wdt,steps", [(2.0, 100), (5.0, 60)])
def test_ccp256_implicit_teacher_forced(wdt, steps):
    # at omega_p dt = 5 the D1/EC discharge heats and ionizes without bound
    # (the oracle does the same; the paper reports no convergence for
    # dt > 2/omega_p), so that run gets room for the children
    wl = W.c3(ppc=40, wdt=wdt)
    for sp in wl["species"]:
        sp["capacity"] = 4 * sp["cell"].size
    ctx = ctx_for(wl)
    rep = teacher_forced(ctx, wl, steps)
    print(rep)
    assert_report(rep)


@pytest.mark.parametrize("scheme,gather", [(0, 0), (1, 0), (1, 2)])
def test_ionizing_beam_teacher_forced(scheme, gather):
    # 100 eV isotropic electrons in dense gas: every electron is a candidate
    # in every step and about 5 % of them ionize, i.e. more ionizations per
    # collision workgroup than its LDS queue holds, so both the queued and
    # the immediate child paths run (implicit: most candidates collide for
    # real, so the deposit of their null prediction is undone)
    wl = W.c1(collisions=1, np_per_species=8192 + 33, scheme=scheme)
    wl["case"]["gather"] = gather
    wl["case"]["gas_density_m3"] = W.gas_density(1000.0)
    e = wl["species"][0]
    n = e["cell"].size
    rng = np.random.Generator(np.random.PCG64(0xBEA))
    v = math.sqrt(2.0 * 100.0 * 1.602176634e-19 / 9.1093837015e-31)
    mu = rng.uniform(-1.0, 1.0, n)
    ph = rng.uniform(0.0, 2.0 * math.pi, n)
    sn = np.sqrt(1.0 - mu * mu)
    e["vx"] = (v * mu).astype(np.float32)
    e["vy"] = (v * sn * np.cos(ph)).astype(np.float32)
    e["vz"] = (v * sn * np.sin(ph)).astype(np.float32)
    for sp in wl["species"]:
        sp["capacity"] = 3 * sp["cell"].size // 2
    tile = 8192
    n_wg = -(-wl["species"][0]["capacity"] // tile)   # electron workgroups
    probe = ctx_for(wl, tile=tile)
    probe.step(1)
    n_ion = int(probe.ledger()["n_coll"][0][2])
    probe.close()
    assert n_ion > 128 * n_wg, (n_ion, n_wg)   # so one workgroup holds > 128
    ctx = ctx_for(wl, tile=tile)
    rep = teacher_forced(ctx, wl, 8)
    print(n_ion, rep)
    assert_report(rep)


@pytest.mark.parametrize("scheme,gather", [(0, 0), (1, 0), (1, 2)])
def test_max_cells_teacher_forced(scheme, gather):
    # the largest grid the library takes (PIC_MAX_CELLS = 4096 cells: the
    # deposit grid and the field fill the most LDS, with m = 2 implicit also
    # the susceptibility words), 300 V, 30 mTorr
    wl = W.ccp_workload("ccp4096", n_cells=4096, np_per_species=40000 + 11, volts=300.0,
                        dt=1.0 / (2000.0 * 13.56e6), p_mtorr=30.0, scheme=scheme, seed=0x4096)
    wl["case"]["gather"] = gather
    ctx = ctx_for(wl, tile=4096)
    rep = teacher_forced(ctx, wl, 20)
    print(rep)
    assert_report(rep)


def test_ccp64_mc_explicit_teacher_forced():
    # the momentum-conserving gather (CIC of the nodal field) on the RF
    # discharge with electrodes and collisions
    wl = W.c1(collisions=1, np_per_species=16384 + 77)
    wl["case"]["gather"] = 1
    ctx = ctx_for(wl)
    rep = teacher_forced(ctx, wl, 60)
    print(rep)
    assert_report(rep)


def test_ccp256_mc_implicit_teacher_forced():
    # D1 implicit with the momentum-conserving gather
    wl = W.c3(ppc=40, wdt=2.0)
    wl["case"]["gather"] = 1
    for sp in wl["species"]:
        sp["capacity"] = 2 * sp["cell"].size
    ctx = ctx_for(wl)
    rep = teacher_forced(ctx, wl, 40)
    print(rep)
    assert_report(rep)


def test_ccp64_ec2_explicit_teacher_forced():
    # m = 2 read as spline degree: quadratic deposit (folded at the
    # electrodes), linear interpolation of the half-grid field
    wl = W.c1(collisions=1, np_per_species=16384 + 77)
    wl["case"]["gather"] = 2
    ctx = ctx_for(wl)
    rep = teacher_forced(ctx, wl, 60)
    print(rep)
    assert_report(rep)


def test_ccp256_ec2_implicit_teacher_forced():
    # D1 implicit with m = 2: quadratic deposit of the predicted positions and
    # the row-sum susceptibility of the dual grid (electrode half cells
    # included: the sheaths hold ions there)
    wl = W.c3(ppc=40, wdt=2.0)
    wl["case"]["gather"] = 2
    for sp in wl["species"]:
        sp["capacity"] = 2 * sp["cell"].size
    ctx = ctx_for(wl)
    rep = teacher_forced(ctx, wl, 40)
    print(rep)
    assert_report(rep)


def test_periodic_ec2_implicit_teacher_forced():
    # the periodic dual grid: the centre left of cell 0 is the last centre
    wl = W.c2(ratio=5.0, gather=2, ppc=100, n_cells=32, wdt=1.5)
    wl["case"]["scheme"] = 1
    ctx = ctx_for(wl)
    rep = teacher_forced(ctx, wl, 60)
    print(rep)
    assert_report(rep)


@pytest.mark.parametrize("scheme,steps_per_period,gather", [(0, 400, 0), (1, 100, 0),
                                                           (0, 400, 1), (1, 100, 1),
                                                           (0, 400, 2), (1, 100, 2)])
def test_ccp64_nonuniform_teacher_forced(scheme, steps_per_period, gather):
    # sheath-refined grid: cells about 4x narrower within 15 % of the gap
    # from either electrode; the implicit run takes 4x the time step, so that
    # fast electrons cross several narrow cells in one move (EC, MC and
    # m = 2 gathers)
    f = 13.56e6
    wl = W.ccp_workload("ccp64_nonuniform", n_cells=64, np_per_species=16384 + 77,
                        volts=100.0, p_mtorr=50.0, dt=1.0 / (steps_per_period * f),
                        scheme=scheme, collisions=1, seed=0x64 + scheme,
                        cell_dx=W.sheath_refined_widths(64, 0.025), gather=gather)
    ctx = ctx_for(wl)
    rep = teacher_forced(ctx, wl, 60)
    print(rep)
    assert_report(rep)


@pytest.mark.parametrize("gather,nonuniform", [(1, False), (2, False), (0, True), (2, True)])
def test_ccp64_subcycled_ions_implicit_gathers_teacher_forced(gather, nonuniform):
    # D1 with ions every 4th step under the MC and m = 2 weightings and on the
    # sheath-refined grid: the ions' node charges, moment words (m = 2) and
    # left-side sums (m = 2, nonuniform) stand between their pushes, and
    # their susceptibility enters only the solve before a push
    kw = dict(cell_dx=W.sheath_refined_widths(64, 0.025)) if nonuniform else {}
    wl = W.ccp_workload("ccp64_sub_d1", n_cells=64, np_per_species=16384 + 77, volts=100.0,
                        p_mtorr=500.0, scheme=1, collisions=1, seed=0x5D1 + gather,
                        gather=gather, **kw)
    wl["case"]["ion_subcycle"] = 4
    ctx = ctx_for(wl)
    rep = teacher_forced(ctx, wl, 14)
    print(rep)
    assert_report(rep)


@pytest.mark.parametrize("scheme", [0, 1])
def test_dense_candidate_lists_teacher_forced(scheme):
    # one workgroup per species at tile 16384: at 50 mTorr over half of the
    # electrons are candidates every step, so the first workgroup's list
    # holds thousands of candidates (the k_collide workgroup of a dense list
    # loops over many blocks); the 77-particle tail is a list of its own
    wl = W.c1(collisions=1, np_per_species=16384 + 77, scheme=scheme)
    ctx = ctx_for(wl, tile=16384)
    rep = teacher_forced(ctx, wl, 30)
    print(rep)
    assert_report(rep)
    assert ctx.ledger()["n_candidates"][0] >= 4096 + 77


@pytest.mark.parametrize("K,step0,scheme", [(4, 0, 0), (7, 5, 0), (4, 0, 1), (7, 5, 1)])
def test_ccp64_subcycled_ions_teacher_forced(K, step0, scheme):
    # ions pushed, absorbed and collided every K-th step with K dt; in
    # between their deposit stays on the grid (high pressure: ion
    # collisions in most push steps).  D1: the ions' susceptibility, with
    # (K dt)^2, only in the solve before a push step
    wl = W.c1(collisions=1, np_per_species=16384 + 77, scheme=scheme)
    wl["case"]["ion_subcycle"] = K
    wl["case"]["step0"] = step0
    wl["case"]["gas_density_m3"] = W.gas_density(500.0)
    ctx = ctx_for(wl)
    rep = teacher_forced(ctx, wl, 6 * K)
    print(rep)
    assert_report(rep)
