"""Long free-running comparison of the HIP path with the FP64 oracle.

Both start from the same 64-cell capacitive discharge (16k electrons and 16k
ions, 50 mTorr, 100 V at 13.56 MHz) and run 10 RF periods on their own.
Float32 particle state against float64 makes the two microstates drift apart
(the motion is chaotic), so they are compared through statistics over the
last 4 periods: the time-averaged node densities, the electron energy
distribution and the power absorbed from the field (the field work summed
over cells and species), each to 2 %.  The GPU side also exercises the
diagnostics accumulators (density, heating, EEDF sampled every step); the
oracle side samples its particle state after every step of the window."""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

E = 1.602176634e-19
ME = 9.1093837015e-31
PERIOD = 400          # steps per RF period at dt = 1/(400 f)
TOL = 0.02


def test_ccp64_ten_periods_statistics_match_oracle():
    import paper_1310_5284_amd as P
    wl = W.c1(collisions=1, np_per_species=16384)
    N = wl["case"]["n_cells"]
    dx = wl["case"]["gap_m"] / N
    t0, tw = 6 * PERIOD, 4 * PERIOD

    ctx = P.PicContext([wl])
    ctx.set_schedule(sort_every=64, diag_every=0, tile=2048)
    ctx.step(t0)
    ctx.reset_accumulators()
    ctx.set_schedule(sort_every=64, diag_every=1, tile=2048)
    ctx.step(tw)
    dens_g, n_samples = ctx.density()
    heat_g = ctx.heating()
    eedf_g, bin_eV, e_samples = ctx.eedf()
    ctx.close()
    assert n_samples == tw and e_samples == tw

    case, sps, procs = W.to_oracle(wl)
    sim = oracle.Sim(case, sps, procs)
    sim.step(t0)
    h0 = sim.heating()
    dens_o = [np.zeros(N + 1), np.zeros(N + 1)]
    eedf_o = np.zeros(eedf_g.size)
    for _ in range(tw):
        sim.step(1)
        for s in range(2):
            sp = sim.species(s)
            dens_o[s] += oracle.deposit_linear(N, sp["xi"]) * sim.w[s]
            if s == 0:
                eps = 0.5 * ME * (sp["vx"] ** 2 + sp["vy"] ** 2 + sp["vz"] ** 2) / E
                b = np.minimum(np.floor(eps / bin_eV).astype(np.int64), eedf_g.size - 1)
                eedf_o += np.bincount(b, minlength=eedf_g.size)
    h1 = sim.heating()

    vol = np.full(N + 1, dx)
    vol[0] = vol[-1] = dx / 2          # half cells at the electrodes
    for s in range(2):
        do = dens_o[s] / tw / vol
        err = np.linalg.norm(dens_g[s] - do) / np.linalg.norm(do)
        print(f"density species {s}: relative L2 {err:.4f}")
        assert err < TOL, (s, err)

    # EEDF: 1 eV bins (pairs of the 0.5 eV bins), L1 distance of the
    # normalised distributions, and the mean energy
    pg = eedf_g.reshape(-1, 2).sum(1) / eedf_g.sum()
    po = eedf_o.reshape(-1, 2).sum(1) / eedf_o.sum()
    l1 = np.abs(pg - po).sum()
    c = (np.arange(pg.size) + 0.5) * 2 * bin_eV
    mg, mo = (pg * c).sum(), (po * c).sum()
    print(f"EEDF: L1 {l1:.4f}, mean energy {mg:.4f} / {mo:.4f} eV")
    assert l1 < TOL
    assert abs(mg - mo) / mo < TOL

    pg_abs = sum(h.sum() for h in heat_g)
    po_abs = sum((h1[s] - h0[s]).sum() for s in range(2))
    err = abs(pg_abs - po_abs) / abs(po_abs)
    print(f"absorbed energy over the window: {pg_abs:.5e} / {po_abs:.5e} J/m^2 ({err:.4f})")
    assert err < TOL
