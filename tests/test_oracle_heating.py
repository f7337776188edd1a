"""Pin of the oracle's per-cell heating profile (the field work of a step
attributed to the cell where the particle's force is gathered; Sec. III's
heating profiles are this quantity summed over time).

The expected profile is built from the oracle's own input and output states,
not from its push: each particle's kinetic-energy change in x over the step,
1/2 m w (v_after^2 - v_before^2), binned by the cell it was gathered in
(explicit: floor of its position at the start of the step; implicit: floor
of the predicted position x~ the state holds).  A wrong cell index, a dropped
half-kick term or a species mix-up fails it.  Collisions are off and the
particles stay away from the electrodes, so every particle survives the
step."""
import numpy as np
import pytest

import workloads as W


def setup(orc, scheme, gather, N=24, n=3000, seed=7):
    rng = np.random.Generator(np.random.PCG64(seed))
    wl = W.ccp_workload("heat_pin", n_cells=N, np_per_species=n, volts=50.0, p_mtorr=50.0,
                        scheme=scheme, collisions=0, seed=seed, gather=gather,
                        dt=1.0 / (400.0 * 13.56e6) if scheme == 0 else 1.0 / (100.0 * 13.56e6))
    case, sps, procs = W.to_oracle(wl)
    for sp in sps:
        # away from the electrodes, and with an arbitrary abar history
        sp["xi"] = 2.0 + (N - 4.0) * rng.random(sp["xi"].size)
        if scheme == 1:
            sp["abar"] = 1e12 * (sp["q"] / abs(sp["q"])) * rng.standard_normal(sp["xi"].size) \
                * (9.1093837015e-31 / sp["m"])
    sim = orc.Sim(dict(case, step0=11), sps, procs, startup=False)
    # a field of every shape: random per cell
    E = 2.0e3 * rng.standard_normal(N)
    return sim, E, sps, case


@pytest.mark.parametrize("scheme", [0, 1])
@pytest.mark.parametrize("gather", [0, 1, 2])
def test_heating_profile_is_the_energy_change_binned_by_gather_cell(orc, scheme, gather):
    sim, E, sps, case = setup(orc, scheme, gather)
    dt = case["dt_s"]
    before = [sim.species(s) for s in range(2)]
    sim.step_with_field(E)
    after = [sim.species(s) for s in range(2)]
    heat = sim.heating()
    N = case["n_cells"]
    for s in range(2):
        b, a = before[s], after[s]
        assert a["id"].size == b["id"].size
        ia = np.argsort(a["id"])
        ib = np.argsort(b["id"])
        assert np.array_equal(a["id"][ia], b["id"][ib])
        if scheme == 0:
            v0, v1 = b["vx"][ib], a["vx"][ia]
        else:
            # the state holds v~ = v_{n-1/2} + dt abar/2 before and
            # v~' = v_{n+1/2} + dt abar_n / 2 after the step
            v0 = b["vx"][ib] - 0.5 * dt * b["abar"][ib]
            v1 = a["vx"][ia] - 0.5 * dt * a["abar"][ia]
        m, w = sps[s]["m"], sps[s]["w"]
        dK = 0.5 * m * w * (v1 ** 2 - v0 ** 2)
        cell = np.floor(b["xi"][ib]).astype(np.int64)
        expect = np.bincount(cell, weights=dK, minlength=N)
        scale = np.abs(dK).sum()
        assert scale > 0
        np.testing.assert_allclose(heat[s], expect, rtol=0, atol=1e-9 * scale)
        assert abs(sim.ledger()["work"][s] - dK.sum()) <= 1e-9 * scale
