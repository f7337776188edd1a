"""Pins of ion subcycling in the oracle (explicit scheme): ions are pushed,
absorbed and collided only in the steps n with n % K == 0, with the time step
K dt, and stand in between.

* in a given uniform field an ion follows leap-frog with the step K dt on
  exactly the steps n % K == 0 (closed form of constant acceleration), while
  electrons move every step;
* ions are null-collision candidates only in those steps, at the rate
  1 - exp(-nu_max K dt) per step taken (binomial bound);
* the energy and particle ledger closes with collisions and absorption on."""
import math

import numpy as np
import pytest

import workloads as W

E = 1.602176634e-19
ME = 9.1093837015e-31
MI = 40 * 1.66053906660e-27


def _field_run(orc, K, step0, nsteps=23):
    N, dx = 16, 1e-3
    rng = np.random.default_rng(K)
    n = 50
    xi = rng.uniform(4.0, 12.0, n)
    vi = rng.normal(0.0, 50.0, n)
    ve = rng.normal(0.0, 2e4, n)
    z = np.zeros(n)
    sps = [dict(q=-E, m=ME, w=1e-30, xi=xi.copy(), vx=ve, vy=z, vz=z, abar=None,
                id=np.arange(n, dtype=np.uint64)),
           dict(q=E, m=MI, w=1e-30, xi=xi.copy(), vx=vi, vy=z, vz=z, abar=None,
                id=np.arange(n, dtype=np.uint64))]
    dt = 2e-10
    case = dict(n_cells=N, gap_m=N * dx, bc=0, scheme=0, gather=0, collisions=0, dt_s=dt,
                step0=step0, ion_subcycle=K)
    sim = orc.Sim(case, sps, [], startup=False)
    Ef = np.full(N, 30.0)                     # V/m, uniform
    for _ in range(nsteps):
        sim.step_with_field(Ef)
    return sim, sps, dt, dx, Ef[0]


@pytest.mark.parametrize("K,step0", [(1, 0), (4, 0), (4, 3), (7, 5)])
def test_ions_follow_leapfrog_with_the_long_step(orc, K, step0):
    nsteps = 23
    sim, sps, dt, dx, Ef = _field_run(orc, K, step0, nsteps)
    m = sum(1 for s in range(step0, step0 + nsteps) if s % K == 0)   # ion pushes
    h = K * dt
    a = E / MI * Ef
    st = sim.species(1)
    o = np.argsort(st["id"])
    v0, x0 = sps[1]["vx"], sps[1]["xi"] * dx
    np.testing.assert_allclose(st["vx"][o], v0 + m * a * h, rtol=1e-12, atol=1e-9)
    x = x0 + h * (m * v0 + a * h * m * (m + 1) / 2)
    np.testing.assert_allclose(st["xi"][o] * dx, x, rtol=0, atol=1e-12)
    # electrons: every step with dt
    se = sim.species(0)
    oe = np.argsort(se["id"])
    ae = -E / ME * Ef
    np.testing.assert_allclose(se["vx"][oe], sps[0]["vx"] + nsteps * ae * dt, rtol=1e-12)


@pytest.mark.parametrize("K", [1, 4])
def test_ion_candidates_only_in_push_steps_at_the_long_step_rate(orc, K):
    wl = W.c1(collisions=1, np_per_species=20000)
    wl["case"]["gas_density_m3"] = W.gas_density(2000.0)   # frequent ion collisions
    wl["case"]["ion_subcycle"] = K
    case, sps, procs = W.to_oracle(wl)
    sim = orc.Sim(case, sps, procs)
    p = 1.0 - math.exp(-sim.numax(1) * case["dt_s"] * K)
    assert 0.02 < p < 0.9
    got, want, var = 0.0, 0.0, 0.0
    for _ in range(3 * K + 2):
        step = sim.step_index
        n = sim.count(1)
        sim.step(1)
        c = int(sim.ledger()["n_candidates"][1])
        if step % K:
            assert c == 0
        else:
            got += c
            want += n * p
            var += n * p * (1 - p)
    assert abs(got - want) < 5 * math.sqrt(var), (got, want)


@pytest.mark.parametrize("K", [3, 8])
def test_ledger_closes_with_subcycled_ions(orc, K):
    wl = W.c1(collisions=1, np_per_species=6000)
    wl["case"]["ion_subcycle"] = K
    case, sps, procs = W.to_oracle(wl)
    sim = orc.Sim(case, sps, procs)
    n_prev = [sim.count(0), sim.count(1)]
    for _ in range(4 * K):
        step = sim.step_index
        sim.step(1)
        L = sim.ledger()
        for sp in range(2):
            lhs = L["K_after"][sp] - L["K_before"][sp]
            rhs = L["work"][sp] - L["absorbed_K"][sp].sum() + L["coll_dK"][sp]
            assert abs(lhs - rhs) <= 1e-11 * max(L["K_before"][sp], 1e-300)
            n_now = sim.count(sp)
            assert n_now == n_prev[sp] - L["absorbed_n"][sp].sum() + L["n_created"][sp]
            n_prev[sp] = n_now
        if step % K:
            assert L["work"][1] == 0.0 and L["absorbed_n"][1].sum() == 0


def test_subcycling_is_explicit_only(orc):
    wl = W.c1(collisions=0, np_per_species=100, scheme=1)
    wl["case"]["ion_subcycle"] = 4
    case, sps, procs = W.to_oracle(wl)
    with pytest.raises(ValueError):
        orc.Sim(case, sps, procs)
