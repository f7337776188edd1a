"""Pins of ion subcycling in the oracle: ions are pushed, absorbed and
collided only in the steps n with n % K == 0, with the time step K dt, and
stand in between.

* in a given uniform field an ion follows leap-frog with the step K dt on
  exactly the steps n % K == 0 (closed form of constant acceleration), while
  electrons move every step; with the D1 scheme it follows the closed form
  of the D1 recurrence in a constant field at K dt;
* D1: a cold ion plasma over a fixed electron background follows the D1
  recurrence at omega_pi K dt (the ions' susceptibility carries (K dt)^2),
  and the implicit field of every step, push step or not, is the plain field
  of the corrected positions (the ions' susceptibility enters only the
  solves whose field they are corrected with);
* ions are null-collision candidates only in those steps, at the rate
  1 - exp(-nu_max K dt) per step taken (binomial bound);
* the energy and particle ledger closes with collisions and absorption on,
  for both schemes."""
import math

import numpy as np
import pytest

import workloads as W

E = 1.602176634e-19
ME = 9.1093837015e-31
MI = 40 * 1.66053906660e-27
EPS0 = 8.8541878128e-12


def _field_run(orc, K, step0, nsteps=23, scheme=0, startup=False):
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
    case = dict(n_cells=N, gap_m=N * dx, bc=0, scheme=scheme, gather=0, collisions=0, dt_s=dt,
                step0=step0, ion_subcycle=K)
    sim = orc.Sim(case, sps, [], startup=startup)
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


def _d1_constant_field(x0, v0, a, h, M):
    """D1 in a constant acceleration a from the stored state (x~ = x0,
    v~ = v0, abar = 0) after M steps of h: abar_m = a (1 - 2^-m),
    v_{m+1/2} = v_{m-1/2} + h abar_m, x_m = x_{m-1} + h v_{m-1/2}; returns the
    stored x~ = x_M + h v~ and v~ = v_{M+1/2} + h abar_M / 2."""
    vt = v0 + h * a * (M - 0.5 + 2.0 ** (-M - 1))
    xM = x0 - h * v0 + h * (M * v0 + h * a * (M * (M - 1) / 2 + 1 - 2.0 ** -M))
    return xM + h * vt, vt, a * (1 - 2.0 ** -M)


@pytest.mark.parametrize("K,step0,startup", [(1, 0, False), (4, 0, False), (4, 3, False),
                                             (7, 5, False), (4, 0, True), (7, 5, True)])
def test_implicit_ions_follow_d1_with_the_long_step(orc, K, step0, startup):
    # with the start-up, the first prediction takes the species' own step:
    # x~ = x_0 + h v
    nsteps = 23
    sim, sps, dt, dx, Ef = _field_run(orc, K, step0, nsteps, scheme=1, startup=startup)
    M = sum(1 for s in range(step0, step0 + nsteps) if s % K == 0)
    for sp, q, m, h, steps in ((1, E, MI, K * dt, M), (0, -E, ME, dt, nsteps)):
        st = sim.species(sp)
        o = np.argsort(st["id"])
        x0 = sps[sp]["xi"] * dx + (h * sps[sp]["vx"] if startup else 0.0)
        x, vt, ab = _d1_constant_field(x0, sps[sp]["vx"], q / m * Ef, h, steps)
        np.testing.assert_allclose(st["vx"][o], vt, rtol=1e-12, atol=1e-9)
        np.testing.assert_allclose(st["abar"][o], ab, rtol=1e-12)
        np.testing.assert_allclose(st["xi"][o] * dx, x, rtol=0, atol=1e-12 + 1e-12 * abs(x).max())


@pytest.mark.parametrize("K,wdt", [(1, 0.6), (3, 0.6), (4, 2.0)])
def test_d1_cold_ion_plasma_follows_recurrence_at_the_long_step(orc, K, wdt):
    # ions displaced over a fixed uniform electron background: each cell an
    # oscillator at omega_pi, stepped by D1 with h = K dt in the push steps
    N, ppc, mode, A, n0 = 16, 8, 2, 0.05, 1e15
    wp = math.sqrt(n0 * E * E / (EPS0 * MI))
    h = wdt / wp
    dt = h / K
    dx = 1e-3
    offs = 0.25 + 0.5 * (np.arange(ppc) + 0.5) / ppc
    j = np.repeat(np.arange(N), ppc)
    base = j + np.tile(offs, N)
    amp = A * np.sin(2 * np.pi * mode * j / N)
    n = N * ppc
    z = np.zeros(n)
    sps = [dict(q=-E, m=ME, w=1.0, xi=np.zeros(0), vx=np.zeros(0), vy=np.zeros(0),
                vz=np.zeros(0), abar=None, id=np.zeros(0, np.uint64)),
           dict(q=E, m=MI, w=n0 * dx / ppc, xi=base + amp, vx=z, vy=z, vz=z, abar=None,
                id=np.arange(n, dtype=np.uint64))]
    case = dict(n_cells=N, gap_m=N * dx, bc=1, scheme=1, gather=0, collisions=0, dt_s=dt,
                background_rho=-n0 * E, ion_subcycle=K)
    sim = orc.Sim(case, sps, [])
    # the D1 recurrence per unit amplitude (start at rest, x~_1 = x_0)
    x, v, ab, xt, ref = 1.0, 0.0, 0.0, 1.0, []
    for _ in range(40):
        xn = xt / (1 + 0.5 * wp ** 2 * h ** 2)
        a = -wp ** 2 * xn
        v = v + 0.5 * h * ab + 0.5 * h * a
        ab = 0.5 * (ab + a)
        xt = xn + h * (v + 0.5 * h * ab)
        ref.append(xt)
    order = np.argsort(sps[1]["id"])
    m = 0
    for step in range(40 * K):
        sim.step(1)
        m += step % K == 0
        st = sim.species(1)
        xi = st["xi"][np.argsort(st["id"])][order]
        np.testing.assert_allclose(xi - base, amp * ref[m - 1], rtol=0, atol=1e-11)


@pytest.mark.parametrize("K,step0", [(4, 0), (3, 2)])
def test_implicit_field_with_subcycled_ions_is_the_field_of_the_corrected_positions(
        orc, K, step0):
    # light ions (50 electron masses) so that their correction weighs: in a
    # push step the solve must take their susceptibility with (K dt)^2, in
    # the others leave it out
    rng = np.random.default_rng(11)
    N, dx = 24, 2e-4
    L = N * dx
    n, n0 = 400, 5e15
    w = n0 * L / n
    wp = math.sqrt(n0 * E * E / (EPS0 * ME))
    dt = 0.2 / wp
    mi = 50 * ME
    z = np.zeros(n)
    sps = [dict(q=-E, m=ME, w=w, xi=rng.integers(0, N, n) + 0.3 + 0.4 * rng.random(n), vx=z,
                vy=z, vz=z, abar=None, id=np.arange(n, dtype=np.uint64)),
           dict(q=E, m=mi, w=w, xi=rng.integers(0, N, n) + 0.3 + 0.4 * rng.random(n), vx=z,
                vy=z, vz=z, abar=None, id=np.arange(n, dtype=np.uint64))]
    case = dict(n_cells=N, gap_m=L, bc=0, scheme=1, gather=0, collisions=0, dt_s=dt,
                rf_volts=3.0, rf_freq_hz=1e7, step0=step0, ion_subcycle=K)
    imp = orc.Sim(case, sps, [], startup=False)
    seen = set()
    for _ in range(K + 1):
        step = imp.step_index
        before = [imp.species(k) for k in range(2)]
        imp.step(1)
        fi = imp.fields()
        moved = []
        for k in range(2):
            after = imp.species(k)
            h = dt * (K if k == 1 else 1)
            push = k == 0 or step % K == 0
            x1 = after["xi"] - after["vx"] * h / dx if push else after["xi"]
            o_b = np.argsort(before[k]["id"]); o_a = np.argsort(after["id"])
            shift = x1[o_a] - before[k]["xi"][o_b]
            assert np.all(np.floor(x1[o_a]) == np.floor(before[k]["xi"][o_b]))   # no crossing
            if push:
                assert np.abs(shift).max() > 1e-4
            else:
                assert np.all(shift == 0)
            moved.append(dict(sps[k], xi=x1, id=after["id"], vx=np.zeros(x1.size),
                              vy=np.zeros(x1.size), vz=np.zeros(x1.size)))
        ex = orc.Sim(dict(case, scheme=0, step0=step + 1, ion_subcycle=1), moved, [])
        ex.compute_fields()
        fe = ex.fields()
        np.testing.assert_allclose(fi["E"], fe["E"], rtol=0, atol=1e-9 * abs(fe["E"]).max())
        seen.add(step % K == 0)
    assert seen == {True, False}


@pytest.mark.parametrize("K,scheme", [(1, 0), (4, 0), (4, 1)])
def test_ion_candidates_only_in_push_steps_at_the_long_step_rate(orc, K, scheme):
    wl = W.c1(collisions=1, np_per_species=20000, scheme=scheme)
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


@pytest.mark.parametrize("K,scheme", [(3, 0), (8, 0), (3, 1), (5, 1)])
def test_ledger_closes_with_subcycled_ions(orc, K, scheme):
    wl = W.c1(collisions=1, np_per_species=6000, scheme=scheme)
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
