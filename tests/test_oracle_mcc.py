"""Pins of the oracle's null-collision Monte Carlo collisions against the
closed forms of the method (Vahedi & Surendra 1995 null-collision scheme,
isotropic scattering, Opal-Peterson-Beaty energy sharing, Maxwellian neutrals).
"""
import math

import numpy as np
import pytest

import workloads as W

QE = 1.602176634e-19
KB = 1.380649e-23


def beam_sim(orc, p_mtorr=50.0, dt=1.8437e-10):
    wl = W.c1(collisions=1, np_per_species=4)
    case, sps, procs = W.to_oracle(wl)
    case = dict(case, gas_density_m3=W.gas_density(p_mtorr), dt_s=dt)
    return orc.Sim(case, sps, procs), case, procs


def speed_of(eps_eV, m):
    return math.sqrt(2 * QE * eps_eV / m)


def sigma_tab(procs, kind, eps):
    p = [q for q in procs if q["kind"] == kind][0]
    if p["threshold_eV"] > 0 and eps <= p["threshold_eV"]:
        return 0.0
    return float(np.interp(eps, p["e0_eV"] + p["de_eV"] * np.arange(p["sigma"].size),
                           p["sigma"]))


@pytest.mark.parametrize("eps", [8.0, 30.0, 120.0])
def test_process_fractions_match_null_collision_law(orc, eps):
    # a candidate undergoes process k with probability n_g sigma_k(eps) v / nu_max
    sim, case, procs = beam_sim(orc)
    numax = sim.numax(0)
    ng = case["gas_density_m3"]
    v = speed_of(eps, W.M_E)
    n = 30000
    counts = {k: 0 for k in (-2, 0, 1, 2)}
    for pid in range(n):
        r = sim.collide_one(0, pid, 17, [v, 0.0, 0.0])[0]
        counts[r] += 1
    for kind in (W.ELASTIC, W.EXCITATION, W.IONIZATION):
        p = ng * sigma_tab(procs, kind, eps) * v / numax
        sd = math.sqrt(n * p * (1 - p)) + 1e-9
        assert abs(counts[kind] - n * p) <= 5 * sd + 1, (kind, counts[kind], n * p)


def _pnull(sim, case, sp):
    return 1 - math.exp(-sim.numax(sp) * case["dt_s"])


def test_waiting_times_are_geometric(orc):
    # the first wait W of a particle loaded at step0 is Geo0(P_null):
    # P(W = k) = (1 - p)^k p; checked on the first few k and the mean
    sim, case, procs = beam_sim(orc, p_mtorr=10.0)
    p = _pnull(sim, case, 0)
    assert 0.05 < p < 0.5
    n = 40000
    ws = np.array([sim.first_wait(0, pid, 7) for pid in range(n)])
    for k in range(4):
        pk = (1 - p) ** k * p
        cnt = int((ws == k).sum())
        assert abs(cnt - n * pk) <= 5 * math.sqrt(n * pk * (1 - pk)), (k, cnt, n * pk)
    assert abs(ws.mean() - (1 - p) / p) <= 5 * math.sqrt((1 - p) / p ** 2 / n)


def test_candidacy_is_bernoulli_per_step(orc):
    # driving the rule over many steps: rate P_null, no correlation between
    # consecutive steps (memoryless), gaps between candidacies geometric
    sim, case, procs = beam_sim(orc, p_mtorr=10.0)
    p = _pnull(sim, case, 0)
    n, T = 3000, 40
    c = np.zeros((n, T), bool)
    for pid in range(n):
        w = sim.first_wait(0, pid, 100)
        for t in range(T):
            c[pid, t], w = sim.wait_step(0, pid, 100 + t, w)
    rate = c.mean()
    N = n * T
    assert abs(rate - p) <= 5 * math.sqrt(p * (1 - p) / N)
    both = (c[:, 1:] & c[:, :-1]).mean()
    assert abs(both - p * p) <= 5 * math.sqrt(p * p * (1 - p * p) / (n * (T - 1))) + 1e-4
    # every step is decided by the stream of that step alone: the same
    # particle run twice gives the same sequence
    w = sim.first_wait(0, 5, 100)
    seq = []
    for t in range(T):
        cand, w = sim.wait_step(0, 5, 100 + t, w)
        seq.append(cand)
    assert np.array_equal(np.array(seq), c[5])


def test_wait_counts_down_and_draws_only_at_zero(orc):
    sim, case, procs = beam_sim(orc, p_mtorr=10.0)
    # a positive wait decrements and never draws, whatever its size
    assert sim.wait_step(0, 3, 12, 5) == (False, 4)
    assert sim.wait_step(0, 3, 12, 1) == (False, 0)
    assert sim.wait_step(0, 3, 12, 10 ** 15) == (False, 10 ** 15 - 1)
    # zero: a candidate, the next wait drawn from the step's stream
    cand, w = sim.wait_step(0, 3, 12, 0)
    assert cand and w >= 0
    assert sim.wait_step(0, 3, 12, 0) == (True, w)


def test_waits_have_no_upper_limit(orc):
    # at a tiny P_null the geometric waits run to ~1/p and beyond: the wait
    # law holds far past any fixed word size (mean (1 - p)/p, and the tail
    # P(W >= k) = (1 - p)^k at k = 2^17 and 2^20)
    sim, case, procs = beam_sim(orc, p_mtorr=50.0)
    numax = sim.numax(0)
    p = 2.0e-6
    case = dict(case, dt_s=-math.log(1 - p) / numax)
    sps = W.to_oracle(W.c1(collisions=1, np_per_species=4))[1]
    sim = orc.Sim(case, sps, procs)
    assert abs(1 - math.exp(-sim.numax(0) * case["dt_s"]) - p) < 1e-12
    n = 30000
    ws = np.array([sim.first_wait(0, pid, 3) for pid in range(n)], dtype=np.float64)
    mean, sd = (1 - p) / p, math.sqrt(1 - p) / p
    assert abs(ws.mean() - mean) <= 5 * sd / math.sqrt(n), (ws.mean(), mean)
    for k in (2 ** 17, 2 ** 20):
        q = (1 - p) ** k
        cnt = int((ws >= k).sum())
        assert abs(cnt - n * q) <= 5 * math.sqrt(n * q * (1 - q)) + 1, (k, cnt, n * q)
    assert ws.max() > 2 ** 22


def test_numax_bounds_every_table_interval(orc):
    sim, case, procs = beam_sim(orc)
    numax = sim.numax(0)
    ng = case["gas_density_m3"]
    e = procs[0]["e0_eV"] + procs[0]["de_eV"] * np.arange(procs[0]["sigma"].size)
    tot = sum(p["sigma"] for p in procs if p["species"] == 0)
    nu = ng * tot * np.sqrt(2 * QE * e / W.M_E)
    assert numax >= nu.max() * (1 - 1e-14)
    # and it is attained at a table point (tight bound for a monotone product)
    assert numax <= nu.max() * (1 + 1e-12)


def _collect(orc, sim, sp, kind, v, n, step=3):
    out = []
    for pid in range(n):
        r, v1, ve, vi, over = sim.collide_one(sp, pid, step, v)
        if r == kind:
            out.append((np.array(v1), np.array(ve), np.array(vi)))
    return out


def test_excitation_removes_threshold_and_scatters_isotropically(orc):
    sim, case, procs = beam_sim(orc, p_mtorr=5000.0)
    eps = 60.0
    v0 = np.array([speed_of(eps, W.M_E), 0.0, 0.0])
    ev = _collect(orc, sim, 0, W.EXCITATION, v0, 60000)
    assert len(ev) > 500
    e1 = np.array([0.5 * W.M_E * (a[0] ** 2).sum() / QE for a in ev])
    np.testing.assert_allclose(e1, eps - 11.5, rtol=1e-12)
    d = np.array([a[0] / np.linalg.norm(a[0]) for a in ev])
    n = len(d)
    for k in range(3):
        assert abs(d[:, k].mean()) < 5 / math.sqrt(3 * n)
        assert abs((d[:, k] ** 2).mean() - 1 / 3) < 5 * math.sqrt(4 / 45 / n)


def test_elastic_energy_follows_recoil_law(orc):
    sim, case, procs = beam_sim(orc, p_mtorr=5000.0)
    eps = 5.0
    v0 = np.array([speed_of(eps, W.M_E) * 0.6, speed_of(eps, W.M_E) * 0.8, 0.0])
    ev = _collect(orc, sim, 0, W.ELASTIC, v0, 12000)
    assert len(ev) > 300
    for v1, _, _ in ev:
        cchi = (v1 @ v0) / (np.linalg.norm(v1) * np.linalg.norm(v0))
        e1 = 0.5 * W.M_E * (v1 ** 2).sum() / QE
        assert e1 == pytest.approx(eps * (1 - 2 * W.M_E / W.M_AR * (1 - cchi)), rel=1e-12)


def test_ionization_energy_sharing(orc):
    sim, case, procs = beam_sim(orc, p_mtorr=20000.0)
    eps = 80.0
    avail = eps - 15.8
    B = 10.0
    v0 = np.array([0.0, 0.0, speed_of(eps, W.M_E)])
    ev = _collect(orc, sim, 0, W.IONIZATION, v0, 60000)
    assert len(ev) > 800
    esc = np.array([0.5 * W.M_E * (a[0] ** 2).sum() / QE for a in ev])
    eej = np.array([0.5 * W.M_E * (a[1] ** 2).sum() / QE for a in ev])
    np.testing.assert_allclose(esc + eej, avail, rtol=1e-12)
    assert np.all(eej <= avail / 2 * (1 + 1e-12))
    # Kolmogorov-Smirnov against F(x) = atan(x/B)/atan(avail/(2B))
    x = np.sort(eej)
    F = np.arctan(x / B) / math.atan(avail / (2 * B))
    n = x.size
    D = max(np.max(np.arange(1, n + 1) / n - F), np.max(F - np.arange(n) / n))
    assert D < 1.63 / math.sqrt(n)  # alpha = 1%
    # new ions are thermal at the gas temperature
    vi = np.array([a[2] for a in ev])
    var = KB * 300.0 / W.M_AR
    assert abs(vi.var() / var - 1) < 5 * math.sqrt(2 / vi.size)


def test_charge_exchange_probability_and_neutral_velocity(orc):
    # a short ion table (to 2 eV) and a long dt make CX frequent enough to test
    wl = W.c1(collisions=1, np_per_species=4)
    case, sps, _ = W.to_oracle(wl)
    procs = W.argon_like_tables(e_max_eV=2.0, de_eV=0.001)
    case = dict(case, dt_s=1e-7)
    sim = orc.Sim(case, sps, procs)
    numax = sim.numax(1)
    dt, ng = case["dt_s"], case["gas_density_m3"]
    assert numax == pytest.approx(ng * 5e-19 * speed_of(2.0, W.M_AR), rel=1e-12)
    # ion at rest: relative speed is the neutral speed, mean sqrt(8kT/(pi M))
    gbar = math.sqrt(8 * KB * 300.0 / (math.pi * W.M_AR))
    n = 40000
    hits = []
    for pid in range(n):
        r, v1, ve, vi, over = sim.collide_one(1, pid, 5, [0.0, 0.0, 0.0])
        if r == W.CHARGE_EXCHANGE:
            hits.append(v1)
    p = ng * 5e-19 * gbar / numax
    sd = math.sqrt(n * p * (1 - p))
    assert abs(len(hits) - n * p) < 5 * sd
    # after CX the ion carries the neutral's velocity, drawn with probability
    # proportional to g: for an ion at rest the speed law is g * Maxwell(g)
    # (a chi law with 4 degrees of freedom), mean E[g^2]/E[g] = 3 kT/M / gbar
    h = np.array(hits)
    sp = np.linalg.norm(h, axis=1)
    expect = 3 * KB * 300.0 / W.M_AR / gbar
    assert abs(sp.mean() / expect - 1) < 5 * 0.37 / math.sqrt(len(h))
    for k in range(3):
        assert abs(h[:, k].mean()) < 5 * sp.std() / math.sqrt(len(h))


def test_over_table_energies_are_flagged(orc):
    sim, case, procs = beam_sim(orc, p_mtorr=5000.0)
    v = speed_of(1500.0, W.M_E)
    flagged = 0
    for pid in range(500):
        r, v1, ve, vi, over = sim.collide_one(0, pid, 1, [v, 0, 0])
        flagged += over
    assert flagged == 500


def test_children_draw_geometric_first_waits(orc):
    # ionization children take their first trial at the next step with a
    # Geo0(P_null) wait of their own: mean (1 - p)/p over many children
    sim, case, procs = beam_sim(orc, p_mtorr=50.0)
    numax = sim.numax(0)
    case = dict(case, dt_s=-math.log(1 - 0.3) / numax)      # P_null = 0.3
    n = 20000
    v80 = speed_of(80.0, W.M_E)
    e = dict(q=-QE, m=W.M_E, w=1e9, xi=np.full(n, 32.5), vx=np.zeros(n), vy=np.zeros(n),
             vz=np.full(n, v80), id=np.arange(n, dtype=np.uint64), abar=None)
    i = dict(q=QE, m=W.M_AR, w=1e9, xi=np.zeros(0), vx=np.zeros(0), vy=np.zeros(0),
             vz=np.zeros(0), id=np.zeros(0, dtype=np.uint64), abar=None)
    sim = orc.Sim(dict(case, rf_volts=0.0), [e, i], procs)
    p = 1 - math.exp(-sim.numax(0) * case["dt_s"])
    assert abs(p - 0.3) < 1e-9
    sim.step(1)
    out = sim.species(0)
    kids = out["wait"][out["id"] >= np.uint64(1 << 63)]
    assert kids.size > 150
    mean, sd = (1 - p) / p, math.sqrt(1 - p) / p
    assert abs(kids.mean() - mean) <= 5 * sd / math.sqrt(kids.size), (kids.mean(), mean)
    pz = (kids == 0).mean()
    assert abs(pz - p) <= 5 * math.sqrt(p * (1 - p) / kids.size)
