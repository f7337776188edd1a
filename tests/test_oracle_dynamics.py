"""Pins of the oracle's particle dynamics against closed forms.

Cold plasma in the EC scheme: when every particle of cell j carries the same
displacement delta_j and no particle crosses a cell edge, linear weighting
(Eq. 2) moves exactly q delta_j / dx of charge from node j to node j+1, so
Gauss's law telescopes and the own-cell field (Eq. 3 with S_0) is exactly
-m omega_p^2 delta_j / q for every wavelength.  Each cell is then a harmonic
oscillator at omega_p and

  * leap-frog gives delta_n = A cos(n theta), cos theta = 1 - (omega_p dt)^2 / 2;
  * the D1 direct-implicit push gives the linear recurrence of
    (x_n, v_{n-1/2}, abar_{n-1}) with x_{n+1} = x~ / (1 + omega_p^2 dt^2 / 2).

A wrong factor anywhere in deposit, solve, gather, push, susceptibility or the
D1 update changes the frequency or the recurrence and fails these tests."""
import math

import numpy as np
import pytest

E = 1.602176634e-19
ME = 9.1093837015e-31
EPS0 = 8.8541878128e-12


def cold_setup(N=16, ppc=8, mode=3, A=0.1, wdt=0.2, scheme=0, n0=1e15):
    wp = math.sqrt(n0 * E * E / (EPS0 * ME))
    dt = wdt / wp
    dx = 1e-3
    L = N * dx
    w = n0 * dx / ppc
    offs = 0.25 + 0.5 * (np.arange(ppc) + 0.5) / ppc
    j = np.repeat(np.arange(N), ppc)
    base = j + np.tile(offs, N)
    amp = A * np.sin(2 * np.pi * mode * j / N)          # cells
    theta_c = 1 - 0.5 * wdt ** 2
    v = amp * (1 - theta_c) * dx / dt                     # v_{-1/2} for a pure cosine
    n = N * ppc
    sp_e = dict(q=-E, m=ME, w=w, xi=base + amp, vx=v, vy=np.zeros(n), vz=np.zeros(n),
                abar=None, id=np.arange(n, dtype=np.uint64))
    sp_i = dict(q=E, m=40 * 1.66053906660e-27, w=w, xi=np.zeros(0), vx=np.zeros(0),
                vy=np.zeros(0), vz=np.zeros(0), abar=None, id=np.zeros(0, np.uint64))
    case = dict(n_cells=N, gap_m=L, bc=1, scheme=scheme, gather=0, collisions=0, dt_s=dt,
                background_rho=n0 * E)
    return case, [sp_e, sp_i], base, amp, dt, dx, wp


@pytest.mark.parametrize("mode,wdt", [(1, 0.2), (3, 0.5), (7, 1.2), (5, 1.9)])
def test_ec_cold_plasma_oscillates_at_exactly_omega_p(orc, mode, wdt):
    case, sps, base, amp, dt, dx, wp = cold_setup(mode=mode, wdt=wdt)
    sim = orc.Sim(case, sps, [])
    theta = math.acos(1 - 0.5 * wdt ** 2)
    order = np.argsort(sps[0]["id"])
    for n in range(1, 101):
        sim.step(1)
        st = sim.species(0)
        xi = st["xi"][np.argsort(st["id"])][order]
        np.testing.assert_allclose(xi - base, amp * math.cos(n * theta), rtol=0, atol=2e-11)
    # the field of the last solve is -m wp^2 delta / q (delta of step 99)
    f = sim.fields()
    d = amp[:: 8] * math.cos(99 * theta) * dx
    np.testing.assert_allclose(f["E"], ME * wp ** 2 * d / E, rtol=0,
                               atol=1e-9 * abs(ME * wp ** 2 * amp.max() * dx / E))


def d1_reference(x0, v0, wdt_s, wp, dt, nsteps):
    """Predicted positions x~_{n+1} of the D1 recurrence for x'' = -wp^2 x."""
    x, v, ab = x0, v0, 0.0
    out = []
    xt = x + dt * (v + 0.5 * dt * ab)           # start-up prediction x~_1
    for _ in range(nsteps):
        xn = xt / (1 + 0.5 * wp ** 2 * dt ** 2)  # corrected x_{n+1}
        a = -wp ** 2 * xn
        vt = v + 0.5 * dt * ab
        v = vt + 0.5 * dt * a                    # v_{n+1/2}
        ab = 0.5 * (ab + a)
        x = xn
        xt = x + dt * (v + 0.5 * dt * ab)        # next prediction
        out.append(xt)
    return np.array(out)


@pytest.mark.parametrize("wdt", [0.2, 1.0, 5.0])
def test_d1_cold_plasma_follows_recurrence(orc, wdt):
    case, sps, base, amp, dt, dx, wp = cold_setup(mode=2, wdt=wdt, A=0.05, scheme=1)
    sps[0]["vx"] = np.zeros_like(sps[0]["vx"])   # start at rest, displaced
    sim = orc.Sim(case, sps, [])
    nsteps = 60
    # per unit amplitude the sequence scales linearly
    ref = d1_reference(1.0, 0.0, wdt, wp, dt, nsteps)
    order = np.argsort(sps[0]["id"])
    for n in range(nsteps):
        sim.step(1)
        st = sim.species(0)
        xi = st["xi"][np.argsort(st["id"])][order]
        np.testing.assert_allclose(xi - base, amp * ref[n], rtol=0, atol=1e-11)
    # damping per step equals the dominant eigenvalue modulus of the D1 map
    M = np.zeros((3, 3))
    for k in range(3):
        e = np.zeros(3); e[k] = 1.0
        x, v, ab = e
        xt = x + dt * (v + 0.5 * dt * ab)
        xn = xt / (1 + 0.5 * wp ** 2 * dt ** 2)
        a = -wp ** 2 * xn
        vn = v + 0.5 * dt * ab + 0.5 * dt * a
        M[:, k] = [xn, vn, 0.5 * (ab + a)]
    lam = np.abs(np.linalg.eigvals(M)).max()
    if wdt >= 1.0:
        # D1 damps oscillations it cannot resolve; the oracle's particles decay too
        assert lam < 1.0
        st = sim.species(0)
        assert np.abs(st["xi"][np.argsort(st["id"])][order] - base).max() < 0.5 * 0.05


def test_implicit_field_equals_explicit_field_at_corrected_positions(orc):
    # the susceptibility is exact while the correction stays inside the cell:
    # E_{n+1} of the implicit solve must equal the plain Poisson field of the
    # charge deposited at the corrected positions x_{n+1}
    rng = np.random.default_rng(9)
    N, dx = 24, 2e-4
    L = N * dx
    n = 400
    n0 = 5e15
    w = n0 * L / n
    wp = math.sqrt(n0 * E * E / (EPS0 * ME))
    dt = 0.3 / wp
    cell = rng.integers(0, N, n)
    off = 0.3 + 0.4 * rng.random(n)
    sp_e = dict(q=-E, m=ME, w=w, xi=cell + off, vx=np.zeros(n), vy=np.zeros(n),
                vz=np.zeros(n), abar=None, id=np.arange(n, dtype=np.uint64))
    mi = 40 * 1.66053906660e-27
    ci = rng.integers(0, N, n)
    sp_i = dict(q=E, m=mi, w=w, xi=ci + 0.5, vx=np.zeros(n), vy=np.zeros(n), vz=np.zeros(n),
                abar=None, id=np.arange(n, dtype=np.uint64))
    case = dict(n_cells=N, gap_m=L, bc=0, scheme=1, gather=0, collisions=0, dt_s=dt,
                rf_volts=3.0, rf_freq_hz=1e7)
    imp = orc.Sim(case, [sp_e, sp_i], [], startup=False)
    before = [imp.species(k) for k in range(2)]
    imp.step(1)
    fi = imp.fields()
    moved = []
    for k, sp in enumerate((sp_e, sp_i)):
        after = imp.species(k)
        # undo the prediction: x_{n+1} = x~_{n+2} - dt v~' / dx
        x1 = after["xi"] - after["vx"] * dt / dx
        o_b = np.argsort(before[k]["id"]); o_a = np.argsort(after["id"])
        assert np.all(np.floor(x1[o_a]) == np.floor(before[k]["xi"][o_b]))  # no crossing
        assert np.abs(x1[o_a] - before[k]["xi"][o_b]).max() > 0
        moved.append(dict(sp, xi=x1, id=after["id"], vx=np.zeros(x1.size),
                          vy=np.zeros(x1.size), vz=np.zeros(x1.size)))
    ex = orc.Sim(dict(case, scheme=0, step0=1), moved, [])
    ex.compute_fields()
    fe = ex.fields()
    np.testing.assert_allclose(fi["E"], fe["E"], rtol=0, atol=1e-9 * abs(fe["E"]).max())


def _implicit_residual(orc, wdt, gather=2, anywhere=False):
    """One implicit step of electrons and ions sitting at cell centres (where
    the m = 2 susceptibility operator is diagonal) or, with anywhere, at
    random positions: the largest difference between the implicit field and
    the plain field of the charge at the corrected positions, relative to
    that field, and the same difference for the field of the uncorrected
    positions."""
    rng = np.random.default_rng(9)
    N, dx = 24, 2e-4
    L = N * dx
    n, n0 = 400, 5e15
    w = n0 * L / n
    wp = math.sqrt(n0 * E * E / (EPS0 * ME))
    dt = wdt / wp
    mi = 40 * 1.66053906660e-27
    z = np.zeros(n)
    def place():
        if anywhere:
            return rng.uniform(0.02, N - 0.02, n)
        return rng.integers(0, N, n) + 0.5
    sps = [dict(q=-E, m=ME, w=w, xi=place(), vx=z, vy=z, vz=z, abar=None,
                id=np.arange(n, dtype=np.uint64)),
           dict(q=E, m=mi, w=w, xi=place(), vx=z, vy=z, vz=z, abar=None,
                id=np.arange(n, dtype=np.uint64))]
    case = dict(n_cells=N, gap_m=L, bc=0, scheme=1, gather=gather, collisions=0, dt_s=dt,
                rf_volts=3.0, rf_freq_hz=1e7)
    imp = orc.Sim(case, sps, [], startup=False)
    imp.step(1)
    moved = []
    for k in range(2):
        after = imp.species(k)
        x1 = after["xi"] - after["vx"] * dt / dx     # x_{n+1} from x~_{n+2}
        moved.append(dict(sps[k], xi=x1, id=after["id"], vx=np.zeros(x1.size),
                          vy=np.zeros(x1.size), vz=np.zeros(x1.size)))
    fields = []
    for sp in (moved, sps):
        ex = orc.Sim(dict(case, scheme=0, step0=1), sp, [])
        ex.compute_fields()
        fields.append(ex.fields()["E"])
    Ei, (E1, E0) = imp.fields()["E"], fields
    scale = np.abs(E1).max()
    return np.abs(Ei - E1).max() / scale, np.abs(E0 - E1).max() / scale


def test_ec2_implicit_field_is_the_corrected_field_to_second_order(orc):
    # The m = 2 deposit is quadratic in a particle's position, so the
    # susceptibility (its linearisation) is exact to first order only: the
    # implicit field misses the field of the corrected positions by O(d^2),
    # d ~ dt^2, a residual that falls 16x per halving of dt.  Without the
    # susceptibility, or with a wrong factor, it falls 4x.
    r = [_implicit_residual(orc, wdt) for wdt in (0.2, 0.1, 0.05)]
    for (a, a0), (b, b0) in zip(r, r[1:]):
        assert 3.5 < a0 / b0 < 4.5          # the correction itself is O(dt^2)
        assert a / b > 12.0
    assert r[-1][0] < 1e-3 * r[-1][1]


def test_ec2_implicit_field_is_the_corrected_field_anywhere(orc):
    # Particles at random positions couple neighbouring centres: with the
    # tridiagonal operator the implicit field still misses the field of the
    # corrected positions by O(d^2) only (16x per halving of dt); its
    # diagonal (row-sum) approximation misses it by O(d) there.
    r = [_implicit_residual(orc, wdt, anywhere=True) for wdt in (0.2, 0.1, 0.05)]
    for (a, a0), (b, b0) in zip(r, r[1:]):
        assert 3.5 < a0 / b0 < 4.5
        assert a / b > 12.0, (a, b)
    assert r[-1][0] < 1e-3 * r[-1][1]


def test_ec2_implicit_damps_the_oscillation_explicit_cannot_follow(orc):
    # omega_p dt = 2.5: leap-frog is unstable (omega_p dt > 2) and the energy
    # of the cold plasma grows; the D1 push with the m = 2 susceptibility
    # damps it.  A susceptibility of the wrong sign or size fails this.
    energy = {}
    for scheme in (0, 1):
        case, sps, base, amp, dt, dx, wp = cold_setup(mode=2, wdt=2.5, A=0.05, scheme=scheme)
        case["gather"] = 2
        sps[0]["vx"] = np.zeros_like(sps[0]["vx"])
        sim = orc.Sim(case, sps, [])
        hist = []
        for _ in range(100):
            sim.step(1)
            L = sim.ledger()
            hist.append(L["WE"] + L["K_after"][0])
        energy[scheme] = hist
    assert energy[0][-1] > 100 * energy[0][0]
    assert energy[1][-1] < 0.01 * energy[1][0]
