"""Pins of the oracle on a nonuniform grid (cells finer in the sheaths, the
multi-scale remedy of the conclusions): positions stay logical (cell index +
offset); a move is made in physical space; node charges are per unit area.

* the solve: uniform charge gives the closed-form quadratic potential at the
  nodes; with a susceptibility the discrete Gauss law and the potential
  difference hold in first-integral form;
* the mover: the physical displacement equals v dt across cells of different
  widths (physical positions rebuilt here from the widths);
* cold plasma: with the particle count of every cell proportional to its
  width (uniform physical density) and a displacement uniform in each cell,
  the EC scheme oscillates at exactly omega_p (leap-frog dispersion) and the
  D1 scheme follows its closed recurrence, which fixes the widths in the
  deposit, solve, gather, susceptibility and mover;
* equal widths reproduce the uniform path."""
import math

import numpy as np
import pytest

E = 1.602176634e-19
ME = 9.1093837015e-31
EPS0 = 8.8541878128e-12

MULT = np.array([1, 1, 2, 3, 5, 5, 3, 2, 1, 1])   # widths in units of the finest cell


def test_solve_uniform_charge_closed_form(orc):
    rng = np.random.default_rng(1)
    w = rng.uniform(0.2e-3, 1.5e-3, 17)
    xn = np.concatenate([[0.0], np.cumsum(w)])
    L = xn[-1]
    rho, V0, VN = 3e-4, 40.0, -5.0
    vol = np.concatenate([[w[0]], 0.5 * (w[:-1] + w[1:]), [w[-1]]])
    phi, Ef = orc.solve_dirichlet_nu(w, rho * vol, V0, VN)
    exact = V0 + (VN - V0 + rho * L * L / (2 * EPS0)) * xn / L - rho * xn ** 2 / (2 * EPS0)
    scale = np.abs(exact).max()
    np.testing.assert_allclose(phi, exact, rtol=0, atol=1e-12 * scale)
    np.testing.assert_allclose(Ef, (exact[:-1] - exact[1:]) / w, rtol=1e-9)


def test_solve_satisfies_gauss_law_with_susceptibility(orc):
    rng = np.random.default_rng(2)
    N = 23
    w = rng.uniform(0.1e-3, 2e-3, N)
    sigma = rng.normal(size=N + 1) * 1e-6
    chi = rng.uniform(0.0, 30.0, N)
    phi, Ef = orc.solve_dirichlet_nu(w, sigma, 12.0, 3.0, chi=chi)
    D = EPS0 * (1.0 + chi) * Ef
    np.testing.assert_allclose(D[1:] - D[:-1], sigma[1:N], rtol=0,
                               atol=1e-9 * np.abs(sigma).max())
    assert abs((Ef * w).sum() - (12.0 - 3.0)) < 1e-9 * 12.0
    np.testing.assert_allclose(phi[:-1] - phi[1:], Ef * w, rtol=1e-10, atol=1e-12)


def _two_species(xe, ve, we, m=ME):
    z = np.zeros(xe.size)
    return [dict(q=-E, m=m, w=we, xi=xe, vx=ve, vy=z, vz=z, abar=None,
                 id=np.arange(xe.size, dtype=np.uint64)),
            dict(q=E, m=40 * 1.66053906660e-27, w=we, xi=np.zeros(0), vx=np.zeros(0),
                 vy=np.zeros(0), vz=np.zeros(0), abar=None, id=np.zeros(0, np.uint64))]


def test_mover_keeps_the_physical_displacement(orc):
    w = 1e-4 * MULT
    edges = np.concatenate([[0.0], np.cumsum(w)])
    dt = 1e-10
    rng = np.random.default_rng(3)
    n = 200
    xi = rng.uniform(0.0, MULT.size, n)
    v = rng.uniform(-3.0, 3.0, n) * w.max() / dt      # up to 3 of the widest cells
    case = dict(n_cells=MULT.size, gap_m=edges[-1], bc=0, scheme=0, gather=0, collisions=0,
                dt_s=dt, cell_dx=w)
    sim = orc.Sim(case, _two_species(xi, v, 1e-30), [], startup=False)
    sim.step(1)
    st = sim.species(0)
    X0 = edges[np.floor(xi).astype(int)] + (xi - np.floor(xi)) * w[np.floor(xi).astype(int)]
    X1_want = X0 + v * dt
    inside = (X1_want > 0) & (X1_want < edges[-1])
    order = np.argsort(st["id"])
    x1 = st["xi"][order]
    c1 = np.floor(x1).astype(int)
    X1 = edges[c1] + (x1 - c1) * w[c1]
    assert x1.size == inside.sum()                   # the others were absorbed
    np.testing.assert_allclose(X1, X1_want[inside], rtol=0, atol=1e-12 * edges[-1])


def cold_nonuniform(wdt, scheme, A=0.06, ppc=6, n0=1e15):
    """Electrons at uniform physical density n0 on a symmetric nonuniform
    grid over a neutralising background; cell c holds MULT_c ppc electrons in
    the middle half of the cell and is displaced by A s_c of the finest cell,
    s antisymmetric about the centre (no mean displacement)."""
    b = 1e-4
    w = b * MULT
    N = MULT.size
    wp = math.sqrt(n0 * E * E / (EPS0 * ME))
    dt = wdt / wp
    weight = n0 * b / ppc
    cells, offs = [], []
    for c, m in enumerate(MULT):
        k = m * ppc
        cells.append(np.full(k, c))
        offs.append(0.25 + 0.5 * (np.arange(k) + 0.5) / k)
    cell = np.concatenate(cells)
    off = np.concatenate(offs)
    s = np.sin(2 * np.pi * (np.arange(N) + 0.5) / N)       # antisymmetric, sum_c s_c w_c = 0
    delta = A * b * s[cell]                                  # physical displacement
    xi = cell + off + delta / w[cell]
    theta_c = 1 - 0.5 * wdt ** 2
    v = delta * (1 - theta_c) / dt if scheme == 0 else np.zeros(cell.size)
    case = dict(n_cells=N, gap_m=w.sum(), bc=0, scheme=scheme, gather=0, collisions=0,
                dt_s=dt, background_rho=n0 * E, cell_dx=w)
    return case, _two_species(xi, v, weight), cell, off, delta, w, dt, wp


@pytest.mark.parametrize("wdt", [0.3, 1.2, 1.9])
def test_ec_cold_plasma_oscillates_at_exactly_omega_p(orc, wdt):
    case, sps, cell, off, delta, w, dt, wp = cold_nonuniform(wdt, 0)
    sim = orc.Sim(case, sps, [])
    theta = math.acos(1 - 0.5 * wdt ** 2)
    for n in range(1, 81):
        sim.step(1)
        st = sim.species(0)
        x = st["xi"][np.argsort(st["id"])]
        got = (x - cell - off) * w[cell]                 # physical displacement
        np.testing.assert_allclose(got, delta * math.cos(n * theta), rtol=0,
                                   atol=1e-10 * np.abs(delta).max())


@pytest.mark.parametrize("wdt", [0.5, 4.0])
def test_d1_cold_plasma_follows_recurrence(orc, wdt):
    case, sps, cell, off, delta, w, dt, wp = cold_nonuniform(wdt, 1)
    sim = orc.Sim(case, sps, [])
    # the D1 map of x'' = -wp^2 x from rest, per unit displacement
    x, v, ab = 1.0, 0.0, 0.0
    xt = x + dt * v
    ref = []
    for _ in range(40):
        xn = xt / (1 + 0.5 * wp ** 2 * dt ** 2)
        a = -wp ** 2 * xn
        v = v + 0.5 * dt * ab + 0.5 * dt * a
        ab = 0.5 * (ab + a)
        xt = xn + dt * (v + 0.5 * dt * ab)
        ref.append(xt)
    for n in range(40):
        sim.step(1)
        st = sim.species(0)
        x1 = st["xi"][np.argsort(st["id"])]
        got = (x1 - cell - off) * w[cell]
        np.testing.assert_allclose(got, delta * ref[n], rtol=0, atol=1e-10 * np.abs(delta).max())


@pytest.mark.parametrize("scheme,gather", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_equal_widths_reproduce_the_uniform_grid(orc, scheme, gather):
    import workloads as W
    wl = W.c1(collisions=1, np_per_species=3000, scheme=scheme)
    wl["case"]["gather"] = gather
    case, sps, procs = W.to_oracle(wl)
    N = case["n_cells"]
    a = orc.Sim(case, sps, procs)
    b = orc.Sim(dict(case, cell_dx=np.full(N, case["gap_m"] / N)), sps, procs)
    a.step(30)
    b.step(30)
    for s in range(2):
        sa, sb = a.species(s), b.species(s)
        assert np.array_equal(sa["id"], sb["id"])
        np.testing.assert_allclose(sb["xi"], sa["xi"], rtol=0, atol=1e-9)
        np.testing.assert_allclose(sb["vx"], sa["vx"], rtol=1e-9, atol=1e-6)
    fa, fb = a.fields(), b.fields()
    np.testing.assert_allclose(fb["E"], fa["E"], rtol=0, atol=1e-9 * np.abs(fa["E"]).max())


def test_rejects_what_the_grid_does_not_support(orc):
    w = np.full(8, 1e-3)
    base = dict(n_cells=8, gap_m=8e-3, bc=0, scheme=0, gather=0, collisions=0, dt_s=1e-11)
    sps = _two_species(np.array([0.5]), np.zeros(1), 1.0)
    for bad in (dict(bc=1), dict(gap_m=9e-3)):
        with pytest.raises(ValueError):
            orc.Sim(dict(base, cell_dx=w, **bad), sps, [])
    with pytest.raises(ValueError):
        orc.Sim(dict(base, cell_dx=np.concatenate([w[:-1], [0.0]])), sps, [])


def test_ec_energy_error_shrinks_like_dt_squared(orc):
    # field energy sum 1/2 eps0 E^2 w_j plus kinetic energy (mean of the two
    # half steps) is conserved up to the leap-frog error
    errs = []
    for wdt in (0.3, 0.15, 0.075):
        case, sps, cell, off, delta, w, dt, wp = cold_nonuniform(wdt, 0)
        sim = orc.Sim(case, sps, [])
        tot = []
        for _ in range(int(round(20 / wdt))):
            sim.step(1)
            L = sim.ledger()
            tot.append(0.5 * (L["K_before"][0] + L["K_after"][0]) + L["WE"])
        tot = np.array(tot)
        errs.append(np.abs(tot / tot[0] - 1).max())
    for a, b in zip(errs, errs[1:]):
        assert 3.0 <= a / b <= 5.5, errs


def test_mc_gather_is_the_centred_potential_difference(orc):
    # the nodal field of the momentum-conserving gather on a nonuniform grid:
    # (phi_{g-1} - phi_{g+1}) / (x_{g+1} - x_{g-1}) from the node positions,
    # the electrode nodes taking their only cell's field; linear in between
    rng = np.random.default_rng(5)
    w = 1e-4 * MULT
    N = w.size
    xn = np.concatenate([[0.0], np.cumsum(w)])
    phi = rng.normal(size=N + 1)
    Ef = (phi[:-1] - phi[1:]) / w
    En = np.empty(N + 1)
    En[1:N] = (phi[:N - 1] - phi[2:]) / (xn[2:] - xn[:N - 1])
    En[0], En[N] = Ef[0], Ef[-1]
    for xi in np.concatenate([rng.uniform(0, N, 50), [0.0, 0.5, N - 1e-9, 3.0]]):
        j = min(int(np.floor(xi)), N - 1)
        f = xi - j
        ref = (1 - f) * En[j] + f * En[j + 1]
        assert abs(orc.gather_mc_nu(w, Ef, xi) - ref) < 1e-12 * np.abs(En).max()


def test_mc_susceptibility_of_a_uniform_plasma_is_the_same_on_every_grid(orc):
    # electrons at uniform physical density (each cell's count proportional
    # to its width, evenly spread): the node susceptibility of the linear
    # weights over the node volumes is beta (omega_p dt)^2 in every cell away
    # from the electrodes, whatever the widths
    case, sps, cell, off, delta, w, dt, wp = cold_nonuniform(0.7, 1)
    N = w.size
    k = MULT * 6
    cells = np.repeat(np.arange(N), k)
    offs = np.concatenate([(np.arange(m) + 0.5) / m for m in k])
    sps[0] = dict(sps[0], xi=cells + offs, vx=np.zeros(cells.size), vy=np.zeros(cells.size),
                  vz=np.zeros(cells.size), id=np.arange(cells.size, dtype=np.uint64))
    sim = orc.Sim(dict(case, gather=1), sps, [], startup=False)
    sim.compute_fields()
    chi = sim.fields()["chi"]
    np.testing.assert_allclose(chi[1:-1], 0.5 * (wp * dt) ** 2, rtol=1e-9)


def test_ec2_gather_is_minus_the_physical_gradient_of_the_deposit_energy(orc):
    # the energy-conserving pair on a nonuniform grid: with E_{j+1/2} =
    # (phi_j - phi_{j+1}) / w_j, the gathered field at a particle equals
    # -d/dX sum_g phi_g w_g(xi(X)), X the physical position (finite
    # differences of the quadratic deposit's own weights, folded at the
    # electrodes)
    rng = np.random.default_rng(8)
    w = 1e-4 * MULT
    N = w.size
    edges = np.concatenate([[0.0], np.cumsum(w)])
    phi = rng.normal(size=N + 1)
    Ef = (phi[:-1] - phi[1:]) / w

    def energy(X):
        c = min(int(np.searchsorted(edges, X, side="right") - 1), N - 1)
        xi = c + (X - edges[c]) / w[c]
        return (orc.deposit_quadratic(N, [xi]) * phi).sum()
    for xi in np.concatenate([rng.uniform(0.05, N - 0.05, 60), [0.3, N - 0.3]]):
        c = int(np.floor(xi))
        o = xi - c
        if min(o, 1 - o) < 1e-3 or abs(o - 0.5) < 1e-3:
            continue   # keep the difference inside one piece of the weights
        X = edges[c] + o * w[c]
        h = 1e-6 * w[c]
        grad = (energy(X + h) - energy(X - h)) / (2 * h)
        assert abs(orc.gather_ec2_nu(w, Ef, xi) + grad) < 1e-5 * np.abs(Ef).max()


def test_ec2_energy_error_shrinks_like_dt_squared_on_a_nonuniform_grid(orc):
    errs = []
    for wdt in (0.3, 0.15, 0.075):
        case, sps, cell, off, delta, w, dt, wp = cold_nonuniform(wdt, 0)
        sim = orc.Sim(dict(case, gather=2), sps, [])
        tot = []
        for _ in range(int(round(20 / wdt))):
            sim.step(1)
            L = sim.ledger()
            tot.append(0.5 * (L["K_before"][0] + L["K_after"][0]) + L["WE"])
        tot = np.array(tot)
        errs.append(np.abs(tot / tot[0] - 1).max())
    for a, b in zip(errs, errs[1:]):
        assert 3.0 <= a / b <= 5.5, errs


# ---------------------------------------------------------------------------
# m = 2 implicit on a nonuniform grid: the operator of F_j = r_j E_j
# ---------------------------------------------------------------------------
def _tri(d, o, F):
    y = d * F
    y[:-1] += o[:-1] * F[1:]
    y[1:] += o[:-1] * F[:-1]
    return y


def test_ec2_nu_operator_is_the_linear_response_of_the_deposit(orc):
    # Move every particle by eps times its m = 2 gather (physical units) and
    # the deposit changes node g by the flux in from centre g - 1 minus the
    # flux out through centre g; to first order the flux through centre h,
    # in logical units, is eps (M (r E))_h / dx, with M the operator of
    # orc_chi_operator_ec2_nu (products of S_1 weights over r_c^2).
    w = 1e-4 * MULT
    N = w.size
    dx = w.sum() / N
    r = w / dx
    rng = np.random.default_rng(31)
    xi = rng.uniform(0.0, N, 300)
    xi[:4] = [0.05, 0.45, N - 0.3, N - 0.02]
    E = rng.normal(size=N)
    d, o = orc.chi_operator_ec2_nu(w, xi)
    flux = _tri(d, o, r * E) / dx
    cell = np.minimum(np.floor(xi).astype(int), N - 1)
    g = np.array([orc.gather_ec2_nu(w, E, x) for x in xi])
    for eps in (2e-9, 1e-9):
        moved = xi + eps * g / w[cell]
        dq = (orc.deposit_quadratic(N, moved) - orc.deposit_quadratic(N, xi)) / eps
        expect = np.concatenate([[0.0], flux]) - np.concatenate([flux, [0.0]])
        assert np.abs(dq - expect).max() < 2e-3 * np.abs(flux).max(), eps


def test_ec2_nu_solve_without_couplings_is_the_nonuniform_solve(orc):
    # (1/r + xd) F = D / eps0 gives E = D / (eps0 (1 + r xd)): the potential-
    # form nonuniform solve with chi = r xd
    w = 1e-4 * MULT
    N = w.size
    dx = w.sum() / N
    rng = np.random.default_rng(8)
    sigma = rng.normal(size=N + 1) * 1e-9
    xd = rng.uniform(0.0, 2.0, N)
    phi_t, E_t = orc.solve_chi_tridiag_nu(w, sigma, xd, np.zeros(N), 1.3)
    phi, Ef = orc.solve_dirichlet_nu(w, sigma, 1.3, 0.0, chi=xd * w / dx)
    np.testing.assert_allclose(E_t, Ef, rtol=1e-10, atol=1e-10 * np.abs(Ef).max())
    np.testing.assert_allclose(phi_t, phi, rtol=1e-10, atol=1e-10 * np.abs(phi).max())


def test_ec2_nu_solve_satisfies_gauss_and_the_potential(orc):
    w = 1e-4 * MULT
    N = w.size
    dx = w.sum() / N
    r = w / dx
    rng = np.random.default_rng(12)
    d, o = orc.chi_operator_ec2_nu(w, rng.uniform(0.0, N, 60))
    xd, xo = 0.4 * d, 0.4 * o
    sigma = rng.normal(size=N + 1) * 1e-9
    V = 2.0
    phi, E = orc.solve_chi_tridiag_nu(w, sigma, xd, xo, V)
    D = EPS0 * (E + _tri(xd, xo, r * E))
    assert np.abs((D[1:] - D[:-1]) - sigma[1:N]).max() < 1e-10 * np.abs(sigma).max()
    assert abs((E * w).sum() - V) < 1e-12
    np.testing.assert_allclose(phi[:-1] - phi[1:], E * w, rtol=1e-12, atol=1e-20)


def _nu_implicit_residual(orc, wdt):
    """One m = 2 implicit step of electrons and ions at random positions on
    the nonuniform grid: the largest difference between the implicit field
    and the plain field of the charge at the corrected positions (relative),
    and the same for the uncorrected positions."""
    rng = np.random.default_rng(21)
    w = 1e-4 * MULT
    N = w.size
    edge = np.concatenate([[0.0], np.cumsum(w)])
    n, n0 = 600, 5e15
    weight = n0 * w.sum() / n
    wp = math.sqrt(n0 * E * E / (EPS0 * ME))
    dt = wdt / wp
    mi = 40 * 1.66053906660e-27
    z = np.zeros(n)
    sps = [dict(q=-E, m=ME, w=weight, xi=rng.uniform(0.02, N - 0.02, n), vx=z, vy=z, vz=z,
                abar=None, id=np.arange(n, dtype=np.uint64)),
           dict(q=E, m=mi, w=weight, xi=rng.uniform(0.02, N - 0.02, n), vx=z, vy=z, vz=z,
                abar=None, id=np.arange(n, dtype=np.uint64))]
    case = dict(n_cells=N, gap_m=w.sum(), bc=0, scheme=1, gather=2, collisions=0, dt_s=dt,
                rf_volts=3.0, rf_freq_hz=1e7, cell_dx=w)
    imp = orc.Sim(case, sps, [], startup=False)
    imp.step(1)

    def phys(x):
        c = np.minimum(np.floor(x).astype(int), N - 1)
        return edge[c] + (x - c) * w[c]

    def logical(X):
        c = np.clip(np.searchsorted(edge, X, side="right") - 1, 0, N - 1)
        return c + (X - edge[c]) / w[c]

    moved = []
    for k in range(2):
        after = imp.species(k)
        X1 = phys(after["xi"]) - after["vx"] * dt      # x_{n+1} from x~_{n+2}
        moved.append(dict(sps[k], xi=logical(X1), id=after["id"], vx=np.zeros(X1.size),
                          vy=np.zeros(X1.size), vz=np.zeros(X1.size)))
    fields = []
    for sp in (moved, sps):
        ex = orc.Sim(dict(case, scheme=0, step0=1), sp, [])
        ex.compute_fields()
        fields.append(ex.fields()["E"])
    Ei, (E1, E0) = imp.fields()["E"], fields
    scale = np.abs(E1).max()
    return np.abs(Ei - E1).max() / scale, np.abs(E0 - E1).max() / scale


def test_ec2_nu_implicit_field_is_the_corrected_field_to_second_order(orc):
    # the operator linearises the quadratic deposit exactly to first order in
    # the D1 displacement, on every width: the residual falls 16x per halving
    # of dt (the correction itself 4x)
    r = [_nu_implicit_residual(orc, wdt) for wdt in (0.2, 0.1, 0.05)]
    for (a, a0), (b, b0) in zip(r, r[1:]):
        assert 3.5 < a0 / b0 < 4.5
        assert a / b > 12.0, (a, b)
    assert r[-1][0] < 1e-3 * r[-1][1]
