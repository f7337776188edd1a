"""Pins of the oracle's grid operations: Eq. (2) weighting, Eq. (3)
interpolation, the explicit and susceptibility-modified field solves.

Each check uses a formulation other than the oracle's own: brute force over
every (particle, node) pair with the spline functions, closed-form potentials,
and dense linear solves of the finite-difference systems."""
import numpy as np
import pytest

EPS0 = 8.8541878128e-12


def S1(x):
    return np.maximum(0.0, 1.0 - np.abs(x))


def S0(x):
    # half-open top hat: a particle exactly on a node belongs to the cell above
    return ((x >= -0.5) & (x < 0.5)).astype(np.float64)


@pytest.mark.parametrize("N,n,periodic", [(5, 37, False), (8, 200, True), (3, 9, False)])
def test_deposit_is_eq2_brute_force(orc, N, n, periodic):
    rng = np.random.default_rng(N * 1000 + n)
    xi = rng.random(n) * N
    xi[:3] = [0.0, N - 1e-9, float(N // 2)]  # node hits and the last edge
    Q = orc.deposit_linear(N, xi, periodic=periodic)
    g = np.arange(N + 1)
    ref = S1(g[:, None] - xi[None, :]).sum(axis=1)
    if periodic:
        # node N is node 0; a particle in the last cell also weights node 0 via N
        ref[0] += ref[N]
        ref[N] = ref[0]
    np.testing.assert_allclose(Q, ref, rtol=0, atol=1e-12)
    # total charge is one per particle (node N duplicates node 0 when periodic)
    tot = Q[:N].sum() if periodic else Q.sum()
    assert abs(tot - n) < 1e-10


def test_ec_gather_is_eq3_brute_force(orc):
    N = 7
    rng = np.random.default_rng(3)
    E = rng.standard_normal(N)
    xi = np.concatenate([rng.random(50) * N, np.arange(N, dtype=float)])
    for x in xi:
        # sum over the half-grid points x_{g+1/2} with S_0
        ref = sum(E[g] * S0(x - g - 0.5) for g in range(N))
        assert orc.gather_ec(N, E, x) == pytest.approx(ref, abs=0, rel=0)


@pytest.mark.parametrize("periodic", [False, True])
def test_mc_gather_brute_force(orc, periodic):
    N = 6
    rng = np.random.default_rng(4)
    E = rng.standard_normal(N)
    # nodal field by centred differences of the potential: (phi_{g-1}-phi_{g+1})/2dx
    Eg = np.zeros(N + 1)
    for g in range(N + 1):
        if periodic:
            Eg[g] = 0.5 * (E[(g - 1) % N] + E[g % N])
        else:
            Eg[g] = E[0] if g == 0 else (E[N - 1] if g == N else 0.5 * (E[g - 1] + E[g]))
    for x in rng.random(40) * N:
        ref = sum(Eg[g] * S1(x - g) for g in range(N + 1))
        assert orc.gather_mc(N, E, x, periodic=periodic) == pytest.approx(ref, rel=1e-13,
                                                                         abs=1e-13)


def test_dirichlet_uniform_rho_closed_form(orc):
    # -eps0 phi'' = rho with phi(0)=V, phi(L)=0 has the quadratic solution
    # phi = V (1 - x/L) + rho x (L - x) / (2 eps0), exact for the 3-point stencil
    N, L, V, rho0 = 64, 0.025, 100.0, 3.2e-5
    dx = L / N
    rho = np.full(N + 1, rho0)
    phi, E = orc.solve_dirichlet(N, dx, rho, V, 0.0)
    x = np.arange(N + 1) * dx
    ref = V * (1 - x / L) + rho0 * x * (L - x) / (2 * EPS0)
    np.testing.assert_allclose(phi, ref, rtol=1e-12, atol=1e-12 * abs(ref).max())
    np.testing.assert_allclose(E, (ref[:-1] - ref[1:]) / dx, rtol=1e-10,
                               atol=1e-10 * abs(E).max())


def _dense_dirichlet(N, dx, rho, chi, V0, VN):
    k = 1.0 + chi
    A = np.zeros((N + 1, N + 1))
    b = np.zeros(N + 1)
    A[0, 0] = 1.0; b[0] = V0
    A[N, N] = 1.0; b[N] = VN
    for g in range(1, N):
        # -(eps0/dx^2) [k_g (phi_{g+1}-phi_g) - k_{g-1}(phi_g - phi_{g-1})] = rho_g
        A[g, g - 1] = -EPS0 * k[g - 1] / dx ** 2
        A[g, g] = EPS0 * (k[g - 1] + k[g]) / dx ** 2
        A[g, g + 1] = -EPS0 * k[g] / dx ** 2
        b[g] = rho[g]
    return np.linalg.solve(A, b)


@pytest.mark.parametrize("with_chi", [False, True])
def test_dirichlet_dense_solve(orc, with_chi):
    rng = np.random.default_rng(11 + with_chi)
    N, dx = 12, 1e-4
    rho = rng.standard_normal(N + 1) * 1e-4
    chi = rng.random(N) * 30 if with_chi else np.zeros(N)
    phi, E = orc.solve_dirichlet(N, dx, rho, 37.0, -5.0, chi=chi if with_chi else None)
    ref = _dense_dirichlet(N, dx, rho, chi, 37.0, -5.0)
    np.testing.assert_allclose(phi, ref, rtol=1e-11, atol=1e-11 * abs(ref).max())


def test_constant_chi_scales_permittivity(orc):
    # constant chi is the plain Poisson equation with eps0 -> eps0 (1+chi)
    rng = np.random.default_rng(2)
    N, dx, c = 20, 2e-4, 4.5
    rho = rng.standard_normal(N + 1) * 1e-5
    phi1, _ = orc.solve_dirichlet(N, dx, rho, 0.0, 0.0, chi=np.full(N, c))
    phi2, _ = orc.solve_dirichlet(N, dx, rho / (1 + c), 0.0, 0.0)
    np.testing.assert_allclose(phi1, phi2, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("with_chi", [False, True])
def test_periodic_dense_solve(orc, with_chi):
    rng = np.random.default_rng(5 + with_chi)
    N, dx = 10, 3e-4
    rho = rng.standard_normal(N + 1) * 1e-5
    rho[:N] -= rho[:N].mean()
    rho[N] = rho[0]
    chi = rng.random(N) * 7 if with_chi else np.zeros(N)
    phi, E = orc.solve_periodic(N, dx, rho, chi=chi if with_chi else None)
    # dense periodic system for phi_0..phi_{N-1} with gauge phi_0 = 0
    k = 1.0 + chi
    A = np.zeros((N, N))
    b = np.zeros(N)
    for g in range(N):
        gl, gr = (g - 1) % N, (g + 1) % N
        A[g, gl] += -EPS0 * k[gl] / dx ** 2
        A[g, g] += EPS0 * (k[gl] + k[g]) / dx ** 2
        A[g, gr] += -EPS0 * k[g] / dx ** 2
        b[g] = rho[g]
    A[0, :] = 0.0
    A[0, 0] = 1.0
    b[0] = 0.0
    ref = np.linalg.solve(A, b)
    np.testing.assert_allclose(phi[:N], ref, rtol=1e-10, atol=1e-10 * abs(ref).max())
    assert abs(phi[N]) < 1e-9 * abs(ref).max()   # periodic potential
    assert abs(E.sum()) < 1e-9 * abs(E).max()


def _chi(orc, N, xi, gather, periodic=False, dx=1e-4, dt=1e-10):
    q, m, w = -1.602176634e-19, 9.1093837015e-31, 1e9
    case = dict(n_cells=N, gap_m=N * dx, bc=1 if periodic else 0, scheme=1, gather=gather,
                collisions=0, dt_s=dt, rf_volts=0.0, rf_freq_hz=0.0,
                background_rho=0.0 if not periodic else 0.0)
    xi = np.asarray(xi, dtype=np.float64)
    z = np.zeros_like(xi)
    sps = [dict(q=q, m=m, w=w, xi=xi, vx=z, vy=z, vz=z, abar=z, id=np.arange(xi.size, dtype=np.uint64)),
           dict(q=-q, m=1e-25, w=w, xi=np.zeros(0), vx=np.zeros(0), vy=np.zeros(0), vz=np.zeros(0),
                abar=np.zeros(0), id=np.zeros(0, dtype=np.uint64))]
    sim = orc.Sim(case, sps, [], startup=False)
    sim.compute_fields()
    K = 0.5 * dt * dt / EPS0 * q * q * w / m      # beta dt^2 q^2 w / (eps0 m)
    return sim.fields()["chi"], K / dx


def test_mc_susceptibility_is_cic_at_nodes_closed_form(orc):
    # 3 electrons at the centre of each of cells 0..3 of 8 (Dirichlet): node
    # weights 1.5, 3, 3, 3, 1.5, 0, ..; densities with half a cell at the
    # electrode node; cell values are the mean of the two nodes
    N = 8
    xi = np.repeat(np.arange(4) + 0.5, 3)
    chi_mc, u = _chi(orc, N, xi, gather=1)
    expect = u * np.array([3.0, 3.0, 3.0, 2.25, 0.75, 0.0, 0.0, 0.0])
    assert np.allclose(chi_mc, expect, rtol=1e-12, atol=0.0)
    # the energy-conserving scheme counts the particles of each cell
    chi_ec, _ = _chi(orc, N, xi, gather=0)
    assert np.allclose(chi_ec, u * np.array([3.0] * 4 + [0.0] * 4), rtol=1e-12, atol=0.0)


@pytest.mark.parametrize("periodic", [False, True])
def test_mc_and_ec_susceptibility_agree_for_uniform_plasma(orc, periodic):
    # c particles at every cell centre: CIC node density equals cell density
    N = 6
    xi = np.repeat(np.arange(N) + 0.5, 5)
    chi_mc, u = _chi(orc, N, xi, gather=1, periodic=periodic)
    chi_ec, _ = _chi(orc, N, xi, gather=0, periodic=periodic)
    assert np.allclose(chi_mc, 5.0 * u, rtol=1e-12)
    assert np.allclose(chi_ec, 5.0 * u, rtol=1e-12)


def S2(x):
    # quadratic B-spline: the convolution of the top hat with S_1
    a = np.abs(x)
    return np.where(a <= 0.5, 0.75 - a * a, np.where(a <= 1.5, 0.5 * (1.5 - a) ** 2, 0.0))


@pytest.mark.parametrize("N,periodic", [(7, False), (9, True), (3, False)])
def test_quadratic_deposit_brute_force(orc, N, periodic):
    # Eq. (2) with m = 2 read as spline degree: every node -1..N+1 takes
    # S_2(node - xi); nodes beyond an electrode fold into it, periodic wrap
    rng = np.random.default_rng(5 + N)
    xi = rng.uniform(0.0, N, 300)
    xi[:3] = [0.0, N - 1e-9, 0.5]
    Q = orc.deposit_quadratic(N, xi, periodic)
    B = np.zeros(N + 3)          # nodes -1 .. N+1
    for p in xi:
        B += S2(np.arange(-1, N + 2) - p)
    if periodic:
        ref = np.zeros(N)
        for g in range(-1, N + 2):
            ref[g % N] += B[g + 1]
        assert np.allclose(Q[:N], ref, rtol=1e-12, atol=1e-12)
        assert Q[N] == Q[0]
        assert abs(Q[:N].sum() - xi.size) < 1e-9
    else:
        ref = B[1:N + 2].copy()
        ref[0] += B[0]
        ref[N] += B[N + 2]
        assert np.allclose(Q, ref, rtol=1e-12, atol=1e-12)
        assert abs(Q.sum() - xi.size) < 1e-9


@pytest.mark.parametrize("periodic", [False, True])
def test_ec2_gather_brute_force(orc, periodic):
    N = 6
    rng = np.random.default_rng(11)
    E = rng.normal(size=N)
    for xi in np.concatenate([rng.uniform(0, N, 40), [0.0, 0.25, 0.5, N - 0.5, N - 1e-9]]):
        ref = 0.0
        for j in range(-1, N + 1):
            if periodic:
                e = E[j % N]
            else:
                e = E[j] if 0 <= j < N else 0.0   # no half-grid field beyond an electrode
            ref += e * S1(xi - (j + 0.5))
        assert abs(orc.gather_ec2(N, E, xi, periodic) - ref) < 1e-12


@pytest.mark.parametrize("periodic", [False, True])
def test_ec2_gather_is_minus_the_gradient_of_the_deposit_energy(orc, periodic):
    # the energy-conserving pair: with E_{j+1/2} = phi_j - phi_{j+1} (dx = 1),
    # the gathered field at xi equals -d/dxi sum_g phi_g w_g(xi), w_g the
    # particle's own node weights (fold and wrap included)
    N = 8
    rng = np.random.default_rng(3)
    phi = rng.normal(size=N + 1)
    if periodic:
        phi[N] = phi[0]
    E = phi[:N] - phi[1:]
    h = 1e-6
    for xi in np.concatenate([rng.uniform(0.02, N - 0.02, 60), [0.3, N - 0.3]]):
        def energy(x):
            w = orc.deposit_quadratic(N, [x], periodic)
            return (w[:N] * phi[:N]).sum() if periodic else (w * phi).sum()
        grad = (energy(xi + h) - energy(xi - h)) / (2 * h)
        assert abs(orc.gather_ec2(N, E, xi, periodic) + grad) < 1e-6


def _ec2_operator(N, xi, periodic):
    # the exact susceptibility operator of the m = 2 implicit scheme, up to
    # its constant: M[h, h'] = sum_p S_1(x_p - x_h) S_1(x_p - x_h') over the
    # N cell centres (minimum-image distances when periodic)
    xc = np.arange(N) + 0.5
    d = xi[:, None] - xc[None, :]
    if periodic:
        d = (d + 0.5 * N) % N - 0.5 * N
    W = S1(d)                     # particles x centres
    return W.T @ W


@pytest.mark.parametrize("N,periodic", [(6, False), (7, True), (2, False)])
def test_ec2_susceptibility_weights_are_row_sums_of_the_operator(orc, N, periodic):
    rng = np.random.default_rng(40 + N)
    xi = rng.uniform(0.0, N, 250)
    xi[:5] = [0.0, 0.25, 0.5, N - 0.5, N - 1e-9]   # electrode half cells and centres
    w = orc.chi_weights_ec2(N, xi, periodic)
    M = _ec2_operator(N, xi, periodic)
    np.testing.assert_allclose(w, M.sum(axis=1), rtol=1e-12, atol=1e-12)
    if periodic:
        # every particle's weights sum to one
        assert abs(w.sum() - xi.size) < 1e-9


@pytest.mark.parametrize("periodic", [False, True])
def test_ec2_susceptibility_at_centres_is_the_cell_count(orc, periodic):
    # a particle at a centre sits on one centre only: the operator is
    # diagonal and the implicit m = 2 solve takes the m = 1 susceptibility
    N = 8
    xi = np.repeat(np.arange(N) + 0.5, np.array([3, 0, 1, 4, 2, 2, 0, 5]))
    chi2, u = _chi(orc, N, xi, gather=2, periodic=periodic)
    chi1, _ = _chi(orc, N, xi, gather=0, periodic=periodic)
    assert np.allclose(chi2, chi1, rtol=1e-12, atol=0.0)
    assert np.allclose(chi1, u * np.array([3, 0, 1, 4, 2, 2, 0, 5]), rtol=1e-12)


def test_ec2_susceptibility_next_to_an_electrode_closed_form(orc):
    # a particle between an electrode and the first centre sees the field of
    # that centre only, with weight 1/2 + xi; it polarises that centre by the
    # square of the weight.  One particle at the middle of two centres gives
    # 1/4 + 1/4 to each (row sum 1/2 per centre)
    N = 4
    chi, u = _chi(orc, N, np.array([0.2]), gather=2)
    assert np.allclose(chi, u * np.array([0.49, 0, 0, 0]), rtol=1e-12, atol=0.0)
    chi, u = _chi(orc, N, np.array([N - 0.1]), gather=2)
    assert np.allclose(chi, u * np.array([0, 0, 0, 0.36]), rtol=1e-12, atol=0.0)
    chi, u = _chi(orc, N, np.array([2.0]), gather=2)
    assert np.allclose(chi, u * np.array([0, 0.5, 0.5, 0]), rtol=1e-12, atol=0.0)


# ---------------------------------------------------------------------------
# The tridiagonal m = 2 susceptibility operator and its solve
# ---------------------------------------------------------------------------
def _apply_tridiag(d, o, E, periodic):
    # (M E)_h for diagonal d and couplings o[h] of centres h, h + 1
    y = d * E + o * np.roll(E, -1) + np.roll(o * E, 1)
    if not periodic:
        y = d * E
        y[:-1] += o[:-1] * E[1:]
        y[1:] += o[:-1] * E[:-1]
    return y


@pytest.mark.parametrize("N,periodic", [(6, False), (7, True), (3, True), (2, False)])
def test_ec2_operator_is_the_gram_matrix_of_the_gather_weights(orc, N, periodic):
    rng = np.random.default_rng(60 + N)
    xi = rng.uniform(0.0, N, 300)
    xi[:5] = [0.0, 0.25, 0.5, N - 0.5, N - 1e-9]
    d, o = orc.chi_operator_ec2(N, xi, periodic)
    M = _ec2_operator(N, xi, periodic)
    np.testing.assert_allclose(d, np.diag(M), rtol=1e-12, atol=1e-12)
    for h in range(N - (0 if periodic else 1)):
        assert abs(o[h] - M[h, (h + 1) % N]) < 1e-9, (h, o[h], M[h, (h + 1) % N])
    if not periodic:
        assert o[N - 1] == 0.0
    # the row sums are the diagonal weights of the nonuniform solve
    E = rng.normal(size=N)
    np.testing.assert_allclose(_apply_tridiag(d, o, E, periodic), M @ E, rtol=1e-10, atol=1e-9)


@pytest.mark.parametrize("N,periodic", [(8, False), (7, True)])
def test_ec2_operator_is_the_linear_response_of_the_deposit(orc, N, periodic):
    # Move every particle by eps times the S_1 gather of a half-grid field E
    # (the direction of the D1 correction).  The quadratic deposit then
    # changes node g by the flux in from centre g - 1 minus the flux out
    # through centre g, and to first order in eps the flux through centre h
    # is eps (M E)_h: the operator is the response of the deposit, not a
    # formula of its own.  (No flux beyond an electrode: the weights that
    # reach past it stay on its node.)
    rng = np.random.default_rng(7 + N)
    xi = rng.uniform(0.0, N, 200)
    xi[:4] = [0.05, 0.45, N - 0.3, N - 0.02]
    E = rng.normal(size=N)
    d, o = orc.chi_operator_ec2(N, xi, periodic)
    flux = _apply_tridiag(d, o, E, periodic)
    for eps in (1e-5, 5e-6):
        g = np.array([orc.gather_ec2(N, E, x, periodic) for x in xi])
        moved = xi + eps * g
        if periodic:
            moved %= N
        dq = (orc.deposit_quadratic(N, moved, periodic) -
              orc.deposit_quadratic(N, xi, periodic)) / eps
        if periodic:
            expect = np.roll(flux, 1) - flux          # node g: centres g - 1 and g
            got = dq[:N]
        else:
            fin = np.concatenate([[0.0], flux])       # into node g from centre g - 1
            fout = np.concatenate([flux, [0.0]])      # out of node g through centre g
            expect, got = fin - fout, dq
        assert np.abs(got - expect).max() < 200 * eps * np.abs(flux).max(), eps


@pytest.mark.parametrize("periodic", [False, True])
def test_tridiag_solve_with_a_diagonal_operator_is_the_diagonal_solve(orc, periodic):
    # without couplings the D-form solve must give the field of the
    # potential-form (Dirichlet) or periodic solve with chi = the diagonal
    N, dx = 9, 2e-4
    rng = np.random.default_rng(11)
    rho = rng.normal(size=N + 1) * 1e-3
    if periodic:
        rho[N] = rho[0]
        rho -= rho[:N].mean()
    xd = rng.uniform(0.0, 3.0, N)
    phi_t, E_t = orc.solve_chi_tridiag(N, dx, rho, xd, np.zeros(N), 1.7, periodic)
    if periodic:
        phi, E = orc.solve_periodic(N, dx, rho, chi=xd)
    else:
        phi, E = orc.solve_dirichlet(N, dx, rho, 1.7, 0.0, chi=xd)
    np.testing.assert_allclose(E_t, E, rtol=1e-10, atol=1e-10 * np.abs(E).max())
    np.testing.assert_allclose(phi_t, phi, rtol=1e-10, atol=1e-10 * np.abs(phi).max())


@pytest.mark.parametrize("periodic", [False, True])
def test_tridiag_solve_satisfies_gauss_and_the_potential(orc, periodic):
    # random couplings: the field satisfies Gauss's law with the displacement
    # eps0 (1 + X) E at every interior node, and the potential difference
    # across the gap (or around the box)
    N, dx = 12, 1e-4
    rng = np.random.default_rng(5)
    xi = rng.uniform(0.0, N, 80)
    d, o = orc.chi_operator_ec2(N, xi, periodic)
    xd, xo = 0.3 * d, 0.3 * o
    rho = rng.normal(size=N + 1) * 1e-3
    if periodic:
        rho[N] = rho[0]
        rho -= rho[:N].mean()
    V = 0.0 if periodic else 2.5
    phi, E = orc.solve_chi_tridiag(N, dx, rho, xd, xo, V, periodic)
    D = EPS0 * (E + _apply_tridiag(xd, xo, E, periodic))
    gauss = (D[1:] - D[:-1]) - dx * rho[1:N]
    assert np.abs(gauss).max() < 1e-10 * np.abs(dx * rho).max()
    if periodic:
        assert abs(D[0] - D[N - 1] - dx * rho[0]) < 1e-10 * np.abs(dx * rho).max()
    assert abs(dx * E.sum() - V) < 1e-12 + 1e-12 * abs(V)
    np.testing.assert_allclose(phi[:-1] - phi[1:], dx * E, rtol=1e-12, atol=1e-20)


@pytest.mark.parametrize("periodic", [False, True])
def test_ec2_exported_susceptibility_is_the_row_sum(orc, periodic):
    # the cell susceptibility exported with the fields is the row sum of the
    # operator, i.e. the diagonal weights of orc_chi_weights_ec2
    N = 10
    xi = np.random.default_rng(3).uniform(0.0, N, 150)
    chi, u = _chi(orc, N, xi, gather=2, periodic=periodic)
    w = orc.chi_weights_ec2(N, xi, periodic)
    np.testing.assert_allclose(chi, u * w, rtol=1e-12, atol=1e-30)
