"""Seeded synthetic inputs for the EC PIC/MCC hot path (arXiv:1310.5284).

This module is the only code shared by the GPU side and the oracle side, and it
holds none of the method's arithmetic: it builds case parameters, particle
loads (uniform positions, Maxwellian velocities) and the analytic synthetic
cross-section tables that stand in for the argon data the paper takes from its
earlier work (Sec. III).  Everything is drawn from numpy's PCG64 with a fixed
seed, so both sides receive byte-identical inputs.

Particle positions are given as an int32 cell index plus a float32 offset in
[0, 1); velocities as float32 m/s; ids as uint64.  ``to_oracle`` only widens
these to float64 (xi = cell + off exactly).
"""
from __future__ import annotations

import math

import numpy as np

# physical constants used to *set up* workloads (the method's own arithmetic
# defines its constants separately on each side)
E_CHARGE = 1.602176634e-19
M_E = 9.1093837015e-31
AMU = 1.66053906660e-27
M_AR = 40.0 * AMU
K_B = 1.380649e-23
TORR = 101325.0 / 760.0
EPS0_SETUP = 8.8541878128e-12

ELASTIC, EXCITATION, IONIZATION, CHARGE_EXCHANGE = 0, 1, 2, 3


def gas_density(p_mtorr: float, T_K: float = 300.0) -> float:
    return p_mtorr * 1e-3 * TORR / (K_B * T_K)


def argon_like_tables(e_max_eV: float = 1000.0, de_eV: float = 0.05):
    """Analytic synthetic cross sections (m^2) on a uniform grid from 0 eV.

    electron elastic 1e-19 (constant); excitation 1e-20 (1 - 11.5/eps) above
    11.5 eV; ionization 3e-20 (1 - 15.8/eps) above 15.8 eV; ion charge exchange
    5e-19 (constant).  These shapes are a workload choice: the paper's argon
    data are not available.
    """
    n = int(round(e_max_eV / de_eV)) + 1
    eps = np.arange(n, dtype=np.float64) * de_eV
    el = np.full(n, 1e-19)
    with np.errstate(divide="ignore", invalid="ignore"):
        ex = np.where(eps > 11.5, 1e-20 * (1.0 - 11.5 / eps), 0.0)
        iz = np.where(eps > 15.8, 3e-20 * (1.0 - 15.8 / eps), 0.0)
    cx = np.full(n, 5e-19)
    mk = lambda sp, kind, thr, s: dict(species=sp, kind=kind, threshold_eV=thr, e0_eV=0.0,
                                       de_eV=de_eV, sigma=s)
    return [mk(0, ELASTIC, 0.0, el), mk(0, EXCITATION, 11.5, ex), mk(0, IONIZATION, 15.8, iz),
            mk(1, CHARGE_EXCHANGE, 0.0, cx)]


def sheath_refined_widths(n_cells, gap_m, ratio=4.0, sheath_frac=0.15):
    """Cell widths of a grid refined next to both electrodes: the cells within
    sheath_frac of the gap from either electrode are about `ratio` times
    narrower than the bulk cells; the widths sum to gap_m."""
    ns = int(round(n_cells * ratio * sheath_frac / ((1 - 2 * sheath_frac) + 2 * ratio * sheath_frac)))
    ns = min(max(ns, 1), (n_cells - 1) // 2)
    nb = n_cells - 2 * ns
    ws = sheath_frac * gap_m / ns
    wb = (1 - 2 * sheath_frac) * gap_m / nb
    w = np.concatenate([np.full(ns, ws), np.full(nb, wb), np.full(ns, ws)])
    return w * (gap_m / w.sum())


def load_species(rng, n, N, q, m, w, T_eV, capacity=None, lo_cell=0, hi_cell=None,
                 id_base=0, widths=None):
    """Uniform positions over cells [lo_cell, hi_cell) (with widths: uniform in
    physical space over the gap) and a Maxwellian at T_eV."""
    hi_cell = N if hi_cell is None else hi_cell
    if widths is None:
        cell = rng.integers(lo_cell, hi_cell, size=n, dtype=np.int64).astype(np.int32)
        off = rng.random(n, dtype=np.float32)
    else:
        edges = np.concatenate([[0.0], np.cumsum(widths)])
        X = rng.random(n) * edges[-1]
        c = np.clip(np.searchsorted(edges, X, side="right") - 1, 0, N - 1)
        cell = c.astype(np.int32)
        off = np.minimum((X - edges[c]) / widths[c], np.nextafter(1.0, 0.0)).astype(np.float32)
        off = np.where(off >= 1.0, np.float32(0.0), off).astype(np.float32)
    vt = math.sqrt(T_eV * E_CHARGE / m)
    v = (vt * rng.standard_normal((3, n))).astype(np.float32)
    return dict(q=q, m=m, w=w, cell=cell, off=off, vx=v[0].copy(), vy=v[1].copy(),
                vz=v[2].copy(), id=(np.arange(n, dtype=np.uint64) + np.uint64(id_base)),
                capacity=int(capacity if capacity is not None else max(n, 1)))


def empty_species(q, m, w=1.0, capacity=1):
    z = np.zeros(0, dtype=np.float32)
    return dict(q=q, m=m, w=w, cell=np.zeros(0, np.int32), off=z, vx=z, vy=z, vz=z,
                id=np.zeros(0, np.uint64), capacity=capacity)


def ccp_case(*, n_cells, gap_m, volts, freq, dt, p_mtorr, scheme=0, collisions=1, seed=0,
             gather=0, T_gas=300.0):
    return dict(n_cells=n_cells, gap_m=gap_m, bc=0, scheme=scheme, gather=gather,
                collisions=collisions, dt_s=dt, step0=0, rf_volts=volts, rf_freq_hz=freq,
                gas_density_m3=gas_density(p_mtorr, T_gas), gas_temp_K=T_gas,
                gas_mass_kg=M_AR, background_rho=0.0, opal_B_eV=10.0, seed=seed)


def ccp_workload(name, *, n_cells, np_per_species, gap_m=0.025, volts=100.0, freq=13.56e6,
                 dt=None, p_mtorr=50.0, n0=1e15, Te=2.0, Ti=0.026, scheme=0, collisions=1,
                 seed=0, steps=1000, capacity_factor=1.25, e_max_eV=1000.0, gather=0,
                 cell_dx=None):
    dt = dt if dt is not None else 1.0 / (400.0 * freq)
    rng = np.random.Generator(np.random.PCG64(seed))
    w = n0 * gap_m / np_per_species
    cap = int(math.ceil(np_per_species * capacity_factor)) + 64
    e = load_species(rng, np_per_species, n_cells, -E_CHARGE, M_E, w, Te, cap, widths=cell_dx)
    i = load_species(rng, np_per_species, n_cells, E_CHARGE, M_AR, w, Ti, cap, widths=cell_dx)
    case = ccp_case(n_cells=n_cells, gap_m=gap_m, volts=volts, freq=freq, dt=dt,
                    p_mtorr=p_mtorr, scheme=scheme, collisions=collisions, seed=seed,
                    gather=gather)
    if cell_dx is not None:
        case["cell_dx"] = np.asarray(cell_dx, dtype=np.float64)
    return dict(name=name, case=case, species=[e, i], processes=argon_like_tables(e_max_eV),
                n_steps=steps, n0=n0, Te=Te)


# ---------------------------------------------------------------------------
# the five synthetic discharges
# ---------------------------------------------------------------------------
def c1(collisions=1, scheme=0, np_per_species=16384, seed=0xC1):
    """Explicit EC CCP: 2.5 cm, 64 cells, 100 V at 13.56 MHz, 50 mTorr,
    16k e + 16k Ar+ at 1e15 m^-3, Te 2 eV, Ti 0.026 eV, dt = 1/(400 f),
    10 RF cycles (4000 steps)."""
    return ccp_workload("ccp64_explicit", n_cells=64, np_per_species=np_per_species,
                        volts=100.0, p_mtorr=50.0, scheme=scheme, collisions=collisions,
                        seed=seed, steps=4000)


def c2(ratio=5.0, gather=0, ppc=1000, n_cells=512, wdt=0.2, seed=0xC2, steps=100000):
    """Periodic collisionless thermal plasma, electrons on a fixed neutralising
    background; dx = ratio * lambda_D, omega_p dt = wdt, ppc electrons/cell."""
    n0, Te = 1e15, 2.0
    lam = math.sqrt(EPS0_SETUP * Te / (n0 * E_CHARGE))
    wp = math.sqrt(n0 * E_CHARGE ** 2 / (EPS0_SETUP * M_E))
    dx = ratio * lam
    L = n_cells * dx
    n = ppc * n_cells
    rng = np.random.Generator(np.random.PCG64(seed))
    w = n0 * L / n
    e = load_species(rng, n, n_cells, -E_CHARGE, M_E, w, Te, n + 64)
    ion = empty_species(E_CHARGE, M_AR, w)
    case = dict(n_cells=n_cells, gap_m=L, bc=1, scheme=0, gather=gather, collisions=0,
                dt_s=wdt / wp, step0=0, rf_volts=0.0, rf_freq_hz=0.0, gas_density_m3=0.0,
                gas_temp_K=300.0, gas_mass_kg=M_AR, background_rho=n0 * E_CHARGE,
                opal_B_eV=10.0, seed=seed)
    return dict(name="periodic_thermal", case=case, species=[e, ion], processes=[],
                n_steps=steps, n0=n0, Te=Te, wp=wp, lambda_D=lam)


def c3(wdt=5.0, scheme=1, ppc=200, collisions=1, seed=0xC3, steps=None):
    """Direct-implicit EC CCP: 2.5 cm, 256 cells (dx = 5 lambda_D at 2.9e17 m^-3,
    Te 2 eV), 100 mTorr, 200 V at 13.56 MHz, 200 particles/cell/species."""
    n0, Te = 2.90e17, 2.0
    wp = math.sqrt(n0 * E_CHARGE ** 2 / (EPS0_SETUP * M_E))
    dt = wdt / wp
    freq = 13.56e6
    per = int(round(1.0 / (freq * dt)))
    return ccp_workload("ccp256_implicit", n_cells=256, np_per_species=ppc * 256, volts=200.0,
                        freq=freq, dt=dt, p_mtorr=100.0, n0=n0, Te=Te, scheme=scheme,
                        collisions=collisions, seed=seed,
                        steps=steps if steps is not None else 100 * per)


def c4(np_per_species=10_000_000, seed=0xC4, scheme=0, cell_dx=None):
    """Production explicit EC CCP: 2048 cells over 2.5 cm, 1e7 e + 1e7 Ar+,
    30 mTorr, 300 V at 13.56 MHz, dt = 1/(2000 f) (cell_dx: a nonuniform grid
    of the same cell count)."""
    freq = 13.56e6
    return ccp_workload("ccp2048_explicit", n_cells=2048, np_per_species=np_per_species,
                        volts=300.0, freq=freq, dt=1.0 / (2000.0 * freq), p_mtorr=30.0,
                        scheme=scheme, seed=seed, steps=2_000_000, cell_dx=cell_dx)


def c5(n_cases=64, seed=5, np_scale=1.0):
    """Batched sweep of uneven discharges (explicit and implicit mixed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    freq = 13.56e6
    for k in range(n_cases):
        p = math.exp(rng.uniform(math.log(10.0), math.log(500.0)))
        V = rng.uniform(50.0, 400.0)
        N = int(round(math.exp(rng.uniform(math.log(128), math.log(1024)))))
        Np = int(round(math.exp(rng.uniform(math.log(1e4), math.log(2e6))) * np_scale))
        scheme = int(rng.integers(0, 2))
        dt = 1.0 / ((400.0 if scheme == 0 else 100.0) * freq)
        out.append(ccp_workload(f"sweep{k:02d}", n_cells=N, np_per_species=max(Np, 16),
                                volts=V, freq=freq, dt=dt, p_mtorr=p, scheme=scheme,
                                seed=(seed << 16) + k, steps=2000))
    return out


# ---------------------------------------------------------------------------
# conversions (no arithmetic of the method)
# ---------------------------------------------------------------------------
def to_oracle(wl) -> tuple:
    """(case, species, processes) in the oracle's float64 form."""
    sps = []
    for sp in wl["species"]:
        sps.append(dict(q=sp["q"], m=sp["m"], w=sp["w"],
                        xi=sp["cell"].astype(np.float64) + sp["off"].astype(np.float64),
                        vx=sp["vx"].astype(np.float64), vy=sp["vy"].astype(np.float64),
                        vz=sp["vz"].astype(np.float64),
                        abar=(sp["abar"].astype(np.float64) if "abar" in sp else None),
                        id=sp["id"]))
    return wl["case"], sps, wl["processes"]
