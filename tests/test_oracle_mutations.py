"""Mutation check of the oracle's pins: each entry below plants one plausible
mistake in a copy of oracle/pic_oracle.c (a dropped term, a wrong sign or
index, a swapped operand, a wrong width or volume, a lost factor), builds the
copy and runs the oracle's pins against it (tests/test_oracle_*.py, through
PIC_ORACLE_LIB).  Every mutant must fail at least one pin; the unmutated copy
must pass them all.  Conventions that only the data layout fixes (the Philox
counter layout, the draw numbers) are not mutated: the GPU parity tests hold
them.  CPU only; the mutants run in parallel processes."""
import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "pic_oracle.c")
PINS = ["test_oracle_rng.py", "test_oracle_grid.py", "test_oracle_heating.py",
        "test_oracle_dynamics.py", "test_oracle_mcc.py", "test_oracle_conservation.py",
        "test_oracle_subcycle.py", "test_oracle_nonuniform.py"]

# (name, text in pic_oracle.c, replacement, which occurrence; None: the
# text must occur exactly once)
MUTANTS = [
    # Philox4x32-10 and the uniforms
    ("philox Weyl constant", "k1 += 0xBB67AE85u;", "k1 += 0xBB67AE84u;", None),
    ("philox multiplier", "(uint64_t)0xCD9E8D57u * (uint64_t)c2", "(uint64_t)0xCD9E8D56u * (uint64_t)c2", None),
    ("u01 even multiple", "(2.0 * (double)(r >> 9) + 1.0)", "(2.0 * (double)(r >> 9) + 0.0)", None),
    # Eq. (2): linear and quadratic deposits
    ("linear weights swapped", "Q[jj] += 1.0 - f;\n        Q[jj + 1] += f;",
     "Q[jj] += f;\n        Q[jj + 1] += 1.0 - f;", None),
    ("periodic fold overwrites", "Q[0] += Q[N];", "Q[0] = Q[N];", None),
    ("quadratic centre weight", "0.75 - d * d", "0.75 - d", None),
    ("quadratic weight dropped beyond electrode", "if (g < 0) g = 0;               /* folded",
     "if (g < 0) continue;               /* folded", None),
    ("cell count index", "cnt[(int64_t)floor(xi[p])] += 1.0;", "cnt[(int64_t)floor(xi[p] + 0.5) % N] += 1.0;", None),
    # field solves
    ("Poisson dx^2 lost", "d[g - 1] = rho[g] * dx * dx / EPS0;", "d[g - 1] = rho[g] * dx / EPS0;", None),
    ("boundary term sign", "d[0] -= a[0] * phi0;\n        d[m - 1] -= c[m - 1] * phiN;\n        /* forward",
     "d[0] += a[0] * phi0;\n        d[m - 1] -= c[m - 1] * phiN;\n        /* forward", None),
    ("chi of the wrong cell", "double kl = 1.0 + (chi ? chi[g - 1] : 0.0);",
     "double kl = 1.0 + (chi ? chi[g] : 0.0);", None),
    ("E sign", "E[j] = (phi[j] - phi[j + 1]) / dx;", "E[j] = (phi[j + 1] - phi[j]) / dx;", None),
    ("periodic constant sign", "double D0 = -num / den;", "double D0 = num / den;", None),
    ("periodic prefix index", "P[j] = P[j - 1] + dx * rho[j];", "P[j] = P[j - 1] + dx * rho[j - 1];", None),
    ("nonuniform solve width", "double kr = (1.0 + (chi ? chi[g] : 0.0)) / w[g];",
     "double kr = (1.0 + (chi ? chi[g] : 0.0)) / w[g - 1];", None),
    ("nonuniform field one width", "E[j] = (phi[j] - phi[j + 1]) / w[j];",
     "E[j] = (phi[j] - phi[j + 1]) / w[0];", None),
    # Eq. (3): gathers
    ("EC gather index", "return E[(int64_t)floor(xi)];", "return E[((int64_t)floor(xi + 0.5)) % N];", None),
    ("MC nodal field one cell", "    return 0.5 * (E[g - 1] + E[g]);\n}\n\ndouble orc_gather_mc(",
     "    return E[g];\n}\n\ndouble orc_gather_mc(", None),
    ("MC interpolation swapped",
     "return (1.0 - f) * nodal_E(N, periodic, E, jj) + f * nodal_E(N, periodic, E, jj + 1);",
     "return f * nodal_E(N, periodic, E, jj) + (1.0 - f) * nodal_E(N, periodic, E, jj + 1);", None),
    ("MC nonuniform plain mean", "return (w[g - 1] * E[g - 1] + w[g] * E[g]) / (w[g - 1] + w[g]);",
     "return 0.5 * (E[g - 1] + E[g]);", None),
    ("m=2 gather half a cell off",
     "double k = floor(xi - 0.5);\n    double t = xi - 0.5 - k;\n    int64_t kk",
     "double k = floor(xi);\n    double t = xi - k;\n    int64_t kk", None),
    ("m=2 field beyond electrode", "if (j < 0 || j >= N) return 0.0;",
     "if (j < 0) return E[0];\n    if (j >= N) return E[N - 1];", None),
    ("m=2 nonuniform gather width", "return ((1.0 - t) * da + t * db) / w[c];",
     "return ((1.0 - t) * da + t * db) / w[0];", None),
    # m = 2 implicit susceptibility weights
    ("m=2 chi plain linear weights", "if (in[e]) w[c[e]] += s1[e] * row;",
     "if (in[e]) w[c[e]] += s1[e];", None),
    ("m=2 chi no electrode rule", "if (in[e]) row += s1[e];", "row += s1[e];", None),
    # m = 2 implicit: the tridiagonal operator and its solve
    ("m=2 operator without couplings", "if (ina && inb) off[a] += wa * wb;",
     "if (ina && inb) off[a] += 0.0 * wa * wb;", None),
    ("m=2 operator coupling weight", "if (ina && inb) off[a] += wa * wb;",
     "if (ina && inb) off[a] += wb * wb;", None),
    ("m=2 operator diagonal weight", "if (ina) diag[a] += wa * wa;",
     "if (ina) diag[a] += wa * wb;", None),
    ("tridiagonal solve D0 sign", "double D0e = (phi0 / dx - sv) / su;   /* D0 / eps0 */",
     "double D0e = (phi0 / dx + sv) / su;", None),
    ("tridiagonal solve sub-diagonal", "double a = j > 0 ? xo[j - 1] : 0.0;",
     "double a = j > 0 ? xo[j] : 0.0;", None),
    ("periodic solve one-sided wrap", "A[(size_t)k * w + j] += xo[j];",
     "A[(size_t)k * w + j] += 0.0 * xo[j];", None),
    ("m=2 nonuniform operator with one power of the width", "double f = 1.0 / (rc * rc);",
     "double f = 1.0 / rc;", None),
    ("m=2 nonuniform field without the width ratio", "E[j] = F * dx / w[j];", "E[j] = F;", None),
    ("m=2 nonuniform diagonal of the reference width", "dg[j] = dx / w[j];", "dg[j] = 1.0;", None),
    ("implicit subcycled ions' susceptibility with one power of K",
     "return p->q * p->q * p->w / p->m * h * h;", "return p->q * p->q * p->w / p->m * h;", None),
    ("subcycled ions' susceptibility in every solve",
     "if (!(p->m > 0.0) || !moves(s, sp)) return 0.0;", "if (!(p->m > 0.0)) return 0.0;", None),
    ("implicit subcycled ions corrected with dt",
     "        double dt = s->c.dt_s * substep(s, k);\n        double qm = p->q / p->m;\n        int64_t i = 0;",
     "        double dt = s->c.dt_s;\n        double qm = p->q / p->m;\n        int64_t i = 0;", None),
    ("implicit subcycled ions corrected in every step",
     "        if (!moves(s, k)) continue;\n        double dt = s->c.dt_s * substep(s, k);\n        double qm",
     "        double dt = s->c.dt_s * substep(s, k);\n        double qm", None),
    ("implicit subcycled ions predicted with dt",
     "double dt = s->c.dt_s * substep(s, k), dt_dx = dt / s->dx;\n        int64_t i = 0;\n        while (i < p->n) {\n            double vt",
     "double dt = s->c.dt_s, dt_dx = dt / s->dx;\n        int64_t i = 0;\n        while (i < p->n) {\n            double vt", None),
    ("implicit start-up of subcycled ions with dt",
     "double dt = s->c.dt_s * substep(s, k), dt_dx = dt / s->dx;\n        int64_t i = 0;\n        while (i < p->n) {\n            p->abar[i] = 0.0;",
     "double dt = s->c.dt_s, dt_dx = dt / s->dx;\n        int64_t i = 0;\n        while (i < p->n) {\n            p->abar[i] = 0.0;", None),
    ("standing ions' kinetic energy from their prediction",
     "const int held = implicit && !moves(s, k);", "const int held = 0;", None),
    ("m=2 nonuniform D0 sign",
     "double D0e = (phi0 / dx - sv) / su;   /* from dx sum_j F_j = phi_0 - phi_N */",
     "double D0e = (phi0 / dx + sv) / su;", None),
    ("m=2 nonuniform potential from E", "phi[j + 1] = phi[j] - dx * F;",
     "phi[j + 1] = phi[j] - dx * E[j];", None),
    ("m=2 exported chi without its left coupling",
     "double left = j > 0 ? s->xo[j - 1] : (periodic ? s->xo[N - 1] : 0.0);",
     "double left = 0.0;", None),
    # explicit push, heating
    ("work without the half kick", "double dK = p->m * p->w * dv * (p->vx[i] + 0.5 * dv);",
     "double dK = p->m * p->w * dv * p->vx[i];", None),
    ("heating in the next cell",
     "s->heat[k][(int64_t)floor(p->xi[i])] += dK;\n            p->vx[i] += dv;",
     "s->heat[k][((int64_t)floor(p->xi[i]) + 1) % s->c.n_cells] += dK;\n            p->vx[i] += dv;", None),
    ("position with the old velocity", "else p->xi[i] += p->vx[i] * dt_dx;\n            int e",
     "else p->xi[i] += (p->vx[i] - dv) * dt_dx;\n            int e", None),
    # D1 implicit push and susceptibility
    ("implicit beta lost", "p->xi[i] += 0.5 * dt * dt * a / s->dx;", "p->xi[i] += dt * dt * a / s->dx;", None),
    ("abar not averaged", "p->abar[i] = 0.5 * (p->abar[i] + a);", "p->abar[i] = a;", None),
    ("implicit velocity kick", "double vnew = p->vx[i] + 0.5 * dt * a;", "double vnew = p->vx[i] + dt * a;", None),
    ("implicit prediction without abar", "double vt = p->vx[i] + 0.5 * dt * p->abar[i];",
     "double vt = p->vx[i];", None),
    ("chi without beta", "s->chi[j] = 0.5 * s->c.dt_s * s->c.dt_s / (EPS0",
     "s->chi[j] = s->c.dt_s * s->c.dt_s / (EPS0", None),
    ("MC chi full volume at electrode", "if (!periodic && (g == 0 || g == N)) vol = 0.5 * s->dx;",
     "if (!periodic && (g == 0 || g == N)) vol = s->dx;", None),
    ("MC chi cell counts", "s->Q[k][g] / vol;", "s->cnt[k][j] / vol;", None),
    ("chi with the reference width", "(EPS0 * (s->cw ? s->cw[j] : s->dx)) * x;", "(EPS0 * s->dx) * x;", None),
    # MCC
    ("nu_max left end only", "double cand = (sl > sr ? sl : sr) * v;", "double cand = sl * v;", None),
    ("P_null linearised", "s->pnull[sp] = 1.0 - exp(-s->numax[sp] * s->c.dt_s * substep(s, sp));",
     "s->pnull[sp] = s->numax[sp] * s->c.dt_s * substep(s, sp);", None),
    ("wait off by one", "if (*wait > 0) {\n        *wait -= 1;", "if (*wait > 1) {\n        *wait -= 1;", None),
    ("geometric draw shifted", "double W = floor(log(u) * s->inv_log1mp[sp]);",
     "double W = ceil(log(u) * s->inv_log1mp[sp]);", None),
    ("children without waits", "orc_mcc_first_wait(s, 0, ide, step));", "0);", None),
    ("process rate without speed", "cum += ng * sig * vm / s->numax[0];", "cum += ng * sig / s->numax[0];", None),
    ("last process wins", "if (u[1] < cum) { chosen = k; break; }", "if (u[1] < cum) { chosen = k; }", None),
    ("elastic recoil sign", "(1.0 - 2.0 * me->m / s->c.gas_mass_kg * (1.0 - cchi))",
     "(1.0 - 2.0 * me->m / s->c.gas_mass_kg * (1.0 + cchi))", None),
    ("excitation loss halved", "double e1 = eps - pr->thr;", "double e1 = eps - 0.5 * pr->thr;", None),
    ("Opal argument", "atan(avail / (2.0 * B))", "atan(avail / B)", None),
    ("CX relative speed one component", "double g = sqrt(g2);", "double g = sqrt(gx * gx);", None),
    ("new ion at the electron mass", "double vti = sqrt(KB_J * s->c.gas_temp_K / s->sp[1].m);",
     "double vti = sqrt(KB_J * s->c.gas_temp_K / me->m);", None),
    ("anisotropic scattering", "double ct = 1.0 - 2.0 * ua;", "double ct = 1.0 - ua;", None),
    # ledger
    ("K_before of the implicit state", "double vx = implicit ? p->vx[i] - 0.5 * hdt * p->abar[i] : p->vx[i];",
     "double vx = p->vx[i];", None),
    ("field energy doubled", "we += 0.5 * EPS0 * s->E[j] * s->E[j] * (s->cw ? s->cw[j] : s->dx);\n    s->led.WE",
     "we += EPS0 * s->E[j] * s->E[j] * (s->cw ? s->cw[j] : s->dx);\n    s->led.WE", None),
    ("children's energy not booked", "s->led.coll_dK[0] += kin(&s->sp[0], ve[0], ve[1], ve[2]);", ";", None),
    ("absorbed energy not booked",
     "s->led.absorbed_K[k][e] += kin(p, p->vx[i], p->vy[i], p->vz[i]);", ";", 0),
    # ion subcycling
    ("subcycle phase", "|| s->step % s->c.ion_subcycle == 0;", "|| s->step % s->c.ion_subcycle == 1;", None),
    ("subcycle long step in the velocity only", "double dt_dx = s->c.dt_s / s->dx * h;",
     "double dt_dx = s->c.dt_s / s->dx;", None),
    ("subcycle long step in the position only", "double qm_dt = p->q / p->m * s->c.dt_s * h;",
     "double qm_dt = p->q / p->m * s->c.dt_s;", None),
    ("subcycled ions collide every step", "if (moves(s, 1)) mcc_species(s, 1, n1, s->step);",
     "mcc_species(s, 1, n1, s->step);", None),
    ("subcycle P_null of the short step", "exp(-s->numax[sp] * s->c.dt_s * substep(s, sp))",
     "exp(-s->numax[sp] * s->c.dt_s)", None),
    # nonuniform grid
    ("mover maps with the old cell's width", "*xi = lo + (X - s->edge[lo]) / s->cw[lo];",
     "*xi = lo + (X - s->edge[lo]) / s->cw[c];", None),
    ("node volume of one cell", ": g == N ? s->cw[N - 1] : 0.5 * (s->cw[g - 1] + s->cw[g]);",
     ": g == N ? s->cw[N - 1] : s->cw[g];", None),
    ("MC node susceptibility volume of the uniform grid",
     "if (s->cw)   /* half of each adjacent cell */\n                    vol = 0.5",
     "if (0)   /* half of each adjacent cell */\n                    vol = 0.5", None),
    ("field energy with the reference width",
     "we += 0.5 * EPS0 * s->E[j] * s->E[j] * (s->cw ? s->cw[j] : s->dx);\n    s->led.WE",
     "we += 0.5 * EPS0 * s->E[j] * s->E[j] * s->dx;\n    s->led.WE", None),
]


def apply(src, old, new, occ):
    pos = -1
    for _ in range((occ or 0) + 1):
        pos = src.find(old, pos + 1)
        assert pos >= 0, f"mutation anchor not found: {old!r}"
    return src[:pos] + new + src[pos + len(old):]


def run_pins(lib_path, timeout=240):
    env = dict(os.environ, PIC_ORACLE_LIB=lib_path, PYTHONDONTWRITEBYTECODE="1",
               OMP_NUM_THREADS="1")
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
           "-m", "not gpu"] + [os.path.join(ROOT, "tests", f) for f in PINS]
    try:
        r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True,
                           timeout=timeout)
    except subprocess.TimeoutExpired:
        return 124, "timeout"
    return r.returncode, (r.stdout + r.stderr)[-600:]


def build(src, path):
    with open(path + ".c", "w") as f:
        f.write(src)
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-w", "-I",
                           os.path.join(ROOT, "oracle"), "-o", path, path + ".c", "-lm"])


def test_every_anchor_is_unique_where_it_must_be():
    src = open(SRC).read()
    for name, old, new, occ in MUTANTS:
        if occ is None:
            assert src.count(old) == 1, (name, src.count(old))
        else:
            assert src.count(old) >= occ + 1, name
        assert apply(src, old, new, occ) != src, name


def test_every_planted_mistake_fails_a_pin():
    src = open(SRC).read()
    tmp = tempfile.mkdtemp(prefix="orc_mut_")
    try:
        base = os.path.join(tmp, "base.so")
        build(src, base)
        rc, out = run_pins(base)
        assert rc == 0, "the unmutated copy must pass every pin:\n" + out

        def one(k):
            name, old, new, occ = MUTANTS[k]
            path = os.path.join(tmp, f"m{k:03d}.so")
            build(apply(src, old, new, occ), path)
            rc, out = run_pins(path)
            return name, rc, out

        workers = max(1, min(8, (os.cpu_count() or 2)))
        with ThreadPoolExecutor(workers) as ex:
            results = list(ex.map(one, range(len(MUTANTS))))
        survivors = [(n, out) for n, rc, out in results if rc == 0]
        print(f"{len(MUTANTS)} mutants, {len(MUTANTS) - len(survivors)} caught")
        assert not survivors, "mutants no pin catches: " + ", ".join(n for n, _ in survivors)
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
