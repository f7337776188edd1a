"""FP64 CPU oracle of the EC electrostatic PIC/MCC step (arXiv:1310.5284).

TEST INFRASTRUCTURE ONLY.  Only the tests, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` import this package.  It wraps the plain C
oracle in ``pic_oracle.c`` with ctypes; it shares no code with the GPU library.

Readings of the paper that the oracle takes (Sec. II, Eqs. (2)-(3); Sec. III):
linear S_1 charge weighting at the nodes, own-cell (S_0) interpolation of the
half-grid field for the EC scheme, CIC of the averaged nodal field for the MC
scheme, leap-frog explicit push, D1 direct-implicit push with beta = 1/2,
null-collision MCC.  Parity pins for every function live in ``tests/``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pic_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

EXPLICIT, IMPLICIT = 0, 1
BC_DIRICHLET, BC_PERIODIC = 0, 1
GATHER_EC, GATHER_MC, GATHER_EC2 = 0, 1, 2
ELASTIC, EXCITATION, IONIZATION, CHARGE_EXCHANGE = 0, 1, 2, 3


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into oracle/liboracle.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".%d.tmp" % os.getpid()   # concurrent test workers each build
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Case(C.Structure):
    _fields_ = [("n_cells", C.c_int32), ("bc", C.c_int32), ("scheme", C.c_int32),
                ("gather", C.c_int32), ("collisions", C.c_int32), ("ion_subcycle", C.c_int32),
                ("gap_m", C.c_double), ("dt_s", C.c_double), ("step0", C.c_int64),
                ("rf_volts", C.c_double), ("rf_freq_hz", C.c_double),
                ("gas_density_m3", C.c_double), ("gas_temp_K", C.c_double),
                ("gas_mass_kg", C.c_double), ("background_rho", C.c_double),
                ("opal_B_eV", C.c_double), ("seed", C.c_uint64),
                ("cell_dx_m", C.POINTER(C.c_double))]


class Ledger(C.Structure):
    _fields_ = [("K_before", C.c_double * 2), ("K_after", C.c_double * 2),
                ("work", C.c_double * 2), ("coll_dK", C.c_double * 2),
                ("absorbed_K", (C.c_double * 2) * 2), ("WE", C.c_double),
                ("absorbed_n", (C.c_int64 * 2) * 2), ("n_coll", (C.c_int64 * 4) * 2),
                ("n_candidates", C.c_int64 * 2), ("n_created", C.c_int64 * 2),
                ("n_over_table", C.c_int64 * 2)]

    def as_dict(self) -> dict:
        return {
            "K_before": np.array(self.K_before[:]), "K_after": np.array(self.K_after[:]),
            "work": np.array(self.work[:]), "coll_dK": np.array(self.coll_dK[:]),
            "absorbed_K": np.array([list(r) for r in self.absorbed_K]),
            "WE": float(self.WE),
            "absorbed_n": np.array([list(r) for r in self.absorbed_n]),
            "n_coll": np.array([list(r) for r in self.n_coll]),
            "n_candidates": np.array(self.n_candidates[:]),
            "n_created": np.array(self.n_created[:]),
            "n_over_table": np.array(self.n_over_table[:]),
        }


_lib = None
_D = C.POINTER(C.c_double)
_U64 = C.POINTER(C.c_uint64)
_U32 = C.POINTER(C.c_uint32)
_I64 = C.POINTER(C.c_int64)


def lib():
    global _lib
    if _lib is None:
        # PIC_ORACLE_LIB: another build of the oracle's source (the mutation
        # test loads copies with planted mistakes this way)
        path = os.environ.get("PIC_ORACLE_LIB")
        if not path:
            path = _LIB
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
        L = C.CDLL(path)
        L.orc_philox4x32_10.argtypes = [_U32, _U32, _U32]
        L.orc_u01.argtypes = [C.c_uint32]
        L.orc_u01.restype = C.c_double
        L.orc_deposit_linear.argtypes = [C.c_int32, C.c_int32, C.c_int64, _D, _D]
        L.orc_count_cells.argtypes = [C.c_int32, C.c_int64, _D, _D]
        L.orc_solve_dirichlet.argtypes = [C.c_int32, C.c_double, _D, _D, C.c_double,
                                          C.c_double, _D, _D]
        L.orc_solve_periodic.argtypes = [C.c_int32, C.c_double, _D, _D, _D, _D]
        L.orc_solve_dirichlet_nu.argtypes = [C.c_int32, _D, _D, _D, C.c_double, C.c_double,
                                             _D, _D]
        L.orc_gather_ec.argtypes = [C.c_int32, _D, C.c_double]
        L.orc_gather_ec.restype = C.c_double
        L.orc_gather_mc.argtypes = [C.c_int32, C.c_int32, _D, C.c_double]
        L.orc_deposit_quadratic.argtypes = [C.c_int32, C.c_int32, C.c_int64, _D, _D]
        L.orc_gather_ec2.argtypes = [C.c_int32, C.c_int32, _D, C.c_double]
        L.orc_gather_ec2.restype = C.c_double
        L.orc_chi_weights_ec2.argtypes = [C.c_int32, C.c_int32, C.c_int64, _D, _D]
        L.orc_chi_operator_ec2.argtypes = [C.c_int32, C.c_int32, C.c_int64, _D, _D, _D]
        L.orc_solve_chi_tridiag.argtypes = [C.c_int32, C.c_int32, C.c_double, _D, _D, _D,
                                            C.c_double, _D, _D]
        L.orc_chi_operator_ec2_nu.argtypes = [C.c_int32, _D, C.c_double, C.c_int64, _D, _D, _D]
        L.orc_solve_chi_tridiag_nu.argtypes = [C.c_int32, _D, C.c_double, _D, _D, _D,
                                               C.c_double, _D, _D]
        L.orc_gather_mc_nu.argtypes = [C.c_int32, _D, _D, C.c_double]
        L.orc_gather_mc_nu.restype = C.c_double
        L.orc_gather_ec2_nu.argtypes = [C.c_int32, _D, _D, C.c_double]
        L.orc_gather_ec2_nu.restype = C.c_double
        L.orc_gather_mc.restype = C.c_double
        L.orc_create.argtypes = [C.POINTER(Case)]
        L.orc_create.restype = C.c_void_p
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_set_species.argtypes = [C.c_void_p, C.c_int32, C.c_double, C.c_double,
                                      C.c_double, C.c_int64, _D, _D, _D, _D, _D, _U64, _I64]
        L.orc_add_process.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_double,
                                      C.c_double, C.c_double, C.c_int32, _D]
        L.orc_prepare.argtypes = [C.c_void_p]
        L.orc_implicit_startup.argtypes = [C.c_void_p]
        L.orc_compute_fields.argtypes = [C.c_void_p]
        L.orc_step.argtypes = [C.c_void_p, C.c_int64]
        L.orc_step_with_field.argtypes = [C.c_void_p, _D]
        L.orc_count.argtypes = [C.c_void_p, C.c_int32]
        L.orc_count.restype = C.c_int64
        L.orc_step_index.argtypes = [C.c_void_p]
        L.orc_step_index.restype = C.c_int64
        L.orc_get_species.argtypes = [C.c_void_p, C.c_int32, _D, _D, _D, _D, _D, _U64, _I64]
        L.orc_mcc_wait_step.argtypes = [C.c_void_p, C.c_int32, C.c_uint64, C.c_int64, _I64]
        L.orc_mcc_wait_step.restype = C.c_int
        L.orc_mcc_first_wait.argtypes = [C.c_void_p, C.c_int32, C.c_uint64, C.c_int64]
        L.orc_mcc_first_wait.restype = C.c_int64
        L.orc_get_fields.argtypes = [C.c_void_p, _D, _D, _D, _D, _D, _D, _D, _D]
        L.orc_get_ledger.argtypes = [C.c_void_p, C.POINTER(Ledger)]
        L.orc_get_heating.argtypes = [C.c_void_p, _D, _D]
        L.orc_numax.argtypes = [C.c_void_p, C.c_int32]
        L.orc_numax.restype = C.c_double
        L.orc_collide_one.argtypes = [C.c_void_p, C.c_int32, C.c_uint64, C.c_int64, _D, _D,
                                      _D, C.POINTER(C.c_int)]
        L.orc_collide_one.restype = C.c_int
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(_D) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------------------
# building blocks
# ---------------------------------------------------------------------------
def philox4x32_10(ctr, key) -> np.ndarray:
    c = (C.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (C.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return np.array(o[:], dtype=np.uint32)


def u01(r: int) -> float:
    return lib().orc_u01(int(r) & 0xFFFFFFFF)


def deposit_linear(N: int, xi, periodic: bool = False) -> np.ndarray:
    xi = _f64(xi)
    Q = np.zeros(N + 1)
    lib().orc_deposit_linear(N, int(periodic), xi.size, _dp(xi), _dp(Q))
    return Q


def deposit_quadratic(N: int, xi, periodic: bool = False) -> np.ndarray:
    xi = _f64(xi)
    Q = np.zeros(N + 1)
    lib().orc_deposit_quadratic(N, int(periodic), xi.size, _dp(xi), _dp(Q))
    return Q


def count_cells(N: int, xi) -> np.ndarray:
    xi = _f64(xi)
    c = np.zeros(N)
    lib().orc_count_cells(N, xi.size, _dp(xi), _dp(c))
    return c


def solve_dirichlet(N, dx, rho, phi0, phiN, chi=None):
    rho = _f64(rho)
    chi = None if chi is None else _f64(chi)
    phi = np.zeros(N + 1)
    E = np.zeros(N)
    lib().orc_solve_dirichlet(N, dx, _dp(rho), _dp(chi), phi0, phiN, _dp(phi), _dp(E))
    return phi, E


def solve_dirichlet_nu(w, sigma, phi0, phiN, chi=None):
    w, sigma = _f64(w), _f64(sigma)
    chi = None if chi is None else _f64(chi)
    N = w.size
    phi = np.zeros(N + 1)
    E = np.zeros(N)
    lib().orc_solve_dirichlet_nu(N, _dp(w), _dp(sigma), _dp(chi), phi0, phiN, _dp(phi), _dp(E))
    return phi, E


def solve_periodic(N, dx, rho, chi=None):
    rho = _f64(rho)
    chi = None if chi is None else _f64(chi)
    phi = np.zeros(N + 1)
    E = np.zeros(N)
    lib().orc_solve_periodic(N, dx, _dp(rho), _dp(chi), _dp(phi), _dp(E))
    return phi, E


def gather_ec(N, E, xi) -> float:
    E = _f64(E)
    return lib().orc_gather_ec(N, _dp(E), float(xi))


def gather_mc(N, E, xi, periodic=False) -> float:
    E = _f64(E)
    return lib().orc_gather_mc(N, int(periodic), _dp(E), float(xi))


def gather_ec2(N, E, xi, periodic=False) -> float:
    E = _f64(E)
    return lib().orc_gather_ec2(N, int(periodic), _dp(E), float(xi))


def gather_mc_nu(w, E, xi) -> float:
    w, E = _f64(w), _f64(E)
    return lib().orc_gather_mc_nu(w.size, _dp(w), _dp(E), float(xi))


def gather_ec2_nu(w, E, xi) -> float:
    w, E = _f64(w), _f64(E)
    return lib().orc_gather_ec2_nu(w.size, _dp(w), _dp(E), float(xi))


def chi_weights_ec2(N: int, xi, periodic: bool = False) -> np.ndarray:
    xi = _f64(xi)
    w = np.zeros(N)
    lib().orc_chi_weights_ec2(N, int(periodic), xi.size, _dp(xi), _dp(w))
    return w


def chi_operator_ec2(N: int, xi, periodic: bool = False):
    """The m = 2 susceptibility operator (orc_chi_operator_ec2): its
    diagonal and its couplings of centres j, j + 1 (the last: the wrap)."""
    xi = _f64(xi)
    d, o = np.zeros(N), np.zeros(N)
    lib().orc_chi_operator_ec2(N, int(periodic), xi.size, _dp(xi), _dp(d), _dp(o))
    return d, o


def chi_operator_ec2_nu(w, xi):
    """The m = 2 operator on a nonuniform grid of widths w
    (orc_chi_operator_ec2_nu)."""
    w, xi = _f64(w), _f64(xi)
    N = w.size
    d, o = np.zeros(N), np.zeros(N)
    lib().orc_chi_operator_ec2_nu(N, _dp(w), float(w.sum() / N), xi.size, _dp(xi), _dp(d),
                                  _dp(o))
    return d, o


def solve_chi_tridiag_nu(w, sigma, xd, xo, phi0: float = 0.0):
    """Field solve with a tridiagonal susceptibility on a nonuniform grid
    (orc_solve_chi_tridiag_nu): returns (phi, E)."""
    w, sigma, xd, xo = _f64(w), _f64(sigma), _f64(xd), _f64(xo)
    N = w.size
    phi, E = np.zeros(N + 1), np.zeros(N)
    lib().orc_solve_chi_tridiag_nu(N, _dp(w), float(w.sum() / N), _dp(sigma), _dp(xd), _dp(xo),
                                   phi0, _dp(phi), _dp(E))
    return phi, E


def solve_chi_tridiag(N: int, dx: float, rho, xd, xo, phi0: float = 0.0,
                      periodic: bool = False):
    """Field solve with a tridiagonal susceptibility (orc_solve_chi_tridiag):
    returns (phi, E)."""
    rho, xd, xo = _f64(rho), _f64(xd), _f64(xo)
    phi, E = np.zeros(N + 1), np.zeros(N)
    lib().orc_solve_chi_tridiag(N, int(periodic), dx, _dp(rho), _dp(xd), _dp(xo), phi0,
                                _dp(phi), _dp(E))
    return phi, E


# ---------------------------------------------------------------------------
# simulation object
# ---------------------------------------------------------------------------
class Sim:
    """One discharge held by the oracle (FP64, single thread)."""

    def __init__(self, case: dict, species: list, processes: list, startup: bool = True):
        c = Case(n_cells=case["n_cells"], bc=case.get("bc", 0), scheme=case.get("scheme", 0),
                 gather=case.get("gather", 0), collisions=case.get("collisions", 0),
                 ion_subcycle=case.get("ion_subcycle", 0),
                 gap_m=case["gap_m"], dt_s=case["dt_s"], step0=case.get("step0", 0),
                 rf_volts=case.get("rf_volts", 0.0), rf_freq_hz=case.get("rf_freq_hz", 0.0),
                 gas_density_m3=case.get("gas_density_m3", 0.0),
                 gas_temp_K=case.get("gas_temp_K", 300.0),
                 gas_mass_kg=case.get("gas_mass_kg", 1.0),
                 background_rho=case.get("background_rho", 0.0),
                 opal_B_eV=case.get("opal_B_eV", 10.0), seed=case.get("seed", 0))
        cdx = case.get("cell_dx")
        self._cdx = None if cdx is None else _f64(cdx)   # held while orc_create copies it
        c.cell_dx_m = _dp(self._cdx)
        self.case = dict(case)
        self.N = int(case["n_cells"])
        self.dx = case["gap_m"] / self.N
        self._h = lib().orc_create(C.byref(c))
        if not self._h:
            raise ValueError("oracle rejected the case")
        for k, sp in enumerate(species):
            xi = _f64(sp["xi"])
            n = xi.size
            ab = sp.get("abar")
            ab = None if ab is None else _f64(ab)
            ids = np.ascontiguousarray(sp["id"], dtype=np.uint64)
            vx, vy, vz = _f64(sp["vx"]), _f64(sp["vy"]), _f64(sp["vz"])
            wt = sp.get("wait")
            wt = None if wt is None else np.ascontiguousarray(wt, dtype=np.int64)
            rc = lib().orc_set_species(self._h, k, sp["q"], sp["m"], sp["w"], n, _dp(xi),
                                       _dp(vx), _dp(vy), _dp(vz), _dp(ab),
                                       ids.ctypes.data_as(_U64),
                                       None if wt is None else wt.ctypes.data_as(_I64))
            if rc:
                raise ValueError("bad species")
        self.q = [sp["q"] for sp in species]
        self.m = [sp["m"] for sp in species]
        self.w = [sp["w"] for sp in species]
        for pr in processes:
            sig = _f64(pr["sigma"])
            rc = lib().orc_add_process(self._h, pr["species"], pr["kind"], pr["threshold_eV"],
                                       pr["e0_eV"], pr["de_eV"], sig.size, _dp(sig))
            if rc:
                raise ValueError("bad process")
        if lib().orc_prepare(self._h):
            raise ValueError("inconsistent cross-section tables")
        if startup and case.get("scheme", 0) == IMPLICIT:
            lib().orc_implicit_startup(self._h)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_destroy(h)
            self._h = None

    def step(self, n: int = 1):
        lib().orc_step(self._h, n)

    def step_with_field(self, E):
        E = _f64(E)
        if E.size != self.N:
            raise ValueError("field must have N values")
        lib().orc_step_with_field(self._h, _dp(E))

    def compute_fields(self):
        lib().orc_compute_fields(self._h)

    @property
    def step_index(self) -> int:
        return lib().orc_step_index(self._h)

    def count(self, sp: int) -> int:
        return lib().orc_count(self._h, sp)

    def numax(self, sp: int) -> float:
        return lib().orc_numax(self._h, sp)

    def species(self, sp: int) -> dict:
        n = self.count(sp)
        out = {k: np.zeros(n) for k in ("xi", "vx", "vy", "vz", "abar")}
        ids = np.zeros(n, dtype=np.uint64)
        wt = np.zeros(n, dtype=np.int64)
        lib().orc_get_species(self._h, sp, _dp(out["xi"]), _dp(out["vx"]), _dp(out["vy"]),
                              _dp(out["vz"]), _dp(out["abar"]), ids.ctypes.data_as(_U64),
                              wt.ctypes.data_as(_I64))
        out["id"] = ids
        out["wait"] = wt
        return out

    def fields(self) -> dict:
        N = self.N
        f = {k: np.zeros(N + 1) for k in ("rho", "phi", "Qe", "Qi")}
        f.update({k: np.zeros(N) for k in ("E", "chi", "cnt_e", "cnt_i")})
        lib().orc_get_fields(self._h, _dp(f["rho"]), _dp(f["phi"]), _dp(f["E"]), _dp(f["chi"]),
                             _dp(f["Qe"]), _dp(f["Qi"]), _dp(f["cnt_e"]), _dp(f["cnt_i"]))
        return f

    def ledger(self) -> dict:
        L = Ledger()
        lib().orc_get_ledger(self._h, C.byref(L))
        return L.as_dict()

    def heating(self):
        he, hi = np.zeros(self.N), np.zeros(self.N)
        lib().orc_get_heating(self._h, _dp(he), _dp(hi))
        return he, hi

    def wait_step(self, sp: int, pid: int, step: int, wait: int):
        """One step of the candidacy rule: (is_candidate, new wait)."""
        w = C.c_int64(int(wait))
        r = lib().orc_mcc_wait_step(self._h, sp, pid, step, C.byref(w))
        return bool(r), int(w.value)

    def first_wait(self, sp: int, pid: int, step: int) -> int:
        """The wait of a particle whose first trial is at `step`."""
        return int(lib().orc_mcc_first_wait(self._h, sp, pid, step))

    def collide_one(self, sp: int, pid: int, step: int, v):
        v = _f64(v).copy()
        ve, vi = np.zeros(3), np.zeros(3)
        over = C.c_int(0)
        r = lib().orc_collide_one(self._h, sp, pid, step, _dp(v), _dp(ve), _dp(vi),
                                  C.byref(over))
        return r, v, ve, vi, bool(over.value)
