"""Python binding of libpicmcc.so, the MI355X (gfx950) hot path of the
energy-conserving electrostatic PIC/MCC method of arXiv:1310.5284.

Argument marshalling only: every step of the method runs in the HIP kernels
behind the C-ABI declared in include/pic.h.  The library owns its device
memory and, unless a raw hipStream_t handle is passed, its own HIP stream.
This module does not import torch: the ROCm torch wheel bundles a second HIP
runtime, and two runtimes in one process do not share streams or memory.
There is no CPU fallback: if the library or a GPU is missing the constructor
raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpicmcc.so")

PIC_OK, PIC_E_INVAL, PIC_E_NOMEM, PIC_E_CAPACITY = 0, -1, -2, -3
PIC_E_UNSTABLE, PIC_E_DEVICE, PIC_E_STATE, PIC_E_DIVERGED = -4, -5, -6, -7
EXPLICIT, IMPLICIT = 0, 1
FLAG_ALLOW_UNSTABLE, FLAG_INTERNAL_UNITS = 1, 2
DIAG_FIELDS, DIAG_LEDGER, DIAG_STATE, DIAG_DENSITY, DIAG_HEATING, DIAG_EEDF = 1, 2, 4, 8, 16, 32
ERRORS = {0: "PIC_OK", -1: "PIC_E_INVAL", -2: "PIC_E_NOMEM", -3: "PIC_E_CAPACITY",
          -4: "PIC_E_UNSTABLE", -5: "PIC_E_DEVICE", -6: "PIC_E_STATE", -7: "PIC_E_DIVERGED"}
EEDF_BINS = 256

_P = C.c_void_p
_D = C.POINTER(C.c_double)
_I64 = C.POINTER(C.c_int64)


class CaseConfig(C.Structure):
    _fields_ = [("n_cells", C.c_int32), ("bc", C.c_int32), ("scheme", C.c_int32),
                ("gather", C.c_int32), ("collisions", C.c_int32), ("history_steps", C.c_int32),
                ("gap_m", C.c_double), ("dt_s", C.c_double), ("start_step", C.c_int64),
                ("rf_volts", C.c_double), ("rf_freq_hz", C.c_double),
                ("gas_density_m3", C.c_double), ("gas_temp_K", C.c_double),
                ("gas_mass_kg", C.c_double), ("background_rho", C.c_double),
                ("opal_B_eV", C.c_double), ("seed", C.c_uint64),
                ("cell_dx_m", C.POINTER(C.c_double)), ("ion_subcycle", C.c_int32),
                ("reserved", C.c_int32)]


# null-collision waiting-time word: count (17 bits) | capped flag
WAIT_MAX = 0x1FFFF
WAIT_CAPPED = 0x20000


class SpeciesInit(C.Structure):
    _fields_ = [("q_C", C.c_double), ("m_kg", C.c_double), ("weight", C.c_double),
                ("n", C.c_int64), ("capacity", C.c_int64), ("cell", _P), ("off", _P),
                ("vx", _P), ("vy", _P), ("vz", _P), ("id", _P), ("abar", _P),
                ("mcc_wait", _P)]


class Xsec(C.Structure):
    _fields_ = [("species", C.c_int32), ("kind", C.c_int32), ("threshold_eV", C.c_double),
                ("e0_eV", C.c_double), ("de_eV", C.c_double), ("n", C.c_int32),
                ("sigma_m2", _P)]


class Ledger(C.Structure):
    _fields_ = [("step", C.c_int64), ("K_before", C.c_double * 2), ("K_after", C.c_double * 2),
                ("work", C.c_double * 2), ("coll_dK", C.c_double * 2),
                ("absorbed_K", (C.c_double * 2) * 2), ("WE", C.c_double),
                ("absorbed_n", (C.c_int64 * 2) * 2), ("n_coll", (C.c_int64 * 4) * 2),
                ("n_candidates", C.c_int64 * 2), ("n_created", C.c_int64 * 2),
                ("n_over_table", C.c_int64 * 2), ("n_lost", C.c_int64 * 2)]

    def as_dict(self) -> dict:
        return {
            "step": int(self.step),
            "K_before": np.array(self.K_before[:]), "K_after": np.array(self.K_after[:]),
            "work": np.array(self.work[:]), "coll_dK": np.array(self.coll_dK[:]),
            "absorbed_K": np.array([list(r) for r in self.absorbed_K]), "WE": float(self.WE),
            "absorbed_n": np.array([list(r) for r in self.absorbed_n]),
            "n_coll": np.array([list(r) for r in self.n_coll]),
            "n_candidates": np.array(self.n_candidates[:]),
            "n_created": np.array(self.n_created[:]),
            "n_over_table": np.array(self.n_over_table[:]), "n_lost": np.array(self.n_lost[:]),
        }


class Diag(C.Structure):
    _fields_ = [("step", C.c_int64), ("n_particles", C.c_int64 * 2), ("n_slots", C.c_int64 * 2),
                ("vel_unit", C.c_double), ("acc_unit", C.c_double),
                ("rho", _P), ("phi", _P), ("E", _P), ("chi", _P), ("qfix", _P * 2),
                ("cell_count", _P * 2), ("ledger", Ledger), ("history", _P),
                ("history_cap", C.c_int64), ("history_n", C.c_int64),
                ("state_cap", C.c_int64 * 2), ("cell", _P * 2), ("off", _P * 2), ("vx", _P * 2),
                ("vy", _P * 2), ("vz", _P * 2), ("id", _P * 2), ("abar", _P * 2),
                ("mcc_wait", _P * 2),
                ("density", _P * 2), ("density_samples", C.c_int64), ("heating", _P * 2),
                ("eedf_bins", C.c_int32), ("eedf_bin_eV", C.c_double), ("eedf", _P),
                ("eedf_samples", C.c_int64)]


_lib = None


def lib():
    """Load libpicmcc.so (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() "
                               "or python paper_1310_5284_amd/build.py")
        L = C.CDLL(LIB_PATH)
        L.pic_init.argtypes = [C.POINTER(C.c_void_p), C.c_int32, C.POINTER(CaseConfig),
                               C.POINTER(SpeciesInit), C.POINTER(Xsec), C.c_int32, _P, C.c_uint32]
        L.pic_step_explicit.argtypes = [_P, C.c_int64]
        L.pic_step_implicit.argtypes = [_P, C.c_int64]
        L.pic_step.argtypes = [_P, C.c_int64]
        L.pic_step_noalloc.argtypes = [_P, C.c_int64]
        L.pic_diagnostics.argtypes = [_P, C.c_int32, C.c_uint32, C.POINTER(Diag)]
        L.pic_set_schedule.argtypes = [_P, C.c_int32, C.c_int32, C.c_int32]
        L.pic_set_launch.argtypes = [_P, C.c_int32, C.c_int32]
        L.pic_set_store_policy.argtypes = [_P, C.c_int32]
        L.pic_autotune.argtypes = [_P, C.POINTER(C.c_int32), C.c_int32, C.POINTER(C.c_int32),
                                   C.c_int32, C.c_int32, C.POINTER(C.c_int32),
                                   C.POINTER(C.c_int32), _D]
        L.pic_reset_accumulators.argtypes = [_P]
        L.pic_fp64_reference_init.argtypes = [_P]
        L.pic_fp64_reference_step.argtypes = [_P, C.c_int64]
        L.pic_fp64_reference_state.argtypes = [_P, C.c_int32, C.c_int32, C.c_int64, _D, _D, _D,
                                               _D, _D, C.POINTER(C.c_uint64), _I64]
        L.pic_fp64_reference_ledger.argtypes = [_P, C.c_int32, C.POINTER(Ledger)]
        L.pic_copy_calibration.argtypes = [C.c_int64, C.c_int32, _D]
        L.pic_destroy.argtypes = [_P]
        L.pic_destroy.restype = None
        L.pic_last_error.argtypes = [_P]
        L.pic_last_error.restype = C.c_char_p
        L.pic_last_timing.argtypes = [_P, _D, _I64]
        L.pic_last_timing_collide.argtypes = [_P, _D, _I64]
        _lib = L
    return _lib


class PicError(RuntimeError):
    def __init__(self, code, msg=""):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


# ---------------------------------------------------------------------------
# One Python function per entry point of include/pic.h, under the same name:
# argument marshalling only; a non-zero return code raises PicError with the
# context's last error text.
# ---------------------------------------------------------------------------
def _ok(h, rc, what):
    if rc != PIC_OK:
        msg = lib().pic_last_error(h) if h else None
        raise PicError(rc, f"{what}: {msg.decode() if msg else ''}")


def pic_last_error(h):
    msg = lib().pic_last_error(h)
    return msg.decode() if msg else ""


def pic_init(cases, species, xs, n_xs, stream=None, flags=0):
    """cases: CaseConfig array, species: SpeciesInit array (2 per case), xs:
    Xsec array with n_xs entries.  Returns the context handle."""
    h = C.c_void_p()
    rc = lib().pic_init(C.byref(h), len(cases), cases, species, xs, int(n_xs), stream,
                        int(flags))
    if rc != PIC_OK:
        raise PicError(rc, "pic_init failed")
    return h


def pic_destroy(h):
    lib().pic_destroy(h)


def pic_step_explicit(h, n):
    _ok(h, lib().pic_step_explicit(h, int(n)), "pic_step_explicit")


def pic_step_implicit(h, n):
    _ok(h, lib().pic_step_implicit(h, int(n)), "pic_step_implicit")


def pic_step(h, n):
    _ok(h, lib().pic_step(h, int(n)), "pic_step")


def pic_step_noalloc(h, n):
    """pic_step with no allocation: host launches, the per-step scratch in the
    library's fixed device array."""
    _ok(h, lib().pic_step_noalloc(h, int(n)), "pic_step_noalloc")


def pic_diagnostics(h, case, mask, diag):
    """Fills the Diag structure `diag` (its pointers name the caller's buffers)."""
    _ok(h, lib().pic_diagnostics(h, int(case), int(mask), C.byref(diag)), "pic_diagnostics")
    return diag


def pic_set_schedule(h, sort_every, diag_every, tile):
    _ok(h, lib().pic_set_schedule(h, int(sort_every), int(diag_every), int(tile)),
        "pic_set_schedule")


def pic_set_launch(h, graph, timing_every):
    _ok(h, lib().pic_set_launch(h, int(graph), int(timing_every)), "pic_set_launch")


def pic_set_store_policy(h, nontemporal):
    _ok(h, lib().pic_set_store_policy(h, int(nontemporal)), "pic_set_store_policy")


def pic_autotune(h, tiles=None, sorts=None, steps_per_trial=32):
    """Returns (tile, sort_every, device ms per step of each trial; the
    last two are the store policies 0 and 1)."""
    def arr(v):
        return (None, 0) if v is None else ((C.c_int32 * len(v))(*v), len(v))
    t, nt = arr(tiles)
    so, ns = arr(sorts)
    n_ms = (nt if tiles is not None else 6) + (ns if sorts is not None else 4) + 2
    ms = (C.c_double * n_ms)()
    tile, sort = C.c_int32(0), C.c_int32(0)
    _ok(h, lib().pic_autotune(h, t, nt, so, ns, int(steps_per_trial), C.byref(tile),
                              C.byref(sort), ms), "pic_autotune")
    return tile.value, sort.value, list(ms)


def pic_reset_accumulators(h):
    _ok(h, lib().pic_reset_accumulators(h), "pic_reset_accumulators")


def pic_fp64_reference_init(h):
    _ok(h, lib().pic_fp64_reference_init(h), "pic_fp64_reference_init")


def pic_fp64_reference_step(h, n):
    _ok(h, lib().pic_fp64_reference_step(h, int(n)), "pic_fp64_reference_step")


def pic_fp64_reference_state(h, case, species, cap):
    """Live particles of the FP64 form: xi (cells), v (cells/step), abar
    (cells/step^2), id."""
    a = {k: np.zeros(cap) for k in ("xi", "vx", "vy", "vz", "abar")}
    ids = np.zeros(cap, np.uint64)
    n = C.c_int64()
    _ok(h, lib().pic_fp64_reference_state(
        h, int(case), int(species), int(cap),
        *(a[k].ctypes.data_as(_D) for k in ("xi", "vx", "vy", "vz", "abar")),
        ids.ctypes.data_as(C.POINTER(C.c_uint64)), C.byref(n)), "pic_fp64_reference_state")
    k = n.value
    out = {key: v[:k].copy() for key, v in a.items()}
    out["id"] = ids[:k].copy()
    return out


def pic_fp64_reference_ledger(h, case):
    """The energy and particle ledger of the FP64 form's last step (dict)."""
    L = Ledger()
    _ok(h, lib().pic_fp64_reference_ledger(h, int(case), C.byref(L)),
        "pic_fp64_reference_ledger")
    return L.as_dict()


def pic_copy_calibration(nbytes, reps=10):
    """Milliseconds per copy of `nbytes` by the library's streaming copy kernel."""
    ms = C.c_double()
    rc = lib().pic_copy_calibration(int(nbytes), int(reps), C.byref(ms))
    if rc != PIC_OK:
        raise PicError(rc, "pic_copy_calibration")
    return ms.value


copy_calibration = pic_copy_calibration


def pic_last_timing(h):
    """(ms, launches) of the timed particle-pass launches of the last step call."""
    ms = C.c_double()
    k = C.c_int64()
    lib().pic_last_timing(h, C.byref(ms), C.byref(k))
    return ms.value, k.value


def pic_last_timing_collide(h):
    """(ms, launches) of the timed collision-kernel launches of the last step call."""
    ms = C.c_double()
    k = C.c_int64()
    lib().pic_last_timing_collide(h, C.byref(ms), C.byref(k))
    return ms.value, k.value


def _ptr(a):
    return None if a is None else a.ctypes.data


class PicContext:
    """A set of discharges advanced together by the GPU library.

    ``workloads`` is a list of workload dicts (see the ``workloads`` module):
    ``case`` parameters, two species with cell/off/vx/vy/vz/id arrays and the
    collision ``processes`` (shared by all cases).
    """

    def __init__(self, workloads, *, flags=0, history_steps=0, stream=None,
                 processes=None):
        self._keep = []
        n = len(workloads)
        cfgs = (CaseConfig * n)()
        sps = (SpeciesInit * (2 * n))()
        self.n_cells = []
        for k, wl in enumerate(workloads):
            c = wl["case"]
            cfgs[k] = CaseConfig(
                n_cells=c["n_cells"], bc=c.get("bc", 0), scheme=c.get("scheme", 0),
                gather=c.get("gather", 0), collisions=c.get("collisions", 0),
                history_steps=c.get("history_steps", history_steps), gap_m=c["gap_m"],
                dt_s=c["dt_s"], start_step=c.get("step0", 0), rf_volts=c.get("rf_volts", 0.0),
                rf_freq_hz=c.get("rf_freq_hz", 0.0), gas_density_m3=c.get("gas_density_m3", 0.0),
                gas_temp_K=c.get("gas_temp_K", 300.0), gas_mass_kg=c.get("gas_mass_kg", 1.0),
                background_rho=c.get("background_rho", 0.0), opal_B_eV=c.get("opal_B_eV", 10.0),
                seed=c.get("seed", 0), ion_subcycle=c.get("ion_subcycle", 0))
            cdx = c.get("cell_dx")
            if cdx is not None:
                cdx = np.ascontiguousarray(cdx, dtype=np.float64)
                self._keep.append(cdx)
                cfgs[k].cell_dx_m = cdx.ctypes.data_as(C.POINTER(C.c_double))
            self.n_cells.append(int(c["n_cells"]))
            for s, sp in enumerate(wl["species"]):
                arrs = {}
                for key, dt in (("cell", np.int32), ("off", np.float32), ("vx", np.float32),
                                ("vy", np.float32), ("vz", np.float32), ("id", np.uint64)):
                    arrs[key] = np.ascontiguousarray(sp[key], dtype=dt)
                ab = sp.get("abar")
                arrs["abar"] = None if ab is None else np.ascontiguousarray(ab, dtype=np.float32)
                wt = sp.get("mcc_wait")
                arrs["mcc_wait"] = None if wt is None else np.ascontiguousarray(wt, dtype=np.uint32)
                self._keep.append(arrs)
                nn = arrs["cell"].size
                sps[2 * k + s] = SpeciesInit(
                    q_C=sp["q"], m_kg=sp["m"], weight=sp["w"], n=nn,
                    capacity=max(int(sp.get("capacity", nn)), nn), cell=_ptr(arrs["cell"]),
                    off=_ptr(arrs["off"]), vx=_ptr(arrs["vx"]), vy=_ptr(arrs["vy"]),
                    vz=_ptr(arrs["vz"]), id=_ptr(arrs["id"]), abar=_ptr(arrs["abar"]),
                    mcc_wait=_ptr(arrs["mcc_wait"]))
        procs = processes if processes is not None else workloads[0].get("processes", [])
        xs = (Xsec * max(len(procs), 1))()
        for i, p in enumerate(procs):
            sig = np.ascontiguousarray(p["sigma"], dtype=np.float64)
            self._keep.append(sig)
            xs[i] = Xsec(species=p["species"], kind=p["kind"], threshold_eV=p["threshold_eV"],
                         e0_eV=p["e0_eV"], de_eV=p["de_eV"], n=sig.size, sigma_m2=sig.ctypes.data)
        try:
            self._h = pic_init(cfgs, sps, xs, len(procs), stream, flags)
        finally:
            self._keep = None
        self.n_cases = n
        self.schemes = [int(w["case"].get("scheme", 0)) for w in workloads]

    # ------------------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            pic_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n=1):
        pic_step(self._h, n)

    def step_noalloc(self, n=1):
        pic_step_noalloc(self._h, n)

    def step_explicit(self, n=1):
        pic_step_explicit(self._h, n)

    def step_implicit(self, n=1):
        pic_step_implicit(self._h, n)

    def set_schedule(self, sort_every=64, diag_every=0, tile=0):
        pic_set_schedule(self._h, sort_every, diag_every, tile)

    def set_launch(self, graph=0, timing_every=1):
        """Host launches (graph=0) or replay of a captured sort period
        (graph=1); HIP-event timing of every timing_every-th step."""
        pic_set_launch(self._h, graph, timing_every)

    def set_store_policy(self, nontemporal):
        """Store policy of the collision kernel: 0 cached (default), 1
        non-temporal; results are identical."""
        pic_set_store_policy(self._h, nontemporal)

    def autotune(self, tiles=None, sorts=None, steps_per_trial=32):
        """Pick the fastest tile, sort period and store policy by timing real
        steps; returns (tile, sort_every, ms per step of each trial, the two
        store policies last)."""
        return pic_autotune(self._h, tiles, sorts, steps_per_trial)

    def reset_accumulators(self):
        pic_reset_accumulators(self._h)

    def sync(self):
        """Wait for the context's stream (pic_diagnostics synchronises it)."""
        self._diag(0, 0, Diag())

    def last_timing(self):
        """(ms, launches) of the particle pass kernel over the last step call."""
        return pic_last_timing(self._h)

    def last_timing_collide(self):
        """(ms, launches) of the collision kernel over the last step call."""
        return pic_last_timing_collide(self._h)

    # ------------------------------------------------------------------
    def _diag(self, case, mask, d):
        return pic_diagnostics(self._h, case, mask, d)

    def counts(self, case=0):
        d = self._diag(case, 0, Diag())
        return dict(step=d.step, n=list(d.n_particles), n_slots=list(d.n_slots),
                    vel_unit=d.vel_unit, acc_unit=d.acc_unit)

    def fields(self, case=0):
        N = self.n_cells[case]
        out = {k: np.zeros(N + 1) for k in ("rho", "phi")}
        out.update({k: np.zeros(N) for k in ("E", "chi")})
        q = [np.zeros(N + 1, np.int64) for _ in range(2)]
        cc = [np.zeros(N, np.int64) for _ in range(2)]
        d = Diag()
        for k in ("rho", "phi", "E", "chi"):
            setattr(d, k, out[k].ctypes.data)
        for s in range(2):
            d.qfix[s] = q[s].ctypes.data
            d.cell_count[s] = cc[s].ctypes.data
        self._diag(case, DIAG_FIELDS, d)
        out["qfix"] = q
        out["cell_count"] = cc
        out["step"] = d.step
        return out

    def ledger(self, case=0):
        d = self._diag(case, DIAG_LEDGER, Diag())
        return d.ledger.as_dict()

    def history(self, case=0, cap=1 << 16):
        rows = (Ledger * cap)()
        d = Diag()
        d.history = C.cast(rows, C.c_void_p)
        d.history_cap = cap
        self._diag(case, DIAG_LEDGER, d)
        return [rows[i].as_dict() for i in range(d.history_n)]

    def state(self, case=0):
        c0 = self.counts(case)
        d = Diag()
        arrs = []
        for s in range(2):
            n = int(c0["n_slots"][s])
            a = dict(cell=np.zeros(n, np.int32), off=np.zeros(n, np.float32),
                     vx=np.zeros(n, np.float32), vy=np.zeros(n, np.float32),
                     vz=np.zeros(n, np.float32), id=np.zeros(n, np.uint64),
                     abar=np.zeros(n, np.float32), mcc_wait=np.zeros(n, np.uint32))
            arrs.append(a)
            d.state_cap[s] = n
            for k in ("cell", "off", "vx", "vy", "vz", "id", "abar", "mcc_wait"):
                getattr(d, k)[s] = a[k].ctypes.data
        self._diag(case, DIAG_STATE, d)
        out = []
        for s in range(2):
            n = int(d.n_particles[s])
            out.append({k: v[:n].copy() for k, v in arrs[s].items()})
        return dict(species=out, vel_unit=d.vel_unit, acc_unit=d.acc_unit, step=d.step)

    # ---- plain FP64 GPU form of the same explicit method ----------------
    def fp64_init(self):
        """Copy the current state into the plain FP64 form (explicit cases)."""
        pic_fp64_reference_init(self._h)

    def fp64_step(self, n=1):
        pic_fp64_reference_step(self._h, n)

    def fp64_state(self, case=0, species=0, cap=None):
        """Live particles of the FP64 form: xi (cells), v (cells/step), id."""
        if cap is None:
            cap = int(self.counts(case)["n_slots"][species]) * 2 + 1024
        return pic_fp64_reference_state(self._h, case, species, cap)

    def fp64_ledger(self, case=0):
        """The energy and particle ledger of the FP64 form's last step."""
        return pic_fp64_reference_ledger(self._h, case)

    def density(self, case=0):
        N = self.n_cells[case]
        a = [np.zeros(N + 1) for _ in range(2)]
        d = Diag()
        for s in range(2):
            d.density[s] = a[s].ctypes.data
        self._diag(case, DIAG_DENSITY, d)
        return a, d.density_samples

    def heating(self, case=0):
        N = self.n_cells[case]
        a = [np.zeros(N) for _ in range(2)]
        d = Diag()
        for s in range(2):
            d.heating[s] = a[s].ctypes.data
        self._diag(case, DIAG_HEATING, d)
        return a

    def eedf(self, case=0):
        h = np.zeros(EEDF_BINS, np.int64)
        d = Diag()
        d.eedf = h.ctypes.data
        self._diag(case, DIAG_EEDF, d)
        return h, d.eedf_bin_eV, d.eedf_samples
