"""CPU checks of the C-ABI library: it loads, exports every entry point that
include/pic.h declares, and its struct layouts match the Python binding."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "include", "pic.h")


def declared_functions():
    src = open(HDR).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pic_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    f = declared_functions()
    for name in ("pic_init", "pic_step_explicit", "pic_step_implicit", "pic_diagnostics",
                 "pic_step", "pic_destroy", "pic_last_error"):
        assert name in f


def test_library_exports_every_declared_symbol():
    import paper_1310_5284_amd as P
    L = P.lib()
    for name in declared_functions():
        assert hasattr(L, name), name


def test_binding_has_a_function_of_the_same_name_for_every_entry_point():
    import inspect

    import paper_1310_5284_amd as P
    for name in declared_functions():
        assert inspect.isfunction(getattr(P, name, None)), name


def test_struct_layouts_match_binding(tmp_path):
    import paper_1310_5284_amd as P
    prog = tmp_path / "sz.c"
    prog.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "pic.h"\n'
                    'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %u %u\\n",'
                    'sizeof(pic_case_config),sizeof(pic_species_init),sizeof(pic_xsec),'
                    'sizeof(pic_ledger),sizeof(pic_diag),offsetof(pic_diag,ledger),'
                    'offsetof(pic_diag,eedf_samples),offsetof(pic_diag,mcc_wait),'
                    'offsetof(pic_species_init,mcc_wait),PIC_WAIT_MAX,PIC_WAIT_CAPPED);'
                    'return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)])
    got = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    want = [C.sizeof(P.CaseConfig), C.sizeof(P.SpeciesInit), C.sizeof(P.Xsec),
            C.sizeof(P.Ledger), C.sizeof(P.Diag), P.Diag.ledger.offset,
            P.Diag.eedf_samples.offset, P.Diag.mcc_wait.offset, P.SpeciesInit.mcc_wait.offset,
            P.WAIT_MAX, P.WAIT_CAPPED]
    assert got == want


def test_init_rejects_bad_input_without_a_gpu():
    # argument validation happens before any device call
    import paper_1310_5284_amd as P
    L = P.lib()
    h = C.c_void_p()
    assert L.pic_init(C.byref(h), 0, None, None, None, 0, None, 0) == P.PIC_E_INVAL
    cfg = (P.CaseConfig * 1)()
    cfg[0].n_cells = 1          # N >= 2 required
    cfg[0].gap_m = 0.01
    cfg[0].dt_s = 1e-10
    sp = (P.SpeciesInit * 2)()
    for s in range(2):
        sp[s].m_kg = 1.0
    assert L.pic_init(C.byref(h), 1, cfg, sp, None, 0, None, 0) == P.PIC_E_INVAL
    # no weighting beyond m = 2
    cfg[0].n_cells = 8
    cfg[0].gather = 3
    assert L.pic_init(C.byref(h), 1, cfg, sp, None, 0, None, 0) == P.PIC_E_INVAL
    # capacity beyond what 32-bit record offsets reach
    cfg[0].gather = 0
    sp[0].capacity = (1 << 28) - 1023
    assert L.pic_init(C.byref(h), 1, cfg, sp, None, 0, None, 0) == P.PIC_E_INVAL
    sp[0].capacity = 0
    # nonuniform grids: EC gather between electrodes, positive widths summing
    # to the gap
    good = (C.c_double * 8)(*([0.01 / 8] * 8))
    cfg[0].bc = 1
    cfg[0].cell_dx_m = C.cast(good, C.POINTER(C.c_double))
    assert L.pic_init(C.byref(h), 1, cfg, sp, None, 0, None, 0) == P.PIC_E_INVAL
    cfg[0].bc = 0
    # m = 2 implicit on a nonuniform grid: its LDS words fit up to 4069 cells
    big = (C.c_double * 4070)(*([0.01 / 4070] * 4070))
    cfg[0].n_cells, cfg[0].scheme, cfg[0].gather = 4070, 1, 2
    cfg[0].cell_dx_m = C.cast(big, C.POINTER(C.c_double))
    assert L.pic_init(C.byref(h), 1, cfg, sp, None, 0, None, 0) == P.PIC_E_INVAL
    cfg[0].n_cells, cfg[0].scheme, cfg[0].gather = 8, 0, 0
    for widths in ([0.01 / 8] * 7 + [0.0], [0.01 / 7] * 8, [0.02] + [-0.01 / 7] * 7):
        arr = (C.c_double * 8)(*widths)
        cfg[0].cell_dx_m = C.cast(arr, C.POINTER(C.c_double))
        assert L.pic_init(C.byref(h), 1, cfg, sp, None, 0, None, 0) == P.PIC_E_INVAL
    cfg[0].cell_dx_m = None
    # ion subcycling: 0 <= K <= 4096
    for K, scheme in ((-1, 0), (4097, 0), (-1, 1)):
        cfg[0].ion_subcycle = K
        cfg[0].scheme = scheme
        assert L.pic_init(C.byref(h), 1, cfg, sp, None, 0, None, 0) == P.PIC_E_INVAL, K
    assert not h.value


def test_product_path_has_no_cpu_fallback():
    # the binding must not import the oracle
    src = open(os.path.join(ROOT, "paper_1310_5284_amd", "__init__.py")).read()
    assert "oracle" not in src.replace("no CPU fallback", "")
