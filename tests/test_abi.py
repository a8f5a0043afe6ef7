"""The C-ABI library loads on the host and exports every entry point that
include/mgr.h declares (no compute calls: no GPU here)."""
import ctypes
import os
import re

from conftest import ROOT


def declared_functions():
    text = open(os.path.join(ROOT, "include", "mgr.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mgr_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("mgr_setup", "mgr_solve", "mgr_destroy", "mgr_pattern_outer", "mgr_status_string",
                     "mgr_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_1801_08464_amd import binding as B
    L = B.load_library()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    assert sorted(B.EXPORTS) == declared_functions()


def test_host_only_entry_points():
    from paper_1801_08464_amd import binding as B
    o = B.default_options()
    assert (o.restart, o.max_iter, o.rp_type, o.global_relax, o.f_sweeps) == (30, 400, 0, 1, 1)
    assert (o.amg_theta, o.amg_pre, o.amg_post, o.amg_coarse_max) == (0.25, 2, 2, 64)
    assert (o.frelax_amg_mask, o.frelax_amg_pre, o.frelax_amg_post, o.cycle_post) == (0, 1, 1, 0)
    assert o.index16 == 1
    assert ctypes.sizeof(o) == 104
    assert B.status_string(B.E_ZERO_FDIAG) == "MGR_E_ZERO_FDIAG"
    assert B.status_string(B.NOT_CONVERGED) == "MGR_NOT_CONVERGED"
    # setup rejects bad arguments before touching the device
    csr = B.MgrCsr(0, 0, None, None, None)
    h = ctypes.c_void_p()
    assert B.load_library().mgr_setup(ctypes.byref(csr), 3, None, ctypes.byref(o), ctypes.byref(h)) == B.E_INVALID
    assert not h.value
    assert B.last_error(None)
    # the handle entry points reject a null handle before touching the device
    L = B.load_library()
    assert L.mgr_update_values(None, None) == B.E_INVALID
    assert L.mgr_solve(None, None, None, 1e-8, None) == B.E_INVALID
    assert L.mgr_apply_preconditioner(None, None, None) == B.E_INVALID
