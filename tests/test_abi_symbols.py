"""The C-ABI library loads on the CPU host and exports every function that
include/hdcg.h declares (no compute call is made without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = []
    for f in os.listdir(os.path.join(ROOT, "include")):
        if f.endswith(".h"):
            src = open(os.path.join(ROOT, "include", f)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names += re.findall(r"^\s*(?:const\s+)?[a-z_]+\s*\**\s*([a-z_0-9]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("dwf_create", "mpc_dag_mpc_apply", "cg_solve", "dwf_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_1402_2585_amd._lib import LIB_PATH

    lib = ctypes.CDLL(LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_errors_without_device_calls():
    """Argument validation happens before any device work."""
    import paper_1402_2585_amd as hd

    lib = hd.load()
    h = ctypes.c_void_p()
    dims = (ctypes.c_int * 4)(4, 4, 5, 4)  # odd extent
    rc = lib.dwf_create(ctypes.byref(h), ctypes.byref(dims), 8, 1.8, 0.01, ctypes.c_void_p(1), None, None)
    assert rc == -2 and b"even" in lib.dwf_last_error()
    dims = (ctypes.c_int * 4)(4, 4, 4, 4)
    rc = lib.dwf_create(ctypes.byref(h), ctypes.byref(dims), 0, 1.8, 0.01, ctypes.c_void_p(1), None, None)
    assert rc == -2
    assert lib.mpc_apply(None, None, None, 0, 0, 1, None) == -1


def test_param_struct_layout_matches_the_library():
    """hdcg_default_params (host code only) fills the ctypes mirror of
    struct hdcg_params with the defaults the header documents; a field out
    of step between the two layouts would read back as another value."""
    import paper_1402_2585_amd as hd

    p = hd.hdcg_default_params()
    want = dict(n_ii=0, maxiter_ii=500, n_irs=7, lambda_irs=1.0, coarse_tol=0.04, coarse_maxiter=2000, flexible=1,
                inner_tol=1e-5, inner_maxiter=500, outer_maxiter=50, build_batch=16, coarse_prec=hd.DWF_C64,
                verbose=0, irs_prec=hd.DWF_C64, subspace_gen=0, rat_lo=3e-4, rat_eps=1e-4, rat_tol=1e-6,
                rat_maxiter=10000, wall_noise=0, ldop_defl=1, phi_prec=hd.DWF_C64, ldop_m1=0, m1_lo=0.5,
                m1_hi=0.0, m1_order=16, m1_shift=0.0, surface_depth=0, coarse_persistent=1, graph=1,
                phase_timing=0, mfma_tile=-1, seed=1, keep_subspace_fp64=1, m1_prec=hd.DWF_C64)
    got = {k: getattr(p, k) for k in want}
    assert got == want


def test_stats_struct_size_matches_the_header():
    """The ctypes mirror of struct hdcg_stats has the header's layout: fixed
    fields, six phase times, then the two 64-entry per-RHS arrays."""
    import ctypes as C

    import paper_1402_2585_amd as hd
    from paper_1402_2585_amd._lib import HdcgStats

    assert C.sizeof(HdcgStats) == 6 * 4 + 6 * 8 + 2 * 4 + 6 * 8 + 64 * 8 + 64 * 8
    assert HdcgStats.coarse_iterations_rhs.offset % 8 == 0 and hd.HdcgError is not None
