"""ctypes binding of libhdcg.so: argument marshalling only.

Every function here has the name of the C entry point it calls and does no
arithmetic of its own: it checks that tensors live on the GPU and are
contiguous, passes their device addresses and torch's current stream, and
turns status codes into exceptions.  All compute runs in the HIP library.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhdcg.so")

DWF_OK, DWF_NOT_CONVERGED = 0, 1
DWF_C128, DWF_C64, DWF_BF16, DWF_F16 = 0, 1, 2, 3

_ERRORS = {
    -1: "DWF_ERR_ARG", -2: "DWF_ERR_GEOMETRY", -3: "DWF_ERR_HIP",
    -4: "DWF_ERR_OOM", -5: "DWF_ERR_STATE", -6: "DWF_ERR_NUMERIC",
}


class HdcgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_ERRORS.get(code, code)}: {msg}")
        self.code = code


class SolveStats(C.Structure):
    _fields_ = [("iterations", C.c_int), ("restarts", C.c_int), ("converged", C.c_int),
                ("true_residual", C.c_double), ("seconds", C.c_double), ("matmuls", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class HdcgParams(C.Structure):
    _fields_ = [("n_ii", C.c_int), ("lambda_ii", C.c_double), ("tol_ii", C.c_double),
                ("maxiter_ii", C.c_int), ("n_irs", C.c_int), ("lambda_irs", C.c_double),
                ("coarse_tol", C.c_double), ("coarse_maxiter", C.c_int), ("flexible", C.c_int),
                ("inner_tol", C.c_double), ("inner_maxiter", C.c_int), ("outer_maxiter", C.c_int),
                ("build_batch", C.c_int), ("coarse_prec", C.c_int), ("verbose", C.c_int),
                ("irs_prec", C.c_int), ("subspace_gen", C.c_int), ("rat_lo", C.c_double),
                ("rat_eps", C.c_double), ("rat_tol", C.c_double), ("rat_maxiter", C.c_int),
                ("wall_noise", C.c_int), ("ldop_defl", C.c_int), ("phi_prec", C.c_int),
                ("ldop_m1", C.c_int), ("m1_lo", C.c_double), ("m1_hi", C.c_double), ("m1_order", C.c_int),
                ("m1_shift", C.c_double), ("surface_depth", C.c_int), ("coarse_persistent", C.c_int),
                ("graph", C.c_int), ("phase_timing", C.c_int), ("mfma_tile", C.c_int), ("seed", C.c_ulonglong),
                ("keep_subspace_fp64", C.c_int), ("m1_prec", C.c_int)]


class HdcgStats(C.Structure):
    _fields_ = [("outer_iterations", C.c_int), ("inner_iterations", C.c_int),
                ("coarse_solves", C.c_int), ("coarse_iterations", C.c_int), ("converged", C.c_int),
                ("nrhs", C.c_int), ("true_residual", C.c_double), ("seconds", C.c_double),
                ("setup_seconds", C.c_double), ("matmuls_fp64", C.c_double), ("matmuls_fp32", C.c_double),
                ("matmuls_bf16", C.c_double), ("group_size", C.c_int), ("graph_replays", C.c_int),
                ("t_fine_dp", C.c_double), ("t_fine_sp", C.c_double), ("t_coarse", C.c_double),
                ("t_project_promote", C.c_double), ("t_linalg", C.c_double), ("t_convert", C.c_double),
                ("coarse_iterations_rhs", C.c_longlong * 64), ("true_residual_rhs", C.c_double * 64)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if not k.endswith("_rhs")}
        d["coarse_iterations_rhs"] = list(self.coarse_iterations_rhs[:self.nrhs])
        d["true_residual_rhs"] = list(self.true_residual_rhs[:self.nrhs])
        return d


_lib = None


def load():
    """Load the in-tree library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: run paper_1402_2585_amd.build.build() first")
    # PyTorch ships its own HIP runtime, which its libraries request under a
    # name the dynamic loader does not match to the system runtime's soname.
    # Loaded first, the library would bring in the system runtime and torch a
    # second one; with torch loaded first the library binds to torch's copy.
    import torch  # noqa: F401
    lib = C.CDLL(LIB_PATH)
    vp, i, d, sz = C.c_void_p, C.c_int, C.c_double, C.c_size_t
    dp = C.POINTER(C.c_double)
    sig = {
        "dwf_create": (i, [C.POINTER(vp), C.POINTER(C.c_int * 4), i, d, d, vp, dp, vp]),
        "dwf_create_mobius": (i, [C.POINTER(vp), C.POINTER(C.c_int * 4), i, d, d, d, d, vp, dp, vp]),
        "dwf_destroy": (i, [vp]),
        "dwf_set_hop_shape": (i, [vp, C.POINTER(C.c_int)]),
        "dwf_release_workspace": (i, [vp]),
        "dwf_tune_hop": (i, [vp, i, i, vp]),
        "dwf_get_hop_shape": (i, [vp, i, i, C.POINTER(C.c_int), C.POINTER(C.c_float), C.POINTER(C.c_int)]),
        "dwf_field_bytes": (i, [vp, i, i, C.POINTER(sz)]),
        "dwf_import": (i, [vp, vp, vp, i, i, vp]),
        "dwf_export": (i, [vp, vp, vp, i, i, vp]),
        "dwf_convert": (i, [vp, vp, i, vp, i, i, vp]),
        "mpc_apply": (i, [vp, vp, vp, i, i, i, vp]),
        "mpc_dag_mpc_apply": (i, [vp, vp, vp, i, i, vp]),
        "dwf_norm2": (i, [vp, dp, vp, i, i, vp]),
        "dwf_dot": (i, [vp, dp, vp, vp, i, i, vp]),
        "dwf_cg_update": (i, [vp, vp, vp, vp, vp, dp, dp, i, i, vp]),
        "dwf_xpay": (i, [vp, vp, vp, dp, i, i, vp]),
        "cg_solve": (i, [vp, vp, vp, i, d, i, C.POINTER(SolveStats), vp]),
        "cg_solve_mixed": (i, [vp, vp, vp, i, d, d, i, C.POINTER(SolveStats), vp]),
        "dwf_multishift_cg": (i, [vp, vp, vp, i, dp, i, d, i, C.POINTER(SolveStats), vp]),
        "dwf_last_error": (C.c_char_p, []),
        "hdcg_default_params": (None, [C.POINTER(HdcgParams)]),
        "hdcg_setup": (i, [C.POINTER(vp), vp, C.POINTER(C.c_int * 4), i, vp, C.POINTER(HdcgParams), vp]),
        "hdcg_destroy": (i, [vp]),
        "hdcg_dims": (i, [vp, C.POINTER(C.c_int * 4), C.POINTER(C.c_int), C.POINTER(C.c_int)]),
        "hdcg_project": (i, [vp, vp, vp, i, i, vp]),
        "hdcg_promote": (i, [vp, vp, vp, i, i, vp]),
        "coarse_apply": (i, [vp, vp, vp, i, i, vp]),
        "hdcg_coarse_solve": (i, [vp, vp, vp, i, i, d, i, C.POINTER(C.c_int), vp]),
        "hdcg_mirs": (i, [vp, vp, vp, i, vp]),
        "hdcg_set_params": (i, [vp, C.POINTER(HdcgParams), vp]),
        "hdcg_ldop_setup": (i, [vp, i, vp, d, i, d, vp]),
        "hdcg_export_ldop": (i, [vp, C.POINTER(C.c_int), vp, dp, vp]),
        "hdcg_trunc_apply": (i, [vp, vp, vp, i, i, vp]),
        "hdcg_m1_interval": (i, [vp, dp, dp, vp]),
        "hdcg_chebyshev": (i, [vp, vp, vp, i, i, vp]),
        "hdcg_trunc_cg": (i, [vp, vp, vp, i, i, vp]),
        "hdcg_adef1_precondition": (i, [vp, vp, vp, i, i, vp]),
        "hdcg_export_coarse": (i, [vp, vp, vp]),
        "hdcg_import_coarse": (i, [vp, vp, vp]),
        "hdcg_coarse_iterations": (i, [vp, C.POINTER(C.c_int), i]),
        "hdcg_mfma_tile": (i, [vp, i, i, C.POINTER(C.c_int), C.POINTER(C.c_float), C.POINTER(C.c_int), vp]),
        "hdcg_coarse_solve_noalloc": (i, [vp, vp, vp, i, i, d, i, C.POINTER(C.c_int), vp]),
        "hdcg_export_subspace": (i, [vp, vp, vp]),
        "hdcg_export_block_map": (i, [vp, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
        "hdcg_solve": (i, [vp, vp, vp, i, d, C.POINTER(HdcgStats), vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


# ------------------------------------------------------------- marshalling --
def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _check(rc, allow_soft=False):
    if rc < 0 or (rc > 0 and not allow_soft):
        raise HdcgError(rc, load().dwf_last_error().decode())
    return rc


def _dbl(values, n):
    arr = (C.c_double * n)(*[float(v) for v in np.broadcast_to(np.asarray(values, float), (n,))])
    return arr


# ------------------------------------------------------------ entry points --
def dwf_create(gauge, dims, Ls, M5, mass, bc=(1, 1, 1, -1), stream=None):
    h = C.c_void_p()
    d = (C.c_int * 4)(*[int(x) for x in dims])
    ph = _dbl([v for z in bc for v in (complex(z).real, complex(z).imag)], 8)
    _check(load().dwf_create(C.byref(h), C.byref(d), int(Ls), float(M5), float(mass), _ptr(gauge), ph,
                             _stream(stream)))
    return h


def dwf_create_mobius(gauge, dims, Ls, M5, mass, b5, c5, bc=(1, 1, 1, -1), stream=None):
    h = C.c_void_p()
    d = (C.c_int * 4)(*[int(x) for x in dims])
    ph = _dbl([v for z in bc for v in (complex(z).real, complex(z).imag)], 8)
    _check(load().dwf_create_mobius(C.byref(h), C.byref(d), int(Ls), float(M5), float(mass), float(b5), float(c5),
                                    _ptr(gauge), ph, _stream(stream)))
    return h


def dwf_destroy(op):
    _check(load().dwf_destroy(op))


def dwf_get_hop_shape(op, prec, nrhs=1):
    """(shape (10 ints), ms per candidate (-1: not tuned or not tried), tuned flag)."""
    sh = (C.c_int * 10)()
    ms = (C.c_float * 32)()
    n = C.c_int()
    rc = _check(load().dwf_get_hop_shape(op, int(prec), int(nrhs), sh, ms, C.byref(n)), allow_soft=True)
    return tuple(sh), list(ms[:n.value]), rc == 0


def dwf_tune_hop(op, prec, nrhs=1, stream=None):
    _check(load().dwf_tune_hop(op, int(prec), int(nrhs), _stream(stream)))


def dwf_release_workspace(op):
    _check(load().dwf_release_workspace(op))


def dwf_set_hop_shape(op, shape):
    """shape: 10 ints (bx, by, bz, bt, remap, lds_kb, nt, morton, phases, rg);
    9 take rg = 1."""
    v = [int(x) for x in shape] + ([1] if len(shape) == 9 else [])
    a = (C.c_int * 10)(*v)
    _check(load().dwf_set_hop_shape(op, a))


def dwf_field_bytes(op, prec, nrhs=1):
    n = C.c_size_t()
    _check(load().dwf_field_bytes(op, int(prec), int(nrhs), C.byref(n)))
    return n.value


def dwf_import(op, native, canonical, prec, nrhs=1, stream=None):
    _check(load().dwf_import(op, _ptr(native), _ptr(canonical), int(prec), int(nrhs), _stream(stream)))


def dwf_export(op, canonical, native, prec, nrhs=1, stream=None):
    _check(load().dwf_export(op, _ptr(canonical), _ptr(native), int(prec), int(nrhs), _stream(stream)))


def dwf_convert(op, dst, dst_prec, src, src_prec, nrhs=1, stream=None):
    _check(load().dwf_convert(op, _ptr(dst), int(dst_prec), _ptr(src), int(src_prec), int(nrhs),
                              _stream(stream)))


def mpc_apply(op, out, inp, prec, dagger=0, nrhs=1, stream=None):
    _check(load().mpc_apply(op, _ptr(out), _ptr(inp), int(prec), int(dagger), int(nrhs), _stream(stream)))


def mpc_dag_mpc_apply(op, out, inp, prec, nrhs=1, stream=None):
    _check(load().mpc_dag_mpc_apply(op, _ptr(out), _ptr(inp), int(prec), int(nrhs), _stream(stream)))


def dwf_norm2(op, x, prec, nrhs=1, stream=None):
    out = (C.c_double * nrhs)()
    _check(load().dwf_norm2(op, out, _ptr(x), int(prec), int(nrhs), _stream(stream)))
    return np.array(out[:])


def dwf_dot(op, a, b, prec, nrhs=1, stream=None):
    out = (C.c_double * (2 * nrhs))()
    _check(load().dwf_dot(op, out, _ptr(a), _ptr(b), int(prec), int(nrhs), _stream(stream)))
    v = np.array(out[:])
    return v[0::2] + 1j * v[1::2]


def dwf_cg_update(op, x, r, p, w, alpha, prec, nrhs=1, stream=None):
    rr = (C.c_double * nrhs)()
    _check(load().dwf_cg_update(op, _ptr(x), _ptr(r), _ptr(p), _ptr(w), _dbl(alpha, nrhs), rr,
                                int(prec), int(nrhs), _stream(stream)))
    return np.array(rr[:])


def dwf_xpay(op, p, r, beta, prec, nrhs=1, stream=None):
    _check(load().dwf_xpay(op, _ptr(p), _ptr(r), _dbl(beta, nrhs), int(prec), int(nrhs), _stream(stream)))


def cg_solve(op, x, b, nrhs=1, tol=1e-8, maxiter=100000, stream=None):
    st = SolveStats()
    rc = _check(load().cg_solve(op, _ptr(x), _ptr(b), int(nrhs), float(tol), int(maxiter), C.byref(st),
                                _stream(stream)), allow_soft=True)
    return rc, st.as_dict()


def cg_solve_mixed(op, x, b, nrhs=1, tol=1e-8, inner_tol=1e-5, maxiter=100000, stream=None):
    st = SolveStats()
    rc = _check(load().cg_solve_mixed(op, _ptr(x), _ptr(b), int(nrhs), float(tol), float(inner_tol), int(maxiter),
                                      C.byref(st), _stream(stream)), allow_soft=True)
    return rc, st.as_dict()


def dwf_multishift_cg(op, x, b, shifts, nrhs=1, tol=1e-10, maxiter=100000, stream=None):
    st = SolveStats()
    sh = _dbl(shifts, len(shifts))
    rc = _check(load().dwf_multishift_cg(op, _ptr(x), _ptr(b), int(nrhs), sh, len(shifts), float(tol),
                                         int(maxiter), C.byref(st), _stream(stream)), allow_soft=True)
    return rc, st.as_dict()


def dwf_last_error():
    return load().dwf_last_error().decode()


# ------------------------------------------------------------------- HDCG --
def hdcg_default_params(**overrides):
    p = HdcgParams()
    load().hdcg_default_params(C.byref(p))
    for k, v in overrides.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def hdcg_setup(op, block, nvec, vectors, params=None, stream=None):
    h = C.c_void_p()
    b = (C.c_int * 4)(*[int(x) for x in block])
    p = params if params is not None else hdcg_default_params()
    _check(load().hdcg_setup(C.byref(h), op, C.byref(b), int(nvec), _ptr(vectors), C.byref(p), _stream(stream)))
    return h


def hdcg_destroy(h):
    _check(load().hdcg_destroy(h))


def hdcg_dims(h):
    c = (C.c_int * 4)()
    nc, nv = C.c_int(), C.c_int()
    _check(load().hdcg_dims(h, C.byref(c), C.byref(nc), C.byref(nv)))
    return tuple(c[:]), nc.value, nv.value


def hdcg_project(h, coarse_out, fine_in, prec, nrhs=1, stream=None):
    _check(load().hdcg_project(h, _ptr(coarse_out), _ptr(fine_in), int(prec), int(nrhs), _stream(stream)))


def hdcg_promote(h, fine_out, coarse_in, prec, nrhs=1, stream=None):
    _check(load().hdcg_promote(h, _ptr(fine_out), _ptr(coarse_in), int(prec), int(nrhs), _stream(stream)))


def coarse_apply(h, out, inp, prec, nrhs=1, stream=None):
    _check(load().coarse_apply(h, _ptr(out), _ptr(inp), int(prec), int(nrhs), _stream(stream)))


def hdcg_coarse_solve(h, x, b, prec, nrhs=1, tol=1e-8, maxiter=10000, stream=None):
    it = C.c_int()
    rc = _check(load().hdcg_coarse_solve(h, _ptr(x), _ptr(b), int(prec), int(nrhs), float(tol), int(maxiter),
                                         C.byref(it), _stream(stream)), allow_soft=True)
    return rc, it.value


def hdcg_mfma_tile(h, prec, nrhs_per_launch, stream=None):
    """(tile, ms): tile = (K per MFMA instruction, waves, K steps per wave);
    ms = measured milliseconds of every candidate (-1: not allowed)."""
    t = (C.c_int * 3)()
    ms = (C.c_float * 32)()
    n = C.c_int()
    _check(load().hdcg_mfma_tile(h, int(prec), int(nrhs_per_launch), t, ms, C.byref(n), _stream(stream)))
    return tuple(t), list(ms[:n.value])


def hdcg_coarse_iterations(h, nrhs):
    a = (C.c_int * nrhs)()
    _check(load().hdcg_coarse_iterations(h, a, int(nrhs)))
    return list(a)


def hdcg_coarse_solve_noalloc(h, x, b, prec, nrhs=1, tol=1e-8, maxiter=10000, stream=None):
    it = C.c_int()
    rc = _check(load().hdcg_coarse_solve_noalloc(h, _ptr(x), _ptr(b), int(prec), int(nrhs), float(tol), int(maxiter),
                                                 C.byref(it), _stream(stream)), allow_soft=True)
    return rc, it.value


def hdcg_mirs(h, out, inp, nrhs=1, stream=None):
    _check(load().hdcg_mirs(h, _ptr(out), _ptr(inp), int(nrhs), _stream(stream)))


def hdcg_set_params(h, params, stream=None):
    _check(load().hdcg_set_params(h, C.byref(params), _stream(stream)))


def hdcg_ldop_setup(h, n_extra, noise=None, shift=0.0, n_steps=3, tol=1e-7, stream=None):
    _check(load().hdcg_ldop_setup(h, int(n_extra), _ptr(noise), float(shift), int(n_steps), float(tol),
                                  _stream(stream)))


def hdcg_export_ldop(h, Z=None, stream=None):
    """Returns (n_global, D); fills Z (device complex128 [n][Nc][Nvec]) when given."""
    n = C.c_int()
    load().hdcg_export_ldop(h, C.byref(n), None, None, _stream(stream))
    D = (C.c_double * max(n.value, 1))()
    _check(load().hdcg_export_ldop(h, C.byref(n), _ptr(Z), D, _stream(stream)))
    return n.value, np.array(D[:n.value])


def hdcg_trunc_apply(h, out, inp, prec, nrhs=1, stream=None):
    _check(load().hdcg_trunc_apply(h, _ptr(out), _ptr(inp), int(prec), int(nrhs), _stream(stream)))


def hdcg_m1_interval(h, stream=None):
    lo, hi = C.c_double(), C.c_double()
    _check(load().hdcg_m1_interval(h, C.byref(lo), C.byref(hi), _stream(stream)))
    return lo.value, hi.value


def hdcg_chebyshev(h, y, r, prec, nrhs=1, stream=None):
    _check(load().hdcg_chebyshev(h, _ptr(y), _ptr(r), int(prec), int(nrhs), _stream(stream)))


def hdcg_trunc_cg(h, y, r, prec, nrhs=1, stream=None):
    _check(load().hdcg_trunc_cg(h, _ptr(y), _ptr(r), int(prec), int(nrhs), _stream(stream)))


def hdcg_adef1_precondition(h, y, r, prec, nrhs=1, stream=None):
    _check(load().hdcg_adef1_precondition(h, _ptr(y), _ptr(r), int(prec), int(nrhs), _stream(stream)))


def hdcg_export_coarse(h, out, stream=None):
    _check(load().hdcg_export_coarse(h, _ptr(out), _stream(stream)))


def hdcg_import_coarse(h, A, stream=None):
    _check(load().hdcg_import_coarse(h, _ptr(A), _stream(stream)))


def hdcg_export_subspace(h, out, stream=None):
    _check(load().hdcg_export_subspace(h, _ptr(out), _stream(stream)))


def hdcg_export_block_map(h, vh):
    a = (C.c_int * vh)()
    j = (C.c_int * vh)()
    _check(load().hdcg_export_block_map(h, a, j))
    return np.array(a[:]), np.array(j[:])


def hdcg_solve(h, x, b, nrhs=1, tol=1e-8, stream=None):
    st = HdcgStats()
    rc = _check(load().hdcg_solve(h, _ptr(x), _ptr(b), int(nrhs), float(tol), C.byref(st), _stream(stream)),
                allow_soft=True)
    return rc, st.as_dict()
