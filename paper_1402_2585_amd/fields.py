"""Device-buffer helpers around an operator handle (allocation with PyTorch,
layout conversion through the library).

Handles are released explicitly: close() on each object, or, for whatever is
still open when the interpreter exits, one atexit handler that closes every
HDCG handle and then every operator (an HDCG handle refers to its operator)
while the HIP runtime is still fully up.  A finaliser that runs during
interpreter shutdown does nothing, so no device memory is freed from a
garbage-collection pass at exit."""
from __future__ import annotations

import atexit
import sys
import weakref

import numpy as np

from . import _lib as L

_LIVE_HDCG = weakref.WeakSet()
_LIVE_OPS = weakref.WeakSet()


def close_all():
    """Close every open HDCG handle, then every operator handle."""
    for h in list(_LIVE_HDCG):
        h.close()
    for op in list(_LIVE_OPS):
        op.close()


atexit.register(close_all)

# torch element type of a native field per precision; 16-bit fields are
# bfloat16 tensors holding (re, im) pairs, two elements per complex value
_DT = {L.DWF_C128: "complex128", L.DWF_C64: "complex64", L.DWF_BF16: "bfloat16"}
_ELEM_BYTES = {L.DWF_C128: 16, L.DWF_C64: 8, L.DWF_BF16: 2}


class FineOperator:
    """Owns one dwf_op handle; fields are torch tensors in the native layout."""

    def __init__(self, gauge, dims, Ls, M5, mass, bc=(1, 1, 1, -1), b5=1.0, c5=0.0):
        """Shamir kernel, or Mobius when (b5, c5) is not (1, 0)."""
        import torch

        self.torch = torch
        g = gauge if isinstance(gauge, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(gauge))
        g = g.to(device="cuda", dtype=torch.complex128).contiguous()
        self.dims, self.Ls, self.M5, self.mass, self.bc = tuple(dims), int(Ls), float(M5), float(mass), bc
        self.b5, self.c5 = float(b5), float(c5)
        if (self.b5, self.c5) == (1.0, 0.0):
            self.h = L.dwf_create(g, dims, Ls, M5, mass, bc)
        else:
            self.h = L.dwf_create_mobius(g, dims, Ls, M5, mass, b5, c5, bc)
        torch.cuda.synchronize()
        X, Y, Z, T = dims
        self.Vh = X * Y * Z * T // 2
        self.canonical_shape = (self.Ls, self.Vh, 4, 3)
        _LIVE_OPS.add(self)

    def close(self):
        if self.h is not None:
            L.dwf_destroy(self.h)
            self.h = None
        _LIVE_OPS.discard(self)

    def __del__(self):
        if sys.is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def dtype(self, prec):
        return getattr(self.torch, _DT[prec])

    def new_field(self, prec=L.DWF_C128, nrhs=1, zero=False):
        n = L.dwf_field_bytes(self.h, prec, nrhs) // _ELEM_BYTES[prec]
        f = self.torch.zeros if zero else self.torch.empty
        return f(n, dtype=self.dtype(prec), device="cuda")

    def to_native(self, canonical, prec=L.DWF_C128):
        """canonical: numpy or torch array (nrhs, Ls, Vh, 4, 3) or (Ls, Vh, 4, 3)."""
        t = canonical if isinstance(canonical, self.torch.Tensor) else self.torch.from_numpy(
            np.ascontiguousarray(canonical))
        t = t.to(device="cuda", dtype=self.dtype(prec)).contiguous()
        nrhs = t.numel() // (self.Vh * self.Ls * 12)
        out = self.new_field(prec, nrhs)
        L.dwf_import(self.h, out, t, prec, nrhs)
        return out

    def to_canonical(self, native, prec=L.DWF_C128, nrhs=None):
        nrhs = nrhs or native.numel() // (self.Vh * self.Ls * 12)
        out = self.torch.empty((nrhs,) + self.canonical_shape, dtype=self.dtype(prec), device="cuda")
        L.dwf_export(self.h, out, native, prec, nrhs)
        return out if nrhs > 1 else out[0]

    def convert(self, x, dst_prec, src_prec, nrhs=1):
        """Native field x (src_prec) as a new native field in dst_prec."""
        out = self.new_field(dst_prec, nrhs)
        L.dwf_convert(self.h, out, dst_prec, x, src_prec, nrhs)
        return out

    def mpc(self, x, prec=L.DWF_C128, dagger=0, nrhs=1, out=None):
        out = self.new_field(prec, nrhs) if out is None else out
        L.mpc_apply(self.h, out, x, prec, dagger, nrhs)
        return out

    def H(self, x, prec=L.DWF_C128, nrhs=1, out=None):
        out = self.new_field(prec, nrhs) if out is None else out
        L.mpc_dag_mpc_apply(self.h, out, x, prec, nrhs)
        return out


class HDCG:
    """Owns one hdcg handle built on a FineOperator."""

    def __init__(self, op: FineOperator, block, vectors, params=None, nvec=None, **overrides):
        """vectors: the nvec canonical starting vectors, or None with nvec
        given: the library then draws them from params.seed (Philox4x32-10)."""
        torch = op.torch
        self.op = op
        if vectors is None:
            if not nvec:
                raise ValueError("nvec is needed when no vectors are given")
            v, self.nvec = None, int(nvec)
        else:
            v = vectors if isinstance(vectors, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(vectors))
            v = v.to(device="cuda", dtype=torch.complex128).contiguous()
            self.nvec = v.shape[0]
        p = params if params is not None else L.hdcg_default_params(**overrides)
        self.params = p
        self.h = L.hdcg_setup(op.h, block, self.nvec, v, p)
        self.coarse_dims, self.Nc, _ = L.hdcg_dims(self.h)
        _LIVE_HDCG.add(self)

    def set_params(self, **changes):
        """Change solve-phase parameters (hdcg_set_params) of the built handle."""
        p = L.HdcgParams()
        for k, _ in p._fields_:
            setattr(p, k, getattr(self.params, k))
        for k, v in changes.items():
            if not hasattr(p, k):
                raise KeyError(k)
            setattr(p, k, v)
        L.hdcg_set_params(self.h, p)
        self.params = p

    def close(self):
        if self.h is not None:
            L.hdcg_destroy(self.h)
            self.h = None
        _LIVE_HDCG.discard(self)

    def __del__(self):
        if sys.is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def new_coarse(self, prec=L.DWF_C128, nrhs=1, zero=True):
        f = self.op.torch.zeros if zero else self.op.torch.empty
        return f((nrhs, self.Nc, self.nvec), dtype=self.op.dtype(prec), device="cuda")

    def coarse_matrix(self):
        A = self.op.torch.empty((self.Nc, 81, self.nvec, self.nvec), dtype=self.op.torch.complex128, device="cuda")
        L.hdcg_export_coarse(self.h, A)
        return A

    def subspace(self):
        P = self.op.torch.empty((self.nvec,) + self.op.canonical_shape, dtype=self.op.torch.complex128, device="cuda")
        L.hdcg_export_subspace(self.h, P)
        return P
