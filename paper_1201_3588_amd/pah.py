"""Python binding of the PAH emission step (include/pah.h): argument
marshalling only; the exact solver runs in libmcrt.so."""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from .mcrt import MCRTError, _ptr, _stream, lib as _mcrt_lib


class PahDesc(C.Structure):
    _fields_ = [("M", C.c_int32), ("n_lambda", C.c_int32), ("n_bands", C.c_int32), ("pad", C.c_int32),
                ("T", C.c_void_p), ("U", C.c_void_p), ("lambda_um", C.c_void_p), ("cabs", C.c_void_p),
                ("cband", C.c_void_p), ("ccont", C.c_void_p)]


def lib():
    L = _mcrt_lib()
    if not getattr(L, "_pah_ready", False):
        P = C.c_void_p
        L.pah_tables_bytes.argtypes = [C.POINTER(PahDesc), C.POINTER(C.c_uint64)]
        L.pah_ctx_create.argtypes = [C.POINTER(PahDesc), C.POINTER(P)]
        L.pah_ctx_destroy.argtypes = [P]
        L.pah_ctx_destroy.restype = None
        L.pah_last_error.argtypes = [P]
        L.pah_last_error.restype = C.c_char_p
        L.pah_build_tables.argtypes = [P, P, C.c_uint64, P]
        L.pah_workspace_bytes.argtypes = [P, C.POINTER(C.c_uint64)]
        L.pah_solve_exact.argtypes = [P, P, C.c_int32, C.c_int64, P, P, P, P, C.c_uint64, P]
        for n in ("pah_tables_bytes", "pah_ctx_create", "pah_build_tables", "pah_workspace_bytes",
                  "pah_solve_exact"):
            getattr(L, n).restype = C.c_int32
        L._pah_ready = True
    return L


class PahSolver:
    """Exact P(T) solver for one PAH species on one device."""

    def __init__(self, T, U, lam_um, cabs, cband, ccont, device="cuda"):
        L = lib()
        dev = torch.device(device)
        f64 = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float64)).to(dev)
        self.device = dev
        self.T, self.U, self.lam = f64(T), f64(U), f64(lam_um)
        self.cabs, self.cband, self.ccont = f64(cabs), f64(cband), f64(ccont)
        self.M, self.n_lambda = int(self.T.numel()), int(self.lam.numel())
        self.n_bands = int(np.asarray(cband).shape[0])
        self.n_out = self.n_bands + self.n_lambda
        d = PahDesc(self.M, self.n_lambda, self.n_bands, 0, *(C.c_void_p(t.data_ptr()) for t in
                    (self.T, self.U, self.lam, self.cabs, self.cband, self.ccont)))
        self.desc = d
        nb = C.c_uint64()
        rc = L.pah_tables_bytes(C.byref(d), C.byref(nb))
        if rc != 0:
            raise MCRTError(rc, "pah descriptor")
        ctx = C.c_void_p()
        rc = L.pah_ctx_create(C.byref(d), C.byref(ctx))
        if rc != 0:
            raise MCRTError(rc, "pah_ctx_create")
        self.ctx = ctx
        self.tables = torch.zeros(int(nb.value), dtype=torch.uint8, device=dev)
        self._check(L.pah_build_tables(ctx, _ptr(self.tables), self.tables.numel(), _stream()),
                    "pah_build_tables")
        wb = C.c_uint64()
        self._check(L.pah_workspace_bytes(ctx, C.byref(wb)), "workspace")
        self.ws = torch.empty(int(wb.value), dtype=torch.uint8, device=dev)

    @classmethod
    def from_model(cls, pm, M=500, T_lo=2.7, T_hi=5000.0, device="cuda"):
        T = T_lo * (T_hi / T_lo) ** (np.arange(M) / (M - 1))
        return cls(T, pm.enthalpy(T), pm.lam_um, pm.cabs, pm.cband, pm.ccont, device=device)

    def __del__(self):
        try:
            if getattr(self, "ctx", None):
                lib().pah_ctx_destroy(self.ctx)
                self.ctx = None
        except Exception:
            pass

    def _check(self, rc, what):
        if rc != 0:
            raise MCRTError(rc, f"{what}: {lib().pah_last_error(self.ctx).decode()}")

    def solve(self, J: torch.Tensor, want_P=False, out=None):
        """J: [n, n_lambda] float32 or float64 device tensor -> (out [n, n_out],
        P [n, M] or None, pabs [n]) as float64 device tensors."""
        J = J.contiguous()
        n = int(J.shape[0])
        o = out if out is not None else torch.empty((n, self.n_out), dtype=torch.float64, device=self.device)
        P = torch.empty((n, self.M), dtype=torch.float64, device=self.device) if want_P else None
        pabs = torch.empty(n, dtype=torch.float64, device=self.device)
        self._check(lib().pah_solve_exact(self.ctx, _ptr(J), 1 if J.dtype == torch.float32 else 0, n,
                                          _ptr(o), _ptr(P), _ptr(pabs), _ptr(self.ws), self.ws.numel(),
                                          _stream()), "pah_solve_exact")
        return o, P, pabs
