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
        L.pah_solve_exact.argtypes = [P, P, C.c_int32, C.c_int64, P, P, P, P]
        L.pah_build_rows.argtypes = [P, P, C.c_int64, P, P]
        L.pah_band_power.argtypes = [P, P, C.c_int64, P, P, P]
        for n in ("pah_build_rows", "pah_band_power", "pah_tables_bytes", "pah_ctx_create", "pah_build_tables",
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

    def rows(self, out, rows=None):
        """Re-emission CDF rows [n, n_lambda] (float64) from solver outputs."""
        n = int(out.shape[0])
        r = rows if rows is not None else torch.empty((n, self.n_lambda), dtype=torch.float64, device=self.device)
        self._check(lib().pah_build_rows(self.ctx, _ptr(out.contiguous()), n, _ptr(r), _stream()), "pah_build_rows")
        return r

    def band_power(self, out, weight):
        """Band powers summed over cells, sum_c weight_c out[c, b] (pah_band_power),
        float64 [n_bands] on the device."""
        out, weight = out.contiguous(), weight.contiguous()
        bp = torch.empty(self.n_bands, dtype=torch.float64, device=self.device)
        self._check(lib().pah_band_power(self.ctx, _ptr(out), int(out.shape[0]), _ptr(weight), _ptr(bp),
                                         _stream()), "pah_band_power")
        return bp

    def solve(self, J: torch.Tensor, want_P=False, out=None):
        """J: [n, n_lambda] float32 or float64 device tensor -> (out [n, n_out],
        P [n, M] or None, pabs [n]) as float64 device tensors."""
        J = J.contiguous()
        n = int(J.shape[0])
        o = out if out is not None else torch.empty((n, self.n_out), dtype=torch.float64, device=self.device)
        P = torch.empty((n, self.M), dtype=torch.float64, device=self.device) if want_P else None
        pabs = torch.empty(n, dtype=torch.float64, device=self.device)
        self._check(lib().pah_solve_exact(self.ctx, _ptr(J), 1 if J.dtype == torch.float32 else 0, n,
                                          _ptr(o), _ptr(P), _ptr(pabs), _stream()), "pah_solve_exact")
        return o, P, pabs


OFFSET_NAMES = ["params", "grads", "adam_m", "adam_v", "n_params", "oW1", "ob1", "oW2", "ob2", "oW3",
                "ob3", "W1h", "W2h", "W3h", "x_mu", "x_sd", "x_lo", "x_hi", "y_mu", "y_sd", "X16",
                "Z1", "H1", "Z2", "H2", "Y", "dY16", "dZ2", "dZ1", "loss", "Wpk", "total"]


def _mlp_lib():
    L = lib()
    if not getattr(L, "_mlp_ready", False):
        P = C.c_void_p
        L.pah_mlp_state_bytes.argtypes = [C.c_int32] * 4 + [C.POINTER(C.c_uint64)]
        L.pah_mlp_create.argtypes = [C.c_int32] * 4 + [P, C.c_uint64, C.POINTER(P)]
        L.pah_mlp_destroy.argtypes = [P]
        L.pah_mlp_destroy.restype = None
        L.pah_mlp_last_error.argtypes = [P]
        L.pah_mlp_last_error.restype = C.c_char_p
        L.pah_mlp_offsets.argtypes = [P, C.POINTER(C.c_uint64), C.c_int32]
        L.pah_mlp_load.argtypes = [P, P, P]
        L.pah_mlp_set_norm.argtypes = [P] * 7 + [P]
        L.pah_mlp_forward.argtypes = [P, P, C.c_int32, P, P]
        L.pah_mlp_train_step.argtypes = [P, P, P, C.c_int32, C.c_float, C.c_int32, P]
        L.pah_surrogate_infer.argtypes = [P, P, P, C.c_int64, P, P, P, C.c_float, C.c_float, P]
        L.pah_exact_fallback.argtypes = [P, P, C.c_int64, P, P, P, P]
        L.pah_mlp_prepare.argtypes = [P, P, P, P, P, C.c_int64, P, P, P]
        for n in ("pah_mlp_prepare", "pah_mlp_state_bytes", "pah_mlp_create", "pah_mlp_offsets", "pah_mlp_load",
                  "pah_mlp_set_norm", "pah_mlp_forward", "pah_mlp_train_step", "pah_surrogate_infer",
                  "pah_exact_fallback"):
            getattr(L, n).restype = C.c_int32
        L._mlp_ready = True
    return L


class PahMLP:
    """Surrogate network state on one device (all in one state buffer)."""

    def __init__(self, n_in=200, n_h=256, n_out=217, batch=2048, device="cuda"):
        L = _mlp_lib()
        self.n_in, self.n_h, self.n_out, self.batch = n_in, n_h, n_out, batch
        self.device = torch.device(device)
        nb = C.c_uint64()
        rc = L.pah_mlp_state_bytes(n_in, n_h, n_out, batch, C.byref(nb))
        if rc != 0:
            raise MCRTError(rc, "pah_mlp_state_bytes")
        self.state = torch.zeros(int(nb.value), dtype=torch.uint8, device=self.device)
        h = C.c_void_p()
        rc = L.pah_mlp_create(n_in, n_h, n_out, batch, _ptr(self.state), self.state.numel(), C.byref(h))
        if rc != 0:
            raise MCRTError(rc, "pah_mlp_create")
        self.h = h
        off = (C.c_uint64 * 32)()
        self._check(L.pah_mlp_offsets(h, off, 32), "offsets")
        self.off = dict(zip(OFFSET_NAMES, [int(v) for v in off]))

    def __del__(self):
        try:
            if getattr(self, "h", None):
                _mlp_lib().pah_mlp_destroy(self.h)
                self.h = None
        except Exception:
            pass

    def _check(self, rc, what):
        if rc != 0:
            raise MCRTError(rc, f"{what}: {_mlp_lib().pah_mlp_last_error(self.h).decode()}")

    def checkpoint(self):
        """Host copy of the persistent network state (FP32 masters, gradients,
        Adam moments, bfloat16 copies, normalisation): the state buffer up to
        the batch activations.  With the step count and the batch order it
        resumes training exactly (every training kernel is deterministic)."""
        torch.cuda.current_stream().synchronize()
        return self.state[:self.off["X16"]].cpu().clone()

    def restore(self, ck):
        """Puts back a checkpoint taken from a network of the same shape."""
        n = self.off["X16"]
        if ck.numel() != n:
            raise ValueError("checkpoint of a network of another shape")
        self.state[:n].copy_(ck.to(self.device))
        torch.cuda.current_stream().synchronize()

    def _shapes(self):
        ni, nh, no = self.n_in, self.n_h, self.n_out
        return [("W1", (nh, ni)), ("b1", (nh,)), ("W2", (nh, nh)), ("b2", (nh,)), ("W3", (no, nh)), ("b3", (no,))]

    def load(self, params):
        flat = np.concatenate([np.asarray(params[k], np.float32).reshape(-1) for k, _ in self._shapes()])
        t = torch.as_tensor(flat).to(self.device)
        self._check(_mlp_lib().pah_mlp_load(self.h, _ptr(t), _stream()), "pah_mlp_load")
        torch.cuda.current_stream().synchronize()

    def _block(self, which):
        n = self.off["n_params"]
        f = self.state[self.off[which]:self.off[which] + 4 * n].view(torch.float32)
        out, o = {}, 0
        for k, shp in self._shapes():
            sz = int(np.prod(shp))
            out[k] = f[o:o + sz].view(*shp)
            o += sz
        return out

    def params(self):
        return {k: v.detach().cpu().numpy().astype(np.float64) for k, v in self._block("params").items()}

    def grads(self):
        return {k: v.detach().cpu().numpy().astype(np.float64) for k, v in self._block("grads").items()}

    def param_tensors(self):
        return self._block("params")

    def set_norm(self, x_mu, x_sd, x_lo, x_hi, y_mu, y_sd):
        ts = [torch.as_tensor(np.asarray(a, np.float32)).to(self.device) for a in (x_mu, x_sd, x_lo, x_hi, y_mu, y_sd)]
        self._check(_mlp_lib().pah_mlp_set_norm(self.h, *[_ptr(t) for t in ts], _stream()), "set_norm")
        torch.cuda.current_stream().synchronize()

    def prepare(self, solver, J, out, pabs):
        """Standardised training pairs (X, Y) from solved cells; sets the normalisation."""
        n = int(J.shape[0])
        X = torch.empty((n, self.n_in), dtype=torch.float32, device=self.device)
        Y = torch.empty((n, self.n_out), dtype=torch.float32, device=self.device)
        self._check(_mlp_lib().pah_mlp_prepare(self.h, solver.ctx, _ptr(J.contiguous().float()), _ptr(out),
                                               _ptr(pabs), n, _ptr(X), _ptr(Y), _stream()), "pah_mlp_prepare")
        return X, Y

    def forward(self, X):
        X = X.contiguous().float()
        Y = torch.empty((X.shape[0], self.n_out), dtype=torch.float32, device=self.device)
        self._check(_mlp_lib().pah_mlp_forward(self.h, _ptr(X), int(X.shape[0]), _ptr(Y), _stream()), "forward")
        return Y

    def train_step(self, X, T, lr, step):
        self._check(_mlp_lib().pah_mlp_train_step(self.h, _ptr(X), _ptr(T), int(X.shape[0]), float(lr),
                                                  int(step), _stream()), "train_step")

    def loss(self):
        o = self.off["loss"]
        return float(self.state[o:o + 4].view(torch.float32).item())

    def infer(self, solver, J, in_margin=0.5, balance_tol=0.02):
        J = J.contiguous().float()
        n = int(J.shape[0])
        out = torch.empty((n, self.n_out), dtype=torch.float64, device=self.device)
        ood = torch.empty(n, dtype=torch.uint8, device=self.device)
        pabs = torch.empty(n, dtype=torch.float64, device=self.device)
        self._check(_mlp_lib().pah_surrogate_infer(self.h, solver.ctx, _ptr(J), n, _ptr(out), _ptr(ood),
                                                   _ptr(pabs), float(in_margin), float(balance_tol), _stream()),
                    "pah_surrogate_infer")
        return out, ood, pabs


def exact_fallback(solver, J, ood, out, idx=None):
    """Exact solution for the cells flagged in ood, written into out in place."""
    n = int(J.shape[0])
    if idx is None:
        idx = torch.empty(n + 1, dtype=torch.int64, device=J.device)
    rc = _mlp_lib().pah_exact_fallback(solver.ctx, _ptr(J.contiguous().float()), n, _ptr(ood), _ptr(out),
                                       _ptr(idx), _stream())
    solver._check(rc, "pah_exact_fallback")
    return idx
