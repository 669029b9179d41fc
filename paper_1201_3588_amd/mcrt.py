"""Python binding of libmcrt (the C ABI in include/mcrt.h).

Argument marshalling only: every step of the method runs in the HIP kernels
of libmcrt.so.  PyTorch provides device memory and the current stream.  The
library must be built (``__graft_entry__.build()``); importing this module
without it raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch  # loads the HIP runtime that libmcrt.so binds to

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmcrt.so")

F32, F64 = 0, 1
FLAG_TALLY_J, FLAG_FROZEN_T, FLAG_KILL_ON_ABSORB, FLAG_EXACT_BW, FLAG_PEEL, FLAG_PEEL_SED = 1, 2, 4, 8, 16, 32
PEEL_REC_BYTES = 64
PEEL_UNIT = 1 << 24                     # fixed-point unit of the next-event images
CNT = dict(launched=0, escaped=1, killed=2, terminated=3, scatters=4, absorptions=5,
           crossings=6, tclamp_lo=7, tclamp_hi=8, pah_abs=9, zero_cross=10, jseg=11, peel=12,
           peel_dropped=13)
ERRORS = {0: "OK", -1: "E_INVALID", -2: "E_STATE", -3: "E_HIP", -4: "E_CAPACITY",
          -5: "E_NUMERIC", -6: "E_UNSUPPORTED"}

_dp = C.c_void_p


class Desc(C.Structure):
    _fields_ = [("precision", C.c_int32), ("n_lambda", C.c_int32), ("n_species", C.c_int32),
                ("nb", C.c_int32), ("max_level", C.c_int32), ("K", C.c_int32),
                ("n_cells", C.c_int64), ("n_nodes", C.c_int64),
                ("box_min", C.c_double * 3), ("base_size", C.c_double),
                ("T_lo", C.c_double), ("T_hi", C.c_double),
                ("n_theta", C.c_int32), ("n_phi", C.c_int32),
                ("lambda_um", _dp), ("kabs", _dp), ("ksca", _dp), ("g", _dp), ("kind", _dp),
                ("base_map", _dp), ("nodes", _dp), ("rho", _dp)]


class Source(C.Structure):
    _fields_ = [("pos", C.c_double * 3), ("lum", C.c_double), ("teff", C.c_double),
                ("beam", C.c_double * 3), ("beam_on", C.c_int32)]


class Tallies(C.Structure):
    _fields_ = [("nabs", _dp), ("sed", _dp), ("jq", _dp), ("counters", _dp), ("image", _dp), ("peel", _dp),
                ("peel_sed", _dp)]


class Observers(C.Structure):
    _fields_ = [("n_obs", C.c_int32), ("npix", C.c_int32), ("n_img_lambda", C.c_int32),
                ("img_lambda", C.c_int32 * 8), ("pad", C.c_int32), ("center", C.c_double * 3),
                ("half_width", C.c_double), ("cos_cone", C.c_double), ("dir", (C.c_double * 3) * 8)]


class RunOpts(C.Structure):
    _fields_ = [("n_total", C.c_uint64), ("seed", C.c_uint64), ("max_events", C.c_uint64),
                ("flags", C.c_int32), ("grid_blocks", C.c_int32),
                ("frozen_nabs", _dp), ("pah_rows", _dp), ("trace", _dp), ("trace_len", _dp),
                ("trace_cap", C.c_int32), ("pad", C.c_int32),
                ("peel_queue", _dp), ("peel_capacity", C.c_uint64),
                ("jrec_ws", _dp), ("jrec_capacity", C.c_uint64),
                ("kernel_begin", C.c_void_p), ("kernel_end", C.c_void_p)]


class TableLayout(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in ("nu", "dnu", "src_cdf", "kext", "albedo", "gpar", "sp_cdf",
                                          "Tk", "E", "R", "Bt", "Wt", "xk", "kext32", "g32", "rho_h32", "level", "leaf_lo",
                                          "binfo", "pah_slot", "scratch", "total")]


TRACE_DTYPE = np.dtype([("type", np.int32), ("cell", np.int32), ("j", np.int32),
                        ("pad", np.int32), ("x", np.float64, 3), ("d", np.float64, 3),
                        ("tau", np.float64)])

_lib = None


def lib():
    """Load libmcrt.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.mcrt_version.restype = C.c_int32
        L.mcrt_tables_bytes.argtypes = [C.POINTER(Desc), C.POINTER(C.c_uint64)]
        L.mcrt_ctx_create.argtypes = [C.POINTER(Desc), C.POINTER(P)]
        L.mcrt_ctx_destroy.argtypes = [P]
        L.mcrt_ctx_destroy.restype = None
        L.mcrt_last_error.argtypes = [P]
        L.mcrt_last_error.restype = C.c_char_p
        L.mcrt_table_layout_get.argtypes = [P, C.POINTER(TableLayout)]
        L.mcrt_build_tables.argtypes = [P, C.POINTER(Source), P, C.c_uint64, P]
        L.mcrt_run.argtypes = [P, C.c_uint64, C.c_uint64, C.POINTER(RunOpts), C.POINTER(Tallies), P]
        L.mcrt_temperatures.argtypes = [P, P, C.c_uint64, P, P]
        L.mcrt_mean_intensity.argtypes = [P, P, C.c_uint64, P, P]
        L.mcrt_thin_field.argtypes = [P, P, P]
        L.mcrt_thin_field.restype = C.c_int32
        L.mcrt_cell_mass.argtypes = [P, P, P]
        L.mcrt_cell_mass.restype = C.c_int32
        L.mcrt_set_observers.argtypes = [P, C.POINTER(Observers)]
        L.mcrt_set_observers.restype = C.c_int32
        L.mcrt_read_counters_sync.argtypes = [C.POINTER(Tallies), P, P]
        L.mcrt_read_counters_sync.restype = C.c_int32
        L.mcrt_jrec_ws_bytes.argtypes = [P, C.c_uint64, C.POINTER(C.c_uint64)]
        L.mcrt_jrec_ws_bytes.restype = C.c_int32
        L.mcrt_psf_radius.argtypes = [C.c_double]
        L.mcrt_psf_radius.restype = C.c_int32
        L.mcrt_image_psf.argtypes = [P, C.c_int32, C.c_int32, C.c_double, C.c_double, P, P, P]
        L.mcrt_image_psf.restype = C.c_int32
        L.mcrt_image_psf_static.argtypes = [P, C.c_int32, C.c_int32, C.c_double, C.c_double, P, P]
        L.mcrt_image_psf_static.restype = C.c_int32
        for name in ("mcrt_tables_bytes", "mcrt_ctx_create", "mcrt_table_layout_get", "mcrt_build_tables",
                     "mcrt_run", "mcrt_temperatures", "mcrt_mean_intensity"):
            getattr(L, name).restype = C.c_int32
        _lib = L
    return _lib


class MCRTError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def image_psf(images: torch.Tensor, npix: int, scale: float, fwhm_pix: float) -> torch.Tensor:
    """Images (device int64 tensor of uint64 sums, [..., npix, npix]) times
    scale, convolved with a Gaussian PSF of FWHM fwhm_pix pixels
    (mcrt_image_psf); returns float64 [n_images, npix, npix]."""
    img = images.contiguous()
    n_img = img.numel() // (npix * npix)
    r = lib().mcrt_psf_radius(float(fwhm_pix))
    if r < 0 or n_img * npix * npix != img.numel():
        raise MCRTError(-1, "image_psf: fwhm out of range or shape mismatch")
    w = torch.empty(2 * r + 1, dtype=torch.float64, device=img.device)
    out = torch.empty((n_img, npix, npix), dtype=torch.float64, device=img.device)
    rc = lib().mcrt_image_psf(_ptr(img), n_img, int(npix), float(scale), float(fwhm_pix), _ptr(w), _ptr(out),
                              _stream())
    if rc != 0:
        raise MCRTError(rc, "mcrt_image_psf")
    return out


def image_psf_static(images: torch.Tensor, npix: int, scale: float, fwhm_pix: float,
                     out: torch.Tensor) -> torch.Tensor:
    """image_psf into a caller-given float64 `out` [n_images, npix, npix],
    with the weights in the library's static device array
    (mcrt_image_psf_static: no device memory is allocated)."""
    n_img = images.numel() // (npix * npix)
    if not images.is_contiguous() or not out.is_contiguous() or out.dtype != torch.float64 \
            or out.numel() != n_img * npix * npix or n_img * npix * npix != images.numel():
        raise MCRTError(-1, "image_psf_static: shape, dtype or layout mismatch")
    rc = lib().mcrt_image_psf_static(_ptr(images), n_img, int(npix), float(scale), float(fwhm_pix), _ptr(out),
                                     _stream())
    if rc != 0:
        raise MCRTError(rc, "mcrt_image_psf_static")
    return out


def u64_view(t: torch.Tensor) -> np.ndarray:
    """Host numpy uint64 view of an int64 tally tensor."""
    return t.detach().cpu().numpy().view(np.uint64)


class Engine:
    """One transport problem on one device: uploads the description, builds the
    tables (on the GPU) and runs packets through the C ABI."""

    def __init__(self, lam_um, kabs, ksca, g, kind, nb, max_level, box_min, base_size, base_map,
                 nodes, rho, K=1024, T_lo=3.0, T_hi=5000.0, n_theta=10, n_phi=1, precision="f32",
                 device="cuda"):
        L = lib()
        dev = torch.device(device)
        f64 = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float64)).to(dev)
        i32 = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.int32)).to(dev)
        self.device = dev
        self.lam = f64(lam_um)
        self.kabs = f64(kabs)
        self.ksca = f64(ksca)
        self.g = f64(g)
        self.kind = i32(kind)
        self.base_map = i32(base_map)
        nodes = np.asarray(nodes, np.int32)
        self.nodes = i32(nodes) if nodes.size else None
        self.rho = f64(rho)
        self.n_lambda = int(self.lam.numel())
        self.n_species = int(np.asarray(kind).size)
        self.n_cells = int(self.rho.numel())
        d = Desc()
        d.precision = F64 if precision == "f64" else F32
        d.n_lambda, d.n_species = self.n_lambda, self.n_species
        d.nb, d.max_level, d.K = int(nb), int(max_level), int(K)
        d.n_cells, d.n_nodes = self.n_cells, int(nodes.size // 8)
        d.box_min = (C.c_double * 3)(*[float(v) for v in box_min])
        d.base_size = float(base_size)
        d.T_lo, d.T_hi = float(T_lo), float(T_hi)
        d.n_theta, d.n_phi = int(n_theta), int(n_phi)
        d.lambda_um, d.kabs, d.ksca, d.g = (_ptr(t) for t in (self.lam, self.kabs, self.ksca, self.g))
        d.kind, d.base_map, d.nodes, d.rho = (_ptr(t) for t in (self.kind, self.base_map, self.nodes, self.rho))
        self.desc = d
        self.n_theta, self.n_phi = int(n_theta), int(n_phi)
        nbytes = C.c_uint64()
        rc = L.mcrt_tables_bytes(C.byref(d), C.byref(nbytes))
        if rc != 0:
            raise MCRTError(rc, "invalid descriptor")
        self.tables = torch.zeros(int(nbytes.value), dtype=torch.uint8, device=dev)
        ctx = C.c_void_p()
        rc = L.mcrt_ctx_create(C.byref(d), C.byref(ctx))
        if rc != 0:
            raise MCRTError(rc, "mcrt_ctx_create")
        self.ctx = ctx
        self.source = None

    @classmethod
    def from_workload(cls, w, device="cuda", precision=None):
        g, sp = w.grid, w.species
        return cls(sp.lam_um, sp.kabs, sp.ksca, sp.g, sp.kind, g.nb, g.max_level, g.box_min,
                   g.base_size, g.base_map, g.nodes, g.rho, K=w.K, T_lo=w.T_lo, T_hi=w.T_hi,
                   n_theta=w.n_theta, n_phi=w.n_phi, precision=precision or w.precision,
                   device=device)

    def __del__(self):
        try:
            if getattr(self, "ctx", None):
                lib().mcrt_ctx_destroy(self.ctx)
                self.ctx = None
        except Exception:
            pass

    def _check(self, rc, what):
        if rc != 0:
            raise MCRTError(rc, f"{what}: {lib().mcrt_last_error(self.ctx).decode()}")

    def build_tables(self, pos, lum, teff, beam=None):
        s = Source()
        s.pos = (C.c_double * 3)(*[float(v) for v in pos])
        s.lum, s.teff = float(lum), float(teff)
        if beam is not None:
            s.beam = (C.c_double * 3)(*[float(v) for v in beam])
            s.beam_on = 1
        self.source = s
        self._check(lib().mcrt_build_tables(self.ctx, C.byref(s), _ptr(self.tables),
                                            self.tables.numel(), _stream()), "mcrt_build_tables")

    def set_observers(self, dirs=(), npix=1, half_width=1.0, center=(0.0, 0.0, 0.0), cos_cone=1.0,
                      lambda_bins=(), peel=False, peel_capacity=1 << 22, peel_sed=False):
        """Escape images (see mcrt_observers); no directions turns them off.
        peel: also next-event images (MCRT_FLAG_PEEL) in tallies["peel"], with a
        device queue of peel_capacity records held by the engine.
        peel_sed: also each observer's next-event SED over every bin
        (MCRT_FLAG_PEEL_SED) in tallies["peel_sed"] [n_obs, n_lambda]."""
        ob = Observers()
        ob.n_obs, ob.npix, ob.n_img_lambda = len(dirs), int(npix), len(lambda_bins)
        for q, jb in enumerate(lambda_bins):
            ob.img_lambda[q] = int(jb)
        ob.center = (C.c_double * 3)(*[float(v) for v in center])
        ob.half_width, ob.cos_cone = float(half_width), float(cos_cone)
        for q, dv in enumerate(dirs):
            for a in range(3):
                ob.dir[q][a] = float(dv[a])
        self._check(lib().mcrt_set_observers(self.ctx, C.byref(ob)), "mcrt_set_observers")
        self.image_shape = (len(dirs), len(lambda_bins), int(npix), int(npix)) if len(dirs) else None
        self.peel_on = bool(peel) and len(dirs) > 0
        self.peel_sed_on = self.peel_on and bool(peel_sed)
        if self.peel_on:
            cap = int(peel_capacity)
            if getattr(self, "_peel_q", None) is None or self._peel_q.numel() < cap * PEEL_REC_BYTES:
                self._peel_q = torch.empty(cap * PEEL_REC_BYTES, dtype=torch.uint8, device=self.device)
            self.peel_capacity = cap

    def new_tallies(self, tally_j=True):
        z = lambda n: torch.zeros(int(n), dtype=torch.int64, device=self.device)
        shape = getattr(self, "image_shape", None)
        return dict(nabs=z(self.n_cells * self.n_species),
                    sed=z(self.n_theta * self.n_phi * self.n_lambda),
                    jq=z(self.n_lambda * self.n_cells) if tally_j else None,
                    counters=z(16),
                    image=z(np.prod(shape)) if shape else None,
                    peel=z(np.prod(shape)) if shape and getattr(self, "peel_on", False) else None,
                    peel_sed=z(shape[0] * self.n_lambda) if shape and getattr(self, "peel_sed_on", False)
                    else None)

    def counters_sync(self, tallies):
        """The run counters as numpy uint64, after the stream has drained."""
        t = Tallies(None, None, None, _ptr(tallies["counters"]), None, None)
        out = np.zeros(16, np.uint64)
        rc = lib().mcrt_read_counters_sync(C.byref(t), out.ctypes.data, _stream())
        if rc != 0:
            raise MCRTError(rc, "mcrt_read_counters_sync")
        return out

    def set_deferred_tally(self, capacity):
        """Path-length tally through a record workspace of `capacity` segment
        records (mcrt_jrec_ws_bytes) instead of per-segment atomics; 0 turns
        it off.  Returns False when the grid does not support it."""
        self._jrec = None                  # release the old workspace before sizing a new one
        if not capacity:
            return True
        nbytes = C.c_uint64(0)
        rc = lib().mcrt_jrec_ws_bytes(self.ctx, int(capacity), C.byref(nbytes))
        if rc == -6:
            self._jrec = None
            return False
        self._check(rc, "mcrt_jrec_ws_bytes")
        self._jrec = (torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device), int(capacity))
        return True

    def run(self, tallies, first_id, n, n_total, seed, max_events=1_000_000, flags=None,
            frozen_nabs=None, pah_rows=None, trace_cap=0, grid_blocks=0, kernel_events=None):
        """kernel_events: optional pair of recorded torch.cuda.Events that the
        library records again right around the transport kernel itself."""
        if flags is None:
            flags = FLAG_TALLY_J if tallies.get("jq") is not None else 0
        t = Tallies(_ptr(tallies["nabs"]), _ptr(tallies["sed"]), _ptr(tallies.get("jq")),
                    _ptr(tallies["counters"]), _ptr(tallies.get("image")), _ptr(tallies.get("peel")),
                    _ptr(tallies.get("peel_sed")))
        o = RunOpts()
        o.n_total, o.seed, o.max_events = int(n_total), int(seed), int(max_events)
        o.flags, o.grid_blocks = int(flags), int(grid_blocks)
        if getattr(self, "peel_on", False) and tallies.get("peel") is not None:
            o.flags |= FLAG_PEEL
            if tallies.get("peel_sed") is not None:
                o.flags |= FLAG_PEEL_SED
            o.peel_queue, o.peel_capacity = _ptr(self._peel_q), self.peel_capacity
        if kernel_events is not None:
            if not (kernel_events[0].cuda_event and kernel_events[1].cuda_event):
                raise MCRTError(-1, "kernel_events must have been recorded once (created)")
            o.kernel_begin, o.kernel_end = kernel_events[0].cuda_event, kernel_events[1].cuda_event
        jrec = getattr(self, "_jrec", None)
        if jrec is not None and (o.flags & FLAG_TALLY_J) and tallies.get("jq") is not None:
            o.jrec_ws, o.jrec_capacity = _ptr(jrec[0]), jrec[1]
        keep = []
        if frozen_nabs is not None:
            if isinstance(frozen_nabs, torch.Tensor):
                fz = frozen_nabs.contiguous()
            else:
                fz = torch.as_tensor(np.ascontiguousarray(frozen_nabs, np.uint64).view(np.int64)).to(self.device)
            keep.append(fz)
            o.frozen_nabs = _ptr(fz)
            o.flags |= FLAG_FROZEN_T
        if pah_rows is not None:
            pr = pah_rows if isinstance(pah_rows, torch.Tensor) else torch.as_tensor(
                np.ascontiguousarray(pah_rows, np.float64)).to(self.device)
            keep.append(pr)
            o.pah_rows = _ptr(pr)
        tr = tl = None
        if trace_cap > 0:
            tr = torch.zeros(int(n) * trace_cap * TRACE_DTYPE.itemsize, dtype=torch.uint8, device=self.device)
            tl = torch.zeros(int(n), dtype=torch.int32, device=self.device)
            o.trace, o.trace_len, o.trace_cap = _ptr(tr), _ptr(tl), int(trace_cap)
        self._check(lib().mcrt_run(self.ctx, int(first_id), int(n), C.byref(o), C.byref(t), _stream()),
                    "mcrt_run")
        if tr is not None:
            torch.cuda.synchronize()
            recs = tr.cpu().numpy().view(TRACE_DTYPE)
            lens = tl.cpu().numpy()
            return [recs[k * trace_cap:k * trace_cap + lens[k]] for k in range(int(n))]
        return keep

    def run_batched(self, tallies, first_id, n, n_total, seed, batch, **kw):
        """run() over consecutive id ranges of at most `batch` packets (so that
        the deferred tally's records of each range fit its workspace)."""
        keep = []
        for a in range(0, int(n), int(batch)):
            keep += self.run(tallies, int(first_id) + a, min(int(batch), int(n) - a), n_total, seed, **kw) or []
        return keep

    def temperatures(self, nabs, n_total):
        T = torch.empty(self.n_cells * self.n_species, dtype=torch.float64, device=self.device)
        self._check(lib().mcrt_temperatures(self.ctx, _ptr(nabs), int(n_total), _ptr(T), _stream()),
                    "mcrt_temperatures")
        return T.view(self.n_cells, self.n_species)

    def mean_intensity(self, jq, n_total):
        J = torch.empty(self.n_cells * self.n_lambda, dtype=torch.float32, device=self.device)
        self._check(lib().mcrt_mean_intensity(self.ctx, _ptr(jq), int(n_total), _ptr(J), _stream()),
                    "mcrt_mean_intensity")
        return J.view(self.n_cells, self.n_lambda)

    def cell_mass(self):
        """Dust mass per leaf, rho_c V_c (mcrt_cell_mass), float64 [n_cells]."""
        m = torch.empty(self.n_cells, dtype=torch.float64, device=self.device)
        self._check(lib().mcrt_cell_mass(self.ctx, _ptr(m), _stream()), "mcrt_cell_mass")
        return m

    def thin_field(self):
        J = torch.empty(self.n_cells * self.n_lambda, dtype=torch.float32, device=self.device)
        self._check(lib().mcrt_thin_field(self.ctx, _ptr(J), _stream()), "mcrt_thin_field")
        return J.view(self.n_cells, self.n_lambda)

    def layout(self):
        lay = TableLayout()
        self._check(lib().mcrt_table_layout_get(self.ctx, C.byref(lay)), "layout")
        return {n: int(getattr(lay, n)) for n, _ in TableLayout._fields_}

    def tables_numpy(self):
        """Host copies of the device tables (for inspection and tests)."""
        torch.cuda.synchronize()
        raw = self.tables.cpu().numpy()
        lay = self.layout()
        nl, S = self.n_lambda, self.n_species
        K = self.desc.K
        f8 = lambda off, n: raw[off:off + 8 * n].view(np.float64).copy()
        return dict(nu=f8(lay["nu"], nl), dnu=f8(lay["dnu"], nl), src_cdf=f8(lay["src_cdf"], nl),
                    kext=f8(lay["kext"], nl), albedo=f8(lay["albedo"], nl),
                    sp_cdf=f8(lay["sp_cdf"], nl * S).reshape(nl, S), Tk=f8(lay["Tk"], K),
                    E=f8(lay["E"], S * K).reshape(S, K),
                    R=f8(lay["R"], S * (K - 1) * nl).reshape(S, K - 1, nl),
                    level=raw[lay["level"]:lay["level"] + self.n_cells].view(np.int8).copy())
