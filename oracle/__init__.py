"""CPU oracle (FP64) for the Monte Carlo dust transfer path.

TEST INFRASTRUCTURE ONLY.  Imported by ``tests/``, by the smoke check of
``__graft_entry__`` and by the CPU-baseline leg of ``bench.py``; the product
package never imports it.  The C sources (``mcrt_oracle.c``) are compiled with
gcc into ``liboracle`` on first use (or by ``build()``); the MLP reference is
plain numpy in ``oracle.mlp``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mcrt_oracle.c")
_HDR = os.path.join(_HERE, "mcrt_oracle.h")
_LIB = os.path.join(_HERE, "libmcrt_oracle.so")
_lib = None

CNT = dict(launched=0, escaped=1, killed=2, terminated=3, scatters=4, absorptions=5,
           crossings=6, tclamp_lo=7, tclamp_hi=8, pah_abs=9, zero_cross=10, jseg=11, peel=12)
FLAG_TALLY_J, FLAG_FROZEN_T, FLAG_KILL_ON_ABSORB, FLAG_EXACT_BW, FLAG_PEEL, FLAG_PEEL_SED = 1, 2, 4, 8, 16, 32
PEEL_ONE = 1 << 24                     # fixed-point unit of the next-event images
EV_LAUNCH, EV_CROSS, EV_SCATTER, EV_ABSORB, EV_ESCAPE, EV_KILLED = range(6)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no fast-math, no FP contraction)."""
    cmd = ["gcc", "-O2", "-march=native", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-o", _LIB + ".tmp", _SRC, "-lm"]
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(
            os.path.getmtime(_SRC), os.path.getmtime(_HDR)):
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class TraceRec(C.Structure):
    _fields_ = [("type", C.c_int32), ("cell", C.c_int32), ("j", C.c_int32), ("pad", C.c_int32),
                ("x", C.c_double * 3), ("d", C.c_double * 3), ("tau", C.c_double)]


TRACE_DTYPE = np.dtype([("type", np.int32), ("cell", np.int32), ("j", np.int32),
                        ("pad", np.int32), ("x", np.float64, 3), ("d", np.float64, 3),
                        ("tau", np.float64)])

_dp = C.POINTER(C.c_double)
_i32p = C.POINTER(C.c_int32)
_u64p = C.POINTER(C.c_uint64)


class Problem(C.Structure):
    _fields_ = [("nl", C.c_int32), ("S", C.c_int32),
                ("lam_um", _dp), ("kabs", _dp), ("ksca", _dp), ("g", _dp), ("kind", _i32p),
                ("nb", C.c_int32), ("L", C.c_int32), ("n_cells", C.c_int64), ("n_nodes", C.c_int64),
                ("box_min", C.c_double * 3), ("base_size", C.c_double),
                ("base_map", _i32p), ("nodes", _i32p), ("rho", _dp),
                ("src_pos", C.c_double * 3), ("lum", C.c_double), ("teff", C.c_double),
                ("beam", C.c_double * 3), ("beam_on", C.c_int32),
                ("K", C.c_int32), ("T_lo", C.c_double), ("T_hi", C.c_double),
                ("n_total", C.c_uint64), ("seed", C.c_uint64), ("max_events", C.c_uint64),
                ("n_theta", C.c_int32), ("n_phi", C.c_int32), ("flags", C.c_int32),
                ("n_threads", C.c_int32), ("frozen_nabs", _u64p), ("pah_rows", _dp),
                ("n_obs", C.c_int32), ("npix", C.c_int32), ("n_img_lambda", C.c_int32), ("pad_img", C.c_int32),
                ("img_lambda", C.c_int32 * 8), ("img_center", C.c_double * 3), ("img_half_width", C.c_double),
                ("img_cos_cone", C.c_double), ("obs_dir", (C.c_double * 3) * 8),
                ("pah_row_map", _i32p)]


class Tables(C.Structure):
    _fields_ = [(n, _dp) for n in ("nu", "dnu", "src_cdf", "kext", "albedo", "sp_cdf", "Tk", "E", "R")]


class Out(C.Structure):
    _fields_ = [("nabs", _u64p), ("sed", _u64p), ("jq", _u64p), ("counters", _u64p), ("image", _u64p),
                ("trace", C.c_void_p), ("trace_len", _i32p), ("trace_cap", C.c_int64),
                ("peel", _u64p), ("peel_sed", _u64p)]


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = C.CDLL(_LIB)
        L.orc_philox4x32_10.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)]
        L.orc_u24.restype = C.c_double
        L.orc_u24.argtypes = [C.c_uint32]
        L.orc_planck_nu.restype = C.c_double
        L.orc_planck_nu.argtypes = [C.c_double, C.c_double]
        L.orc_lambda_bins.argtypes = [C.c_int32, _dp, _dp, _dp]
        L.orc_build_tables.argtypes = [C.POINTER(Problem), C.POINTER(Tables)]
        L.orc_locate.restype = C.c_int
        L.orc_locate.argtypes = [C.POINTER(Problem), C.POINTER(C.c_int64), _i32p, C.POINTER(C.c_int64)]
        L.orc_transport.restype = C.c_int
        L.orc_transport.argtypes = [C.POINTER(Problem), C.POINTER(Tables), C.c_uint64, C.c_uint64, C.POINTER(Out)]
        L.orc_temperatures.argtypes = [C.POINTER(Problem), C.POINTER(Tables), _u64p, _dp]
        L.orc_mean_intensity.argtypes = [C.POINTER(Problem), C.POINTER(Tables), _u64p, _dp]
        L.orc_pah_solve.argtypes = [C.c_int32, _dp, _dp, C.c_int32, _dp, _dp, _dp, C.c_int32, _dp, _dp,
                                    C.c_int64, _dp, _dp, _dp, C.c_int32]
        L.orc_pah_rates.argtypes = [C.c_int32, _dp, _dp, C.c_int32, _dp, _dp, _dp, _dp, _dp]
        L.orc_thin_field.argtypes = [C.POINTER(Problem), C.POINTER(Tables), _dp]
        L.orc_pah_rows.argtypes = [C.c_int32, C.c_int32, _dp, _dp, _dp, C.c_int64, _dp]
        _lib = L
    return _lib


def _p(a, typ=_dp):
    return a.ctypes.data_as(typ) if a is not None else None


def philox(ctr, key):
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def u24(w):
    return lib().orc_u24(int(w) & 0xFFFFFFFF)


def planck_nu(nu, T):
    return lib().orc_planck_nu(float(nu), float(T))


def lambda_bins(lam_um):
    lam = np.ascontiguousarray(lam_um, dtype=np.float64)
    nu = np.empty_like(lam)
    dnu = np.empty_like(lam)
    lib().orc_lambda_bins(lam.size, _p(lam), _p(nu), _p(dnu))
    return nu, dnu


class Session:
    """Holds the ctypes problem for one workload (keeps its arrays alive)."""

    def __init__(self, w, n_threads: int = 1, n_total: int | None = None, seed: int | None = None,
                 flags: int | None = None, frozen_nabs=None, pah_rows=None, max_events=None,
                 observers=None, pah_row_map=None):
        """pah_rows: dense [n_pah][n_cells][nl] CDF rows, or with pah_row_map
        (int32 [n_pah * n_cells]) a compact table [n_rows][nl] indexed by it."""
        g, sp, src = w.grid, w.species, w.source
        self.w = w
        self._keep = []

        def keep(a, dt):
            a = np.ascontiguousarray(a, dtype=dt)
            self._keep.append(a)
            return a
        p = Problem()
        p.nl, p.S = sp.n_lambda, sp.n_species
        p.lam_um = _p(keep(sp.lam_um, np.float64))
        p.kabs = _p(keep(sp.kabs, np.float64))
        p.ksca = _p(keep(sp.ksca, np.float64))
        p.g = _p(keep(sp.g, np.float64))
        p.kind = _p(keep(sp.kind, np.int32), _i32p)
        p.nb, p.L = g.nb, g.max_level
        p.n_cells, p.n_nodes = g.n_cells, g.n_nodes
        p.box_min = (C.c_double * 3)(*g.box_min)
        p.base_size = g.base_size
        p.base_map = _p(keep(g.base_map, np.int32), _i32p)
        p.nodes = _p(keep(g.nodes if g.nodes.size else np.zeros(8, np.int32), np.int32), _i32p)
        p.rho = _p(keep(g.rho, np.float64))
        p.src_pos = (C.c_double * 3)(*src.pos)
        p.lum, p.teff = src.lum, src.teff
        if src.beam is not None:
            p.beam = (C.c_double * 3)(*src.beam)
            p.beam_on = 1
        p.K, p.T_lo, p.T_hi = w.K, w.T_lo, w.T_hi
        p.n_total = int(n_total if n_total is not None else w.n_packets)
        p.seed = int(seed if seed is not None else w.seed)
        p.max_events = int(max_events if max_events is not None else w.max_events)
        p.n_theta, p.n_phi = w.n_theta, w.n_phi
        p.flags = int(flags if flags is not None else (FLAG_TALLY_J if w.tally_j else 0))
        p.n_threads = int(n_threads)
        if frozen_nabs is not None:
            p.frozen_nabs = _p(keep(frozen_nabs, np.uint64), _u64p)
            p.flags |= FLAG_FROZEN_T
        if pah_rows is not None:
            p.pah_rows = _p(keep(pah_rows, np.float64))
        if pah_row_map is not None:
            rm = keep(pah_row_map, np.int32)
            n_pah = int((np.asarray(sp.kind) == 1).sum())
            n_rows = np.asarray(pah_rows).reshape(-1, sp.n_lambda).shape[0]
            assert rm.size == n_pah * g.n_cells and rm.min() >= 0 and rm.max() < n_rows
            p.pah_row_map = _p(rm, _i32p)
        if observers is not None:
            ob = observers
            p.n_obs, p.npix = len(ob["dirs"]), int(ob["npix"])
            p.n_img_lambda = len(ob["lambda_bins"])
            for q, jb in enumerate(ob["lambda_bins"]):
                p.img_lambda[q] = int(jb)
            p.img_center = (C.c_double * 3)(*ob["center"])
            p.img_half_width, p.img_cos_cone = float(ob["half_width"]), float(ob["cos_cone"])
            for q, dv in enumerate(ob["dirs"]):
                for a in range(3):
                    p.obs_dir[q][a] = float(dv[a])
        self.p = p
        self.tables = self._build_tables()

    def _build_tables(self):
        p = self.p
        nl, S, K = p.nl, p.S, p.K
        t = dict(nu=np.zeros(nl), dnu=np.zeros(nl), src_cdf=np.zeros(nl), kext=np.zeros(nl),
                 albedo=np.zeros(nl), sp_cdf=np.zeros(nl * S), Tk=np.zeros(K), E=np.zeros(S * K),
                 R=np.zeros(S * (K - 1) * nl))
        T = Tables(**{k: _p(v) for k, v in t.items()})
        lib().orc_build_tables(C.byref(p), C.byref(T))
        self._T = T
        self._tarr = t
        out = dict(t)
        out["sp_cdf"] = t["sp_cdf"].reshape(nl, S)
        out["E"] = t["E"].reshape(S, K)
        out["R"] = t["R"].reshape(S, K - 1, nl)
        return out

    def transport(self, first_id: int = 0, n: int | None = None, trace_cap: int = 0):
        p = self.p
        n = int(n if n is not None else p.n_total)
        nabs = np.zeros(p.n_cells * p.S, np.uint64)
        sed = np.zeros(p.n_theta * p.n_phi * p.nl, np.uint64)
        jq = np.zeros(p.nl * p.n_cells, np.uint64) if (p.flags & FLAG_TALLY_J) else None
        cnt = np.zeros(16, np.uint64)
        img = np.zeros(p.n_obs * p.n_img_lambda * p.npix * p.npix, np.uint64) if p.n_obs > 0 else None
        peel = np.zeros_like(img) if (img is not None and p.flags & FLAG_PEEL) else None
        psed = np.zeros(p.n_obs * p.nl, np.uint64) if (peel is not None and p.flags & FLAG_PEEL_SED) else None
        o = Out(nabs=_p(nabs, _u64p), sed=_p(sed, _u64p), jq=_p(jq, _u64p), counters=_p(cnt, _u64p),
                image=_p(img, _u64p), peel=_p(peel, _u64p), peel_sed=_p(psed, _u64p))
        tr = tl = None
        if trace_cap > 0:
            tr = np.zeros(n * trace_cap, TRACE_DTYPE)
            tl = np.zeros(n, np.int32)
            o.trace = tr.ctypes.data
            o.trace_len = _p(tl, _i32p)
            o.trace_cap = trace_cap
        rc = lib().orc_transport(C.byref(p), C.byref(self._T), first_id, n, C.byref(o))
        if rc != 0:
            raise RuntimeError(f"orc_transport failed: {rc}")
        res = dict(nabs=nabs.reshape(p.n_cells, p.S),
                   sed=sed.reshape(p.n_theta, p.n_phi, p.nl), counters=cnt,
                   jq=jq.reshape(p.nl, p.n_cells) if jq is not None else None,
                   image=img.reshape(p.n_obs, p.n_img_lambda, p.npix, p.npix) if img is not None else None,
                   peel=peel.reshape(p.n_obs, p.n_img_lambda, p.npix, p.npix) if peel is not None else None,
                   peel_sed=psed.reshape(p.n_obs, p.nl) if psed is not None else None)
        if tr is not None:
            res["trace"] = [tr[k * trace_cap:k * trace_cap + tl[k]] for k in range(n)]
        return res

    def accumulate(self, acc, first_id: int, n: int):
        """Run packets [first_id, first_id+n) adding into acc (dict of uint64 arrays
        nabs, sed, jq, counters as made by new_accumulator)."""
        o = Out(nabs=_p(acc["nabs"], _u64p), sed=_p(acc["sed"], _u64p),
                jq=_p(acc.get("jq"), _u64p), counters=_p(acc["counters"], _u64p),
                image=_p(acc.get("image"), _u64p), peel=_p(acc.get("peel"), _u64p),
                peel_sed=_p(acc.get("peel_sed"), _u64p))
        rc = lib().orc_transport(C.byref(self.p), C.byref(self._T), first_id, n, C.byref(o))
        if rc != 0:
            raise RuntimeError(f"orc_transport failed: {rc}")
        return acc

    def new_accumulator(self):
        p = self.p
        return dict(nabs=np.zeros(p.n_cells * p.S, np.uint64),
                    sed=np.zeros(p.n_theta * p.n_phi * p.nl, np.uint64),
                    jq=np.zeros(p.nl * p.n_cells, np.uint64) if (p.flags & FLAG_TALLY_J) else None,
                    counters=np.zeros(16, np.uint64),
                    image=np.zeros(p.n_obs * p.n_img_lambda * p.npix * p.npix, np.uint64) if p.n_obs else None,
                    peel=np.zeros(p.n_obs * p.n_img_lambda * p.npix * p.npix, np.uint64)
                    if (p.n_obs and p.flags & FLAG_PEEL) else None,
                    peel_sed=np.zeros(p.n_obs * p.nl, np.uint64)
                    if (p.n_obs and p.flags & FLAG_PEEL and p.flags & FLAG_PEEL_SED) else None)

    def temperatures(self, nabs):
        p = self.p
        nabs = np.ascontiguousarray(nabs, np.uint64).reshape(-1)
        T = np.zeros(p.n_cells * p.S)
        lib().orc_temperatures(C.byref(p), C.byref(self._T), _p(nabs, _u64p), _p(T))
        return T.reshape(p.n_cells, p.S)

    def mean_intensity(self, jq):
        p = self.p
        jq = np.ascontiguousarray(jq, np.uint64).reshape(-1)
        J = np.zeros(p.n_cells * p.nl)
        lib().orc_mean_intensity(C.byref(p), C.byref(self._T), _p(jq, _u64p), _p(J))
        return J.reshape(p.n_cells, p.nl)

    def thin_field(self):
        p = self.p
        J = np.zeros(p.n_cells * p.nl)
        lib().orc_thin_field(C.byref(p), C.byref(self._T), _p(J))
        return J.reshape(p.n_cells, p.nl)

    def locate(self, F):
        F = (C.c_int64 * 3)(*[int(v) for v in F])
        lev = C.c_int32()
        lo = (C.c_int64 * 3)()
        c = lib().orc_locate(C.byref(self.p), F, C.byref(lev), lo)
        return c, lev.value, tuple(lo)


def pah_rates(T, U, lam_um, cabs, J):
    M = len(T)
    T, U = np.ascontiguousarray(T, np.float64), np.ascontiguousarray(U, np.float64)
    lam, ca, Jc = (np.ascontiguousarray(a, np.float64) for a in (lam_um, cabs, J))
    A = np.zeros((M, M))
    Ad = np.zeros(M)
    lib().orc_pah_rates(M, _p(T), _p(U), lam.size, _p(lam), _p(ca), _p(Jc), _p(A), _p(Ad))
    return A, Ad


def pah_solve(T, U, lam_um, cabs, cband, ccont, J, n_threads: int = 1, want_P: bool = False):
    """Steady-state P(T) and emission for each field row of J [n, nl].
    Returns (out [n, n_bands+nl], P [n, M] or None, pabs [n])."""
    T, U = np.ascontiguousarray(T, np.float64), np.ascontiguousarray(U, np.float64)
    lam, ca, cb, cc = (np.ascontiguousarray(a, np.float64) for a in (lam_um, cabs, cband, ccont))
    J = np.ascontiguousarray(np.atleast_2d(J), np.float64)
    n, nl = J.shape
    nbd = cb.shape[0]
    out = np.zeros((n, nbd + nl))
    P = np.zeros((n, len(T))) if want_P else None
    pabs = np.zeros(n)
    lib().orc_pah_solve(len(T), _p(T), _p(U), nl, _p(lam), _p(ca), _p(cb), nbd, _p(cc), _p(J), n,
                        _p(out), _p(P), _p(pabs), n_threads)
    return out, P, pabs


def cell_mass(grid):
    """Dust mass per leaf, rho_c V_c, with V_c = (base_size 2^-level_c)^3."""
    side = grid.base_size * np.ldexp(1.0, -np.asarray(grid.leaf_level, np.int64))
    return np.asarray(grid.rho, np.float64) * side ** 3


def band_power(out, mass, n_bands):
    """Emitted band powers summed over cells: sum_c mass_c out[c, b] for the
    first n_bands outputs (the quantity whose change between passes ends the
    PAH iteration)."""
    out = np.asarray(out, np.float64)
    return np.asarray(mass, np.float64) @ out[:, :n_bands]


def pah_rows(lam_um, cband, out):
    """Re-emission CDF rows [n, nl] from solver outputs [n, n_bands + nl]."""
    lam = np.ascontiguousarray(lam_um, np.float64)
    cb = np.ascontiguousarray(cband, np.float64)
    o = np.ascontiguousarray(np.atleast_2d(out), np.float64)
    rows = np.zeros((o.shape[0], lam.size))
    lib().orc_pah_rows(lam.size, cb.shape[0], _p(lam), _p(cb), _p(o), o.shape[0], _p(rows))
    return rows


def psf_convolve(images, scale, fwhm_pix):
    """Images [..., npix, npix] times scale, convolved with a Gaussian point
    spread function of full width at half maximum fwhm_pix pixels (paper
    Sec. 4, Fig. 2): sigma = fwhm / (2 sqrt(2 ln 2)), taps |dx|, |dy| <= r =
    ceil(3 sigma), weights exp(-(dx^2 + dy^2) / (2 sigma^2)) normalised to unit
    sum over that square, zero outside the image.  Plain sum over shifts."""
    img = np.asarray(images, dtype=np.float64) * float(scale)
    sigma = fwhm_pix / (2.0 * np.sqrt(2.0 * np.log(2.0)))
    r = int(np.ceil(3.0 * sigma))
    if sigma > 0:
        d = np.arange(-r, r + 1, dtype=np.float64)
        w1 = np.exp(-d * d / (2.0 * sigma * sigma))
        w1 /= w1.sum()
    else:
        w1 = np.ones(1)
    n = img.shape[-1]
    pad = np.zeros(img.shape[:-2] + (n + 2 * r, n + 2 * r))
    pad[..., r:r + n, r:r + n] = img
    out = np.zeros_like(img)
    for dy in range(-r, r + 1):
        for dx in range(-r, r + 1):
            out += w1[dy + r] * w1[dx + r] * pad[..., r + dy:r + dy + n, r + dx:r + dx + n]
    return out
