"""Seeded synthetic inputs for the Monte Carlo dust transfer path.

This module builds the *inputs* of the method and nothing else: wavelength
grids, synthetic grain and PAH cross-section tables, nested cube/subcube grids
with their cell densities, point sources and synthetic radiation fields.  It
holds none of the method's arithmetic (no Planck tables, no optical-depth
march, no temperature inversion, no P(T) solver).  Both the CPU oracle and the
HIP engine consume exactly these arrays.

The workloads follow the dust model of the paper (Sec. 1: silicate,
amorphous-carbon and graphite grains with n(a) ~ a^-3.5, PAHs with 30 and 200
C atoms, 17 Lorentzian emission bands, abundances 31:150:50:30) and the disk of
Sec. 3 (flared disk, gap and spiral density wave), with synthetic optical data
in place of the Mie/laboratory tables the paper takes from the literature.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

AU = 1.495978707e13          # cm
L_SUN = 3.828e33             # erg s^-1
AMU = 1.66053906660e-24      # g
_C = 2.99792458e10           # cm s^-1 (used only to build synthetic fields)
_H = 6.62607015e-27
_K = 1.380649e-16

EQUIL = 0
PAH = 1


# --------------------------------------------------------------------------
# containers
# --------------------------------------------------------------------------
@dataclass
class Grid:
    """Nested cube/subcube grid (Sec. 2: cubes, optionally divided into subcubes).

    Base cubes: nb^3 cubes of side ``base_size`` (cm) starting at ``box_min``.
    ``base_map[ix + nb*(iy + nb*iz)]`` is a leaf id (>= 0) or ``-(node+1)``.
    ``nodes[8*node + o]`` uses the same encoding for octant
    ``o = bx | by<<1 | bz<<2``.  Leaves carry their level and the integer
    coordinates of their lower corner in finest units (2^max_level per base
    cube).
    """
    nb: int
    max_level: int
    box_min: np.ndarray
    base_size: float
    base_map: np.ndarray
    nodes: np.ndarray
    leaf_level: np.ndarray
    leaf_lo: np.ndarray
    rho: np.ndarray = None

    @property
    def n_cells(self) -> int:
        return int(self.leaf_level.shape[0])

    @property
    def n_nodes(self) -> int:
        return int(self.nodes.shape[0] // 8)

    def leaf_boxes_cm(self):
        """(lo, side) of every leaf in cm."""
        fine = self.base_size / (1 << self.max_level)
        lo = self.box_min[None, :] + self.leaf_lo.astype(np.float64) * fine
        side = self.base_size / (2.0 ** self.leaf_level.astype(np.float64))
        return lo, side


@dataclass
class Species:
    """Opacity per gram of dust mixture for each species (mass weight folded in)."""
    lam_um: np.ndarray            # [nl] bin-centre wavelengths
    kabs: np.ndarray              # [S, nl] cm^2 g^-1
    ksca: np.ndarray              # [S, nl] cm^2 g^-1
    g: np.ndarray                 # [nl] HG asymmetry shared by all species
    kind: np.ndarray              # [S] EQUIL or PAH
    names: list = field(default_factory=list)

    @property
    def n_species(self):
        return int(self.kabs.shape[0])

    @property
    def n_lambda(self):
        return int(self.lam_um.shape[0])


@dataclass
class Source:
    pos: np.ndarray               # cm
    lum: float                    # erg s^-1
    teff: float                   # K
    beam: np.ndarray = None       # unit vector for a pencil beam, None = isotropic


@dataclass
class Workload:
    name: str
    grid: Grid
    species: Species
    source: Source
    n_packets: int
    seed: int
    precision: str = "f32"        # transport arithmetic
    tally_j: bool = True
    n_theta: int = 10
    n_phi: int = 1
    K: int = 1024
    T_lo: float = 3.0
    T_hi: float = 5000.0
    max_events: int = 1_000_000
    pah: list = field(default_factory=list)   # PahModel per PAH species


# --------------------------------------------------------------------------
# wavelength grid
# --------------------------------------------------------------------------
def lambda_grid(nl: int, lo_um: float = 0.1, hi_um: float = 1000.0) -> np.ndarray:
    """nl log-spaced wavelengths from lo to hi (inclusive), in micron."""
    return lo_um * (hi_um / lo_um) ** (np.arange(nl, dtype=np.float64) / (nl - 1))


# --------------------------------------------------------------------------
# grids
# --------------------------------------------------------------------------
def _box_distance(lo, hi, p):
    d = np.maximum(np.maximum(lo - p, 0.0), p - hi)
    return np.sqrt((d * d).sum(axis=-1))


def nested_grid(nb: int, box_min, base_size: float, max_level: int,
                refine_centre=None, refine_radius: float = 0.0) -> Grid:
    """Base grid nb^3; a node is divided 2x2x2 while its level < max_level and
    its closest point to ``refine_centre`` lies within ``refine_radius``.

    Leaves are numbered in base raster order (x fastest); the leaves of a
    divided base cube are numbered depth-first, octant order, in its place.
    """
    box_min = np.asarray(box_min, dtype=np.float64)
    L = int(max_level)
    nf = 1 << L
    fine = base_size / nf
    idx = np.arange(nb ** 3, dtype=np.int64)
    base_lo_f = np.stack([idx % nb, (idx // nb) % nb, idx // (nb * nb)], axis=1) * nf

    def refines(level, lo_f):
        if refine_centre is None or level >= L:
            return np.zeros(lo_f.shape[0], dtype=bool)
        lo = box_min + lo_f * fine
        side = base_size / (1 << level)
        return _box_distance(lo, lo + side, np.asarray(refine_centre, np.float64)) < refine_radius

    def children(level, lo):
        half = 1 << (L - level - 1)
        return [np.array([lo[0] + (o & 1) * half, lo[1] + ((o >> 1) & 1) * half,
                          lo[2] + ((o >> 2) & 1) * half], dtype=np.int64) for o in range(8)]

    def count(level, lo):
        if refines(level, lo[None, :])[0]:
            return sum(count(level + 1, c) for c in children(level, lo))
        return 1

    ref0 = refines(0, base_lo_f)
    counts = np.ones(nb ** 3, dtype=np.int64)
    for b in np.nonzero(ref0)[0]:
        counts[b] = count(0, base_lo_f[b])
    offsets = np.concatenate([[0], np.cumsum(counts)[:-1]]).astype(np.int64)
    n_cells = int(counts.sum())
    base_map = offsets.copy()
    leaf_level = np.zeros(n_cells, dtype=np.int8)
    leaf_lo = np.empty((n_cells, 3), dtype=np.int32)
    plain = ~ref0
    leaf_lo[offsets[plain]] = base_lo_f[plain]
    nodes: list = []

    def build(level, lo, nxt):
        if refines(level, lo[None, :])[0]:
            me = len(nodes)
            nodes.append([0] * 8)
            for o, c in enumerate(children(level, lo)):
                nodes[me][o], nxt = build(level + 1, c, nxt)
            return -(me + 1), nxt
        leaf_level[nxt] = level
        leaf_lo[nxt] = lo
        return nxt, nxt + 1

    for b in np.nonzero(ref0)[0]:
        base_map[b], end = build(0, base_lo_f[b], offsets[b])
        assert end == offsets[b] + counts[b]
    nodes_arr = np.array(nodes, dtype=np.int32).reshape(-1) if nodes else np.zeros(0, np.int32)
    return Grid(nb=nb, max_level=L, box_min=box_min, base_size=float(base_size),
                base_map=base_map.astype(np.int32), nodes=nodes_arr,
                leaf_level=leaf_level, leaf_lo=leaf_lo)


def uniform_grid(nb: int, box_min, base_size: float) -> Grid:
    return nested_grid(nb, box_min, base_size, 0)


def subsample_density(grid: Grid, fn, sub: int = 4, chunk: int = 1 << 18) -> np.ndarray:
    """Cell value = mean of fn(x, y, z) [cm] over sub^3 points per leaf."""
    lo, side = grid.leaf_boxes_cm()
    off = (np.arange(sub) + 0.5) / sub
    ox, oy, oz = np.meshgrid(off, off, off, indexing="ij")
    ofs = np.stack([ox.ravel(), oy.ravel(), oz.ravel()], axis=1)    # [sub^3, 3]
    out = np.empty(grid.n_cells, dtype=np.float64)
    for a in range(0, grid.n_cells, chunk):
        b = min(grid.n_cells, a + chunk)
        pts = lo[a:b, None, :] + side[a:b, None, None] * ofs[None, :, :]
        out[a:b] = fn(pts[..., 0], pts[..., 1], pts[..., 2]).mean(axis=1)
    return out


# --------------------------------------------------------------------------
# synthetic grain optics (stand-ins for the Mie tables of Sec. 1)
# --------------------------------------------------------------------------
_MATERIALS = {
    # name: (beta, grain density g cm^-3, A_abs, B_sca, mass weight, size range um)
    "silicate": (2.0, 3.0, 0.3, 1.0, 31.0, (0.006, 0.25)),
    "amC": (1.0, 1.8, 1.0, 0.5, 150.0, (0.006, 0.25)),
    "graphite": (2.0, 2.2, 0.8, 0.5, 50.0, (0.0005, 0.008)),
}


def _q_grain(mat, a_um, lam_um):
    beta, _, A, B, _, _ = _MATERIALS[mat]
    x = 2.0 * np.pi * a_um / lam_um
    y = A * x * lam_um ** (1.0 - beta)
    if mat == "silicate":
        y = y * (1.0 + 2.0 * np.exp(-0.5 * ((lam_um - 9.7) / 1.2) ** 2)
                 + 1.0 * np.exp(-0.5 * ((lam_um - 18.0) / 2.5) ** 2))
    qabs = y / (1.0 + y)
    w = B * x ** 4
    qsca = 1.5 * w / (1.0 + w)
    return qabs, qsca


def grain_species(lam_um, n_sizes=8, materials=("silicate", "amC", "graphite"),
                  extra_weight=0.0):
    """Per-species opacity per gram of the whole mixture.

    Mass weights of the materials follow the abundances 31:150:50 (and
    ``extra_weight`` for PAH, normalised together); sizes are n_sizes log bins
    with number weights from n(a) ~ a^-3.5.
    Returns (kabs, ksca, names, kext_V) with kext_V at 0.55 um.
    """
    wsum = sum(_MATERIALS[m][4] for m in materials) + extra_weight
    kabs, ksca, names, kV = [], [], [], 0.0
    for m in materials:
        beta, rho_gr, _, _, wm, (alo, ahi) = _MATERIALS[m]
        edges = alo * (ahi / alo) ** (np.arange(n_sizes + 1) / n_sizes)
        a = np.sqrt(edges[:-1] * edges[1:])
        nnum = (edges[:-1] ** -2.5 - edges[1:] ** -2.5) / 2.5
        mass = nnum * (4.0 / 3.0) * np.pi * (a * 1e-4) ** 3 * rho_gr
        frac = (wm / wsum) * mass / mass.sum()
        for b in range(n_sizes):
            area = np.pi * (a[b] * 1e-4) ** 2
            m1 = (4.0 / 3.0) * np.pi * (a[b] * 1e-4) ** 3 * rho_gr
            qa, qs = _q_grain(m, a[b], lam_um)
            kabs.append(frac[b] * area * qa / m1)
            ksca.append(frac[b] * area * qs / m1)
            qaV, qsV = _q_grain(m, a[b], np.array([0.55]))
            kV += float(frac[b] * area * (qaV[0] + qsV[0]) / m1)
            names.append(f"{m}_{b}")
    return np.array(kabs), np.array(ksca), names, kV


def hg_g_disk(lam_um):
    """g = 0.6 at 0.1 um falling linearly in log(lambda) to 0 at 10 um, 0 beyond."""
    g = 0.6 * (1.0 - (np.log10(lam_um) + 1.0) / 2.0)
    return np.clip(g, 0.0, 0.6)


# --------------------------------------------------------------------------
# synthetic PAH model (stand-in for the Sec. 1 PAH data)
# --------------------------------------------------------------------------
# 17 Lorentzian bands: centre [um], FWHM [um], integrated strength per C atom
# [cm^2 um].  Synthetic values placed on the usual 3.3-17 um features.
PAH_BANDS = np.array([
    (3.30, 0.040, 3.0e-21), (3.40, 0.030, 0.5e-21), (5.25, 0.060, 0.3e-21),
    (5.70, 0.080, 0.4e-21), (6.20, 0.140, 3.0e-21), (6.90, 0.200, 0.5e-21),
    (7.60, 0.300, 4.0e-21), (7.85, 0.300, 3.5e-21), (8.60, 0.280, 2.5e-21),
    (11.00, 0.100, 0.3e-21), (11.30, 0.180, 4.0e-21), (12.00, 0.300, 1.0e-21),
    (12.70, 0.350, 2.0e-21), (13.55, 0.250, 0.4e-21), (14.20, 0.250, 0.3e-21),
    (16.40, 0.200, 0.4e-21), (17.00, 0.500, 0.8e-21),
])


@dataclass
class PahModel:
    """Synthetic PAH: cross-sections on the wavelength grid and a heat capacity.

    Enthalpy U(T) = N_m k theta (T/theta - atan(T/theta)), N_m = 3 N_C - 6
    vibrational modes: heat capacity ~ T^2 when cold, N_m k when hot.
    """
    n_c: int
    theta: float
    lam_um: np.ndarray
    cabs: np.ndarray          # [nl] cm^2 per molecule (continuum + bands)
    cband: np.ndarray         # [17, nl] band parts
    ccont: np.ndarray         # [nl] non-band part
    mass: float               # g per molecule

    @property
    def n_modes(self):
        return 3 * self.n_c - 6

    def enthalpy(self, T):
        T = np.asarray(T, dtype=np.float64)
        return self.n_modes * _K * self.theta * (T / self.theta - np.arctan(T / self.theta))


def pah_model(n_c: int, lam_um) -> PahModel:
    lam = np.asarray(lam_um, dtype=np.float64)
    x = 1.0 / lam
    drude = (x * 1.0) ** 2 / ((x * x - 4.6 ** 2) ** 2 + (x * 1.0) ** 2)
    fuv = np.where(x > 5.9, 0.1 * (x - 5.9) ** 2, 0.0)
    base = 0.3 + 0.1 * x
    lam_c = 0.35 if n_c <= 50 else 0.60
    y = lam_c / lam
    cut = np.arctan(1.0e3 * (y - 1.0) ** 3 / y) / np.pi + 0.5
    sig_uv = 1.0e-17 * (2.0 * drude + fuv + base) * cut
    # beyond 17 eV (hard UV to X-rays) the per-atom photo-absorption falls as
    # E^-2 from its 17 eV value, a smooth stand-in for the graphite-like
    # scaling the paper uses up to 1 keV (grids that start at 0.1 um never
    # reach it)
    x17 = 17.0 / 1.2398419843320026           # 1/um at 17 eV
    if np.any(x > x17):
        drude17 = x17 ** 2 / ((x17 * x17 - 4.6 ** 2) ** 2 + x17 ** 2)
        s17 = 2.0 * drude17 + 0.1 * (x17 - 5.9) ** 2 + 0.3 + 0.1 * x17
        sig_uv = np.where(x > x17, 1.0e-17 * s17 * (x17 / x) ** 2, sig_uv)
    sig_ir = 2.0e-22 * (lam / 10.0) ** -1.0
    cband = np.empty((PAH_BANDS.shape[0], lam.size))
    for b, (l0, fw, S) in enumerate(PAH_BANDS):
        half = 0.5 * fw
        cband[b] = n_c * S / np.pi * half / ((lam - l0) ** 2 + half * half)
    ccont = n_c * (sig_uv + sig_ir)
    cabs = ccont + cband.sum(axis=0)
    return PahModel(n_c=n_c, theta=800.0, lam_um=lam, cabs=cabs, cband=cband,
                    ccont=ccont, mass=n_c * 12.0 * AMU)


def hard_photon_case(energies_ev=(3.8, 13.6, 50.0, 100.0, 300.0, 1000.0), flux=1.0e4, nl=241,
                     M=1000, n_c=100):
    """The paper's Fig. 3 set-up: a PAH with n_c C atoms in monochromatic
    radiation of flux `flux` (erg s^-1 cm^-2) at each photon energy.
    Wavelength grid 0.001-1000 um (down to 1.24 keV), M enthalpy bins on
    T = 2.7 K .. 5e4 K (the top bin holds more than 1 keV).  Each field lights
    the one bin nearest the energy: 4 pi J_j dnu_j = flux.  Returns a dict
    with lam, the PAH model, T, U, the lit bins and the fields [n_e, nl]."""
    lam = lambda_grid(nl, 0.001, 1000.0)
    pm = pah_model(n_c, lam)
    T = 2.7 * (5.0e4 / 2.7) ** (np.arange(M) / (M - 1))
    U = pm.enthalpy(T)
    ed = np.empty(nl + 1)
    ed[1:-1] = np.sqrt(lam[:-1] * lam[1:])
    ed[0] = lam[0] ** 2 / ed[1]
    ed[-1] = lam[-1] ** 2 / ed[-2]
    nu = _C / (lam * 1e-4)
    dnu = _C / (ed[:-1] * 1e-4) - _C / (ed[1:] * 1e-4)
    hnu_ev = _H * nu / 1.602176634e-12
    bins = [int(np.argmin(np.abs(np.log(hnu_ev / e)))) for e in energies_ev]
    J = np.zeros((len(bins), nl))
    for k, j in enumerate(bins):
        J[k, j] = flux / (4.0 * np.pi * dnu[j])
    return dict(lam=lam, pm=pm, T=T, U=U, bins=bins, hnu_ev=hnu_ev[bins], J=J, flux=flux)


def blackbody_field(lam_um, G0, T_h):
    """J_nu [erg s^-1 cm^-2 Hz^-1 sr^-1] on the grid: shape of a T_h blackbody,
    scaled so that 4 pi * int J_lambda d lambda = G0 * 1.6e-3 erg s^-1 cm^-2
    (trapezoid rule in lambda, over the grid)."""
    lam = np.asarray(lam_um, dtype=np.float64)[None, :] * 1e-4
    G0 = np.atleast_1d(np.asarray(G0, dtype=np.float64))[:, None]
    T_h = np.atleast_1d(np.asarray(T_h, dtype=np.float64))[:, None]
    ex = np.minimum(_H * _C / (lam * _K * T_h), 700.0)
    Blam = 2 * _H * _C ** 2 / lam ** 5 / np.expm1(ex)
    tot = 4 * np.pi * np.trapezoid(Blam, lam[0], axis=1)[:, None]
    Jlam = Blam * (G0 * 1.6e-3) / tot
    return Jlam * lam ** 2 / _C


def pah_fields(n: int, lam_um, seed: int = 4):
    """Synthetic radiation fields: log10 G0 ~ N(3, 1.2^2) truncated to [0, 6],
    blackbody hardness T_h log-uniform in [3000, 40000] K."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lg = np.empty(n)
    filled = 0
    while filled < n:
        draw = rng.normal(3.0, 1.2, size=2 * (n - filled) + 16)
        draw = draw[(draw >= 0.0) & (draw <= 6.0)]
        take = min(n - filled, draw.size)
        lg[filled:filled + take] = draw[:take]
        filled += take
    Th = np.exp(rng.uniform(np.log(3000.0), np.log(40000.0), size=n))
    return blackbody_field(lam_um, 10.0 ** lg, Th), 10.0 ** lg, Th


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------
def pah_test_rows(n_pah: int, n_cells: int, nl: int, seed: int = 3) -> np.ndarray:
    """Seeded stand-in re-emission rows [n_pah][n_cells][nl] for transport
    tests: per cell the running sum of uniform random weights over the bins,
    divided by its total, last entry set to exactly 1 (a valid CDF)."""
    rng = np.random.default_rng(seed)
    rows = np.cumsum(rng.random((n_pah, n_cells, nl)), axis=2)
    rows /= rows[:, :, -1:]
    rows[:, :, -1] = 1.0
    return rows


def c1_sphere(n_packets: int = 100_000, seed: int = 1, nl: int = 100, nb: int = 32,
              tau_v: float = 1.0) -> Workload:
    """Uniform dust sphere R = 10 AU around a 4000 K, 1 L_sun star, 32^3 cells.

    Opacity: lambda <= 1 um gray with albedo 0.5; beyond, kabs ~ lambda^-1.5,
    ksca ~ lambda^-4 (albedo falls to 0).  Isotropic scattering.
    """
    lam = lambda_grid(nl)
    k0 = 1.0e4
    kabs = np.where(lam <= 1.0, k0, k0 * lam ** -1.5)[None, :]
    ksca = np.where(lam <= 1.0, k0, k0 * lam ** -4.0)[None, :]
    R = 10.0 * AU
    rho0 = tau_v / (2.0 * k0 * R)
    grid = uniform_grid(nb, [-R, -R, -R], 2.0 * R / nb)
    lo, side = grid.leaf_boxes_cm()
    c = lo + 0.5 * side[:, None]
    grid.rho = np.where(np.sqrt((c * c).sum(1)) <= R, rho0, 0.0)
    sp = Species(lam_um=lam, kabs=kabs, ksca=ksca, g=np.zeros(nl),
                 kind=np.array([EQUIL], np.int32), names=["gray"])
    src = Source(pos=np.zeros(3), lum=L_SUN, teff=4000.0)
    return Workload("c1_sphere32", grid, sp, src, n_packets, seed, precision="f64",
                    tally_j=False, n_theta=10, n_phi=1)


def _disk_density(rho0, gap_spiral=False):
    r0 = AU

    def fn(x, y, z):
        r = np.sqrt(x * x + y * y)
        rr = np.maximum(r, 1e-30) / r0
        h = 0.1 * r0 * rr ** 1.125
        rho = rho0 / rr * np.exp(-z * z / (2 * h * h))
        rho = np.where((r >= 0.1 * AU) & (r <= 100.0 * AU), rho, 0.0)
        if gap_spiral:
            rau = r / AU
            rho = rho * (1.0 - 0.99 * np.exp(-(rau - 20.0) ** 2 / (2 * 2.0 ** 2)))
            phi = np.arctan2(y, x)
            tp = math.tan(math.radians(15.0))
            d = np.full_like(rau, np.inf)
            for k in range(-5, 2):
                rs = 20.0 * np.exp((phi + 2 * np.pi * k) * tp)
                d = np.minimum(d, np.abs(rau - rs))
            d = d * math.cos(math.radians(15.0))
            rho = rho * (1.0 + 0.5 * np.exp(-d * d / (2 * 1.0 ** 2)))
        return rho
    return fn


def _disk_workload(name, nb, n_packets, seed, nl, gap_spiral, with_pah, n_sizes=8,
                   max_level=3, sub=4):
    lam = lambda_grid(nl)
    extra = 30.0 if with_pah else 0.0
    kabs, ksca, names, kV = grain_species(lam, n_sizes=n_sizes, extra_weight=extra)
    kind = [EQUIL] * kabs.shape[0]
    pahs = []
    if with_pah:
        wsum = 31.0 + 150.0 + 50.0 + 30.0
        for nc in (30, 200):
            pm = pah_model(nc, lam)
            frac = 0.5 * 30.0 / wsum
            kabs = np.vstack([kabs, frac * pm.cabs / pm.mass])
            ksca = np.vstack([ksca, np.zeros(nl)])
            i55 = pah_model(nc, np.array([0.55]))
            kV += float(frac * i55.cabs[0] / i55.mass)
            kind.append(PAH)
            names.append(f"pah{nc}")
            pahs.append(pm)
    tau_mid = 100.0
    rho0 = tau_mid / (kV * AU * math.log(1000.0))
    box = 100.0 * AU
    grid = nested_grid(nb, [-box, -box, -box], 2 * box / nb, max_level,
                       refine_centre=np.zeros(3), refine_radius=1.0 * AU)
    grid.rho = subsample_density(grid, _disk_density(rho0, gap_spiral), sub=sub)
    sp = Species(lam_um=lam, kabs=kabs, ksca=ksca, g=hg_g_disk(lam),
                 kind=np.array(kind, np.int32), names=names)
    src = Source(pos=np.zeros(3), lum=L_SUN, teff=5800.0)
    return Workload(name, grid, sp, src, n_packets, seed, precision="f32", tally_j=True,
                    n_theta=10, n_phi=8 if gap_spiral else 1, pah=pahs)


def c2_disk(n_packets: int = 10_000_000, seed: int = 2, nl: int = 200, nb: int = 64) -> Workload:
    """Flared disk, 64^3 base cubes + 2x2x2 refinement to depth 3 inside 1 AU,
    3 materials x 8 sizes, 200 wavelengths, HG g(lambda), 1e7 packets."""
    return _disk_workload(f"c2_disk{nb}", nb, n_packets, seed, nl, False, False)


def c3_gap_spiral(n_packets: int = 100_000_000, seed: int = 3, nl: int = 200,
                  nb: int = 128) -> Workload:
    """C2 disk x planet gap at 20 AU x log spiral (pitch 15 deg), 128^3 base,
    plus PAH species with 30 and 200 C atoms."""
    return _disk_workload(f"c3_gapspiral{nb}", nb, n_packets, seed, nl, True, True)


def c5_full(n_packets: int = 1_000_000_000, seed: int = 5, nl: int = 200, nb: int = 256) -> Workload:
    """C3 physics on a 256^3 base grid refined to depth 3 inside 1 AU
    (16,784,776 leaves), 1e9 packets.  Cell densities are means over 2^3
    sub-samples per leaf (4^3 for the smaller disks) to keep the build short."""
    return _disk_workload(f"c5_gapspiral{nb}", nb, n_packets, seed, nl, True, True, sub=2)


def small_disk(n_packets: int = 20_000, seed: int = 2, nl: int = 40, nb: int = 16,
               n_sizes: int = 2, max_level: int = 3, with_pah: bool = False,
               gap_spiral: bool = False) -> Workload:
    """Reduced disk with the C2 structure (nested grid, several species, HG;
    optionally the C3 gap, spiral and PAH species) sized for the oracle to
    finish in seconds."""
    return _disk_workload(f"small_disk{nb}", nb, n_packets, seed, nl, gap_spiral, with_pah,
                          n_sizes=n_sizes, max_level=max_level)


def uniform_cube(n: int, alpha_per_cell: float, albedo: float = 0.0, nl: int = 4,
                 seed: int = 7, n_packets: int = 1000, precision: str = "f64",
                 g: float = 0.0) -> Workload:
    """n^3 unit-density cube of side n cm (cells of 1 cm) with a gray opacity
    giving ``alpha_per_cell`` extinction per cell side; star at the centre."""
    lam = lambda_grid(nl)
    kext = alpha_per_cell
    kabs = np.full((1, nl), kext * (1.0 - albedo))
    ksca = np.full((1, nl), kext * albedo)
    grid = uniform_grid(n, [0.0, 0.0, 0.0], 1.0)
    grid.rho = np.ones(grid.n_cells)
    sp = Species(lam_um=lam, kabs=kabs, ksca=ksca, g=np.full(nl, g),
                 kind=np.array([EQUIL], np.int32), names=["gray"])
    src = Source(pos=np.full(3, n / 2.0), lum=1.0, teff=5000.0)
    return Workload(f"cube{n}", grid, sp, src, n_packets, seed, precision=precision,
                    tally_j=True, n_theta=4, n_phi=1)
