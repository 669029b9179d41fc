#!/usr/bin/env python3
"""Benchmark of the Monte Carlo dust transfer hot path on one MI355X.

Headline workload (the largest configuration): the gap + spiral
proto-planetary disk with PAHs on a 256^3 base grid refined 2x2x2 to depth 3
inside 1 AU (16,784,776 leaves), 24 grain species (3 materials x 8 sizes) and
2 PAH species (30 and 200 C atoms), 200 wavelengths, Henyey-Greenstein
scattering, 1e9 packets per pass from a 5800 K, 1 L_sun star; FP32 geometry,
FP64 tables and temperatures, integer tallies, path-length J tally on, the
surrogate network in the loop for the PAH emission with the exact solver as
fallback on flagged cells.

One step = one pass of the PAH iteration through every step of the hot path:
  table build -> PAH emission of both PAH species from the previous pass's
  mean intensity (surrogate + exact fallback) and their re-emission rows ->
  transport of all 1e9 packets (path-length tally through segment records,
  id ranges that fit the record workspace) -> temperatures -> mean intensity
  -> band powers (the iteration's stop quantity).
Before the timed region (untimed): the grid, pass 0 (thin starlight field,
exact PAH emission, one transport pass) and the surrogates' training on
exactly solved cells of that pass's field plus synthetic fields.  Inputs are
resident in device memory when the timed region starts.  Prints one JSON line;
extra blocks time the smaller disks, the re-emission law comparison and the
paper's Fig. 2 / Fig. 3 set-ups.  The CPU oracle is timed on a bounded sample
of the same workload for reference.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "photon packets/sec + cell-crossings/sec (1 GPU); PAH cells/sec surrogate vs exact"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print("bench: " + msg, file=sys.stderr, flush=True)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_transport_gap_spiral_256_pmc.md")
TRAFFIC_SOURCES = ("mcrt_transport.hip", "mcrt_internal.h")


def committed_traffic():
    """HBM bytes per packet of k_transport from the committed counter summary,
    if it was taken on the current source of that kernel; else None."""
    import hashlib
    try:
        h = hashlib.sha256()
        for f in TRAFFIC_SOURCES:
            h.update(open(os.path.join(ROOT, "paper_1201_3588_amd", "csrc", f), "rb").read())
        kv = dict(l.strip().split(": ", 1) for l in open(TRAFFIC_FILE)
                  if l.startswith(("traffic_bytes_per_packet:", "source_sha256:")))
        if kv.get("source_sha256") == h.hexdigest():
            return float(kv["traffic_bytes_per_packet"])
    except (OSError, ValueError, KeyError):
        pass
    return None


def random_atomic_rate(n_slots, stream):
    """Achievable rate of random 64-bit atomic adds over a table of n_slots
    words (the size of the path-length tally), measured with HIP events."""
    import ctypes as C
    import torch
    from paper_1201_3588_amd import mcrt
    table = torch.zeros(n_slots, dtype=torch.int64, device="cuda")
    n_ops = 1 << 28
    L = mcrt.lib()
    L.mcrt_bench_random.argtypes = [C.c_void_p, C.c_uint64, C.c_void_p, C.c_uint64, C.c_uint64,
                                    C.c_uint64, C.c_int32, C.c_void_p, C.c_void_p]
    s = C.c_void_p(stream.cuda_stream)
    L.mcrt_bench_random(C.c_void_p(table.data_ptr()), n_slots, None, 0, n_ops, 1, 0, None, s)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    L.mcrt_bench_random(C.c_void_p(table.data_ptr()), n_slots, None, 0, n_ops, 2, 0, None, s)
    e1.record(stream)
    torch.cuda.synchronize()
    issued = int(table.sum().item()) // 2
    del table
    return issued / (e0.elapsed_time(e1) / 1e3)


def c3_block(n_packets, micro, stream, iterate=True):
    """The gap + spiral disk with PAHs (128^3 base, depth 3, 2,098,552 leaves,
    26 species, 200 bins): PAH re-emission rows from the optically thin field
    (first pass of the PAH iteration, exact solver), then one timed transport
    pass whose 3.4 GB path-length tally is HBM resident."""
    import torch
    import synth
    from paper_1201_3588_amd import mcrt
    from paper_1201_3588_amd.pipeline import PahLoop
    t0 = time.perf_counter()
    w = synth.c3_gap_spiral(n_packets=n_packets)
    t_synth = time.perf_counter() - t0
    loop = PahLoop(w)
    eng = loop.eng
    N = w.n_packets
    # deferred path tally: about 131 segment records per packet here; the
    # workspace takes the device memory that is free (up to 2^33 records, 137 GB)
    # and the pass runs in id ranges whose records fit it with 8 % to spare
    free = torch.cuda.mem_get_info()[0]
    cap = min(1 << 33, max(1 << 22, (free - (24 << 30)) // 16)) // 4096 * 4096
    deferred = eng.set_deferred_tally(cap)
    batch = min(N, int(cap / (1.08 * 131))) if deferred else N
    J = eng.thin_field()
    torch.cuda.synchronize()
    p0 = torch.cuda.Event(enable_timing=True)
    p1 = torch.cuda.Event(enable_timing=True)
    p0.record(stream)
    loop.emission(J)
    p1.record(stream)
    del J
    tal = eng.new_tallies(tally_j=True)
    eng.run(tal, 0, min(N, 2_000_000), N, w.seed, pah_rows=loop.rows)        # warm-up
    for v in (t for t in tal.values() if t is not None):
        v.zero_()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    eng.run_batched(tal, 0, N, N, w.seed, batch, pah_rows=loop.rows)
    e1.record(stream)
    torch.cuda.synchronize()
    dt = e0.elapsed_time(e1) / 1e3
    c = mcrt.u64_view(tal["counters"])
    cnt = {k: int(c[v]) for k, v in mcrt.CNT.items()}
    assert cnt["launched"] == N and cnt["launched"] == cnt["escaped"] + cnt["killed"] + cnt["terminated"]
    alg = 8 * cnt["crossings"] + 16 * (cnt["jseg"] + cnt["absorptions"] + cnt["escaped"])
    res = {"workload": "gap_spiral_disk_128cube_depth3_2098552leaves_26species_200lambda_1e8packets_pah",
           "leaves": w.grid.n_cells, "packets": N, "transport_kernel_ms": dt * 1e3,
           "path_tally": f"deferred records, id ranges of {batch} packets" if deferred else "atomic",
           "packets_per_s": N / dt, "crossings_per_s": cnt["crossings"] / dt, "per_pass_counts": cnt,
           "pah_rows_from_thin_field_ms": p0.elapsed_time(p1),
           "pah_cells_solved": 2 * w.grid.n_cells, "synth_build_s": t_synth,
           "roofline": {"bound": "hbm", "achieved": alg / dt / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": alg / dt / 1e9 / HBM_PEAK_GBS, "traffic": None,
                        "kernel": "transport pass (k_transport + record passes per id range)" if deferred
                                  else "k_transport<float,false,false,false>",
                        "alg_bytes_per_launch": alg}}
    res["images"] = images_block(w, eng, loop.rows, stream, dt, batch)
    if iterate:
        # the PAH iteration to convergence (emitted band power of both PAH
        # species changing by less than 1 % between passes), from the thin field
        t_it = time.perf_counter()
        it = loop.run(n_iter=6, tol=0.01, batch=batch)
        torch.cuda.synchronize()
        hist = it["history"]
        res["pah_iteration"] = {"passes": len(hist), "wall_s": time.perf_counter() - t_it,
                                "converged": hist[-1]["change"] is not None and hist[-1]["change"] < 0.01,
                                "band_power_change_per_pass": [h["change"] for h in hist],
                                "pah_absorptions_per_pass": [h["pah_abs"] for h in hist]}
        del it
    del tal, loop, eng
    if micro:
        rate = random_atomic_rate(w.species.n_lambda * w.grid.n_cells, stream)
        tr = (cnt["jseg"] + cnt["absorptions"] + cnt["escaped"]) / dt
        res["random_access_ceiling"] = {"atomics_per_s": rate, "table_bytes": w.species.n_lambda * w.grid.n_cells * 8,
                                        "tally_updates_per_s": tr, "frac_of_ceiling": tr / rate}
    return res


def reemission_block(w, stream, label):
    """The re-emission law: the paper's (bracket of the temperature before the
    absorption) against the Bjorkman-Wood difference spectrum of the
    absorption's own temperature rise, one full pass of each with the same
    seed and running absorption counts.  Reports the transport rate of each,
    the mean relative temperature difference per decade of absorptions in the
    (cell, species) pair with its standard error, and the total-variation
    distance between the escaping spectra beside that of two seeds of the
    paper's law (the Monte Carlo noise floor)."""
    import torch
    from paper_1201_3588_amd import mcrt
    eng = mcrt.Engine.from_workload(w)
    eng.build_tables(w.source.pos, w.source.lum, w.source.teff)
    N = w.n_packets
    runs = {}
    for name, flags, seed in (("before", 0, w.seed), ("exact_bw", mcrt.FLAG_EXACT_BW, w.seed),
                              ("before_seed2", 0, w.seed + 7)):
        tal = eng.new_tallies(tally_j=w.tally_j)
        fl = flags | (mcrt.FLAG_TALLY_J if w.tally_j else 0)
        eng.run(tal, 0, min(N, 1_000_000), N, seed, flags=fl)                 # warm-up
        for v in (t for t in tal.values() if t is not None):
            v.zero_()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        eng.run(tal, 0, N, N, seed, flags=fl)
        e1.record(stream)
        T = eng.temperatures(tal["nabs"], N)
        torch.cuda.synchronize()
        sed = tal["sed"].reshape(-1, w.species.n_lambda).sum(0).double()
        runs[name] = dict(ms=e0.elapsed_time(e1), T=T.reshape(-1),
                          n=tal["nabs"].reshape(-1).double(), sed=sed / sed.sum())
        del tal
    a, b = runs["before"], runs["exact_bw"]
    both = (a["n"] > 0) & (b["n"] > 0)
    nmean = 0.5 * (a["n"] + b["n"])
    rel = a["T"] / b["T"] - 1.0
    bins = []
    for lo in (1, 10, 100, 1000, 10000, 100000):
        m = both & (nmean >= lo) & (nmean < 10 * lo)
        k = int(m.sum().item())
        if k < 10:
            continue
        r = rel[m]
        bins.append({"n_abs_from": lo, "pairs": k, "mean_rel_T_diff": float(r.mean().item()),
                     "stderr": float((r.std() / k ** 0.5).item()),
                     "median_rel_T_diff": float(r.median().item())})
    tv = 0.5 * float((a["sed"] - b["sed"]).abs().sum().item())
    tv0 = 0.5 * float((a["sed"] - runs["before_seed2"]["sed"]).abs().sum().item())
    absorbed = float(a["n"].sum().item())
    return {"workload": label, "packets": N, "absorptions_per_dusty_pair": absorbed / int((a["n"] > 0).sum().item()),
            "transport_ms": {"before": a["ms"], "exact_bw": b["ms"]},
            "packets_per_s": {"before": N / a["ms"] * 1e3, "exact_bw": N / b["ms"] * 1e3},
            "T_before_over_T_exact_bw_minus_1_by_n_abs": bins,
            "sed_total_variation": tv, "sed_total_variation_two_seeds": tv0}


def images_block(w, eng, rows, stream, plain_s, batch):
    """The paper's Fig. 2 on the gap + spiral disk: next-event images at the
    bins holding 10 and 11.3 um, face-on and inclined by 60 deg, 401 x 401
    pixels over the 200 AU box, one full pass with the images on (its extra
    time over the plain pass is the image cost); then the ELT point spread
    function (50 mas FWHM at 50 pc, 2.5 AU) and the face-on 11.3 um radial
    profile across the planet's gap at 20 AU, before and after the PSF."""
    import numpy as np
    import torch
    import synth
    from paper_1201_3588_amd import mcrt
    AU, PC = synth.AU, 3.0856775814913673e18
    lam = np.asarray(w.species.lam_um)
    bins = [int(np.argmin(np.abs(np.log(lam / t)))) for t in (10.0, 11.3)]
    npix, half = 401, 100.0 * AU
    incl = np.radians(60.0)
    eng.set_observers(dirs=[(0.0, 0.0, 1.0), (0.0, -np.sin(incl), np.cos(incl))], npix=npix, half_width=half,
                      center=(0.0, 0.0, 0.0), cos_cone=float(np.cos(np.radians(10.0))), lambda_bins=bins,
                      peel=True, peel_capacity=1 << 25)
    tal = eng.new_tallies(tally_j=True)
    N = w.n_packets
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    eng.run_batched(tal, 0, N, N, w.seed, batch, pah_rows=rows)
    e1.record(stream)
    c = eng.counters_sync(tal)
    t_img = e0.elapsed_time(e1) / 1e3
    pix_au = 2.0 * half / npix / AU
    fwhm_pix = 2.5 / pix_au
    p0 = torch.cuda.Event(enable_timing=True)
    p1 = torch.cuda.Event(enable_timing=True)
    eps = w.source.lum / N
    D = 50.0 * PC
    dnu = torch.as_tensor(eng.tables_numpy()["dnu"][bins], device="cuda")
    p0.record(stream)
    conv = mcrt.image_psf(tal["peel"], npix, eps / (4 * np.pi * D * D) / mcrt.PEEL_UNIT, fwhm_pix)
    p1.record(stream)
    raw = tal["peel"].double().reshape(2, 2, npix, npix) * (eps / (4 * np.pi * D * D) / mcrt.PEEL_UNIT)
    conv = conv.reshape(2, 2, npix, npix)
    torch.cuda.synchronize()
    jy = 1e23 / dnu.reshape(1, 2, 1, 1)                 # erg s^-1 cm^-2 per bin -> Jy

    def radial(img):
        yy, xx = torch.meshgrid(torch.arange(npix, device="cuda"), torch.arange(npix, device="cuda"), indexing="ij")
        rr = torch.sqrt(((xx - npix // 2) * pix_au) ** 2 + ((yy - npix // 2) * pix_au) ** 2)
        prof = {}
        for r_au in (15.0, 20.0, 25.0):
            m = (rr >= r_au - 1.0) & (rr < r_au + 1.0)
            prof[r_au] = float(img[m].mean().item())
        return prof
    pr, pc = radial(raw[0, 1] * jy[0, 1]), radial(conv[0, 1] * jy[0, 1])
    return {"bins": bins, "lambda_um": [float(lam[b]) for b in bins], "npix": npix, "pixel_au": pix_au,
            "pass_with_images_ms": t_img * 1e3, "pass_plain_ms": plain_s * 1e3,
            "image_cost_fraction": t_img / plain_s - 1.0,
            "next_event_records": int(c[mcrt.CNT["peel"]]), "dropped": int(c[mcrt.CNT["peel_dropped"]]),
            "psf_fwhm_pix": fwhm_pix, "psf_ms_4_images": p0.elapsed_time(p1),
            "total_flux_jy": (raw * jy).sum(dim=(2, 3)).tolist(),
            "faceon_11um_gap_contrast_raw": {"I20_over_I15": pr[20.0] / pr[15.0], "I20_over_I25": pr[20.0] / pr[25.0]},
            "faceon_11um_gap_contrast_psf": {"I20_over_I15": pc[20.0] / pc[15.0], "I20_over_I25": pc[20.0] / pc[25.0]}}


def hard_photon_block(stream):
    """The paper's Fig. 3: P(T) of a 100 C atom PAH in monochromatic radiation
    of flux 1e4 erg s^-1 cm^-2 at 3.8, 13.6, 50, 100, 300 eV and 1 keV (1000
    enthalpy bins to 5e4 K, 241 wavelength bins down to 1.24 keV), from the
    exact solver; per energy the median temperature, the 99 % and 99.99 %
    points of P(T), and the share of time above 1000 K."""
    import numpy as np
    import torch
    import synth
    from paper_1201_3588_amd import pah
    case = synth.hard_photon_case()
    pm, T = case["pm"], case["T"]
    s = pah.PahSolver(T, case["U"], case["lam"], pm.cabs, pm.cband, pm.ccont)
    J = torch.as_tensor(case["J"]).cuda()
    s.solve(J, want_P=True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    out, P, pabs = s.solve(J, want_P=True)
    e1.record(stream)
    torch.cuda.synchronize()
    P = P.cpu().numpy()
    rows = []
    for k, e in enumerate(case["hnu_ev"]):
        c = np.cumsum(P[k])
        q = lambda v: float(T[np.searchsorted(c, v)])
        rows.append({"hnu_ev": float(e), "T_median": q(0.5), "T_99": q(0.99), "T_9999": q(0.9999),
                     "P_above_1000K": float(P[k][T > 1000.0].sum())})
    return {"n_c": 100, "flux": case["flux"], "M": len(T), "n_lambda": len(case["lam"]),
            "solve_ms_6_fields": e0.elapsed_time(e1), "P_of_T": rows,
            "energy_deposition": "every absorbed photon deposits its full energy (the Dwek & Smith loss of "
                                 "kinetic energy above 100 eV is not modelled): the 300 eV and 1 keV "
                                 "distributions are upper bounds on the heating"}


def random_load_rate(n_load, stream):
    """Achievable rate of random 4-byte loads from a buffer of n_load floats
    (the size of the transport's per-crossing gathers), HIP events."""
    import ctypes as C
    import torch
    from paper_1201_3588_amd import mcrt
    buf = torch.ones(n_load, dtype=torch.float32, device="cuda")
    sink = torch.zeros(1, dtype=torch.float32, device="cuda")
    n_ops = 1 << 30
    L = mcrt.lib()
    L.mcrt_bench_random.argtypes = [C.c_void_p, C.c_uint64, C.c_void_p, C.c_uint64, C.c_uint64,
                                    C.c_uint64, C.c_int32, C.c_void_p, C.c_void_p]
    s = C.c_void_p(stream.cuda_stream)
    L.mcrt_bench_random(None, 0, C.c_void_p(buf.data_ptr()), n_load, n_ops, 1, 1, C.c_void_p(sink.data_ptr()), s)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    L.mcrt_bench_random(None, 0, C.c_void_p(buf.data_ptr()), n_load, n_ops, 2, 1, C.c_void_p(sink.data_ptr()), s)
    e1.record(stream)
    torch.cuda.synchronize()
    ncu = torch.cuda.get_device_properties(0).multi_processor_count
    q = 16 * 256 * ncu
    issued = (n_ops + q - 1) // q * q
    del buf, sink
    return issued / (e0.elapsed_time(e1) / 1e3)


def c2_block(steps, stream, micro):
    """The flared disk (64^3 base, depth 3, 262,480 leaves, 24 species, 200
    bins, 1e7 packets): one transport pass (deferred path tally) +
    temperatures + mean intensity per step; its grid and tallies sit in the
    L2 / Infinity Cache, so its random-access ceiling is measured at its own
    sizes."""
    import torch
    import synth
    from paper_1201_3588_amd import mcrt
    w = synth.c2_disk()
    N = w.n_packets
    eng = mcrt.Engine.from_workload(w)
    eng.build_tables(w.source.pos, w.source.lum, w.source.teff)
    deferred = eng.set_deferred_tally(min(1 << 31, max(1 << 20, 100 * N)))
    tal = eng.new_tallies(tally_j=True)
    ev = []

    def step():
        for v in (t for t in tal.values() if t is not None):
            v.zero_()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        eng.run(tal, 0, N, N, w.seed)
        e1.record(stream)
        ev.append((e0, e1))
        eng.temperatures(tal["nabs"], N)
        eng.mean_intensity(tal["jq"], N)

    step()
    torch.cuda.synchronize()
    ev.clear()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    k = sum(a.elapsed_time(b) for a, b in ev) / len(ev) / 1e3
    c = mcrt.u64_view(tal["counters"])
    cnt = {kk: int(c[v]) for kk, v in mcrt.CNT.items()}
    assert cnt["launched"] == N and cnt["launched"] == cnt["escaped"] + cnt["killed"] + cnt["terminated"]
    alg = 8 * cnt["crossings"] + 16 * (cnt["jseg"] + cnt["absorptions"] + cnt["escaped"])
    res = {"workload": "flared_disk_64cube_depth3_262480leaves_24species_200lambda_1e7packets",
           "packets_per_s": N * steps / wall, "ms_per_step": wall / steps * 1e3,
           "transport_pass_ms": k * 1e3, "transport_packets_per_s": N / k,
           "transport_crossings_per_s": cnt["crossings"] / k, "per_pass_counts": cnt,
           "path_tally": "deferred records" if deferred else "atomic",
           "pass_roofline": {"bound": "hbm", "achieved": alg / k / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": alg / k / 1e9 / HBM_PEAK_GBS, "alg_bytes_per_pass": alg,
                             "byte_model": "8 B per crossing, 16 B per tally read-modify-write "
                                           "(path segment, absorption, escape)"}}
    if micro:
        loads = random_load_rate(w.grid.nb ** 3 * 2, stream)
        atom = random_atomic_rate(w.species.n_lambda * w.grid.n_cells, stream)
        res["random_access_ceiling"] = {
            "where": "grid (2 MB) and tallies (470 MB) resident in L2 / Infinity Cache",
            "random_4B_loads_per_s": loads, "random_8B_atomics_per_s": atom,
            "crossings_per_s_over_load_rate": cnt["crossings"] / k / loads,
            "tally_updates_per_s_over_atomic_rate": (cnt["jseg"] + cnt["absorptions"] + cnt["escaped"]) / k / atom}
    del tal, eng
    return res


class C5Run:
    """The headline workload and its pass (see the module docstring)."""

    def __init__(self, args, stream):
        import torch
        import synth
        from paper_1201_3588_amd import mcrt
        from paper_1201_3588_amd.pah import PahSolver
        self.args, self.stream = args, stream
        t0 = time.perf_counter()
        self.w = w = synth.c5_full(n_packets=args.packets)
        self.synth_s = time.perf_counter() - t0
        log(f"grid built in {self.synth_s:.1f} s ({w.grid.n_cells} leaves)")
        self.eng = mcrt.Engine.from_workload(w)
        self.eng.build_tables(w.source.pos, w.source.lum, w.source.teff)
        self.N, self.nc, self.nl = w.n_packets, w.grid.n_cells, w.species.n_lambda
        self.solvers = [PahSolver.from_model(pm) for pm in w.pah]
        self.rows = torch.empty((len(self.solvers), self.nc, self.nl), dtype=torch.float64, device="cuda")
        self.mass = self.eng.cell_mass()
        self.tal = self.eng.new_tallies(tally_j=True)
        # deferred path tally: the record workspace takes the device memory
        # left after the pass's own buffers (two fields, temperatures, a PAH
        # output chunk, the surrogates and their training set: ~60 GB); the
        # pass runs in id ranges whose records fit it (~250 records per packet)
        free = torch.cuda.mem_get_info()[0]
        cap = min(1 << 35, max(1 << 22, (free - (60 << 30)) // 16)) // 4096 * 4096
        self.deferred = self.eng.set_deferred_tally(cap)
        self.capacity = cap if self.deferred else 0
        self.batch = (args.batch or cap // 300) if self.deferred else self.N
        self.chunk = 1 << 22
        self.surs = None
        self.last = {}

    def pah_step(self, J, exact=False):
        """PAH emission of both species from J and their re-emission rows;
        returns (band powers [n_pah, 17], flagged-cell count tensor)."""
        import torch
        bps, n_flag = [], torch.zeros((), dtype=torch.int64, device="cuda")
        for p, s in enumerate(self.solvers):
            bp = torch.zeros(s.n_bands, dtype=torch.float64, device="cuda")
            for a in range(0, self.nc, self.chunk):
                b = min(self.nc, a + self.chunk)
                if exact or self.surs is None:
                    out = s.solve(J[a:b])[0]
                else:
                    out, ood = self.surs[p].solve(J[a:b])[:2]
                    n_flag += (ood != 0).sum()
                s.rows(out, rows=self.rows[p, a:b])
                bp += s.band_power(out, self.mass[a:b])
                del out
            bps.append(bp)
        return torch.stack(bps), n_flag

    def one_pass(self, J, seed, exact=False):
        """One pass (the timed step).  Returns the new field; per-pass figures
        in self.last (HIP events, read after the caller synchronises)."""
        import torch
        st = self.stream
        ev = lambda: torch.cuda.Event(enable_timing=True)
        e_start, e_pah, e_tr, e_end = ev(), ev(), ev(), ev()
        e_start.record(st)
        self.eng.build_tables(self.w.source.pos, self.w.source.lum, self.w.source.teff)
        bp, n_flag = self.pah_step(J, exact)
        e_pah.record(st)
        for v in (t for t in self.tal.values() if t is not None):
            v.zero_()
        kev = []
        for a in range(0, self.N, self.batch):
            k0, k1 = ev(), ev()
            k0.record(st)                 # creates the events; the library records them again
            k1.record(st)                 # around the transport kernel of this id range
            kev.append((k0, k1))
            self.eng.run(self.tal, a, min(self.batch, self.N - a), self.N, seed, pah_rows=self.rows,
                         kernel_events=(k0, k1))
        e_tr.record(st)
        T = self.eng.temperatures(self.tal["nabs"], self.N)
        Jn = self.eng.mean_intensity(self.tal["jq"], self.N)
        e_end.record(st)
        self.last = dict(events=(e_start, e_pah, e_tr, e_end), kev=kev, bp=bp, n_flag=n_flag, T=T)
        return Jn

    def pass_figures(self):
        """Times and counts of the last pass (after a synchronise)."""
        from paper_1201_3588_amd import mcrt
        e_start, e_pah, e_tr, e_end = self.last["events"]
        c = mcrt.u64_view(self.tal["counters"])
        cnt = {k: int(c[v]) for k, v in mcrt.CNT.items()}
        k_ms = [a.elapsed_time(b) for a, b in self.last["kev"]]
        return dict(pass_ms=e_start.elapsed_time(e_end), pah_ms=e_start.elapsed_time(e_pah),
                    transport_ms=e_pah.elapsed_time(e_tr), post_ms=e_tr.elapsed_time(e_end),
                    k_transport_ms=k_ms, counts=cnt, n_flag=int(self.last["n_flag"].item()))

    def train(self, J1):
        """Surrogates for both PAH species, trained on exactly solved cells:
        1e6 lit cells of the pass-1 field and 4e5 synthetic fields; held out:
        2e5 other lit cells of that field (disjoint from the training cells)
        and 5e4 synthetic fields of another seed."""
        import numpy as np
        import torch
        import synth
        from paper_1201_3588_amd.surrogate import Surrogate, band_error
        t0 = time.perf_counter()
        lit = torch.nonzero(J1.sum(1) > 0).squeeze(1)
        g = torch.Generator(device="cuda")
        g.manual_seed(5)
        perm = lit[torch.randperm(lit.numel(), generator=g, device="cuda")]
        n_tr = min(self.args.train_cells, perm.numel() // 2)
        tr_idx, ho_idx = perm[:n_tr], perm[n_tr:n_tr + 200_000]
        lam = self.w.species.lam_um
        Jsyn = torch.as_tensor(synth.pah_fields(self.args.train_synthetic, lam, seed=4)[0].astype(np.float32)).cuda()
        Jsyn_ho = torch.as_tensor(synth.pah_fields(50_000, lam, seed=14)[0].astype(np.float32)).cuda()
        Jtr = torch.cat([J1.index_select(0, tr_idx), Jsyn])
        Jho = J1.index_select(0, ho_idx)
        surs, info = [], []

        def err(sur, J):
            pred, ood, _ = sur.predict(J)
            ex, _ = sur.exact(J)
            ok = (ood == 0) & (ex[:, :17].sum(1) > 0)
            e = band_error(pred, ex)[ok]
            return {"cells": int(J.shape[0]), "p95": float(torch.quantile(e, 0.95).item()),
                    "median": float(e.median().item()), "flagged": float((ood != 0).float().mean().item())}
        for s, pm in zip(self.solvers, self.w.pah):
            sur = Surrogate(s, batch=2048, seed=4)
            out, pabs = sur.exact(Jtr)
            hist = sur.fit(Jtr, out, pabs, epochs=self.args.epochs, lr=2e-3)
            sub = Jtr[:: max(1, Jtr.shape[0] // 100_000)][:100_000]
            info.append({"n_c": pm.n_c, "train_cells": int(Jtr.shape[0]), "epochs": self.args.epochs,
                         "loss_first": hist[0], "loss_last": hist[-1],
                         "band_error_training_cells_in_distribution": err(sur, sub),
                         "band_error_held_out_disk_cells": err(sur, Jho),
                         "band_error_held_out_synthetic_fields": err(sur, Jsyn_ho)})
            surs.append(sur)
        torch.cuda.synchronize()
        self.surs = surs
        return {"species": info, "setup_s": time.perf_counter() - t0,
                "held_out": "2e5 lit cells of the pass-1 field not among the training cells "
                            "(disjoint slices of one permutation) and 5e4 synthetic fields of another seed"}


def pah_kernel_rooflines(R, J, stream):
    """The PAH step's kernels on their own, against their rooflines:
    the fused surrogate inference (k_mlp_infer) on 4,194,304 cells of the
    field, the exact solver (k_pah_solve) on 262,144 of them, and surrogate
    training (forward + backward + Adam, batch 2048) on a fresh network."""
    import torch
    from paper_1201_3588_amd.surrogate import Surrogate
    ev = lambda: torch.cuda.Event(enable_timing=True)
    sur, s = R.surs[0], R.solvers[0]
    Jc = J[: 1 << 22].contiguous()
    n = Jc.shape[0]
    sur.predict(Jc[:65536])
    e0, e1 = ev(), ev()
    e0.record(stream)
    sur.predict(Jc)
    e1.record(stream)
    Jx = Jc[: 1 << 18]
    s.solve(Jx[:4096])
    x0, x1 = ev(), ev()
    x0.record(stream)
    s.solve(Jx)
    x1.record(stream)
    # training throughput on a throwaway network (its normalisation is refitted)
    t = Surrogate(s, batch=2048, seed=9)
    nt = 2048 * 64
    out, pabs = t.exact(Jc[:nt])
    X, Y = t.net.prepare(s, Jc[:nt], out, pabs)
    for k in range(4):
        t.net.train_step(X[k * 2048:(k + 1) * 2048], Y[k * 2048:(k + 1) * 2048], 1e-3, k + 1)
    steps = 60
    t0, t1 = ev(), ev()
    t0.record(stream)
    for k in range(steps):
        a = (k % 64) * 2048
        t.net.train_step(X[a:a + 2048], Y[a:a + 2048], 1e-3, k + 5)
    t1.record(stream)
    torch.cuda.synchronize()
    ti, tx, tt = e0.elapsed_time(e1) / 1e3, x0.elapsed_time(x1) / 1e3, t0.elapsed_time(t1) / 1e3
    ni, nh, no = s.n_lambda + 1, 256, s.n_out
    fl_inf = 2 * (ni * nh + nh * nh + nh * no)
    fl_train = 3 * fl_inf - 2 * ni * nh                  # forward, backward (no input gradient)
    by_inf = 4 * s.n_lambda + 8 * no + 8 + 1             # J in (FP32); outputs, P_abs out (FP64); flag
    inf_rate = n / ti
    inf_roof = min(2.5e15 / fl_inf, 8e12 / by_inf)
    ex_rate = Jx.shape[0] / tx
    fl_ex = 0.35e6
    tr_rate = steps * 2048 / tt
    return {
        "k_mlp_infer": {"cells": n, "ms": ti * 1e3, "cells_per_s": inf_rate, "flop_per_cell": fl_inf,
                        "hbm_bytes_per_cell": by_inf, "roofline_cells_per_s": inf_roof, "frac": inf_rate / inf_roof,
                        "bound": "hbm" if 8e12 / by_inf < 2.5e15 / fl_inf else "mfma",
                        "peaks": "BF16 dense MFMA 2.5 PFLOP/s, HBM 8 TB/s"},
        "k_pah_solve": {"cells": int(Jx.shape[0]), "ms": tx * 1e3, "cells_per_s": ex_rate, "flop_per_cell": fl_ex,
                        "achieved_tflops": ex_rate * fl_ex / 1e12, "peak_tflops": 78.6,
                        "frac": ex_rate * fl_ex / 78.6e12, "bound": "fp64"},
        "training": {"batch": 2048, "steps": steps, "ms_per_step": tt / steps * 1e3, "samples_per_s": tr_rate,
                     "flop_per_sample": fl_train, "achieved_tflops": tr_rate * fl_train / 1e12,
                     "peak_tflops": 2500.0, "frac": tr_rate * fl_train / 2.5e15, "bound": "mfma"},
    }


def cpu_baseline_c5(w, n_s):
    """The oracle (FP64 C, threaded over the host cores) on the first n_s
    packet ids of the headline workload, path-length tally on, running
    absorption counts.  Its PAH re-emission rows are seeded stand-in rows
    (a table of 65,536 random CDF rows, cell c using row c mod 65,536), so it
    does not need the 27 GB of per-cell rows."""
    import numpy as np
    import oracle
    import synth
    threads = min(16, len(os.sched_getaffinity(0)))
    n_pah = int((w.species.kind == 1).sum())
    table = synth.pah_test_rows(n_pah, 65536, w.species.n_lambda, seed=77).reshape(n_pah * 65536, -1)
    rmap = (np.arange(w.grid.n_cells, dtype=np.int64) % 65536).astype(np.int32)
    rmap = np.concatenate([rmap + 65536 * p for p in range(n_pah)]).astype(np.int32)
    s = oracle.Session(w, n_threads=threads, pah_rows=table, pah_row_map=rmap)
    acc = s.new_accumulator()
    for v in acc.values():
        if v is not None:
            v.fill(0)                    # touch the pages before the clock starts
    tc0 = time.perf_counter()
    s.accumulate(acc, 0, n_s)
    tc = time.perf_counter() - tc0
    return {"value": n_s / tc, "unit": "packets/s", "cores": threads, "kind": "oracle",
            "sample": f"first {n_s} packet ids of the 256^3 gap + spiral disk (1e9-packet pass), transport "
                      f"with path-length tally and running counts, PAH rows from a seeded stand-in table, "
                      f"{tc:.1f} s wall"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--packets", type=int, default=1_000_000_000)
    ap.add_argument("--batch", type=int, default=0,
                    help="packets per transport call (0: sized so that the records of a range fit the "
                         "workspace, from the records per packet of pass 0)")
    ap.add_argument("--cpu-sample", type=int, default=1_000_000)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-micro", action="store_true")
    ap.add_argument("--train-cells", type=int, default=1_000_000)
    ap.add_argument("--train-synthetic", type=int, default=400_000)
    ap.add_argument("--epochs", type=int, default=12)
    ap.add_argument("--plain", action=argparse.BooleanOptionalAction, default=True,
                    help="also time one pass with the exact PAH solver instead of the surrogate")
    ap.add_argument("--extra", action=argparse.BooleanOptionalAction, default=True,
                    help="also run the smaller disks, the re-emission law comparison and the Fig. 3 set-up")
    ap.add_argument("--c3-iterate", action=argparse.BooleanOptionalAction, default=True)
    ap.add_argument("--pah-kernels", action=argparse.BooleanOptionalAction, default=True,
                    help="time the PAH step's kernels alone against their rooflines")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run one elementwise copy of 256 MiB (read) -> 256 MiB (write) first, "
                         "the reference for scaling hardware byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU design "
              "shards packet ids across devices and sums the integer tallies", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    if args.copy_probe:
        a = torch.ones(1 << 26, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        del a, b
    R = C5Run(args, stream)
    N = R.N
    # pass 0 from the optically thin starlight field, exact PAH emission
    t0 = time.perf_counter()
    J = R.one_pass(R.eng.thin_field(), R.w.seed + 1000, exact=True)
    torch.cuda.synchronize()
    p0 = R.pass_figures()
    if R.deferred and not args.batch:
        # id ranges whose records fit the workspace with 8 % to spare
        R.batch = int(R.capacity / (1.08 * p0["counts"]["jseg"] / N))
    log(f"workspace {R.capacity} records, id ranges of {R.batch} packets")
    log(f"pass 0 (exact PAH emission) in {time.perf_counter() - t0:.1f} s")
    training = R.train(J)
    log(f"surrogates trained in {training['setup_s']:.1f} s")
    pah_roof = pah_kernel_rooflines(R, J, stream) if args.pah_kernels else None
    plain = None
    if args.plain:
        # one pass in the plain form (exact solver for every PAH cell), same field
        Jp = R.one_pass(J, R.w.seed + 999, exact=True)
        torch.cuda.synchronize()
        plain = R.pass_figures()
        del Jp
    seed = R.w.seed
    for k in range(args.warmup):
        J = R.one_pass(J, seed + k)
    torch.cuda.synchronize()
    log("timed steps")
    figs, bps = [], []
    t0 = time.perf_counter()
    for k in range(args.steps):
        J = R.one_pass(J, seed + args.warmup + k)
        torch.cuda.synchronize()
        figs.append(R.pass_figures())
        bps.append(R.last["bp"].cpu().numpy())
    t1 = time.perf_counter()
    wall = t1 - t0
    cnt = figs[-1]["counts"]
    for f in figs:
        c = f["counts"]
        assert c["launched"] == N and c["launched"] == c["escaped"] + c["killed"] + c["terminated"]
    changes = [None] + [float(np.max(np.abs(b - a) / np.maximum(np.abs(a), 1e-300))) for a, b in zip(bps[:-1], bps[1:])]
    k_all = [t for f in figs for t in f["k_transport_ms"]]
    k_avg = sum(k_all) / len(k_all) / 1e3
    n_launch = len(figs[-1]["k_transport_ms"])
    tr_ms = sum(f["transport_ms"] for f in figs) / len(figs)
    pah_ms = sum(f["pah_ms"] for f in figs) / len(figs)
    cr = sum(f["counts"]["crossings"] for f in figs) / len(figs)
    # algorithmic bytes of the transport kernel per launch (one id range):
    # per crossing the base-cube entry with the density term (8 B); per path
    # segment its 8 B record; per absorption and per escape one 8 B atomic
    # read-modify-write (16 B)
    alg_pass = 8 * cnt["crossings"] + 8 * cnt["jseg"] + 16 * (cnt["absorptions"] + cnt["escaped"])
    alg_launch = alg_pass / n_launch
    achieved = alg_launch / k_avg / 1e9
    n_pah_cells = len(R.solvers) * R.nc
    per_packet = committed_traffic()
    traffic = per_packet * N / n_launch if per_packet is not None else None
    out = {
        "metric": METRIC,
        "value": N * args.steps / wall,
        "unit": "packets/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "gap_spiral_disk_256cube_depth3_16784776leaves_26species_200lambda_1e9packets_pah",
                   "packets_per_step": N, "leaves": R.nc, "n_lambda": R.nl, "species": int(R.w.species.n_species),
                   "pah_species": len(R.solvers), "transport": "f32 geometry, f64 tables/T",
                   "tally_j": True, "pah_emission": "surrogate in the loop, exact fallback"},
        "crossings_per_s": cr * args.steps / wall,
        "per_step_counts": cnt,
        "step_breakdown_ms": {"pah_emission_and_rows": pah_ms, "transport_pass": tr_ms,
                              "k_transport_sum": sum(k_all) / len(figs),
                              "record_passes_and_launch_gaps": tr_ms - sum(k_all) / len(figs),
                              "temperatures_and_mean_intensity": sum(f["post_ms"] for f in figs) / len(figs)},
        "transport_packets_per_s": N / (tr_ms / 1e3),
        "transport_crossings_per_s": cr / (tr_ms / 1e3),
        "path_tally": {"mode": f"deferred records, id ranges of {R.batch} packets" if R.deferred else "atomic",
                       "workspace_records": R.capacity, "segments_per_packet": cnt["jseg"] / N},
        "pah": {"molecule_cells_per_pass": n_pah_cells,
                "surrogate_in_loop_cells_per_s": n_pah_cells / (pah_ms / 1e3),
                "exact_cells_per_s": n_pah_cells / (plain["pah_ms"] / 1e3) if plain else None,
                "speedup": (plain["pah_ms"] / pah_ms) if plain else None,
                "fallback_fraction": figs[-1]["n_flag"] / n_pah_cells,
                "surrogate_training": training,
                "iteration_band_power_change_per_step": changes,
                "pass_plain_s": plain["pass_ms"] / 1e3 if plain else None,
                "pass_surrogate_s": wall / args.steps,
                "kernels": pah_roof},
        "pass0": {"pass_ms": p0["pass_ms"], "pah_exact_ms": p0["pah_ms"], "transport_ms": p0["transport_ms"]},
        "synth_build_s": R.synth_s,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_transport<float,false,false,true>",
                     "launches_per_step": n_launch, "avg_launch_ms": k_avg * 1e3,
                     "alg_bytes_per_launch": alg_launch,
                     "byte_model": "8 B per crossing (base-cube entry + density), 8 B per path-segment record, "
                                   "16 B per absorption and per escape (8 B atomic read-modify-write)"},
    }
    del J
    R.tal = None
    if not args.no_micro:
        loads = random_load_rate(R.w.grid.nb ** 3 * 2, stream)
        out["random_access_ceiling"] = {
            "random_4B_loads_per_s": loads,
            "buffer_bytes": R.w.grid.nb ** 3 * 8,
            "crossings_per_s_in_k_transport": cnt["crossings"] / n_launch / k_avg,
            "frac_of_load_rate": cnt["crossings"] / n_launch / k_avg / loads,
            "note": "one dependent 8 B gather per crossing against random 4 B loads over the grid's size"}
    w5 = R.w
    del R
    torch.cuda.empty_cache()
    if args.extra:
        out["c2"] = c2_block(5, stream, not args.no_micro)
        out["reemission_law"] = [
            reemission_block(synth.c1_sphere(n_packets=n), stream,
                             f"uniform_sphere_32cube_100lambda_{n:.0e}packets_f64".replace("+0", ""))
            for n in (100_000, 1_000_000, 10_000_000)]
        out["reemission_law"].append(reemission_block(synth.c2_disk(), stream,
                                                      "flared_disk_64cube_depth3_262480leaves_1e7packets"))
        out["pah_hard_photons"] = hard_photon_block(stream)
        out["c3"] = c3_block(100_000_000, not args.no_micro, stream, iterate=args.c3_iterate)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline_c5(w5, args.cpu_sample)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
