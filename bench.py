#!/usr/bin/env python3
"""Benchmark of the Monte Carlo dust transfer hot path on one MI355X.

One step = one pass of the hot path over the flared proto-planetary disk
workload (64^3 base cubes refined 2x2x2 to depth 3 inside 1 AU = 262,480
leaves, 3 materials x 8 grain sizes, 200 wavelengths, Henyey-Greenstein
scattering, 1e7 packets from a 5800 K, 1 L_sun star, FP32 geometry, FP64
tables and temperatures, path-length J tally on):
  table build -> transport of all packets (path-length tally through per-segment
  records and LDS sums; --atomic-tally for per-segment atomics) -> temperatures
  -> mean intensity -> PAH (30 C) emission of every dusty cell from its field:
  surrogate network with exact fallback on flagged cells -> PAH re-emission rows.
The exact PAH solver is timed on the same cells beside the step.  The
surrogate is trained before the timed region on exactly solved cells (the
disk's fields plus synthetic fields).  Inputs are resident in device memory
before the timed region.  Prints one JSON line.  The CPU oracle is timed on a
bounded sample for reference.
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
    # deferred path tally: about 140 segment records per packet here, so the
    # pass runs in id ranges of 12 M packets against a 2^31-record workspace
    deferred = eng.set_deferred_tally(1 << 31)
    batch = 12_000_000 if deferred else N
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
            "solve_ms_6_fields": e0.elapsed_time(e1), "P_of_T": rows}


def c5_block(n_packets, stream):
    """The gap + spiral disk with PAHs on a 256^3 base grid (depth 3,
    16,784,776 leaves, 26 species, 200 bins, 1e9 packets), one pass timed end
    to end in both forms from the same field: plain (exact PAH solver for both
    PAH species) and with the surrogate in the loop (exact fallback on flagged
    cells).  A pass = PAH emission and re-emission rows from the previous
    field + transport + temperatures + mean intensity.  The surrogates are
    trained on the disk's own first-pass fields."""
    import numpy as np
    import torch
    import synth
    from paper_1201_3588_amd import mcrt
    from paper_1201_3588_amd.pah import PahSolver
    from paper_1201_3588_amd.surrogate import Surrogate, band_error
    t0 = time.perf_counter()
    w = synth.c5_full(n_packets=n_packets)
    t_synth = time.perf_counter() - t0
    eng = mcrt.Engine.from_workload(w)
    eng.build_tables(w.source.pos, w.source.lum, w.source.teff)
    N, nc, nl = w.n_packets, w.grid.n_cells, w.species.n_lambda
    solvers = [PahSolver.from_model(pm) for pm in w.pah]
    rows = torch.empty((len(solvers), nc, nl), dtype=torch.float64, device="cuda")
    chunk = 1 << 22

    def pah_step(J, surs=None):
        n_flag = 0
        for p, s in enumerate(solvers):
            for a in range(0, nc, chunk):
                b = min(nc, a + chunk)
                if surs is None:
                    out = s.solve(J[a:b])[0]
                else:
                    out, ood = surs[p].solve(J[a:b])[:2]
                    n_flag += int((ood != 0).sum().item())
                s.rows(out, rows=rows[p, a:b])
        return n_flag

    def one_pass(J, seed, surs=None):
        tal = eng.new_tallies(tally_j=True)
        torch.cuda.synchronize()
        t = time.perf_counter()
        n_flag = pah_step(J, surs)
        eng.run(tal, 0, N, N, seed, pah_rows=rows)
        T = eng.temperatures(tal["nabs"], N)
        Jn = eng.mean_intensity(tal["jq"], N)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        c = mcrt.u64_view(tal["counters"])
        del tal, T
        return Jn, dt, c, n_flag

    J1, t_first, c1, _ = one_pass(eng.thin_field(), w.seed)
    assert int(c1[0]) == N and int(c1[0]) == int(c1[1] + c1[2] + c1[3])
    # surrogates trained on a sample of the first pass's lit cells plus synthetic fields
    t_train = time.perf_counter()
    lit = torch.nonzero(J1.sum(1) > 0).squeeze(1)
    g = torch.Generator(device="cuda")
    g.manual_seed(5)
    samp = lit[torch.randperm(lit.numel(), generator=g, device="cuda")[:1_000_000]]
    Jtr = torch.cat([J1.index_select(0, samp),
                     torch.as_tensor(synth.pah_fields(400_000, w.species.lam_um, seed=4)[0].astype(np.float32)).cuda()])
    surs, errs = [], []
    held = lit[torch.randperm(lit.numel(), generator=g, device="cuda")[:200_000]]
    for s in solvers:
        sur = Surrogate(s, batch=2048, seed=4)
        out, pabs = sur.exact(Jtr)
        sur.fit(Jtr, out, pabs, epochs=12, lr=2e-3)
        Jh = J1.index_select(0, held)
        pred, ood, _ = sur.predict(Jh)
        ex, _ = sur.exact(Jh)
        ok = (ood == 0) & (ex[:, :17].sum(1) > 0)
        errs.append(float(torch.quantile(band_error(pred, ex)[ok], 0.95).item()))
        surs.append(sur)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t_train
    _, t_plain, c_plain, _ = one_pass(J1, w.seed + 1)
    _, t_sur, c_sur, n_flag = one_pass(J1, w.seed + 1, surs)
    for c in (c_plain, c_sur):
        assert int(c[0]) == N and int(c[0]) == int(c[1] + c[2] + c[3])
    return {"workload": "gap_spiral_disk_256cube_depth3_16784776leaves_26species_200lambda_1e9packets_pah",
            "leaves": nc, "packets": N, "synth_build_s": t_synth,
            "pass_plain_s": t_plain, "pass_surrogate_s": t_sur,
            "packets_per_s_plain": N / t_plain, "packets_per_s_surrogate": N / t_sur,
            "crossings_per_pass": int(c_plain[6]), "pah_absorptions_per_pass": int(c_plain[9]),
            "pah_cells_per_pass": len(solvers) * nc, "surrogate_flagged_per_pass": n_flag,
            "surrogate_band_error_p95": errs, "surrogate_training_s": t_train}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--packets", type=int, default=10_000_000)
    ap.add_argument("--cpu-sample", type=int, default=400_000)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-micro", action="store_true")
    ap.add_argument("--no-pah", action="store_true")
    ap.add_argument("--train-synthetic", type=int, default=400_000)
    ap.add_argument("--epochs", type=int, default=12)
    ap.add_argument("--train-passes", type=int, default=3,
                    help="transport passes (other seeds) whose disk fields join the training set")
    ap.add_argument("--c3", action=argparse.BooleanOptionalAction, default=True,
                    help="also time one pass of the gap + spiral disk with PAHs (HBM-resident tallies)")
    ap.add_argument("--c3-packets", type=int, default=100_000_000)
    ap.add_argument("--c3-iterate", action=argparse.BooleanOptionalAction, default=True,
                    help="also iterate the gap + spiral disk's PAH emission to convergence")
    ap.add_argument("--atomic-tally", action="store_true",
                    help="path-length tally by per-segment atomics instead of the deferred records")
    ap.add_argument("--reemission", action=argparse.BooleanOptionalAction, default=True,
                    help="compare the paper's re-emission law with the Bjorkman-Wood one")
    ap.add_argument("--c5", action="store_true",
                    help="also time the 256^3 gap + spiral disk (1e9 packets) end to end, plain and "
                         "with the surrogate in the loop (minutes; needs ~150 GB of device memory)")
    ap.add_argument("--c5-packets", type=int, default=1_000_000_000)
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
    from paper_1201_3588_amd import mcrt

    torch.cuda.set_device(0)
    if args.copy_probe:
        a = torch.ones(1 << 26, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        del a, b
    w = synth.c2_disk(n_packets=args.packets)
    N = w.n_packets
    eng = mcrt.Engine.from_workload(w)
    # path-length tally through segment records (about 64 per packet here)
    # instead of one atomic per segment
    deferred = (not args.atomic_tally) and eng.set_deferred_tally(min(1 << 31, max(1 << 20, 100 * N)))
    tal = eng.new_tallies(tally_j=True)
    stream = torch.cuda.current_stream()
    ev = []
    dusty = torch.as_tensor(np.nonzero(w.grid.rho > 0)[0]).cuda()
    sur = None
    info = {}
    if not args.no_pah:
        from paper_1201_3588_amd import pah
        from paper_1201_3588_amd.surrogate import Surrogate, band_error
        pm = synth.pah_model(30, w.species.lam_um)
        solver = pah.PahSolver.from_model(pm)
        sur = Surrogate(solver, batch=2048, seed=4)
        # training cells: the disk's own fields (one pass) plus synthetic fields
        eng.build_tables(w.source.pos, w.source.lum, w.source.teff)
        t_prep = time.perf_counter()
        Jd = []
        for k in range(args.train_passes):
            for v in (t for t in tal.values() if t is not None):
                v.zero_()
            eng.run(tal, 0, N, N, w.seed + 101 * (k + 1))
            Jd.append(eng.mean_intensity(tal["jq"], N).index_select(0, dusty))
        Js = torch.as_tensor(synth.pah_fields(args.train_synthetic, w.species.lam_um, seed=4)[0]
                             .astype(np.float32)).cuda()
        Jtr = torch.cat(Jd + [Js])
        keep = Jtr.sum(1) > 0
        Jtr = Jtr[keep].contiguous()
        print(f"bench: exact solve of {Jtr.shape[0]} training cells", file=sys.stderr, flush=True)
        out_tr, pabs_tr = sur.exact(Jtr)
        torch.cuda.synchronize()
        print(f"bench: solved in {time.perf_counter() - t_prep:.1f} s; training", file=sys.stderr, flush=True)
        hist = sur.fit(Jtr, out_tr, pabs_tr, epochs=args.epochs, lr=2e-3,
                       log=lambda m: print("bench: " + m, file=sys.stderr, flush=True))
        torch.cuda.synchronize()
        info["surrogate_training"] = {"cells": int(Jtr.shape[0]), "epochs": args.epochs,
                                      "loss_first": hist[0], "loss_last": hist[-1],
                                      "setup_s": time.perf_counter() - t_prep}
        rows = torch.empty((dusty.numel(), w.species.n_lambda), dtype=torch.float64, device="cuda")
    pah_t = []

    def step():
        for v in (t for t in tal.values() if t is not None):
            v.zero_()
        eng.build_tables(w.source.pos, w.source.lum, w.source.teff)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        eng.run(tal, 0, N, N, w.seed)
        e1.record(stream)
        ev.append((e0, e1))
        T = eng.temperatures(tal["nabs"], N)
        J = eng.mean_intensity(tal["jq"], N)
        if sur is not None:
            Jc = J.index_select(0, dusty)
            p0 = torch.cuda.Event(enable_timing=True)
            p1 = torch.cuda.Event(enable_timing=True)
            p0.record(stream)
            out, ood, pabs, idx = sur.solve(Jc)
            sur.solver.rows(out, rows=rows)
            p1.record(stream)
            pah_t.append((p0, p1, ood))
        return T, J

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev.clear()
    pah_t.clear()
    print("bench: timed steps", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    k_ms = [a.elapsed_time(b) for a, b in ev]
    k_avg = sum(k_ms) / len(k_ms) / 1e3
    if sur is not None:
        n_c = int(dusty.numel())
        s_ms = [a.elapsed_time(b) for a, b, _ in pah_t]
        s_avg = sum(s_ms) / len(s_ms) / 1e3
        frac_ood = float((pah_t[-1][2] != 0).float().mean().item())
        # exact solver on the same cells, and the surrogate's band error against it
        Jc = eng.mean_intensity(tal["jq"], N).index_select(0, dusty)
        torch.cuda.synchronize()
        x0 = torch.cuda.Event(enable_timing=True)
        x1 = torch.cuda.Event(enable_timing=True)
        x0.record(stream)
        ex, _pabs_ex = sur.exact(Jc)
        x1.record(stream)
        pred, ood, _ = sur.predict(Jc)
        torch.cuda.synchronize()
        t_ex = x0.elapsed_time(x1) / 1e3
        err = band_error(pred, ex)
        okm = (ood == 0) & (ex[:, :17].sum(1) > 0)
        cpu_pah = None
        if not args.no_cpu:
            import oracle
            threads = min(16, len(os.sched_getaffinity(0)))
            sample = Jc[:: max(1, n_c // 4000)][:4000].double().cpu().numpy()
            Tg = 2.7 * (5000.0 / 2.7) ** (np.arange(500) / 499)
            tc0 = time.perf_counter()
            oracle.pah_solve(Tg, pm.enthalpy(Tg), w.species.lam_um, pm.cabs, pm.cband, pm.ccont, sample,
                             n_threads=threads)
            cpu_pah = {"value": sample.shape[0] / (time.perf_counter() - tc0), "unit": "cells/s",
                       "cores": threads, "kind": "oracle",
                       "sample": f"{sample.shape[0]} of the disk's dusty cells, exact P(T) solver"}
        info["pah"] = {"cells": n_c, "exact_cells_per_s": n_c / t_ex, "cpu_baseline_exact": cpu_pah,
                       "surrogate_in_loop_cells_per_s": n_c / s_avg,
                       "speedup": t_ex / s_avg, "ood_fraction": frac_ood,
                       "ood_input_fraction": float(((ood & 1) != 0).float().mean().item()),
                       "ood_balance_fraction": float(((ood & 2) != 0).float().mean().item()),
                       "exact_balance_dev_p99": float(torch.quantile(
                           (ex.sum(1) / _pabs_ex - 1).abs()[ex.sum(1) > 0], 0.99).item()),
                       "band_error_p95": float(torch.quantile(err[okm], 0.95).item()),
                       "band_error_median": float(err[okm].median().item())}
    c = mcrt.u64_view(tal["counters"])
    cnt = {k: int(c[v]) for k, v in mcrt.CNT.items()}
    assert cnt["launched"] == N and cnt["launched"] == cnt["escaped"] + cnt["killed"] + cnt["terminated"]

    # algorithmic bytes of one transport pass: per crossing the density (4 B)
    # and base-map entry (4 B); per path-tally segment one 8 B read-modify-write
    # (16 B); per absorption and per escape one 8 B atomic (16 B).  With the
    # deferred tally the pass is the transport kernel plus the record passes
    # (count, scan, scatter, sum), all inside the timed run.
    alg_bytes = 8 * cnt["crossings"] + 16 * cnt["jseg"] + 16 * cnt["absorptions"] + 16 * cnt["escaped"]
    achieved = alg_bytes / k_avg / 1e9
    # HBM bytes of one launch from the committed counter summary, if it was taken
    # on the current transport kernel source
    traffic = None
    try:
        import hashlib
        h = hashlib.sha256()
        for f in ("mcrt_transport.hip", "mcrt_jdefer.hip"):
            h.update(open(os.path.join(ROOT, "paper_1201_3588_amd", "csrc", f), "rb").read())
        sha = h.hexdigest()
        kv = dict(l.split(": ", 1) for l in open(os.path.join(ROOT, "profiles", "transport_flared_disk_pmc.md"))
                  if l.startswith(("traffic_bytes_per_launch:", "source_sha256:")))
        if kv.get("source_sha256", "").strip() == sha and N == 10_000_000:
            traffic = int(kv["traffic_bytes_per_launch"])
    except OSError:
        pass
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
        "config": {"workload": "flared_disk_64cube_depth3_262480leaves_24species_200lambda_1e7packets",
                   "packets_per_step": N, "leaves": w.grid.n_cells, "n_lambda": w.species.n_lambda,
                   "species": w.species.n_species, "transport": "f32 geometry, f64 tables/T",
                   "tally_j": True},
        "crossings_per_s": cnt["crossings"] * args.steps / wall,
        "transport_kernel_ms": k_avg * 1e3,
        "transport_packets_per_s": N / k_avg,
        "transport_crossings_per_s": cnt["crossings"] / k_avg,
        "per_step_counts": cnt,
        **info,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": ("transport pass: k_transport<float,false,false,true> + k_jr_count, k_scan_*, "
                                "k_jr_scatter, k_jr_items, k_jr_sum") if deferred else
                               "k_transport<float,false,false,false>",
                     "alg_bytes_per_launch": alg_bytes},
        "path_tally": {"mode": "deferred records" if deferred else "atomic",
                       "segments_per_s": cnt["jseg"] / k_avg},
    }

    if not args.no_micro:
        atom_rate = random_atomic_rate(w.species.n_lambda * w.grid.n_cells, stream)
        # the tally updates of the pass (path segments, absorptions, escapes)
        # per second against the measured rate of random 64-bit atomics over a
        # table of the path tally's size: above 1 once the path segments no
        # longer go through atomics
        tr_atoms = (cnt["jseg"] + cnt["absorptions"] + cnt["escaped"]) / k_avg
        out["random_access_ceiling"] = {
            "atomics_per_s": atom_rate, "table_bytes": w.species.n_lambda * w.grid.n_cells * 8,
            "gbs_at_16B_per_op": atom_rate * 16 / 1e9,
            "tally_updates_per_s": tr_atoms, "frac_of_ceiling": tr_atoms / atom_rate}

    if args.reemission:
        out["reemission_law"] = [
            reemission_block(synth.c1_sphere(n_packets=n), stream,
                             f"uniform_sphere_32cube_100lambda_{n:.0e}packets_f64".replace("+0", ""))
            for n in (100_000, 1_000_000, 10_000_000)]
        out["reemission_law"].append(reemission_block(synth.c2_disk(n_packets=N), stream,
                                                      out["config"]["workload"]))
    if not args.no_pah:
        out["pah_hard_photons"] = hard_photon_block(stream)
    if args.c3:
        out["c3"] = c3_block(args.c3_packets, not args.no_micro, stream, iterate=args.c3_iterate)
    if args.c5:
        out["c5"] = c5_block(args.c5_packets, stream)

    if not args.no_cpu:
        import oracle
        try:
            threads = min(16, len(os.sched_getaffinity(0)))
        except AttributeError:
            threads = min(16, os.cpu_count() or 1)
        n_s = min(args.cpu_sample, N)
        s = oracle.Session(w, n_threads=threads)
        acc = s.new_accumulator()
        tc0 = time.perf_counter()
        s.accumulate(acc, 0, n_s)
        tc = time.perf_counter() - tc0
        out["cpu_baseline"] = {"value": n_s / tc, "unit": "packets/s", "cores": threads, "kind": "oracle",
                               "sample": f"first {n_s} packet ids of the same workload, transport only, "
                                         f"{tc:.1f} s wall"}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
