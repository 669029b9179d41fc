#!/usr/bin/env python3
"""Benchmark of the Monte Carlo dust transfer hot path on one MI355X.

One step = one pass of the hot path over the flared proto-planetary disk
workload (64^3 base cubes refined 2x2x2 to depth 3 inside 1 AU = 262,480
leaves, 3 materials x 8 grain sizes, 200 wavelengths, Henyey-Greenstein
scattering, 1e7 packets from a 5800 K, 1 L_sun star, FP32 geometry, FP64
tables and temperatures, path-length J tally on):
  table build -> transport of all packets -> temperatures -> mean intensity.
Inputs are resident in device memory before the timed region.  Prints one
JSON line.  The CPU oracle is timed on a bounded sample for reference.
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--packets", type=int, default=10_000_000)
    ap.add_argument("--cpu-sample", type=int, default=400_000)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-micro", action="store_true")
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
    w = synth.c2_disk(n_packets=args.packets)
    N = w.n_packets
    eng = mcrt.Engine.from_workload(w)
    tal = eng.new_tallies(tally_j=True)
    stream = torch.cuda.current_stream()
    ev = []

    def step():
        for v in tal.values():
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
        return T, J

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev.clear()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    k_ms = [a.elapsed_time(b) for a, b in ev]
    k_avg = sum(k_ms) / len(k_ms) / 1e3
    c = mcrt.u64_view(tal["counters"])
    cnt = {k: int(c[v]) for k, v in mcrt.CNT.items()}
    assert cnt["launched"] == N and cnt["launched"] == cnt["escaped"] + cnt["killed"] + cnt["terminated"]

    # algorithmic bytes of one transport launch: per crossing the density (4 B)
    # and base-map entry (4 B); per path-tally segment one 8 B read-modify-write
    # (16 B); per absorption and per escape one 8 B atomic (16 B)
    alg_bytes = 8 * cnt["crossings"] + 16 * cnt["jseg"] + 16 * cnt["absorptions"] + 16 * cnt["escaped"]
    achieved = alg_bytes / k_avg / 1e9
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
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_transport<float>", "alg_bytes_per_launch": alg_bytes},
    }

    if not args.no_micro:
        # achievable random 64-bit atomic rate over a table of the J tally's size
        n_slots = w.species.n_lambda * w.grid.n_cells
        table = torch.zeros(n_slots, dtype=torch.int64, device="cuda")
        n_ops = 1 << 28
        L = mcrt.lib()
        import ctypes as C
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
        dt = e0.elapsed_time(e1) / 1e3
        atom_rate = issued / dt
        out["random_access_ceiling"] = {
            "atomics_per_s": atom_rate, "table_bytes": n_slots * 8,
            "gbs_at_16B_per_op": atom_rate * 16 / 1e9,
            "transport_jseg_per_s": cnt["jseg"] / k_avg,
            "frac_of_ceiling": (alg_bytes / k_avg) / (atom_rate * 16)}
        del table

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
