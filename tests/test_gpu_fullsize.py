"""Parity at the benchmark's full size: the flared disk (262,480 leaves, 24
species, 200 wavelengths) with 1e7 packets in the launch configuration that
bench.py times.  The oracle cannot redo the whole pass, so it checks sampled
outputs one by one and properties that hold at any size:
  * exact integer bookkeeping of the full pass;
  * with a frozen absorption field (an oracle run of 2e5 packets, scaled),
    sampled packet ids anywhere in [0, 1e7) retrace the oracle's histories;
  * temperatures of sampled cells and the mean intensity of every cell from
    seeded tallies of the pass's size (no oracle input comes from the GPU);
  * the exact PAH solver on sampled cells' Monte Carlo fields (oracle run);
  * 3 sigma agreement of SED bins and per-cell absorptions at 2e6 packets
    (frozen field from an oracle run);
  * with a frozen field, the full pass's path-length tally through records (the
    benchmark's path) equals the per-segment atomic one bit for bit.
"""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu
mcrt = pytest.importorskip("paper_1201_3588_amd.mcrt")

from test_gpu_transport import _compare_traces, conservation, host, statistical_check  # noqa: E402


@pytest.fixture(scope="module")
def full_pass():
    w = synth.c2_disk()
    e = mcrt.Engine.from_workload(w)
    e.build_tables(w.source.pos, w.source.lum, w.source.teff)
    assert e.set_deferred_tally(min(1 << 31, 100 * w.n_packets))        # as bench.py
    tal = e.new_tallies(tally_j=True)
    e.run(tal, 0, w.n_packets, w.n_packets, w.seed)
    T = e.temperatures(tal["nabs"], w.n_packets)
    J = e.mean_intensity(tal["jq"], w.n_packets)
    torch.cuda.synchronize()
    return w, e, host(tal), T.cpu().numpy(), J.cpu().numpy()


def test_full_pass_bookkeeping(full_pass):
    w, e, r, T, J = full_pass
    conservation(r, w.n_packets)
    c = r["counters"]
    assert c[2] == 0                                   # nothing hit the event cap
    assert c[6] > 5e8 and c[11] > 4e8                  # crossings, path-tally segments
    assert np.all(np.isfinite(T)) and np.all(np.isfinite(J))


def test_sampled_packets_retrace_oracle(full_pass):
    # frozen field: an oracle run of 2e5 packets, scaled to the 1e7-packet pass
    w, e, r, T, J = full_pass
    frozen = oracle.Session(w, n_threads=8, flags=0).transport(n=200_000)["nabs"] * np.uint64(50)
    s = oracle.Session(w, frozen_nabs=frozen)
    ids = np.linspace(0, w.n_packets - 1, 160).astype(np.int64)
    same = 0
    parted = []
    for pid in ids:
        tal = e.new_tallies(tally_j=True)
        gt = e.run(tal, int(pid), 1, w.n_packets, w.seed, frozen_nabs=frozen, trace_cap=400,
                   flags=mcrt.FLAG_TALLY_J | mcrt.FLAG_FROZEN_T)
        ot = s.transport(int(pid), 1, trace_cap=400)["trace"]
        same += _compare_traces(gt, ot, 1e-5, float(w.grid.nb), parted=parted)
    assert same >= 0.97 * len(ids), parted


def seeded_tallies(w, seed, n_pick=300):
    """Seeded absorption counts (sampled dusty cells, every species) and path
    sums (every bin of every dusty cell) of the sizes a full pass gives."""
    S, nl = w.species.n_species, w.species.n_lambda
    rng = np.random.default_rng(seed)
    dusty = np.nonzero(w.grid.rho > 0)[0]
    pick = rng.choice(dusty, n_pick, replace=False)
    nabs = np.zeros((w.grid.n_cells, S), np.uint64)
    nabs[pick] = rng.integers(0, 100_000, (n_pick, S)).astype(np.uint64)
    jq = np.zeros((nl, w.grid.n_cells), np.uint64)
    jq[:, dusty] = rng.integers(0, 1 << 40, (nl, dusty.size), dtype=np.uint64)
    return pick, nabs, jq


def test_sampled_temperatures_and_all_intensities(full_pass):
    # the temperature and mean-intensity kernels at full size, on seeded
    # tallies of the pass's magnitude; the pass's own fields are finite
    w, e, r, T, J = full_pass
    S = w.species.n_species
    assert np.all(np.isfinite(T)) and np.all(np.isfinite(J))
    pick, nabs, jq = seeded_tallies(w, 1)
    Tg = e.temperatures(torch.as_tensor(nabs.reshape(-1).view(np.int64)).cuda(), w.n_packets).cpu().numpy()
    Jg = e.mean_intensity(torch.as_tensor(jq.reshape(-1).view(np.int64)).cuda(), w.n_packets).cpu().numpy()
    s = oracle.Session(w, n_threads=8)
    To = s.temperatures(nabs)
    assert np.allclose(Tg.reshape(-1, S)[pick], To[pick], rtol=1e-11, atol=0)
    Jo = s.mean_intensity(jq)
    assert np.allclose(Jg, Jo, rtol=2e-7, atol=1e-30 * Jo.max())


def test_pah_exact_on_sampled_disk_fields(full_pass):
    # Monte Carlo fields of the disk from an oracle run of 2e5 packets
    from paper_1201_3588_amd import pah
    w, e, r, T, J = full_pass
    s = oracle.Session(w, n_threads=8)
    J = s.mean_intensity(s.transport(n=200_000)["jq"]).astype(np.float32)
    dusty = np.nonzero((w.grid.rho > 0) & (J.sum(1) > 0))[0]
    pick = np.random.default_rng(2).choice(dusty, 40, replace=False)
    pm = synth.pah_model(30, w.species.lam_um)
    s = pah.PahSolver.from_model(pm)
    g_out, _, _ = s.solve(torch.as_tensor(J[pick]).cuda())
    g_out = g_out.cpu().numpy()
    Tg = 2.7 * (5000.0 / 2.7) ** (np.arange(500) / 499)
    o_out, _, _ = oracle.pah_solve(Tg, pm.enthalpy(Tg), w.species.lam_um, pm.cabs, pm.cband, pm.ccont,
                                   J[pick].astype(np.float64), n_threads=8)
    for c in range(len(pick)):
        m = o_out[c] > 1e-12 * o_out[c].max()
        assert np.max(np.abs(g_out[c][m] / o_out[c][m] - 1)) < 1e-10


def test_full_grid_statistics_frozen():
    # the full 262,480-leaf grid, 2e6 packets per side with a frozen
    # temperature field (from an oracle run of 2e5 packets), seeds differing:
    # absorptions per cell (summed over the 24 species) and SED bins within
    # 3 sigma (statparity's criteria)
    w2 = synth.c2_disk(n_packets=2_000_000)
    frozen = oracle.Session(w2, n_threads=8).transport(n=200_000)["nabs"]

    def per_cell(d, w):
        return dict(sed=d["sed"].astype(np.float64),
                    nabs=d["nabs"].reshape(w.grid.n_cells, -1).astype(np.float64).sum(1))
    res = statistical_check(w2, frozen=frozen, summarize=per_cell)
    for k, (ok, v) in res.items():
        assert ok and v["n"] >= 300, (k, v)


def test_full_pass_deferred_tally_equals_atomic(full_pass):
    w, e, r, T, J = full_pass
    frozen = torch.as_tensor(r["nabs"].view(np.int64)).cuda()
    flags = mcrt.FLAG_TALLY_J | mcrt.FLAG_FROZEN_T
    out = {}
    for mode in ("deferred", "atomic"):
        if mode == "atomic":
            e.set_deferred_tally(0)
        tal = e.new_tallies(tally_j=True)
        e.run(tal, 0, w.n_packets, w.n_packets, w.seed, frozen_nabs=frozen, flags=flags)
        out[mode] = host(tal)
        del tal
    for k in ("nabs", "sed", "jq", "counters"):
        assert np.array_equal(out["atomic"][k], out["deferred"][k]), k
