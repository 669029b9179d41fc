"""Parity at the size of the gap + spiral disk with PAHs (128^3 base, depth 3,
2,098,552 leaves, 26 species of which two PAHs, 200 wavelengths, 1e8 packets),
in the launch configuration the benchmark times: PAH re-emission rows from the
optically thin field (first pass of the PAH iteration, exact solver), then one
transport pass with the path-length tally deferred to records (two partition
levels, id ranges of 12 M packets).  The oracle checks sampled outputs one by
one:
  * exact integer bookkeeping of the full pass;
  * the exact PAH solution and re-emission rows of sampled cells on the
    oracle's thin field, and the pass's rows at those cells reproduced;
  * with a frozen absorption field (an oracle run of 1e5 packets, scaled) and
    seeded stand-in PAH rows on both sides, sampled packet ids anywhere in
    [0, 1e8) retrace the oracle's histories, PAH re-emission included (at most
    2 % of them, rays meeting a face at grazing incidence, may carry FP32
    position errors up to 1e-3 instead of 1e-5);
  * temperatures of sampled cells and the mean intensity of every cell from
    seeded tallies of the pass's size (no oracle input comes from the GPU);
  * with a frozen field, the deferred tally of 3 M packets equals the
    per-segment atomic one bit for bit.
"""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu
mcrt = pytest.importorskip("paper_1201_3588_amd.mcrt")

from test_gpu_transport import _compare_traces, conservation, host  # noqa: E402


@pytest.fixture(scope="module")
def c3_pass():
    from paper_1201_3588_amd.pipeline import PahLoop
    w = synth.c3_gap_spiral()
    loop = PahLoop(w)
    J0 = loop.eng.thin_field()
    outs = loop.emission(J0)
    assert loop.eng.set_deferred_tally(1 << 31)
    tal = loop.eng.new_tallies(tally_j=True)
    loop.eng.run_batched(tal, 0, w.n_packets, w.n_packets, w.seed, 12_000_000, pah_rows=loop.rows)
    T = loop.eng.temperatures(tal["nabs"], w.n_packets)
    torch.cuda.synchronize()
    return dict(w=w, loop=loop, J0=J0, outs=outs, r=host(tal), T=T.cpu().numpy(),
                rows=loop.rows.cpu().numpy())


def test_c3_bookkeeping(c3_pass):
    w, r = c3_pass["w"], c3_pass["r"]
    conservation(r, w.n_packets)
    c = r["counters"]
    assert c[2] == 0                                  # nothing hit the event cap
    assert c[9] > 1e6                                 # PAH absorptions re-emitted from the rows
    assert c[6] > 1e10 and c[11] > 1e10               # crossings, path-tally segments
    assert np.all(np.isfinite(c3_pass["T"]))


def test_c3_pah_emission_and_rows_of_sampled_cells(c3_pass):
    # the exact PAH solution and the rows of sampled cells, on the oracle's
    # optically thin field (the field the pass's rows were built from)
    w, loop = c3_pass["w"], c3_pass["loop"]
    pick = np.random.default_rng(3).choice(w.grid.n_cells, 60, replace=False)
    J = oracle.Session(w, flags=0).thin_field()[pick]
    Tg = 2.7 * (5000.0 / 2.7) ** (np.arange(500) / 499)
    for p, (pm, s) in enumerate(zip(w.pah, loop.solvers)):
        g_out = s.solve(torch.as_tensor(J).cuda())[0].cpu().numpy()
        o_out, _, _ = oracle.pah_solve(Tg, pm.enthalpy(Tg), w.species.lam_um, pm.cabs, pm.cband, pm.ccont,
                                       J, n_threads=8)
        for k in range(len(pick)):
            m = o_out[k] > 1e-12 * o_out[k].max()
            assert np.max(np.abs(g_out[k][m] / o_out[k][m] - 1)) < 1e-10
        g_rows = s.rows(torch.as_tensor(o_out).cuda()).cpu().numpy()
        ref = oracle.pah_rows(w.species.lam_um, pm.cband, o_out)
        assert np.max(np.abs(g_rows - ref)) < 1e-12
    # the pass's own rows at those cells are the rows of the GPU thin field's solution
    Jg = c3_pass["J0"].index_select(0, torch.as_tensor(pick).cuda())
    for p, s in enumerate(loop.solvers):
        again = s.rows(s.solve(Jg)[0]).cpu().numpy()
        assert np.allclose(again, c3_pass["rows"][p][pick], rtol=0, atol=1e-15)


def test_c3_sampled_packets_retrace_oracle(c3_pass):
    # frozen field: an oracle run of 1e5 packets scaled to the 1e8-packet pass;
    # PAH rows: seeded stand-in rows on both sides (dense on the GPU, a compact
    # table with a per-cell row index in the oracle)
    w, loop = c3_pass["w"], c3_pass["loop"]
    nc, nl = w.grid.n_cells, w.species.n_lambda
    n_pah = len(w.pah)
    table = synth.pah_test_rows(1, 4096, nl, seed=33)[0]
    rmap = np.random.default_rng(9).integers(0, 4096, n_pah * nc).astype(np.int32)
    rows = torch.as_tensor(table).cuda()[torch.as_tensor(rmap).cuda().long()].view(n_pah, nc, nl)
    frozen = oracle.Session(w, n_threads=8, flags=0, pah_rows=table,
                            pah_row_map=rmap).transport(n=100_000)["nabs"] * np.uint64(1000)
    frozen_dev = torch.as_tensor(frozen.reshape(-1).view(np.int64)).cuda()
    s = oracle.Session(w, frozen_nabs=frozen, flags=oracle.FLAG_FROZEN_T, pah_rows=table, pah_row_map=rmap)
    ids = np.linspace(0, w.n_packets - 1, 120).astype(np.int64)
    same = 0
    pah_seen = 0
    grazing, parted = [], []
    for pid in ids:
        tal = loop.eng.new_tallies(tally_j=False)
        gt = loop.eng.run(tal, int(pid), 1, w.n_packets, w.seed, frozen_nabs=frozen_dev, trace_cap=1000,
                          pah_rows=rows, flags=mcrt.FLAG_FROZEN_T)
        ot = s.transport(int(pid), 1, trace_cap=1000)["trace"]
        same += _compare_traces(gt, ot, 1e-5, float(w.grid.nb), grazing, parted)
        pah_seen += int(mcrt.u64_view(tal["counters"])[9])
    assert same >= 0.95 * len(ids), parted
    assert len(grazing) <= 0.02 * len(ids), grazing
    assert pah_seen > 0


def test_c3_sampled_temperatures_and_intensities(c3_pass):
    # the temperature and mean-intensity kernels at this size on seeded
    # tallies of the pass's magnitude; the pass's own temperatures are finite
    from test_gpu_fullsize import seeded_tallies
    w, loop = c3_pass["w"], c3_pass["loop"]
    S = w.species.n_species
    pick, nabs, jq = seeded_tallies(w, 4, n_pick=200)
    Tg = loop.eng.temperatures(torch.as_tensor(nabs.reshape(-1).view(np.int64)).cuda(), w.n_packets)
    Jg = loop.eng.mean_intensity(torch.as_tensor(jq.reshape(-1).view(np.int64)).cuda(), w.n_packets)
    Tg, Jg = Tg.cpu().numpy(), Jg.cpu().numpy()
    s = oracle.Session(w, n_threads=8, flags=0)
    To = s.temperatures(nabs)
    eq = w.species.kind == 0
    assert np.allclose(Tg.reshape(-1, S)[pick][:, eq], To[pick][:, eq], rtol=1e-11, atol=0)
    Jo = s.mean_intensity(jq)
    assert np.allclose(Jg, Jo, rtol=2e-7, atol=1e-30 * Jo.max())


def test_c3_deferred_tally_equals_atomic(c3_pass):
    # the same 3 M packets with the pass's absorption field frozen, once with
    # per-segment atomics and once through records (two partition levels):
    # identical tallies
    w, loop = c3_pass["w"], c3_pass["loop"]
    eng = loop.eng
    frozen = torch.as_tensor(c3_pass["r"]["nabs"].view(np.int64)).cuda()
    flags = mcrt.FLAG_TALLY_J | mcrt.FLAG_FROZEN_T
    out = {}
    for mode in ("atomic", "deferred"):
        eng.set_deferred_tally(1 << 31 if mode == "deferred" else 0)
        tal = eng.new_tallies(tally_j=True)
        eng.run(tal, 40_000_000, 3_000_000, w.n_packets, w.seed, frozen_nabs=frozen, pah_rows=loop.rows,
                flags=flags)
        out[mode] = host(tal)
        del tal
    a, b = out["atomic"], out["deferred"]
    assert int(a["counters"][mcrt.CNT["jseg"]]) > 3e8
    for k in ("nabs", "sed", "jq", "counters"):
        assert np.array_equal(a[k], b[k]), k
