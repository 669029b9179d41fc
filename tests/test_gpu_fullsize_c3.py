"""Parity at the size of the gap + spiral disk with PAHs (128^3 base, depth 3,
2,098,552 leaves, 26 species of which two PAHs, 200 wavelengths, 1e8 packets),
in the launch configuration the benchmark times: PAH re-emission rows from the
optically thin field (first pass of the PAH iteration, exact solver), then one
transport pass with the path-length tally deferred to records (two partition
levels, id ranges of 12 M packets).  The oracle checks sampled outputs one by
one:
  * exact integer bookkeeping of the full pass;
  * the exact PAH solution and re-emission rows of sampled cells;
  * with the pass's own absorption field frozen, sampled packet ids anywhere in
    [0, 1e8) retrace the oracle's histories, PAH re-emission included (at most
    2 % of them, rays meeting a face at grazing incidence, may carry FP32
    position errors up to 1e-3 instead of 1e-5);
  * temperatures of sampled cells and the mean intensity of every cell,
    recomputed by the oracle from the GPU's tallies;
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
    w, loop = c3_pass["w"], c3_pass["loop"]
    pick = np.random.default_rng(3).choice(w.grid.n_cells, 60, replace=False)
    pk = torch.as_tensor(pick).cuda()
    J = c3_pass["J0"].index_select(0, pk).cpu().numpy().astype(np.float64)
    Tg = 2.7 * (5000.0 / 2.7) ** (np.arange(500) / 499)
    for p, pm in enumerate(w.pah):
        g_out = c3_pass["outs"][p].index_select(0, pk).cpu().numpy()
        o_out, _, _ = oracle.pah_solve(Tg, pm.enthalpy(Tg), w.species.lam_um, pm.cabs, pm.cband, pm.ccont,
                                       J, n_threads=8)
        for k in range(len(pick)):
            m = o_out[k] > 1e-12 * o_out[k].max()
            assert np.max(np.abs(g_out[k][m] / o_out[k][m] - 1)) < 1e-10
        ref = oracle.pah_rows(w.species.lam_um, pm.cband, g_out)
        assert np.max(np.abs(c3_pass["rows"][p][pick] - ref)) < 1e-12


def test_c3_sampled_packets_retrace_oracle(c3_pass):
    w, loop, r = c3_pass["w"], c3_pass["loop"], c3_pass["r"]
    frozen = r["nabs"].reshape(w.grid.n_cells, w.species.n_species)
    frozen_dev = torch.as_tensor(frozen.view(np.int64)).cuda()
    s = oracle.Session(w, frozen_nabs=frozen, pah_rows=c3_pass["rows"])
    ids = np.linspace(0, w.n_packets - 1, 120).astype(np.int64)
    same = 0
    pah_seen = 0
    grazing = []
    for pid in ids:
        tal = loop.eng.new_tallies(tally_j=True)
        gt = loop.eng.run(tal, int(pid), 1, w.n_packets, w.seed, frozen_nabs=frozen_dev, trace_cap=600,
                          pah_rows=loop.rows, flags=mcrt.FLAG_TALLY_J | mcrt.FLAG_FROZEN_T)
        ot = s.transport(int(pid), 1, trace_cap=600)["trace"]
        same += _compare_traces(gt, ot, 1e-5, float(w.grid.nb), grazing)
        pah_seen += int(mcrt.u64_view(tal["counters"])[9])
    assert same >= 0.97 * len(ids)
    assert len(grazing) <= 0.02 * len(ids), grazing
    assert pah_seen > 0


def test_c3_sampled_temperatures_and_intensities(c3_pass):
    w, loop, r = c3_pass["w"], c3_pass["loop"], c3_pass["r"]
    S = w.species.n_species
    nabs = r["nabs"].reshape(w.grid.n_cells, S)
    hot = np.nonzero(nabs.sum(1) > 0)[0]
    pick = np.random.default_rng(4).choice(hot, 200, replace=False)
    sub = np.zeros_like(nabs)
    sub[pick] = nabs[pick]
    s = oracle.Session(w, n_threads=8, pah_rows=c3_pass["rows"])
    To = s.temperatures(sub)
    eq = w.species.kind == 0
    assert np.allclose(c3_pass["T"].reshape(-1, S)[pick][:, eq], To[pick][:, eq], rtol=1e-11, atol=0)
    J = loop.eng.mean_intensity(torch.as_tensor(r["jq"].view(np.int64)).cuda(), w.n_packets).cpu().numpy()
    Jo = s.mean_intensity(r["jq"])
    assert np.allclose(J, Jo, rtol=2e-7, atol=1e-30 * Jo.max())


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
