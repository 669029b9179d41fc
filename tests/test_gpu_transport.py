"""GPU parity of the transport engine against the CPU oracle (through the C ABI).

* tables: FP64 device tables equal the oracle's to rounding;
* traces: with the temperature field frozen, a packet's history is a pure
  function of (seed, id); FP64 geometry reproduces the oracle's histories
  (event types and cells exact, positions to 1e-12), FP32 geometry to 1e-5,
  and a packet whose FP32 history parts from the oracle's parts at a tie;
* integer bookkeeping identities hold exactly;
* statistics: independent GPU and oracle runs agree within 3 sigma per
  output (per-cell absorptions, path sums and SED bins; paired batch means
  over 32 packet-id batches, tests/statparity.py);
* temperatures and mean intensity equal the oracle's for the same tallies.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import statparity
import synth

pytestmark = pytest.mark.gpu

mcrt = pytest.importorskip("paper_1201_3588_amd.mcrt")


def engine(w, precision=None):
    e = mcrt.Engine.from_workload(w, precision=precision)
    e.build_tables(w.source.pos, w.source.lum, w.source.teff, beam=w.source.beam)
    return e


def host(tal):
    torch.cuda.synchronize()
    return {k: (mcrt.u64_view(v) if v is not None else None) for k, v in tal.items()}


def conservation(r, n):
    c = r["counters"]
    assert c[0] == n
    assert c[0] == c[1] + c[2] + c[3]
    assert int(r["nabs"].sum()) == int(c[5])
    assert int(r["sed"].sum()) == int(c[1])


# --------------------------------------------------------------------------
def test_tables_match_oracle():
    for w in (synth.c1_sphere(n_packets=10), synth.small_disk(n_packets=10)):
        e = engine(w)
        g = e.tables_numpy()
        t = oracle.Session(w).tables
        for k in ("nu", "dnu", "src_cdf", "kext", "albedo", "Tk", "E"):
            assert np.allclose(g[k], t[k], rtol=1e-13, atol=0), k
        assert np.allclose(g["sp_cdf"], t["sp_cdf"], rtol=1e-13, atol=1e-15)
        assert np.allclose(g["R"], t["R"], rtol=1e-12, atol=1e-15)
        assert np.all(g["R"][..., -1] == 1.0)
        assert np.array_equal(g["level"], w.grid.leaf_level)


def _first_split(a, b):
    """Index of the first record where two traces differ in (type, cell, bin),
    or None when they agree throughout."""
    n = min(len(a), len(b))
    for i in range(n):
        if a["type"][i] != b["type"][i] or a["cell"][i] != b["cell"][i] or a["j"][i] != b["j"][i]:
            return i
    return None if len(a) == len(b) else n


def _compare_traces(gt, ot, pos_tol, extent, grazing=None, parted=None):
    """Number of packets whose (type, cell, bin) sequences agree.  For those,
    the position at every event must agree to pos_tol relative to the larger of
    the grid extent and the path length travelled so far (rounding accumulates
    along a path), directions and optical depths to 10 pos_tol.  A ray that
    meets a face at grazing incidence (|d| along the face normal small) turns
    a rounding of its position across the face into an error 1/|d| larger
    along it; with `grazing` (a list) such packets may exceed pos_tol up to
    100 pos_tol and are appended to the list instead of failing.

    A packet whose sequences part must part at a tie decided by rounding: up
    to the first differing record the two histories agree as above, and at
    that record the two sides stand at the same point to within 10 pos_tol
    (a crossing against an interaction just short of the face, or two
    neighbouring cells across an edge or a corner).  With `parted` (a list)
    the split index and that distance are appended for each such packet."""
    same = 0
    for a, b in zip(gt, ot):
        path = np.concatenate([[0.0], np.cumsum(np.linalg.norm(np.diff(b["x"], axis=0), axis=1))])
        k = _first_split(a, b)
        m = len(b) if k is None else k
        if m:
            err = np.linalg.norm(a["x"][:m] - b["x"][:m], axis=1) / np.maximum(extent, path[:m])
            if grazing is not None and np.max(err) >= pos_tol:
                assert np.max(err) < 100 * pos_tol
                if k is None:
                    grazing.append(float(np.max(err)))
            else:
                assert np.max(err) < pos_tol, (k, np.max(err))
            assert np.max(np.abs(a["d"][:m] - b["d"][:m])) < pos_tol * 10
            assert np.max(np.abs(a["tau"][:m] - b["tau"][:m]) / np.maximum(1.0, np.abs(b["tau"][:m]))) < pos_tol * 10
        if k is None:
            same += 1
            continue
        assert 0 < k < min(len(a), len(b)), (k, len(a), len(b))
        gap = float(np.linalg.norm(a["x"][k] - b["x"][k]) / max(extent, path[k]))
        lim = 100 * pos_tol if grazing is not None else 10 * pos_tol
        assert gap < lim, ("parted away from a tie", k, gap, a[k - 1:k + 1], b[k - 1:k + 1])
        if parted is not None:
            parted.append((k, gap))
    return same


@pytest.mark.parametrize("precision,tol,min_frac", [("f64", 1e-12, 0.999), ("f32", 1e-5, 0.98)])
def test_fixed_random_traces(precision, tol, min_frac):
    for w in (synth.small_disk(n_packets=400, nl=32, n_sizes=2, nb=8),
              synth.uniform_cube(8, 0.7, albedo=0.5, g=0.6, n_packets=400)):
        base = oracle.Session(w).transport(n=2000)["nabs"]
        e = engine(w, precision)
        tal = e.new_tallies(tally_j=True)
        gt = e.run(tal, 100, 400, w.n_packets, w.seed, frozen_nabs=base, trace_cap=600,
                   flags=mcrt.FLAG_TALLY_J | mcrt.FLAG_FROZEN_T)
        ot = oracle.Session(w, frozen_nabs=base).transport(100, 400, trace_cap=600)["trace"]
        parted = []
        same = _compare_traces(gt, ot, tol, float(w.grid.nb), parted=parted)
        assert same >= min_frac * 400, (precision, same)
        assert same + len(parted) == 400


@pytest.mark.parametrize("precision,tol", [("f64", 1e-12), ("f32", 1e-5)])
@pytest.mark.parametrize("beam", [(0.0, 0.0, 1.0), (-1.0, 0.0, 0.0)])
def test_axis_aligned_beam_traces(precision, tol, beam):
    # a pencil beam along a grid axis from the star on a grid vertex: until
    # its first scattering a packet does not move along two axes and sits on
    # their faces, so their exits are at infinity (FP32: a reciprocal of -inf,
    # and 0 * inf on the low face, which the minimum must skip)
    w = synth.uniform_cube(8, 0.7, albedo=0.5, g=0.6, n_packets=400)
    w.source.beam = np.array(beam)
    base = oracle.Session(w).transport(n=2000)["nabs"]
    e = engine(w, precision)
    tal = e.new_tallies(tally_j=True)
    gt = e.run(tal, 0, 400, w.n_packets, w.seed, frozen_nabs=base, trace_cap=600,
               flags=mcrt.FLAG_TALLY_J | mcrt.FLAG_FROZEN_T)
    ot = oracle.Session(w, frozen_nabs=base).transport(0, 400, trace_cap=600)["trace"]
    assert np.allclose(ot[0]["d"][0], beam) and ot[0]["type"][0] == 0
    parted = []
    same = _compare_traces(gt, ot, tol, float(w.grid.nb), parted=parted)
    assert same >= (0.999 if precision == "f64" else 0.98) * 400, (precision, same, parted)
    assert same + len(parted) == 400


def disk_observers(w, npix=25):
    # face-on, edge-on and inclined views of the disk, centred on the star,
    # field of view the whole grid, three near- and mid-infrared bins; an odd
    # pixel count puts the star at a pixel centre (direct starlight projects to
    # the centre up to rounding, which must not decide the pixel)
    half = 0.5 * w.grid.nb * w.grid.base_size
    return dict(dirs=[(0, 0, 1), (1, 0, 0), (0, 0.5, 0.866)], npix=npix, half_width=1.2 * half,
                center=list(w.source.pos), cos_cone=float(np.cos(np.radians(35.0))), lambda_bins=[10, 14, 16])


@pytest.mark.parametrize("law", ["before", "exact_bw"])
def test_fp64_frozen_tallies_equal_oracle(law):
    # law: re-emission from the bracket holding T_before (the paper's method)
    # or from the Bjorkman-Wood difference spectrum of the temperature rise
    extra = mcrt.FLAG_EXACT_BW if law == "exact_bw" else 0
    w = synth.small_disk(n_packets=3000, nl=32, n_sizes=2, nb=8)
    w.precision = "f64"
    base = oracle.Session(w).transport()["nabs"]
    e = engine(w)
    obs = disk_observers(w)
    e.set_observers(**obs, peel=True)
    tal = e.new_tallies()
    e.run(tal, 0, 3000, 3000, w.seed, frozen_nabs=base, flags=mcrt.FLAG_TALLY_J | mcrt.FLAG_FROZEN_T | extra)
    g = host(tal)
    o = oracle.Session(w, frozen_nabs=base, observers=obs,
                       flags=oracle.FLAG_TALLY_J | oracle.FLAG_PEEL | extra).transport()
    assert np.array_equal(g["counters"], o["counters"])
    assert int(o["counters"][oracle.CNT["peel"]]) > 1000
    # next-event weights: the same events and lines of sight; the optical
    # depths of the two sides differ in the last bits (cell-local against
    # global coordinates), which can move a rounding to 2^-24 by one unit
    gp, op = g["peel"].astype(np.int64), o["peel"].reshape(-1).astype(np.int64)
    assert op.sum() > 1000 * oracle.PEEL_ONE
    assert np.abs(gp - op).max() <= 2
    assert abs(int(gp.sum()) - int(op.sum())) <= 1e-12 * op.sum() + 50
    assert np.array_equal(g["nabs"], o["nabs"].reshape(-1))
    assert np.array_equal(g["sed"], o["sed"].reshape(-1))
    assert np.array_equal(g["jq"], o["jq"].reshape(-1))
    assert o["image"].sum() > 100
    assert np.array_equal(g["image"], o["image"].reshape(-1))
    assert np.array_equal(e.counters_sync(tal), o["counters"])
    if extra:
        d = oracle.Session(w, frozen_nabs=base, flags=oracle.FLAG_TALLY_J).transport()
        assert not np.array_equal(d["sed"], o["sed"])


def test_fp64_frozen_azimuth_bins_equal_oracle():
    # the gap + spiral disk with PAHs, escapes binned in 10 equal-cos theta x
    # 8 phi bins (the SEDs of the non-axisymmetric disk): with FP64 geometry,
    # a frozen temperature field and equal seeds, every (theta, phi, bin)
    # count equals the oracle's
    w = synth.small_disk(n_packets=6000, nl=32, n_sizes=1, nb=8, with_pah=True, gap_spiral=True)
    w.precision = "f64"
    assert (w.n_theta, w.n_phi) == (10, 8)
    n_pah = int((w.species.kind == 1).sum())
    rows = synth.pah_test_rows(n_pah, w.grid.n_cells, w.species.n_lambda, seed=13)
    base = oracle.Session(w, pah_rows=rows).transport(n=2000)["nabs"]
    e = engine(w)
    tal = e.new_tallies()
    flags = mcrt.FLAG_TALLY_J | mcrt.FLAG_FROZEN_T
    e.run(tal, 0, w.n_packets, w.n_packets, w.seed, frozen_nabs=base, pah_rows=rows, flags=flags)
    g = host(tal)
    o = oracle.Session(w, frozen_nabs=base, pah_rows=rows).transport()
    assert np.array_equal(g["counters"], o["counters"])
    assert np.array_equal(g["sed"], o["sed"].reshape(-1))
    assert np.array_equal(g["nabs"], o["nabs"].reshape(-1))
    assert np.array_equal(g["jq"], o["jq"].reshape(-1))
    # every azimuth bin is populated, so a wrong phi bin cannot hide
    per_phi = o["sed"].sum(axis=(0, 2))
    assert per_phi.shape == (8,) and per_phi.min() > 200, per_phi
    assert int(o["counters"][oracle.CNT["pah_abs"]]) > 50


def test_peel_fp32_and_queue_overflow():
    # FP32 transport against the FP64 oracle with equal random numbers: the
    # direct starlight (star pixel) agrees to FP32 rounding of the optical
    # depth, every image's total to the few packets whose histories part;
    # a queue too small for the run keeps what fits and counts the rest
    w = synth.small_disk(n_packets=3000, nl=32, n_sizes=2, nb=8)
    base = oracle.Session(w).transport()["nabs"]
    obs = disk_observers(w)
    e = engine(w)
    e.set_observers(**obs, peel=True)
    tal = e.new_tallies()
    e.run(tal, 0, 3000, 3000, w.seed, frozen_nabs=base, flags=mcrt.FLAG_TALLY_J | mcrt.FLAG_FROZEN_T)
    g = host(tal)
    o = oracle.Session(w, frozen_nabs=base, observers=obs, flags=oracle.FLAG_TALLY_J | oracle.FLAG_PEEL).transport()
    gp = g["peel"].reshape(o["peel"].shape).astype(np.float64)
    op = o["peel"].astype(np.float64)
    c = obs["npix"] // 2
    assert g["counters"][mcrt.CNT["peel_dropped"]] == 0
    assert abs(int(g["counters"][mcrt.CNT["peel"]]) - int(o["counters"][oracle.CNT["peel"]])) <= 0.02 * o["counters"][oracle.CNT["peel"]]
    for ob in range(op.shape[0]):
        for l in range(op.shape[1]):
            assert abs(gp[ob, l].sum() - op[ob, l].sum()) <= 0.03 * op[ob, l].sum() + oracle.PEEL_ONE
    # the star's pixel: launches are identical on both sides
    assert np.allclose(gp[:, :, c, c], op[:, :, c, c], rtol=0.03)
    e.set_observers(**obs, peel=True, peel_capacity=50)
    small = e.new_tallies()
    e.run(small, 0, 3000, 3000, w.seed, frozen_nabs=base, flags=mcrt.FLAG_TALLY_J | mcrt.FLAG_FROZEN_T)
    s = host(small)
    n_ev = int(s["counters"][mcrt.CNT["peel"]])
    assert n_ev == int(g["counters"][mcrt.CNT["peel"]])
    assert int(s["counters"][mcrt.CNT["peel_dropped"]]) == n_ev - 50
    assert 0 < s["peel"].sum() < g["peel"].sum()


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_peel_sed_equals_oracle(precision):
    # each observer's next-event SED over every bin (emissions and
    # scatterings in any bin are queued and marched): FP64 with a frozen
    # field and equal seeds gives the oracle's weights to the rounding unit
    # per bin; FP32 agrees to the packets whose histories part (a few %)
    w = synth.small_disk(n_packets=3000, nl=32, n_sizes=2, nb=8)
    w.precision = precision
    base = oracle.Session(w).transport()["nabs"]
    e = engine(w)
    obs = disk_observers(w)
    e.set_observers(**obs, peel=True, peel_sed=True, peel_capacity=1 << 16)
    tal = e.new_tallies()
    assert tal["peel_sed"] is not None and tal["peel_sed"].numel() == 3 * w.species.n_lambda
    e.run(tal, 0, 3000, 3000, w.seed, frozen_nabs=base, flags=mcrt.FLAG_TALLY_J | mcrt.FLAG_FROZEN_T)
    g = host(tal)
    o = oracle.Session(w, frozen_nabs=base, observers=obs,
                       flags=oracle.FLAG_TALLY_J | oracle.FLAG_PEEL | oracle.FLAG_PEEL_SED).transport()
    gs = g["peel_sed"].reshape(3, -1).astype(np.int64)
    os_ = o["peel_sed"].astype(np.int64)
    n_ev = int(o["counters"][oracle.CNT["peel"]])
    assert n_ev > 3000 and int(g["counters"][mcrt.CNT["peel_dropped"]]) == 0
    assert os_.sum() > 1000 * oracle.PEEL_ONE and np.count_nonzero(os_[0]) > 20
    if precision == "f64":
        assert np.array_equal(g["counters"], o["counters"])
        assert np.abs(gs - os_).max() <= 2
        assert np.abs(g["peel"].astype(np.int64) - o["peel"].reshape(-1).astype(np.int64)).max() <= 2
    else:
        assert abs(int(g["counters"][mcrt.CNT["peel"]]) - n_ev) <= 0.02 * n_ev
        for ob in range(3):
            assert abs(gs[ob].sum() - os_[ob].sum()) <= 0.03 * os_[ob].sum()
    # the images at the imaged bins are the SED's weights where the events project inside
    img = g["peel"].reshape(3, 3, -1).astype(np.int64).sum(2)
    for l, jb in enumerate(obs["lambda_bins"]):
        assert np.all(img[:, l] <= gs[:, jb])


def test_images_count_every_in_cone_escape():
    # FP32 transport, traced: each image holds exactly the escapes whose
    # direction lies in the observer's cone (the field of view encloses every
    # back-projected point), and nothing of other bins
    w = synth.small_disk(n_packets=3000, nl=32, n_sizes=2, nb=8)
    e = engine(w)
    obs = disk_observers(w, npix=16)
    obs["half_width"] = 4.0 * w.grid.nb * w.grid.base_size
    e.set_observers(**obs)
    tal = e.new_tallies()
    tr = e.run(tal, 0, 3000, 3000, w.seed, trace_cap=400)
    img = host(tal)["image"].reshape(3, 3, 16, 16)
    last = [t[-1] for t in tr]
    assert all(r["type"] == 4 for r in last)
    d = np.array([r["d"] for r in last])
    jj = np.array([r["j"] for r in last])
    for o, dv in enumerate(obs["dirs"]):
        n = np.asarray(dv, float) / np.linalg.norm(dv)
        for l, jb in enumerate(obs["lambda_bins"]):
            assert img[o, l].sum() == np.sum((d @ n >= obs["cos_cone"]) & (jj == jb)), (o, l)
    assert img.sum() > 100
    e.set_observers()                       # off again: runs need no image tally
    tal2 = e.new_tallies()
    assert tal2["image"] is None
    e.run(tal2, 0, 100, 3000, w.seed)


def test_shards_add_up_bit_exact():
    w = synth.small_disk(n_packets=20000, nl=32, n_sizes=2, nb=8)
    base = np.zeros((w.grid.n_cells, w.species.n_species), np.uint64) + 3
    e = engine(w)
    flags = mcrt.FLAG_TALLY_J | mcrt.FLAG_FROZEN_T
    full = e.new_tallies()
    e.run(full, 0, 20000, 20000, 5, frozen_nabs=base, flags=flags)
    part = e.new_tallies()
    e.run(part, 0, 7000, 20000, 5, frozen_nabs=base, flags=flags)
    e.run(part, 7000, 13000, 20000, 5, frozen_nabs=base, flags=flags, grid_blocks=3)
    a, b = host(full), host(part)
    for k in ("nabs", "sed", "jq", "counters"):
        assert np.array_equal(a[k], b[k]), k


def test_conservation_full_sphere():
    w = synth.c1_sphere()            # 1e5 packets, FP64
    e = engine(w)
    tal = e.new_tallies(tally_j=False)
    e.run(tal, 0, w.n_packets, w.n_packets, w.seed, flags=0)
    conservation(host(tal), w.n_packets)


def shells(nabs, w, n_shell=12):
    lo, side = w.grid.leaf_boxes_cm()
    r = np.linalg.norm(lo + 0.5 * side[:, None] - w.source.pos, axis=1)
    idx = np.minimum((r / (r.max() + 1e-30) * n_shell).astype(int), n_shell - 1)
    S = w.species.n_species
    nabs = nabs.reshape(-1, S).astype(np.float64)
    out = np.stack([np.bincount(idx, weights=nabs[:, s], minlength=n_shell) for s in range(S)], 1)
    return out.reshape(-1)


def summaries(d, w, per_cell=True):
    """Outputs compared statistically: SED bins, absorptions per (cell,
    species) (or, without per_cell, in radial shells per species), and the
    path-length tally per (bin, cell)."""
    out = dict(sed=d["sed"].astype(np.float64))
    if per_cell:
        out["nabs"] = d["nabs"].astype(np.float64).reshape(-1)
    else:
        out["shells"] = shells(d["nabs"], w)
    if d.get("jq") is not None:
        out["jq"] = d["jq"].astype(np.float64).reshape(-1)
    return out


def batch_runs(run, B):
    """run(b) -> cumulative tallies after batch b; returns per-batch summaries [B, n]."""
    prev, rows = None, []
    for b in range(B):
        cur = {k: v.copy() for k, v in run(b).items() if v is not None}
        d = cur if prev is None else {k: cur[k] - prev[k] for k in cur}
        rows.append(d)
        prev = cur
    return rows


def statistical_check(w, B=32, seed_gpu=None, seed_orc=None, frozen=None, extra_flags=0, summarize=None):
    """B packet-id batches run one after the other on each side (one launch
    per batch on the GPU), seeds differing; returns statparity's verdict per
    output kind of summarize(tallies, w) (default: summaries)."""
    summarize = summarize or summaries
    nb_ = w.n_packets // B
    e = engine(w)
    tal = e.new_tallies(tally_j=w.tally_j)
    sg = seed_gpu if seed_gpu is not None else w.seed
    so = seed_orc if seed_orc is not None else 1000 + w.seed
    flags = (mcrt.FLAG_TALLY_J if w.tally_j else 0) | (mcrt.FLAG_FROZEN_T if frozen is not None else 0)
    flags |= extra_flags

    def gpu_run(b):
        e.run(tal, b * nb_, nb_, w.n_packets, sg, frozen_nabs=frozen, flags=flags)
        return host(tal)

    s = oracle.Session(w, seed=so, n_threads=8, frozen_nabs=frozen,
                       flags=(oracle.FLAG_TALLY_J if w.tally_j else 0) | extra_flags)
    acc = s.new_accumulator()

    def orc_run(b):
        return s.accumulate(acc, b * nb_, nb_)

    G = [summarize(d, w) for d in batch_runs(gpu_run, B)]
    O = [summarize(d, w) for d in batch_runs(orc_run, B)]
    res = {}
    for k in G[0]:
        ga = np.stack([g[k] for g in G])
        oa = np.stack([o[k] for o in O])
        res[k] = statparity.compare(ga, oa)
    conservation(host(tal), w.n_packets)
    return res


@pytest.mark.parametrize("name", ["c1", "c1_exact_bw", "disk", "disk_frozen", "disk_frozen_f64"])
def test_statistical_parity(name):
    """c1: the dust sphere with the full method (running absorption counts),
    path-length tally on; c1_exact_bw: the same with the Bjorkman-Wood law;
    disk: the gap + spiral disk (nested grid, two grain materials, 8 azimuth
    bins) with running counts; disk_frozen(_f64): the disk in FP32 (FP64)
    with the temperature bracket taken from a frozen absorption field.
    Compared outputs: every (cell, species) absorption count, every SED bin
    and every (bin, cell) path sum whose mean over the two runs is at least
    100 (counts; path sums in their fixed-point unit), each against its
    paired batch-means sigma; the criteria of tests/statparity.py (at most
    0.5 % beyond 3 sigma, none beyond 5, chi^2/dof in [0.9, 1.1] for
    n >= 2500 outputs, else its central 99.98 % interval)."""
    frozen = None
    extra = mcrt.FLAG_EXACT_BW if name.endswith("exact_bw") else 0
    if name.startswith("c1"):
        w = synth.c1_sphere(n_packets=1_600_000)
        w.tally_j = True
    else:
        w = synth.small_disk(n_packets=800_000, nl=40, n_sizes=2, nb=16, gap_spiral=True)
        if name.endswith("f64"):
            w.precision = "f64"
        if "frozen" in name:
            frozen = oracle.Session(w, n_threads=8).transport(n=200_000)["nabs"]
    res = statistical_check(w, frozen=frozen, extra_flags=extra)
    for k, (ok, v) in res.items():
        assert ok, (name, k, v)
        assert v["n"] >= (300 if k != "jq" else 10000), (name, k, v)


def test_temperatures_and_intensity_equal_oracle():
    w = synth.small_disk(n_packets=20000, nl=40, n_sizes=2, nb=16)
    s = oracle.Session(w, n_threads=8)
    r = s.transport()
    T_o = s.temperatures(r["nabs"])
    J_o = s.mean_intensity(r["jq"])
    e = engine(w)
    nabs = torch.as_tensor(r["nabs"].reshape(-1).view(np.int64)).cuda()
    jq = torch.as_tensor(r["jq"].reshape(-1).view(np.int64)).cuda()
    T_g = e.temperatures(nabs, w.n_packets).cpu().numpy()
    J_g = e.mean_intensity(jq, w.n_packets).cpu().numpy()
    assert np.allclose(T_g, T_o, rtol=1e-11, atol=0)
    assert (T_o > w.T_lo).sum() > 100
    assert np.allclose(J_g, J_o, rtol=2e-7, atol=1e-30 * J_o.max())


def test_invalid_inputs_are_rejected():
    w = synth.small_disk(n_packets=10, nl=16, n_sizes=1, nb=8)
    w.grid.rho = w.grid.rho.copy()
    w.grid.rho[5] = np.nan
    e = mcrt.Engine.from_workload(w)
    with pytest.raises(mcrt.MCRTError) as ei:
        e.build_tables(w.source.pos, w.source.lum, w.source.teff)
    assert ei.value.code == -5
    w = synth.small_disk(n_packets=10, nl=16, n_sizes=1, nb=8)
    bm = w.grid.base_map.copy()
    bm[0] = w.grid.n_cells + 5
    w.grid.base_map = bm
    e = mcrt.Engine.from_workload(w)
    with pytest.raises(mcrt.MCRTError) as ei:
        e.build_tables(w.source.pos, w.source.lum, w.source.teff)
    assert ei.value.code == -1


def test_thin_field_matches_oracle():
    w = synth.small_disk(n_packets=10, nl=24, n_sizes=1, nb=8)
    e = engine(w)
    Jg = e.thin_field().cpu().numpy()
    Jo = oracle.Session(w).thin_field()
    assert np.allclose(Jg, Jo, rtol=2e-6, atol=0)


def test_pah_reemission_in_transport_equals_oracle():
    """PAH species absorb and re-emit from per-cell rows: FP64 with a frozen
    temperature field and fixed rows reproduces the oracle's tallies exactly."""
    w = synth.small_disk(n_packets=4000, nl=32, n_sizes=1, nb=8, with_pah=True)
    w.precision = "f64"
    n_pah = int((w.species.kind == 1).sum())
    assert n_pah == 2
    rng = np.random.default_rng(3)
    pdf = rng.random((n_pah, w.grid.n_cells, w.species.n_lambda))
    rows = np.cumsum(pdf, axis=2)
    rows /= rows[:, :, -1:]
    rows[:, :, -1] = 1.0
    frozen = np.full((w.grid.n_cells, w.species.n_species), 2, np.uint64)
    e = engine(w)
    tal = e.new_tallies()
    e.run(tal, 0, 4000, 4000, 9, frozen_nabs=frozen, pah_rows=rows, flags=mcrt.FLAG_TALLY_J | mcrt.FLAG_FROZEN_T)
    g = host(tal)
    o = oracle.Session(w, seed=9, frozen_nabs=frozen, pah_rows=rows).transport()
    assert int(g["counters"][9]) > 100            # PAH absorptions happened
    assert np.array_equal(g["counters"], o["counters"])
    assert np.array_equal(g["nabs"], o["nabs"].reshape(-1))
    assert np.array_equal(g["sed"], o["sed"].reshape(-1))
    assert np.array_equal(g["jq"], o["jq"].reshape(-1))


def test_pah_loop_converges():
    # the PAH iteration from the thin starlight field: the first pass moves
    # the emitted band power a lot, later passes by less and less, and the
    # iteration stops once the change is below the 1 % tolerance (the noise
    # of a pass of 1e6 packets is a few tenths of a per cent here)
    from paper_1201_3588_amd.pipeline import PahLoop
    w = synth.small_disk(n_packets=1_000_000, nl=200, n_sizes=1, nb=16, with_pah=True)
    res = PahLoop(w).run(n_iter=6, tol=0.01)
    h = res["history"]
    ch = [x["change"] for x in h[1:]]
    assert len(h) >= 3 and all(x["pah_abs"] > 1000 for x in h)
    conservation(host(res["tallies"]), w.n_packets)
    assert ch[0] > 0.05, ch
    assert ch[-1] < 0.01 and ch[-1] < 0.2 * ch[0], ch


def test_exact_bw_correction_vanishes_with_many_absorptions():
    """The paper drops the Bjorkman-Wood correction, arguing it is negligible
    once a cell has absorbed many packets (Sec. 2).  On the dust sphere the
    escaping spectra of the two laws (same seed, running counts) differ by a
    total-variation distance far above the Monte Carlo noise at ~3 absorptions
    per cell and fall to that noise at ~200; the exact law costs no speed."""
    def sed_dist(n, flags, seed):
        w = synth.c1_sphere(n_packets=n)
        e = engine(w)
        tal = e.new_tallies(tally_j=False)
        e.run(tal, 0, n, n, seed, flags=flags)
        s = tal["sed"].reshape(-1, w.species.n_lambda).sum(0).double()
        return s / s.sum()

    tv, noise = {}, {}
    for n in (100_000, 10_000_000):
        a = sed_dist(n, 0, 1)
        b = sed_dist(n, mcrt.FLAG_EXACT_BW, 1)
        c = sed_dist(n, 0, 8)
        tv[n] = 0.5 * float((a - b).abs().sum())
        noise[n] = 0.5 * float((a - c).abs().sum())
    assert tv[100_000] > 4 * noise[100_000], (tv, noise)
    assert tv[10_000_000] < 0.05 * tv[100_000], (tv, noise)
    assert tv[10_000_000] < 3 * noise[10_000_000], (tv, noise)


@pytest.mark.parametrize("precision,capacity,nb,nl", [("f64", 1 << 22, 16, 32), ("f32", 1 << 22, 16, 32),
                                                      ("f32", 4096 * 3, 16, 32), ("f32", 1 << 22, 72, 200)])
def test_deferred_tally_equals_atomic(precision, capacity, nb, nl):
    # the path-length tally through segment records, partition and LDS sums
    # is the tally of per-segment atomics, bit for bit (frozen temperatures
    # make every packet's path independent of the others); a workspace far
    # too small sends the overflow to direct adds, still exact.  The 72^3 grid
    # with 200 bins has 1834 buckets of tally words: two partition levels.
    w = synth.small_disk(n_packets=20000, nl=nl, n_sizes=2, nb=nb)
    w.precision = precision
    base = oracle.Session(w, n_threads=8).transport(n=4000)["nabs"]
    e = engine(w)
    ref = e.new_tallies()
    flags = mcrt.FLAG_TALLY_J | mcrt.FLAG_FROZEN_T
    e.run(ref, 0, 20000, 20000, w.seed, frozen_nabs=base, flags=flags)
    assert e.set_deferred_tally(capacity)
    tal = e.new_tallies()
    e.run(tal, 0, 12000, 20000, w.seed, frozen_nabs=base, flags=flags)
    e.run(tal, 12000, 8000, 20000, w.seed, frozen_nabs=base, flags=flags)
    a, b = host(ref), host(tal)
    n_seg = int(a["counters"][mcrt.CNT["jseg"]])
    assert n_seg > 8 * capacity if capacity < 1 << 20 else n_seg < capacity
    for k in ("nabs", "sed", "jq", "counters"):
        assert np.array_equal(a[k], b[k]), k
    e.set_deferred_tally(0)


def _jrec_overflow(e):
    # records of the last id range that fell past their bucket regions and
    # were added to the tally directly (header word 2 of the workspace)
    return int(e._jrec[0][:64].view(torch.int64)[2].item())


@pytest.mark.parametrize("nb,nl", [(16, 32), (48, 200), (56, 200), (64, 200), (72, 200)])
def test_deferred_tally_chain_of_ranges_equals_atomic(nb, nl):
    # consecutive id ranges of one pass: the first counts its records for
    # its bucket regions, the later ones size them from the totals of the
    # ranges before.  A workspace barely above a range's records shrinks
    # those regions, so records past a region's end are added directly: the
    # tally is still the atomic one bit for bit.  16^3 with 32 bins: one partition
    # level of 4 buckets; 48^3, 56^3 and 64^3 with 200 bins: one level of 545,
    # 865 and 1290 buckets (scatter blocks of 512 threads claiming for two
    # buckets each, of 1024 claiming for one and for two); 72^3: two levels.
    n, step = 40000, 8000
    w = synth.small_disk(n_packets=n, nl=nl, n_sizes=2, nb=nb)
    w.precision = "f32"
    base = oracle.Session(w, n_threads=8).transport(n=4000)["nabs"]
    e = engine(w)
    flags = mcrt.FLAG_TALLY_J | mcrt.FLAG_FROZEN_T
    ref = e.new_tallies()
    e.run(ref, 0, n, n, w.seed, frozen_nabs=base, flags=flags)
    a = host(ref)
    per_range = int(a["counters"][mcrt.CNT["jseg"]]) * step // n
    capacity = (per_range + 4095) // 4096 * 4096
    assert e.set_deferred_tally(capacity)
    tal = e.new_tallies()
    ovf = []
    for first in range(0, n, step):
        e.run(tal, first, step, n, w.seed, frozen_nabs=base, flags=flags)
        ovf.append(_jrec_overflow(e))
    b = host(tal)
    for k in ("nabs", "sed", "jq", "counters"):
        assert np.array_equal(a[k], b[k]), k
    assert ovf[0] == 0 and sum(ovf[1:]) > 0, ovf
    e.set_deferred_tally(0)


def test_deferred_tally_chain_with_arbitrary_workspace_contents():
    # a chain of ranges whose workspace is overwritten with arbitrary bytes
    # between ranges (as when it is freed and allocated again at the same
    # address): the next range sizes its regions from whatever the workspace
    # holds, the regions still fit the record arrays, and the tally is the
    # atomic one bit for bit (two partition levels)
    n, step = 40000, 8000
    w = synth.small_disk(n_packets=n, nl=200, n_sizes=2, nb=72)
    w.precision = "f32"
    base = oracle.Session(w, n_threads=8).transport(n=4000)["nabs"]
    e = engine(w)
    flags = mcrt.FLAG_TALLY_J | mcrt.FLAG_FROZEN_T
    ref = e.new_tallies()
    e.run(ref, 0, n, n, w.seed, frozen_nabs=base, flags=flags)
    assert e.set_deferred_tally(1 << 22)
    tal = e.new_tallies()
    g = torch.Generator(device="cuda")
    g.manual_seed(3)
    ws = e._jrec[0]
    for first in range(0, n, step):
        if first >= 2 * step:
            ws.copy_(torch.randint(0, 256, ws.shape, dtype=torch.uint8, device="cuda", generator=g))
        e.run(tal, first, step, n, w.seed, frozen_nabs=base, flags=flags)
    a, b = host(ref), host(tal)
    for k in ("nabs", "sed", "jq", "counters"):
        assert np.array_equal(a[k], b[k]), k
    e.set_deferred_tally(0)
