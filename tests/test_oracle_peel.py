"""Pins of the oracle's next-event (peel-off) images: the dust-free star,
closed-form attenuation of direct starlight, a brute-force recount from packet
traces with the optical depth from the box geometry, and agreement with the
escape images, which count the packets that actually leave (paper Sec. 2 and
Fig. 2: the model seen from chosen directions at 11.3 and 10 um)."""
import math

import numpy as np
from scipy import integrate

import oracle
import synth

ONE = oracle.PEEL_ONE


def _obs(w, dirs, npix=9, bins=(3, 7), cos_cone=0.5, half=None):
    half = half if half is not None else 0.6 * w.grid.nb * w.grid.base_size
    return dict(dirs=dirs, npix=npix, half_width=half, center=list(w.source.pos),
                cos_cone=cos_cone, lambda_bins=list(bins))


def test_star_alone_every_launch_in_the_centre_pixel():
    w = synth.uniform_cube(8, 0.0, nl=16, n_packets=3000)
    obs = _obs(w, [(0, 0, 1), (0, 0.6, 0.8), (-1, 0, 0)])
    r = oracle.Session(w, observers=obs, flags=oracle.FLAG_PEEL).transport()
    launched = r["sed"].sum(axis=(0, 1))
    c = obs["npix"] // 2
    for o in range(3):
        for l, jb in enumerate(obs["lambda_bins"]):
            img = r["peel"][o, l].astype(np.int64)
            assert img[c, c] == int(launched[jb]) * ONE
            assert img.sum() == img[c, c]
    assert int(r["counters"][oracle.CNT["peel"]]) == int(launched[[3, 7]].sum())


def test_direct_starlight_attenuation_closed_form():
    # pure absorber that ends each packet at its first absorption: only the
    # star's emissions are peeled; star on the vertex at the cube's centre,
    # tau to the edge = alpha * (distance along n to the first face)
    w = synth.uniform_cube(8, 0.3, albedo=0.0, nl=16, n_packets=2000)
    dirs = [(0, 0, 1), (0, 0.6, 0.8), (-1, 0, 0)]
    obs = _obs(w, dirs)
    r = oracle.Session(w, observers=obs, flags=oracle.FLAG_PEEL | oracle.FLAG_KILL_ON_ABSORB).transport(trace_cap=4)
    per_bin = np.bincount([t[0]["j"] for t in r["trace"]], minlength=16)
    c = obs["npix"] // 2
    for o, n in enumerate(dirs):
        n = np.array(n, float) / np.linalg.norm(n)
        dist = min((8.0 - 4.0) / a if a > 0 else (0.0 - 4.0) / a for a in n if a != 0)
        unit = math.exp(-0.3 * dist) * ONE
        for l, jb in enumerate(obs["lambda_bins"]):
            img = r["peel"][o, l].astype(np.int64)
            assert img.sum() == img[c, c]
            assert abs(img[c, c] - per_bin[jb] * unit) <= per_bin[jb] * 0.5 + 1


def _box_tau(x, n, alpha, size):
    t = min(((size - x[a]) / n[a]) if n[a] > 0 else (-x[a] / n[a]) for a in range(3) if n[a] != 0)
    return alpha * t


def _hg(g, mu):
    return (1 - g * g) / (1 + g * g - 2 * g * mu) ** 1.5


def test_brute_force_recount_from_traces():
    # non-gray cube with anisotropic scattering and re-emission: every peeled
    # event (launch, scattering with the incoming direction, re-emission at
    # the new bin) is recounted from the traces with tau from the box geometry
    nl = 16
    w = synth.uniform_cube(6, 0.4, albedo=0.5, nl=nl, n_packets=1500, g=0.6)
    w.species.kabs = w.species.kabs * (1.0 + np.arange(nl) / nl)
    w.source.pos = np.array([2.3, 3.1, 2.7])
    dirs = [(0, 0, 1), (0.3, -0.5, 0.81), (-1, 0.2, 0.1)]
    obs = _obs(w, dirs, npix=15, bins=(2, 9, 13), half=4.5)
    s = oracle.Session(w, observers=obs, flags=oracle.FLAG_PEEL, max_events=400)
    r = s.transport(trace_cap=2000)
    kext = s.tables["kext"]
    size = 6.0
    want = np.zeros_like(r["peel"], dtype=np.int64)
    count = 0
    for tr in r["trace"]:
        assert tr[-1]["type"] == oracle.EV_ESCAPE
        for k, ev in enumerate(tr):
            typ = int(ev["type"])
            if typ not in (oracle.EV_LAUNCH, oracle.EV_SCATTER, oracle.EV_ABSORB) or ev["cell"] < 0:
                continue
            j = int(ev["j"])
            if j not in obs["lambda_bins"]:
                continue
            count += 1
            l = obs["lambda_bins"].index(j)
            for o, n in enumerate(dirs):
                n = np.array(n, float) / np.linalg.norm(n)
                rr = math.hypot(n[0], n[1])
                e1 = np.array([-n[1], n[0], 0.0]) / rr if rr > 1e-12 else np.array([1.0, 0.0, 0.0])
                e2 = np.cross(n, e1)
                X = ev["x"] * w.grid.base_size - w.source.pos
                px = math.floor((X @ e1 + 4.5) / 9.0 * 15)
                py = math.floor((X @ e2 + 4.5) / 9.0 * 15)
                if not (0 <= px < 15 and 0 <= py < 15):
                    continue
                ph = _hg(0.6, float(tr[k - 1]["d"] @ n)) if typ == oracle.EV_SCATTER else 1.0
                want[o, l, py, px] += round(ph * math.exp(-_box_tau(ev["x"], n, kext[j], size)) * ONE)
    assert count > 300
    assert int(r["counters"][oracle.CNT["peel"]]) == count
    got = r["peel"].astype(np.int64)
    assert np.abs(got - want).max() <= 3
    assert want.sum() > 100 * ONE


def _hg_cone(g, beam, n, cos_c):
    """(1 / 4 pi) * integral of the Henyey-Greenstein function of the angle to
    `beam` over the cone of directions within acos(cos_c) of n."""
    n = np.asarray(n, float) / np.linalg.norm(n)
    u = np.cross(n, [0.0, 0.0, 1.0])
    u = u / np.linalg.norm(u)
    v = np.cross(n, u)

    def f(b, a):
        om = math.cos(a) * n + math.sin(a) * (math.cos(b) * u + math.sin(b) * v)
        return _hg(g, float(om @ beam)) * math.sin(a)
    val, _ = integrate.dblquad(f, 0.0, math.acos(cos_c), 0.0, 2.0 * math.pi, epsabs=1e-12, epsrel=1e-10)
    return val / (4.0 * math.pi)


def test_scattered_beam_agrees_with_escape_cones():
    # pencil beam along +x through an optically thin pure scatterer (g = 0.6,
    # tau = 0.05 along the beam): the escapes in a cone about n count the
    # scattered light that leaves within the cone, whose expectation is the
    # peel-off weight towards n times the cone integral of the phase function
    # over its value at n (single scattering of the beam; a few per cent of
    # multiple scattering shares the estimate).  The escape side comes from
    # the deflection sampler, so a wrong normalisation of the phase function
    # in the peel-off weight fails here.
    g = 0.6
    w = synth.uniform_cube(8, 0.00625, albedo=1.0, nl=4, n_packets=2_000_000, g=g)
    w.source.pos = np.array([0.0, 4.3, 4.6])
    w.source.beam = np.array([1.0, 0.0, 0.0])
    cos_c = math.cos(math.radians(20.0))
    ths = (30.0, 60.0, 90.0, 135.0)
    dirs = [(math.cos(math.radians(t)), math.sin(math.radians(t)), 0.0) for t in ths]
    obs = dict(dirs=dirs, npix=3, half_width=20.0, center=[4.0, 4.0, 4.0], cos_cone=cos_c,
               lambda_bins=[0, 1, 2, 3])
    r = oracle.Session(w, observers=obs, flags=oracle.FLAG_PEEL, n_threads=8).transport()
    beam = np.array([1.0, 0.0, 0.0])
    for o, n in enumerate(dirs):
        esc = float(r["image"][o].sum())
        peel = float(r["peel"][o].sum()) / ONE
        ratio = _hg_cone(g, beam, n, cos_c) / _hg(g, float(np.dot(beam, n)))
        assert esc > 400
        assert abs(esc - ratio * peel) < 4.0 * math.sqrt(esc) + 0.02 * esc, (ths[o], esc, ratio * peel)


# --------------------------------------------------------------------------
# next-event SEDs (ORC_FLAG_PEEL_SED): per observer, every bin
def test_peel_sed_star_alone_is_the_launch_spectrum():
    # dust-free: every launch weighs 1 towards every observer, in its own bin
    w = synth.uniform_cube(8, 0.0, nl=16, n_packets=3000)
    obs = _obs(w, [(0, 0, 1), (0.3, -0.5, 0.2)], bins=(3,))
    r = oracle.Session(w, observers=obs, flags=oracle.FLAG_PEEL | oracle.FLAG_PEEL_SED).transport()
    launched = r["sed"].sum(axis=(0, 1)).astype(np.int64)
    assert launched.sum() == 3000 and np.count_nonzero(launched) >= 6
    for o in range(2):
        assert np.array_equal(r["peel_sed"][o].astype(np.int64), launched * ONE)
    assert int(r["counters"][oracle.CNT["peel"]]) == 3000       # every event queued, not only bin 3


def test_peel_sed_direct_starlight_closed_form():
    # pure absorber, packets end at their first absorption: each launch in
    # bin j adds round(2^24 exp(-tau)) towards observer n, tau = alpha times
    # the distance along n from the star (cube centre) to the first face
    w = synth.uniform_cube(8, 0.3, albedo=0.0, nl=16, n_packets=2000)
    dirs = [(0, 0, 1), (0, 0.6, 0.8), (-1, 0, 0)]
    obs = _obs(w, dirs, bins=(5,))
    r = oracle.Session(w, observers=obs, flags=oracle.FLAG_PEEL | oracle.FLAG_PEEL_SED |
                       oracle.FLAG_KILL_ON_ABSORB).transport(trace_cap=4)
    per_bin = np.bincount([t[0]["j"] for t in r["trace"]], minlength=16).astype(np.int64)
    for o, n in enumerate(dirs):
        n = np.array(n, float) / np.linalg.norm(n)
        dist = min((8.0 - 4.0) / a if a > 0 else (0.0 - 4.0) / a for a in n if a != 0)
        unit = int(round(math.exp(-0.3 * dist) * ONE))
        got = r["peel_sed"][o].astype(np.int64)
        assert np.all(np.abs(got - per_bin * unit) <= per_bin // 2 + 1), (o, got, per_bin * unit)


def test_peel_sed_at_imaged_bins_equals_image_totals():
    # scattering, re-emitting disk; a field of view enclosing every projected
    # event: at an imaged bin the SED holds the same weights as the image
    w = synth.small_disk(n_packets=3000, nl=32, n_sizes=2, nb=8)
    half = 4.0 * w.grid.nb * w.grid.base_size
    obs = _obs(w, [(0, 0, 1), (1, 0, 0), (0, 0.5, 0.866)], npix=15, bins=(10, 14, 16), half=half)
    base = oracle.Session(w).transport()["nabs"]
    r = oracle.Session(w, frozen_nabs=base, observers=obs,
                       flags=oracle.FLAG_TALLY_J | oracle.FLAG_PEEL | oracle.FLAG_PEEL_SED).transport()
    img = r["peel"].astype(np.int64)
    sed = r["peel_sed"].astype(np.int64)
    for o in range(3):
        for l, jb in enumerate(obs["lambda_bins"]):
            assert img[o, l].sum() == sed[o, jb] and sed[o, jb] > 5 * ONE
    # every bin with escaping light has a next-event estimate
    esc = r["sed"].sum(axis=(0, 1))
    assert np.all(sed[:, esc > 50] > 0)
    # without the SED flag nothing changes in the images
    r0 = oracle.Session(w, frozen_nabs=base, observers=obs, flags=oracle.FLAG_TALLY_J | oracle.FLAG_PEEL).transport()
    assert np.array_equal(r0["peel"], r["peel"]) and r0["peel_sed"] is None
