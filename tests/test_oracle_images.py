"""Pins of the oracle's escape images: a packet in an imaged bin that leaves
within an observer's cone is placed where its ray, extended backwards, crosses
the image plane through the centre perpendicular to the line of sight."""
import numpy as np

import oracle
import synth


def _obs(dirs, npix, w, center, cos_cone, bins):
    return dict(dirs=dirs, npix=npix, half_width=w, center=center, cos_cone=cos_cone, lambda_bins=bins)


def test_direct_starlight_lands_in_the_centre_pixel():
    # empty cube, star at the image centre: every in-cone packet of an imaged
    # bin is counted once, in the centre pixel of a 9 x 9 image
    w = synth.uniform_cube(8, 0.0, nl=16, n_packets=4000)
    c = list(w.source.pos)
    dirs = [(0, 0, 1), (1, 1, 1), (-1, 0, 0)]
    cosc = np.cos(np.radians(25.0))
    s = oracle.Session(w, observers=_obs(dirs, 9, 3.0, c, cosc, [3, 5]))
    r = s.transport(trace_cap=32)
    img = r["image"]
    assert img.shape == (3, 2, 9, 9)
    for o, dv in enumerate(dirs):
        n = np.asarray(dv, float) / np.linalg.norm(dv)
        for l, jb in enumerate([3, 5]):
            want = sum(1 for t in r["trace"] if t[-1]["type"] == oracle.EV_ESCAPE and t[-1]["j"] == jb
                       and np.dot(t[-1]["d"], n) >= cosc)
            assert want > 0
            assert img[o, l, 4, 4] == want
            assert img[o, l].sum() == want


def test_pencil_beam_pixel_by_hand():
    # beam along +z from a star offset by (0.3 w, -0.55 w, 0) from the centre,
    # 10 x 10 pixels of half width w = 2 cm:
    #  observer +z: plane axes (x, y); the ray meets the plane at (0.3 w, -0.55 w)
    #    -> pixel (px, py) = (floor(6.5), floor(2.25)) = (6, 2)
    #  observer (0, 0.6, 0.8): axes e1 = (-1, 0, 0), e2 = (0, -0.8, 0.6); the ray
    #    x = X + t z meets X . n = 0 at t = 0.55 w 0.6 / 0.8 = 0.4125 w, i.e. at
    #    (0.3 w, -0.55 w, 0.4125 w): coordinates (-0.3 w, 0.6875 w) -> (3, 8)
    #  observer +x: outside the 40 degree cone -> nothing
    w = synth.uniform_cube(8, 0.0, nl=16, n_packets=500)
    c = np.full(3, 4.0)
    hw = 2.0
    w.source.pos = c + np.array([0.3 * hw, -0.55 * hw, 0.0])
    w.source.beam = np.array([0.0, 0.0, 1.0])
    s = oracle.Session(w, observers=_obs([(0, 0, 1), (0, 0.6, 0.8), (1, 0, 0)], 10, hw, c,
                                         np.cos(np.radians(40.0)), [2, 3, 4, 5]))
    r = s.transport()
    img = r["image"]
    assert r["counters"][oracle.CNT["escaped"]] == 500
    per_bin = r["sed"].sum(axis=(0, 1))[2:6]
    assert per_bin.min() > 10
    for l in range(4):
        assert img[0, l, 2, 6] == per_bin[l] and img[0, l].sum() == per_bin[l]
        assert img[1, l, 8, 3] == per_bin[l] and img[1, l].sum() == per_bin[l]
    assert img[2].sum() == 0


def test_scattered_light_counts_every_in_cone_escape():
    # a scattering cube: with a field of view wide enough for any back-projected
    # point, the image of each observer and bin holds exactly the escapes whose
    # direction lies in its cone
    w = synth.uniform_cube(6, 0.4, albedo=0.9, nl=16, n_packets=3000, g=0.3)
    c = list(w.source.pos)
    dirs = [(0, 0, 1), (0.3, -0.5, 0.2), (0, -1, 0)]
    cosc = np.cos(np.radians(30.0))
    hw = 2 * 6 * np.sqrt(3) / cosc
    s = oracle.Session(w, observers=_obs(dirs, 16, hw, c, cosc, [3, 4]))
    r = s.transport(trace_cap=400)
    assert all(t[-1]["type"] == oracle.EV_ESCAPE for t in r["trace"])
    esc = np.array([t[-1]["d"] for t in r["trace"]])
    jj = np.array([t[-1]["j"] for t in r["trace"]])
    assert r["counters"][oracle.CNT["scatters"]] > 1000
    for o, dv in enumerate(dirs):
        n = np.asarray(dv, float) / np.linalg.norm(dv)
        for l, jb in enumerate([3, 4]):
            assert r["image"][o, l].sum() == np.sum((esc @ n >= cosc) & (jj == jb))
    # scattered light does not all come from one spot
    assert np.count_nonzero(r["image"][0, 0]) >= 4
