"""Pins of the oracle's temperature inversion and mean-intensity estimator."""
import math

import numpy as np

import oracle
import synth

AU = synth.AU


def test_temperature_round_trip():
    w = synth.small_disk(n_packets=10)
    s = oracle.Session(w, n_total=1)
    E, Tk = s.tables["E"], s.tables["Tk"]
    g = w.grid
    lo, side = g.leaf_boxes_cm()
    c = int(np.argmax(g.rho))
    vol = side[c] ** 3
    for sp in range(w.species.n_species):
        for k in (5, 300, 777, 1000):
            # one packet carrying exactly E_s(T_k) rho V
            w.source.lum = E[sp, k] * g.rho[c] * vol
            s2 = oracle.Session(w, n_total=1)
            nabs = np.zeros((g.n_cells, w.species.n_species), np.uint64)
            nabs[c, sp] = 1
            T = s2.temperatures(nabs)
            assert abs(T[c, sp] / Tk[k] - 1) < 1e-12
            assert np.all(T[np.arange(g.n_cells) != c, sp] == w.T_lo)


def test_temperature_clamps():
    w = synth.small_disk(n_packets=10)
    s = oracle.Session(w, n_total=1)
    g = w.grid
    c = int(np.argmax(g.rho))
    nabs = np.zeros((g.n_cells, w.species.n_species), np.uint64)
    nabs[c, :] = 2 ** 62
    T = s.temperatures(nabs)
    assert np.all(T[c] == w.T_hi)


def test_mean_intensity_thin_point_source():
    # J_nu dnu summed over bins: 4 pi sum_j J_j dnu_j = L <r^-2>_cell / (4 pi)
    nb = 4
    Rb = 2.0 * AU
    w = synth.uniform_cube(nb, 1.0, albedo=0.0, nl=50, n_packets=1000000, seed=21)
    w.grid.box_min = np.full(3, -Rb)
    w.grid.base_size = 2 * Rb / nb
    w.source.pos = np.zeros(3)
    w.source.lum = synth.L_SUN
    w.species.kabs = np.full((1, 50), 1e-6 / w.grid.base_size)   # tau = 1e-6 per cell
    w.species.ksca = np.zeros((1, 50))
    s = oracle.Session(w, n_threads=4)
    r = s.transport()
    J = s.mean_intensity(r["jq"])
    nu, dnu = oracle.lambda_bins(w.species.lam_um)
    tot = 4 * np.pi * (J * dnu[None, :]).sum(1)
    lo, side = w.grid.leaf_boxes_cm()
    rng = np.random.default_rng(2)
    for c in range(w.grid.n_cells):
        pts = lo[c] + side[c] * rng.random((400000, 3))
        ref = w.source.lum * (1.0 / (pts ** 2).sum(1)).mean() / (4 * np.pi)
        # inner cells: path-length estimator noise ~1/sqrt(#crossings)
        assert abs(tot[c] / ref - 1) < 0.03
    # spectrum of J in a thin medium follows the source spectrum
    B = np.array([oracle.planck_nu(n, w.source.teff) for n in nu]) * dnu
    inner = np.argsort(-tot)[:8]
    spec = (J[inner] * dnu).sum(0)
    main = B / B.sum() > 0.02
    assert np.allclose(spec[main] / spec.sum(), (B / B.sum())[main], rtol=0.05)


def test_thin_field_is_the_mean_intensity_of_a_thin_medium():
    # far from the star the analytic thin field equals the path-length estimate
    nb = 6
    Rb = 3.0 * AU
    w = synth.uniform_cube(nb, 1.0, albedo=0.0, nl=50, n_packets=1000000, seed=23)
    w.grid.box_min = np.full(3, -Rb)
    w.grid.base_size = 2 * Rb / nb
    w.source.pos = np.zeros(3)
    w.source.lum = synth.L_SUN
    w.species.kabs = np.full((1, 50), 1e-6 / w.grid.base_size)
    w.species.ksca = np.zeros((1, 50))
    s = oracle.Session(w, n_threads=8)
    J = s.mean_intensity(s.transport()["jq"])
    Jt = s.thin_field()
    nu, dnu = oracle.lambda_bins(w.species.lam_um)
    lo, side = w.grid.leaf_boxes_cm()
    r = np.linalg.norm(lo + 0.5 * side[:, None], axis=1)
    far = r > 2.5 * side[0]
    tot, tott = (J * dnu).sum(1), (Jt * dnu).sum(1)
    # <r^-2> over a cell differs from r_c^-2 by O((side/r)^2 / 12): a few percent here
    assert np.all(np.abs(tot[far] / tott[far] - 1) < 0.06)
    assert far.sum() > 50
