"""Pins of the oracle's spectral tables against closed forms."""
import numpy as np

import oracle
import synth

C = 2.99792458e10
H = 6.62607015e-27
K = 1.380649e-16
SIGMA = 2 * np.pi ** 5 * K ** 4 / (15 * H ** 3 * C ** 2)


def gray_cube(nl=2000, lo=0.01, hi=1e5, T_lo=3.0, T_hi=5000.0, Kn=64, teff=5000.0):
    w = synth.uniform_cube(2, 1.0, nl=nl)
    w.species.lam_um = synth.lambda_grid(nl, lo, hi)
    w.species.kabs = np.ones((1, nl))
    w.species.ksca = np.zeros((1, nl))
    w.species.g = np.zeros(nl)
    w.K, w.T_lo, w.T_hi = Kn, T_lo, T_hi
    w.source.teff = teff
    return w


def test_lambda_bins_telescoping_and_positive():
    lam = synth.lambda_grid(100)
    nu, dnu = oracle.lambda_bins(lam)
    assert np.all(dnu > 0)
    assert np.allclose(nu, C / (lam * 1e-4), rtol=1e-15)
    step = np.sqrt(lam[1] / lam[0])
    lo, hi = lam[0] / step * 1e-4, lam[-1] * step * 1e-4
    assert abs(dnu.sum() - (C / lo - C / hi)) < 1e-12 * (C / lo)


def test_planck_integral_is_stefan_boltzmann():
    lam = synth.lambda_grid(3000, 0.01, 1e5)
    nu, dnu = oracle.lambda_bins(lam)
    for T in (30.0, 300.0, 3000.0):
        s = sum(oracle.planck_nu(n, T) * d for n, d in zip(nu, dnu))
        assert abs(s / (SIGMA * T ** 4 / np.pi) - 1) < 2e-4


def test_planck_limits():
    # Rayleigh-Jeans and Wien limits
    T = 1000.0
    nu = 1e9
    assert abs(oracle.planck_nu(nu, T) / (2 * nu ** 2 * K * T / C ** 2) - 1) < 1e-4
    nu = 1e15
    wien = 2 * H * nu ** 3 / C ** 2 * np.exp(-H * nu / (K * T))
    assert abs(oracle.planck_nu(nu, T) / wien - 1) < 1e-12


def test_gray_emission_table_is_4_kappa_sigma_T4():
    w = gray_cube()
    s = oracle.Session(w)
    Tk, E = s.tables["Tk"], s.tables["E"][0]
    assert np.allclose(Tk[[0, -1]], [w.T_lo, w.T_hi], rtol=1e-14)
    assert np.allclose(np.diff(np.log(Tk)), np.log(w.T_hi / w.T_lo) / (w.K - 1), rtol=1e-10)
    sel = (Tk > 20) & (Tk < 4000)
    assert np.allclose(E[sel], 4 * SIGMA * Tk[sel] ** 4, rtol=3e-4)
    assert np.all(np.diff(E) > 0)


def test_difference_rows_tend_to_dB_dT():
    # With T_{k+1} -> T_k the row pdf is kabs dB/dT dnu, normalised.
    w = gray_cube(nl=300, lo=0.1, hi=1000.0, T_lo=300.0, T_hi=300.0 * (1 + 1e-6), Kn=2)
    rng = np.random.default_rng(3)
    w.species.kabs = rng.uniform(0.5, 2.0, size=(1, 300))
    s = oracle.Session(w)
    R = s.tables["R"][0, 0]
    pdf = np.diff(np.concatenate([[0.0], R]))
    nu, dnu = oracle.lambda_bins(w.species.lam_um)
    T = 300.0
    x = H * nu / (K * T)
    B = np.array([oracle.planck_nu(n, T) for n in nu])
    dBdT = B * x * np.exp(x) / np.expm1(x) / T
    ref = w.species.kabs[0] * dBdT * dnu
    ref /= ref.sum()
    assert np.max(np.abs(pdf - ref)) < 1e-5 * ref.max()
    assert R[-1] == 1.0 and np.all(np.diff(R) >= 0)


def test_source_cdf_and_species_cdf():
    w = synth.small_disk()
    s = oracle.Session(w)
    t = s.tables
    nu, dnu = oracle.lambda_bins(w.species.lam_um)
    B = np.array([oracle.planck_nu(n, w.source.teff) for n in nu]) * dnu
    assert np.allclose(np.diff(np.concatenate([[0.0], t["src_cdf"]])), B / B.sum(), atol=1e-14)
    ka = w.species.kabs
    ref = np.cumsum(ka, axis=0) / ka.sum(axis=0)
    assert np.allclose(t["sp_cdf"], ref.T, atol=1e-14)
    assert np.all(t["sp_cdf"][:, -1] == 1.0)
    kext = (w.species.kabs + w.species.ksca).sum(0)
    assert np.allclose(t["kext"], kext, rtol=1e-14)
    assert np.allclose(t["albedo"], w.species.ksca.sum(0) / kext, rtol=1e-14)
