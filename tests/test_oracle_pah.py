"""Pins of the oracle's PAH steady-state solver (transient heating, P(T))."""
import numpy as np
import pytest
from scipy.optimize import brentq

import oracle
import synth

LAM = synth.lambda_grid(200)
M = 500


def grid_for(pm, M=M, Ttop=5000.0):
    T = 2.7 * (Ttop / 2.7) ** (np.arange(M) / (M - 1))
    return T, pm.enthalpy(T)


def solve(pm, J, M=M, **kw):
    T, U = grid_for(pm, M)
    return oracle.pah_solve(T, U, LAM, pm.cabs, pm.cband, pm.ccont, J, want_P=True, **kw)


@pytest.mark.parametrize("nc", [30, 200])
def test_recurrence_equals_dense_solve(nc):
    pm = synth.pah_model(nc, LAM)
    T, U = grid_for(pm)
    J = synth.blackbody_field(LAM, [10.0, 1e5], [20000.0, 4000.0])
    _, P, _ = solve(pm, J)
    for c in range(2):
        A, Ad = oracle.pah_rates(T, U, LAM, pm.cabs, J[c])
        W = np.tril(A, -1).copy()            # W[f, i]: rate i -> f
        W[np.arange(M - 1), np.arange(1, M)] = Ad[1:]
        Q = W - np.diag(W.sum(0))
        Q[0, :] = 1.0
        b = np.zeros(M)
        b[0] = 1.0
        Pd = np.linalg.solve(Q, b)
        # a dense LU resolves entries only down to ~1e-14 of the largest
        m = P[c] > 1e-9 * P[c].max()
        assert m.sum() > 100
        assert np.max(np.abs(Pd[m] / P[c][m] - 1)) < 1e-10


def test_three_state_by_hand():
    pm = synth.pah_model(30, LAM)
    T = np.array([20.0, 600.0, 1500.0])
    U = pm.enthalpy(T)
    J = synth.blackbody_field(LAM, [1e4], [15000.0])
    A, Ad = oracle.pah_rates(T, U, LAM, pm.cabs, J[0])
    out, P, _ = oracle.pah_solve(T, U, LAM, pm.cabs, pm.cband, pm.ccont, J, want_P=True)
    # flux balance across each boundary:  P1 Ad1 = P0 (A10 + A20);  P2 Ad2 = P0 A20 + P1 A21
    p0 = 1.0
    p1 = p0 * (A[1, 0] + A[2, 0]) / Ad[1]
    p2 = (p0 * A[2, 0] + p1 * A[2, 1]) / Ad[2]
    ref = np.array([p0, p1, p2]) / (p0 + p1 + p2)
    assert np.allclose(P[0], ref, rtol=1e-13)


@pytest.mark.parametrize("nc", [30, 200])
def test_discrete_energy_identity(nc):
    # absorbed: sum_{i<f} P_i A_fi (U_f - U_i) ; emitted: all outputs.  Each
    # absorption raises the mean enthalpy by exactly h nu, so while no jump
    # passes the top bin the absorbed power is 4 pi sum C J dnu itself.
    pm = synth.pah_model(nc, LAM)
    T, U = grid_for(pm)
    J = synth.blackbody_field(LAM, [3.0, 3e3, 1e6], [30000.0, 8000.0, 20000.0])
    out, P, pabs = solve(pm, J)
    for c in range(3):
        A, Ad = oracle.pah_rates(T, U, LAM, pm.cabs, J[c])
        dU = U[:, None] - U[None, :]
        absorbed = (np.tril(A, -1) * dU * P[c][None, :]).sum()
        assert abs(out[c].sum() / absorbed - 1) < 1e-11
        assert abs(absorbed / pabs[c] - 1) < 1e-11


H = 6.62607015e-27


def _photon_rates(pm, J):
    nu, dnu = oracle.lambda_bins(LAM)
    return 4 * np.pi * pm.cabs * J * dnu / (H * nu), H * nu, dnu


def test_rates_conserve_energy_and_photons_per_state():
    pm = synth.pah_model(30, LAM)
    T, U = grid_for(pm)
    J = synth.blackbody_field(LAM, [1e2], [15000.0])[0]
    A, _ = oracle.pah_rates(T, U, LAM, pm.cabs, J)
    N, E, dnu = _photon_rates(pm, J)
    pabs = 4 * np.pi * (pm.cabs * J * dnu).sum()
    gain = ((U[:, None] - U[None, :]) * np.tril(A, -1)).sum(0)      # per initial state
    below_top = U + E.max() < U[-1]
    assert below_top.sum() > 300
    assert np.allclose(gain[below_top], pabs, rtol=1e-12)
    # states whose smallest photon already clears the next bin make a transition
    # for every photon absorbed
    clear = np.zeros(M, bool)
    clear[:-1] = U[:-1] + E.min() >= U[1:]
    assert clear.sum() > 20
    assert np.allclose(np.tril(A, -1).sum(0)[clear], N.sum(), rtol=1e-12)
    # the top state has nowhere to go; jumps past the top land in it
    assert np.all(A[:, -1] == 0.0)
    i = M - 2
    assert np.isclose(A[-1, i], N.sum(), rtol=1e-12)


def test_line_field_splits_between_two_bins():
    # one wavelength bin lit: from state i the photons land on the two bin
    # centres around U_i + E with weights making the mean gain exactly E
    pm = synth.pah_model(30, LAM)
    T, U = grid_for(pm)
    j = int(np.argmin(np.abs(LAM - 0.2)))
    J = np.zeros(LAM.size)
    J[j] = 1e-18
    A, _ = oracle.pah_rates(T, U, LAM, pm.cabs, J)
    N, E, _ = _photon_rates(pm, J)
    for i in (0, 40, 200):
        x = U[i] + E[j]
        k = np.searchsorted(U, x, side="right") - 1
        assert np.isclose(A[k, i], N[j] * (U[k + 1] - x) / (U[k + 1] - U[k]), rtol=1e-12)
        assert np.isclose(A[k + 1, i], N[j] * (x - U[k]) / (U[k + 1] - U[k]), rtol=1e-12)
        assert np.count_nonzero(A[:, i]) == 2


def test_sparse_noisy_fields_balance_exactly():
    # Monte Carlo fields: a few lit bins with Poisson counts
    pm = synth.pah_model(30, LAM)
    J0 = synth.blackbody_field(LAM, [1e3] * 6, [10000.0] * 6)
    rng = np.random.default_rng(5)
    k = rng.poisson(J0 / J0.sum(1, keepdims=True) * 60.0)
    J = k / 60.0 * J0.sum(1, keepdims=True)
    assert np.all((k > 0).sum(1) < 50)
    out, _, pabs = solve(pm, J)
    assert np.allclose(out.sum(1), pabs, rtol=1e-11)


@pytest.mark.parametrize("nc", [30, 200])
def test_linear_regime(nc):
    # weak fields: single-photon heating, band and mid-IR emission scale with G0
    # (the far-IR of barely excited molecules also feels ground-state depletion)
    pm = synth.pah_model(nc, LAM)
    J = synth.blackbody_field(LAM, [1e-3, 1e-2], [10000.0, 10000.0])
    out, P, _ = solve(pm, J)
    assert P[1][0] > 0.99
    mid_ir = np.concatenate([np.ones(17, bool), LAM < 30.0])
    m = (out[0] > 1e-6 * out[0].sum()) & mid_ir
    assert m.sum() > 40
    assert np.max(np.abs(out[1][m] / out[0][m] / 10.0 - 1)) < 1e-5


def test_strong_field_large_molecule_reaches_equilibrium():
    pm = synth.pah_model(20000, LAM)
    J = synth.blackbody_field(LAM, [1e6], [10000.0])
    out, P, pabs = solve(pm, J)
    T, _ = grid_for(pm)
    nu, dnu = oracle.lambda_bins(LAM)
    pem = lambda t: 4 * np.pi * sum(pm.cabs[j] * oracle.planck_nu(nu[j], t) * dnu[j] for j in range(LAM.size))
    Teq = brentq(lambda t: pem(t) - pabs[0], 3.0, 4999.0)
    assert abs(T[np.argmax(P[0])] / Teq - 1) < 0.02
    assert abs((P[0] * T).sum() / Teq - 1) < 0.02


def test_small_molecule_fluctuates_and_top_bin_empty():
    # transient heating: a 30 C PAH in a moderate field spends most time cold
    # but reaches far above the equilibrium temperature
    pm = synth.pah_model(30, LAM)
    J = synth.blackbody_field(LAM, [1e2, 1e6], [20000.0, 40000.0])
    out, P, pabs = solve(pm, J)
    T, _ = grid_for(pm)
    assert T[np.argmax(P[0])] < 30.0
    assert P[0][T > 500].sum() > 1e-6
    assert P[0][-1] < 1e-10 and P[1][-1] < 1e-10


def test_reemission_rows():
    # the row's increments add up the continuum bin powers and the band powers
    pm = synth.pah_model(30, LAM)
    J = synth.blackbody_field(LAM, [1e3, 1e5], [20000.0, 6000.0])
    out, _, _ = solve(pm, J)
    rows = oracle.pah_rows(LAM, pm.cband, out)
    assert np.all(np.diff(rows, axis=1) >= 0) and np.all(rows[:, -1] == 1.0)
    tot = out.sum(1)
    pdf = np.diff(np.concatenate([np.zeros((2, 1)), rows], axis=1), axis=1)
    nu, dnu = oracle.lambda_bins(LAM)
    # a bin far from every band carries only its continuum power
    far = np.argmin(np.abs(LAM - 1.0))
    assert np.allclose(pdf[:, far] * tot, out[:, 17 + far], rtol=1e-6)
    # bins around 11.3 um carry the 11.3 um band: integrated excess = band power share
    b = 10
    w = pm.cband[b] * dnu / (pm.cband[b] * dnu).sum()
    near = w > 1e-3
    excess = (pdf[:, near] * tot[:, None] - out[:, 17:][:, near]).sum(1)
    others = sum(out[:, k] * (pm.cband[k] * dnu / (pm.cband[k] * dnu).sum())[near].sum()
                 for k in range(17) if k != b)
    assert np.allclose(excess, out[:, b] * w[near].sum() + others, rtol=1e-9)


def test_hard_photons_broaden_the_temperature_distribution():
    # the paper's Fig. 3: a 100 C atom PAH in monochromatic radiation of fixed
    # flux 1e4 erg s^-1 cm^-2 at 3.8 eV .. 1 keV.  Absorbed power is C F
    # (one lit bin); the molecule emits it; at fixed flux harder photons come
    # more rarely and each lifts the molecule further, so P(T) moves to low
    # temperatures (median falls) while its hot tail stays (the spread from
    # the median to the 99.99 % point widens)
    case = synth.hard_photon_case()
    pm, T, U = case["pm"], case["T"], case["U"]
    out, P, pabs = oracle.pah_solve(T, U, case["lam"], pm.cabs, pm.cband, pm.ccont, case["J"],
                                    want_P=True, n_threads=4)
    C = pm.cabs[case["bins"]]
    assert np.allclose(pabs, C * case["flux"], rtol=1e-12)
    assert np.allclose(out.sum(1), pabs, rtol=1e-12)
    med, spread = [], []
    for p in P:
        c = np.cumsum(p)
        q = lambda v: T[np.searchsorted(c, v)]
        med.append(q(0.5))
        spread.append(q(0.9999) / q(0.5))
    assert all(a > b for a, b in zip(med[1:], med[2:]))           # 13.6 eV onwards
    assert all(a < b for a, b in zip(spread[:-1], spread[1:]))
    assert spread[-1] > 5 * spread[0]


def test_band_power_and_cell_mass_definitions():
    # leaf masses add up to the grid's mass by brute force over a fine
    # sampling (a density constant per leaf), and a single-cell, single-band
    # case reduces to mass times that band's power
    import oracle as O
    w = synth.small_disk(n_packets=10, nl=16, n_sizes=1, nb=4)
    m = O.cell_mass(w.grid)
    lo, side = w.grid.leaf_boxes_cm()
    assert np.allclose(m, w.grid.rho * side ** 3, rtol=1e-15)
    vol = (side ** 3).sum()
    assert abs(vol / (w.grid.nb * w.grid.base_size) ** 3 - 1) < 1e-12
    out = np.zeros((3, 20))
    out[1, 4] = 2.5
    assert np.allclose(O.band_power(out, [1.0, 3.0, 5.0], 17), np.eye(17)[4] * 7.5)
