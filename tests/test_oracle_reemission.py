"""Pins of the re-emission law: the frequency a packet gets after an absorption.

Paper, Sec. 2: the new frequency is drawn with the cell temperature before the
absorption, and the Bjorkman & Wood (2001) correction for the temperature rise
the absorption causes is dropped.  The default law samples
kabs [B(T_{k+1}) - B(T_k)] of the table bracket holding T_before; with
FLAG_EXACT_BW the oracle samples kabs [B(T_after) - B(T_before)] of the
absorption's own rise.  For a gray absorber whose brackets end on table points
both distributions are closed forms in the Planck function, independent of the
difference-emissivity rows the oracle draws from."""
import numpy as np
from scipy import stats

import oracle
import synth

NL = 40


def _gray_cell(n_packets, eps, seed=31):
    # one 1 cm cube of unit density, gray pure absorber with tau = 2 from the
    # centre to a face: a packet is absorbed about five times before it leaves
    w = synth.uniform_cube(1, 4.0, albedo=0.0, nl=NL, n_packets=n_packets, seed=seed)
    w.source.lum = eps * n_packets       # eps / (rho V) = eps
    w.tally_j = False
    return w


def _reemitted(w, flags, n0):
    s = oracle.Session(w, flags=flags, frozen_nabs=np.array([n0], np.uint64), max_events=60)
    tr = s.transport(trace_cap=64)["trace"]
    return np.array([e["j"] for t in tr for e in t if e["type"] == 3]), s


def _planck_rows(s, T):
    nu, dnu = s.tables["nu"], s.tables["dnu"]
    return np.array([oracle.planck_nu(v, T) for v in nu]) * dnu


def _chi2_pvalue(bins, expected_shape):
    counts = np.bincount(bins, minlength=NL).astype(float)
    exp = expected_shape / expected_shape.sum() * counts.sum()
    keep = exp >= 5.0
    obs = np.append(counts[keep], counts[~keep].sum())
    ex = np.append(exp[keep], exp[~keep].sum())
    if ex[-1] < 5.0:                     # fold a small remainder into the largest bin
        m = int(np.argmax(ex[:-1]))
        obs[m] += obs[-1]
        ex[m] += ex[-1]
        obs, ex = obs[:-1], ex[:-1]
    assert counts[~keep].sum() <= max(10.0, 5 * exp[~keep].sum())
    return stats.chisquare(obs, ex).pvalue


def _tables():
    s = oracle.Session(_gray_cell(10, 1.0))
    return s.tables["E"][0], s.tables["Tk"]


def test_exact_bw_samples_planck_difference_of_the_rise():
    # N_before = 0 and eps / (rho V) = E(T_k2): the rise spans T_0 .. T_k2 and
    # the sampled spectrum is B(T_k2) - B(T_0) plus the part below E(T_0),
    # which the clamp to the first bracket draws from B(T_1) - B(T_0)
    E, Tk = _tables()
    k2 = int(np.searchsorted(Tk, 40.0))
    w = _gray_cell(6000, E[k2])
    bins, s = _reemitted(w, oracle.FLAG_EXACT_BW, 0)
    assert bins.size > 20000
    b0, b1, b2 = (_planck_rows(s, Tk[k]) for k in (0, 1, k2))
    expected = (b2 - b0) + E[0] / (E[1] - E[0]) * (b1 - b0)
    assert _chi2_pvalue(bins, expected) > 1e-4
    # the default law with the same tallies stays in the first bracket
    bins_d, _ = _reemitted(w, 0, 0)
    assert _chi2_pvalue(bins_d, b1 - b0) > 1e-4
    # ... whose photons are an order of magnitude redder
    nu = s.tables["nu"]
    assert nu[bins].mean() > 5.0 * nu[bins_d].mean()


def test_default_law_samples_the_bracket_before_absorption():
    # N_before = 3 with eps chosen so that 3 eps lies inside bracket kb: every
    # re-emission follows B(T_{kb+1}) - B(T_kb), whatever the rise
    E, Tk = _tables()
    kb = int(np.searchsorted(Tk, 25.0))
    eps = (0.3 * E[kb] + 0.7 * E[kb + 1]) / 3.0
    w = _gray_cell(6000, eps)
    bins, s = _reemitted(w, 0, 3)
    expected = _planck_rows(s, Tk[kb + 1]) - _planck_rows(s, Tk[kb])
    assert _chi2_pvalue(bins, expected) > 1e-4


def test_exact_bw_is_hotter_and_laws_meet_as_counts_grow():
    # same random numbers, gray absorber: the paths do not depend on the
    # frequency, so the two laws see identical events and differ only in the
    # drawn bin.  With eps / (rho V) = E(30 K) / N_before the rise is a factor
    # (1 + 1/N_before) in absorbed power: at N_before = 2 the exact law (the
    # rise above T_before) emits visibly bluer photons; as N_before grows the
    # rise shrinks inside one bracket and the two laws draw the same bins
    E, Tk = _tables()
    k = int(np.searchsorted(Tk, 30.0))
    diffs = []
    for n0 in (2, 20, 200):
        w = _gray_cell(1500, E[k] / n0)
        a, s = _reemitted(w, 0, n0)
        b, _ = _reemitted(w, oracle.FLAG_EXACT_BW, n0)
        assert a.size == b.size > 5000
        nu = s.tables["nu"]
        if n0 == 2:
            assert nu[b].mean() > 1.03 * nu[a].mean()
        assert nu[b].mean() >= nu[a].mean()
        diffs.append(np.mean(a != b))
    assert diffs[0] > 0.1
    assert diffs[1] < 0.25 * diffs[0]
    assert diffs[2] < 0.002
