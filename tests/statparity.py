"""Statistical parity of two independent Monte Carlo runs ("within 3 sigma").

Each run is split into B consecutive packet-id batches, run in the same order
on both sides.  With running absorption counts the batches are not identically
distributed: cell temperatures, and with them the re-emitted spectra, rise
over the pass, so the spread of one run's batch values overstates its noise
(the escaping spectrum's chi^2/dof between two oracle seeds comes out near
0.5).  Batch b of one run and batch b of the other, however, see the same
stage of the pass, so the paired differences D_b = G_b - O_b have mean zero
under parity whatever the drift, and their spread gives the standard error of
the difference of the totals (batch means on the differences).  For every
output whose mean of the two totals is at least `min_count` (a cut on
the sum, not on either side, so that it does not select on the difference):

    t = sum_b D_b / sqrt(B s_D^2),    s_D^2 the sample variance of the D_b,

which follows Student's t with B - 1 degrees of freedom (at B = 32 a 3-sigma
excess is 1.6 times more frequent than for the normal law, a 5-sigma one 30
times), so t is mapped to the normal deviate z of equal two-sided tail
probability.  The criteria on z:

* at most 0.5 % of the outputs beyond 3 (0.27 % expected), or, for fewer than
  about 2000 outputs, at most the 99.99 % point of Binomial(n, 0.0027);
* none beyond 5;
* chi^2 / dof = mean(z^2) in [0.9, 1.1] when n >= 2500, else within the
  central 99.98 % interval of chi^2_n / n.
"""
from __future__ import annotations

import numpy as np
from scipy import stats

P3 = 2.0 * stats.norm.sf(3.0)


def batch_z(ga, oa, min_count=100.0):
    """ga, oa: [B, n] per-batch values of the two runs, batch b of each from
    the same stage of its pass.  Returns (z of the compared outputs, their
    indices)."""
    ga = np.asarray(ga, np.float64)
    oa = np.asarray(oa, np.float64)
    B = ga.shape[0]
    assert oa.shape == ga.shape and B >= 8
    gs, os_ = ga.sum(0), oa.sum(0)
    v = B * (ga - oa).var(0, ddof=1)
    m = (0.5 * (gs + os_) >= min_count) & (v > 0)
    idx = np.nonzero(m)[0]
    t = (gs[m] - os_[m]) / np.sqrt(v[m])
    z = np.sign(t) * stats.norm.isf(stats.t.sf(np.abs(t), B - 1))
    return z, idx


def verdict(z):
    """The criteria above; returns (ok, summary dict)."""
    z = np.asarray(z, np.float64)
    n = int(z.size)
    if n == 0:
        return False, {"n": 0}
    n3 = int(np.sum(np.abs(z) > 3.0))
    lim3 = max(0.005 * n, float(stats.binom.ppf(0.9999, n, P3)))
    zmax = float(np.max(np.abs(z)))
    chi2 = float(np.mean(z * z))
    if n >= 2500:
        lo, hi = 0.9, 1.1
    else:
        lo, hi = stats.chi2.ppf(1e-4, n) / n, stats.chi2.ppf(1 - 1e-4, n) / n
    ok = n3 <= lim3 and zmax < 5.0 and lo <= chi2 <= hi
    return ok, {"n": n, "beyond3": n3, "beyond3_limit": lim3, "zmax": zmax, "chi2_dof": chi2,
                "chi2_window": (float(lo), float(hi))}


def compare(ga, oa, min_count=100.0):
    z, _ = batch_z(ga, oa, min_count)
    return verdict(z)
