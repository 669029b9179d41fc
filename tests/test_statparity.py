"""Pins of the statistical-parity criterion (tests/statparity.py) itself:
seeded synthetic batch tallies with known truth, and two oracle runs of the
full method (running absorption counts) under different seeds."""
import numpy as np

import oracle
import statparity
import synth


def poisson_batches(rng, mean, B=32):
    return rng.poisson(mean / B, size=(B, mean.size)).astype(np.float64)


def test_equal_distributions_pass_and_a_half_sigma_bias_fails():
    rng = np.random.default_rng(5)
    mean = rng.uniform(150, 2000, size=6000)
    passed = 0
    for _ in range(20):
        ok, v = statparity.compare(poisson_batches(rng, mean), poisson_batches(rng, mean))
        passed += ok
        assert v["n"] == 6000
    assert passed >= 19
    # every output shifted by half its standard deviation: chi^2/dof ~ 1.25
    sd = np.sqrt(2 * mean)
    ok, v = statparity.compare(poisson_batches(rng, mean + 0.5 * sd), poisson_batches(rng, mean))
    assert not ok and v["chi2_dof"] > 1.1
    # one output 8 sigma off
    g = poisson_batches(rng, mean)
    g[:, 17] += 8 * sd[17] / 32
    ok, v = statparity.compare(g, poisson_batches(rng, mean))
    assert not ok and v["zmax"] > 5


def test_common_drift_across_batches_cancels():
    # both runs drift the same way over the pass (rising temperatures): the
    # paired differences keep the criterion's scale; a one-run spread would
    # be inflated by the drift and hide a bias
    rng = np.random.default_rng(6)
    B, n = 32, 3000
    mean = rng.uniform(200, 1000, size=n)
    ramp = np.linspace(0.6, 1.4, B)[:, None]
    g = rng.poisson(ramp * mean / B).astype(np.float64)
    o = rng.poisson(ramp * mean / B).astype(np.float64)
    ok, v = statparity.compare(g, o)
    assert ok, v
    assert 0.9 < v["chi2_dof"] < 1.1


def test_two_oracle_seeds_agree_with_running_counts():
    # the gap + spiral disk (8 azimuth bins), running counts: each run's
    # batches drift strongly over the pass (about +10 % absorptions per batch
    # from first to last quarter), the paired criterion still holds
    w = synth.small_disk(n_packets=800_000, nl=40, n_sizes=2, nb=16, gap_spiral=True)
    B = 32
    nb = w.n_packets // B
    runs = []
    for seed in (11, 1011):
        s = oracle.Session(w, seed=seed, n_threads=8)
        acc = s.new_accumulator()
        prev, rows = None, []
        for b in range(B):
            s.accumulate(acc, b * nb, nb)
            cur = {k: acc[k].astype(np.float64) for k in ("nabs", "sed")}
            rows.append(cur if prev is None else {k: cur[k] - prev[k] for k in cur})
            prev = cur
        runs.append({k: np.stack([r[k] for r in rows]) for k in ("nabs", "sed")})
    for k in ("nabs", "sed"):
        ok, v = statparity.compare(runs[0][k], runs[1][k])
        assert ok and v["n"] > 300, (k, v)
