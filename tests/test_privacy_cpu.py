"""The shuffle-amplified DP bound and the output-noise statistics (host arithmetic of
paper Sec. 5), pinned by special cases, limits and the exact Gaussian-mechanism
privacy curve (Balle and Wang 2018) -- not by retyping the formulas."""
import math

import numpy as np
import pytest
from scipy.stats import norm

from paper_2509_01253_amd import privacy as P


def test_no_local_privacy_loss_gives_no_loss():
    # eps0 = 0: (e^0 - 1) = 0 kills the amplified term; delta' = delta + 2 * 3/2 * n * delta0
    eps, d = P.amplified_dp(0.0, 1e-9, 10_000, 1e-6)
    assert eps == 0.0
    assert d == pytest.approx(1e-6 + 3 * 10_000 * 1e-9)


def test_amplification_monotone_and_vanishing():
    n, delta = 100_000, 1e-6
    e = [P.amplified_dp(e0, 0.0, n, delta)[0] for e0 in (0.1, 0.5, 1.0, 2.0)]
    assert all(a < b for a, b in zip(e, e[1:]))          # more local loss, more central loss
    assert all(x < e0 for x, e0 in zip(e, (0.1, 0.5, 1.0, 2.0)))  # shuffling amplifies
    m = [P.amplified_dp(1.0, 0.0, k, delta)[0] for k in (10 ** 4, 10 ** 5, 10 ** 6, 10 ** 8)]
    assert all(a > b for a, b in zip(m, m[1:]))
    # large n: eps ~ tanh(eps0/2) * 8 sqrt(e^eps0 ln(4/delta)) / sqrt(n)  (log1p(x) ~ x,
    # (e^a - 1)/(e^a + 1) = tanh(a/2), the 1/n term negligible)
    big = 10 ** 12
    eps = P.amplified_dp(1.0, 0.0, big, delta)[0]
    lead = math.tanh(0.5) * 8 * math.sqrt(math.e * math.log(4 / delta)) / math.sqrt(big)
    assert eps == pytest.approx(lead, rel=1e-4)


def test_theorem_range_enforced():
    n, delta = 1000, 1e-6
    lim = math.log(n / (16 * math.log(2 / delta)))
    P.amplified_dp(lim * 0.999, 0.0, n, delta)
    with pytest.raises(ValueError):
        P.amplified_dp(lim * 1.001, 0.0, n, delta)
    with pytest.raises(ValueError):
        P.amplified_dp(0.1, 0.0, 100, delta)  # too few outputs for any eps0 at this delta


@pytest.mark.parametrize("sigma,s,delta0", [(4.0, 0.5, 1e-5), (1e-6, 1e-7, 1e-9), (2.0, 0.3, 1e-3)])
def test_gaussian_eps0_is_valid_for_the_exact_privacy_curve(sigma, s, delta0):
    """The classical calibration is conservative: at its eps0 (below 1) the exact
    delta of the Gaussian mechanism, Phi(s/2sigma - eps sigma/s) - e^eps Phi(-s/2sigma
    - eps sigma/s), is at most delta0."""
    eps0 = P.gaussian_eps0(sigma, s, delta0)
    assert 0 < eps0 < 1
    a, b = s / (2 * sigma), eps0 * sigma / s
    exact = norm.cdf(a - b) - math.exp(eps0) * norm.cdf(-a - b)
    assert exact <= delta0
    # and not absurdly loose: halving eps0 breaks it for the larger deltas
    if delta0 >= 1e-5:
        b2 = 0.5 * eps0 * sigma / s
        assert norm.cdf(a - b2) - math.exp(0.5 * eps0) * norm.cdf(-a - b2) > delta0


def test_noise_histogram_of_gaussian_samples():
    rng = np.random.default_rng(7)
    e = rng.normal(0.0, 2.5e-7, 200_000)
    h = P.noise_histogram(e, bins=41, bound=1e-6)
    assert sum(h["counts"]) == e.size and len(h["edges"]) == 42
    assert h["std"] == pytest.approx(float(np.std(e)))
    assert abs(h["skewness"]) < 0.02 and abs(h["excess_kurtosis"]) < 0.05
    assert h["inside_bound"] == pytest.approx(float(np.mean(np.abs(e) <= 1e-6)))
    # a uniform error is visibly not Gaussian (excess kurtosis -1.2)
    u = P.noise_histogram(rng.uniform(-1, 1, 200_000))
    assert u["excess_kurtosis"] == pytest.approx(-1.2, abs=0.02)


def test_round_report_fields():
    rng = np.random.default_rng(8)
    rep = P.round_report(rng.normal(0, 1e-6, 10_000), n_shuffled=10 ** 6, sensitivity=1e-7)
    assert rep["eps0"] == pytest.approx(P.gaussian_eps0(rep["noise"]["std"], 1e-7, 1e-9))
    assert rep["eps"] is not None and rep["eps"] < rep["eps0"]
    small = P.round_report(rng.normal(0, 1e-6, 1000), n_shuffled=16, sensitivity=1e-7)
    assert small["eps"] is None and "range" in small["note"]
