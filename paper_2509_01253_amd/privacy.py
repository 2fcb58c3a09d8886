"""Output-noise statistics and the shuffle-amplified differential-privacy bound of a
server round (paper Sec. 5, Theorem "DP amplification" and its remarks; appendix
"FHE Noise").

The paper's argument: the noise the scheme leaves on every linear-layer output is
(empirically) Gaussian, so each output, seen alone, is an (eps0, delta0)-locally
differentially private release; the server shuffles the n outputs of a layer with a
fresh secret permutation every round, and shuffling amplifies local DP to central DP
(Feldman, McMillan, Talwar 2022, Theorem 3.8).  This module holds that arithmetic
only (host side, no scheme operations): a histogram of decrypted-output errors, the
Gaussian-mechanism eps0 of a measured noise level, and the amplified (eps, delta).

Readings where the paper leaves the quantities open:
  * local randomizer = one output value plus the scheme's output noise, modelled as
    N(0, sigma^2) with sigma measured from decryptions;
  * neighbouring inputs differ in that output by at most `sensitivity` (a caller's
    choice; the paper fixes none);
  * eps0 from the classical Gaussian mechanism (Dwork and Roth 2014, Theorem A.1):
    sigma >= sensitivity * sqrt(2 ln(1.25 / delta0)) / eps0, valid for eps0 < 1;
  * n = the number of outputs one round's permutation shuffles (output neurons of
    an FC layer, output channels of a convolution).
"""
from __future__ import annotations

import math

import numpy as np


def noise_histogram(errors, bins: int = 41, bound: float | None = None) -> dict:
    """Histogram and moments of decrypted-output errors (decrypted minus exact layer
    output).  `bound`, if given, is the error below which decryption is correct (the
    paper's [-1/2p, 1/2p] band; here the caller's tolerance) and the fraction inside
    it is reported."""
    e = np.asarray(errors, np.float64).ravel()
    n = e.size
    mean = float(e.mean()) if n else 0.0
    std = float(e.std()) if n else 0.0
    z = (e - mean) / std if std > 0 else np.zeros_like(e)
    lim = float(np.abs(e).max()) if n else 0.0
    counts, edges = np.histogram(e, bins=bins, range=(-lim, lim) if lim > 0 else (-1, 1))
    out = {"n": int(n), "mean": mean, "std": std, "max_abs": lim,
           "skewness": float(np.mean(z ** 3)) if n else 0.0,
           "excess_kurtosis": float(np.mean(z ** 4) - 3.0) if n else 0.0,
           "counts": counts.tolist(), "edges": edges.tolist()}
    if bound is not None:
        out["bound"] = float(bound)
        out["inside_bound"] = float(np.mean(np.abs(e) <= bound)) if n else 1.0
    return out


def gaussian_eps0(sigma: float, sensitivity: float, delta0: float) -> float:
    """eps0 of the classical Gaussian mechanism with noise sigma, sensitivity and
    delta0: eps0 = sensitivity sqrt(2 ln(1.25/delta0)) / sigma (meaningful for
    eps0 < 1)."""
    if sigma <= 0 or sensitivity < 0 or not 0 < delta0 < 1:
        raise ValueError("need sigma > 0, sensitivity >= 0, 0 < delta0 < 1")
    return sensitivity * math.sqrt(2.0 * math.log(1.25 / delta0)) / sigma


def amplified_dp(eps0: float, delta0: float, n: int, delta: float) -> tuple:
    """(eps, delta') of n shuffled (eps0, delta0)-locally private outputs (paper's
    Theorem on DP amplification by the per-round shuffle):
        eps <= ln(1 + (e^eps0 - 1)/(e^eps0 + 1) (8 sqrt(e^eps0 ln(4/delta)) / sqrt(n)
                                                 + 8 e^eps0 / n)),
        delta' = delta + (e^eps + 1)(e^-eps0 / 2 + 1) n delta0,
    valid when eps0 <= ln(n / (16 ln(2/delta))); ValueError otherwise."""
    if n < 1 or not 0 < delta <= 1 or eps0 < 0 or delta0 < 0:
        raise ValueError("need n >= 1, 0 < delta <= 1, eps0 >= 0, delta0 >= 0")
    limit = n / (16.0 * math.log(2.0 / delta))
    if limit <= 1.0 or eps0 > math.log(limit):
        raise ValueError(f"eps0 = {eps0:.4g} outside the theorem's range (eps0 <= ln(n / (16 ln(2/delta))))")
    e0 = math.exp(eps0)
    core = 8.0 * math.sqrt(e0 * math.log(4.0 / delta)) / math.sqrt(n) + 8.0 * e0 / n
    eps = math.log1p((e0 - 1.0) / (e0 + 1.0) * core)
    delta_out = delta + (math.exp(eps) + 1.0) * (math.exp(-eps0) / 2.0 + 1.0) * n * delta0
    return eps, delta_out


def round_report(errors, n_shuffled: int, sensitivity: float, delta0: float = 1e-9, delta: float = 1e-6,
                 bound: float | None = None) -> dict:
    """Noise histogram of one round's decrypted outputs and the DP guarantee of the
    shuffled round: eps0 from the measured sigma, eps from the amplification theorem
    (None where the theorem does not apply)."""
    h = noise_histogram(errors, bound=bound)
    rep = {"noise": h, "n_shuffled": int(n_shuffled), "sensitivity": float(sensitivity), "delta0": delta0,
           "delta": delta}
    if h["std"] > 0:
        e0 = gaussian_eps0(h["std"], sensitivity, delta0)
        rep["eps0"] = e0
        try:
            rep["eps"], rep["delta_total"] = amplified_dp(e0, delta0, n_shuffled, delta)
        except ValueError as exc:
            rep["eps"], rep["delta_total"], rep["note"] = None, None, str(exc)
    return rep
