"""Posterior quantities of BayesLSH in FP64 (oracle; test infrastructure only).

After comparing n hashes of a pair and seeing m agreements (the event
M(m, n)), the likelihood is Binomial(n, S) (Section 4, eqn likelihood).
BayesLSH needs three numbers from the posterior p(S | M(m, n)):

  prune probability   Pr[S >= t | M(m,n)]             (Section 4, eqn pruneProb)
  MAP estimate        S_hat = argmax_s p(s | M(m,n))    (Section 4, eqn map)
  concentration       Pr[|S - S_hat| < delta | M(m,n)]  (Section 4, eqn concentrateProb)

Jaccard (Section 4.1): prior Beta(alpha, beta), posterior
Beta(m + alpha, n - m + beta); the prune probability is 1 - I_t(a, b) and the
concentration is I_{S_hat+delta}(a, b) - I_{S_hat-delta}(a, b), with I the
regularized incomplete beta function.  The regularized incomplete beta comes
from scipy (the paper also defers to a library routine for it).

Cosine (Section 4.2): the hash family estimates r = 1 - theta/pi on
[0.5, 1]; the prior on r is uniform on [0.5, 1]; r2c(r) = cos(pi (1 - r)) and
c2r(c) = 1 - arccos(c)/pi map between r and the cosine.  Every posterior
probability is a ratio of integrals of r^m (1-r)^(n-m) over sub-intervals of
[0.5, 1].  With a = m + 1, b = n - m + 1 (integers) the standard identity

    int_x^1 r^m (1-r)^(n-m) dr = B(a, b) * Pr[Binomial(n + 1, x) <= m]

turns each integral into a binomial lower tail, which is summed here in log
space so that ratios of very small tails (m << n/2) neither underflow nor
cancel.  B(a, b) cancels in every ratio.

Readings of the paper taken here:
  * Jaccard MAP is the Beta mode (m+alpha-1)/(n+alpha+beta-2), clamped to
    [0, 1]; the text derives the mode but the printed formula has -1 in the
    denominator.
  * Cosine MAP: the posterior of r lives on [0.5, 1], so its argmax is
    max(0.5, m/n); S_hat = r2c of that.
  * The concentration interval is clipped to the support ([0,1] for Jaccard,
    r in [0.5, 1] for cosine).
  * A pair survives a check iff the prune probability is >= epsilon (the
    algorithm prunes on "< epsilon"); a pair is concentrated iff the
    concentration probability is >= 1 - gamma (guarantee 2 of Section 1; the
    printed test in Algorithm 1 is garbled).
"""
from __future__ import annotations

import math
from functools import lru_cache

import numpy as np
from scipy.special import betainc, betaincc, gammaln

JACCARD = 0
COSINE = 1


# --------------------------------------------------------------------------
# Jaccard, Beta(alpha, beta) prior  (Section 4.1)
# --------------------------------------------------------------------------
def jaccard_prune_prob(m: int, n: int, t: float, alpha: float = 1.0, beta: float = 1.0) -> float:
    """Pr[S >= t | M(m,n)] = 1 - I_t(m + alpha, n - m + beta).

    scipy's ``betaincc`` returns 1 - I_x(a, b) without forming the difference.
    """
    return float(betaincc(m + alpha, n - m + beta, t))


def jaccard_map(m: int, n: int, alpha: float = 1.0, beta: float = 1.0) -> float:
    """Mode of Beta(m + alpha, n - m + beta), clamped to [0, 1]."""
    s = (m + alpha - 1.0) / (n + alpha + beta - 2.0)
    return min(1.0, max(0.0, s))


def jaccard_concentration(m: int, n: int, delta: float, alpha: float = 1.0, beta: float = 1.0) -> float:
    """Pr[|S - S_hat| < delta | M(m,n)] = I_hi(a,b) - I_lo(a,b), interval clipped to [0, 1]."""
    s = jaccard_map(m, n, alpha, beta)
    a, b = m + alpha, n - m + beta
    hi = min(1.0, s + delta)
    lo = max(0.0, s - delta)
    return float(betainc(a, b, hi) - betainc(a, b, lo))


def fit_beta_moments(sims) -> tuple[float, float, bool]:
    """Learned Jaccard prior (Section 4.1): the Beta(alpha, beta) whose mean and
    variance equal the sample mean and the sample variance (sum of squared
    deviations divided by the sample size).  With mean s and variance v,
    alpha = s (s(1-s)/v - 1) and beta = (1-s)(s(1-s)/v - 1).  Returns
    (alpha, beta, fell_back): no Beta has the sample's moments when fewer than
    two values are given, v = 0 or v >= s(1-s), and a fit above 1e6 is beyond
    the tables' range; all of these give the uniform prior (1, 1)."""
    x = np.asarray(sims, dtype=np.float64)
    if x.size < 2:
        return 1.0, 1.0, True
    s = float(x.mean())
    v = float(((x - s) ** 2).mean())
    if not (v > 0.0) or not (v < s * (1.0 - s)):
        return 1.0, 1.0, True
    c = s * (1.0 - s) / v - 1.0
    a, b = s * c, (1.0 - s) * c
    if not (0.0 < a <= 1e6 and 0.0 < b <= 1e6):
        return 1.0, 1.0, True
    return a, b, False


# --------------------------------------------------------------------------
# Cosine, uniform prior on r in [0.5, 1]  (Section 4.2)
# --------------------------------------------------------------------------
def r2c(r: float) -> float:
    """Angle similarity r = 1 - theta/pi -> cosine."""
    return math.cos(math.pi * (1.0 - r))


def c2r(c: float) -> float:
    """Cosine -> angle similarity r = 1 - arccos(c)/pi."""
    return 1.0 - math.acos(c) / math.pi


def log_upper_mass(m: int, n: int, x: float) -> float:
    """log of int_x^1 r^m (1-r)^(n-m) dr / B(m+1, n-m+1) = log Pr[Bin(n+1, x) <= m]."""
    if x >= 1.0:
        return -math.inf
    if x <= 0.0:
        return 0.0
    j = np.arange(m + 1, dtype=np.float64)
    log_comb = gammaln(n + 2.0) - gammaln(j + 1.0) - gammaln(n + 2.0 - j)
    terms = log_comb + j * math.log(x) + (n + 1.0 - j) * math.log1p(-x)
    top = terms.max()
    return float(top + math.log(np.exp(terms - top).sum()))


def cosine_prune_prob(m: int, n: int, t: float) -> float:
    """Pr[S >= t | M(m,n)] = int_{t_r}^1 / int_{0.5}^1 of r^m (1-r)^(n-m), t_r = c2r(t)."""
    tr = c2r(t)
    return math.exp(log_upper_mass(m, n, tr) - log_upper_mass(m, n, 0.5))


def cosine_map(m: int, n: int) -> float:
    """S_hat = r2c(argmax over [0.5, 1] of r^m (1-r)^(n-m)) = r2c(max(0.5, m/n))."""
    return r2c(max(0.5, m / n))


def cosine_concentration(m: int, n: int, delta: float) -> float:
    """Pr[S_hat - delta < S < S_hat + delta | M(m,n)], mapped to r and clipped to [0.5, 1]."""
    s = cosine_map(m, n)
    r_lo = max(0.5, c2r(max(-1.0, s - delta)))
    r_hi = c2r(min(1.0, s + delta))
    base = log_upper_mass(m, n, 0.5)
    return math.exp(log_upper_mass(m, n, r_lo) - base) - math.exp(log_upper_mass(m, n, r_hi) - base)


# --------------------------------------------------------------------------
# Dispatch by measure
# --------------------------------------------------------------------------
def prune_prob(measure: int, m: int, n: int, t: float, alpha=1.0, beta=1.0) -> float:
    if measure == JACCARD:
        return jaccard_prune_prob(m, n, t, alpha, beta)
    return cosine_prune_prob(m, n, t)


def map_estimate(measure: int, m: int, n: int, alpha=1.0, beta=1.0) -> float:
    if measure == JACCARD:
        return jaccard_map(m, n, alpha, beta)
    return cosine_map(m, n)


def concentration(measure: int, m: int, n: int, delta: float, alpha=1.0, beta=1.0) -> float:
    if measure == JACCARD:
        return jaccard_concentration(m, n, delta, alpha, beta)
    return cosine_concentration(m, n, delta)


# --------------------------------------------------------------------------
# Memo of the per-(m, n) decisions, as the paper's own inference cache does
# (Section 4.3).  Every entry is the posterior evaluated directly above; no
# threshold search or monotonicity is assumed.
# --------------------------------------------------------------------------
@lru_cache(maxsize=64)
def decision_memo(measure: int, t: float, epsilon: float, delta: float, gamma: float,
                  alpha: float, beta: float, k: int, n_levels: int, with_concentration: bool = True):
    """Per level j (n = (j+1) k) and m in [0, n]:

      survive[j, m]  = Pr[S >= t | M(m,n)] >= epsilon
      accept[j, m]   = survive and Pr[|S - S_hat| < delta | M(m,n)] >= 1 - gamma
      shat[j, m]     = MAP estimate
      p_ge[j, m], conc[j, m]  the raw probabilities (conc is NaN where not evaluated)

    Arrays have shape [n_levels, n_levels*k + 1]; entries with m > n are unused.
    """
    n_max = n_levels * k
    survive = np.zeros((n_levels, n_max + 1), np.uint8)
    accept = np.zeros((n_levels, n_max + 1), np.uint8)
    shat = np.zeros((n_levels, n_max + 1), np.float64)
    p_ge = np.full((n_levels, n_max + 1), np.nan)
    conc = np.full((n_levels, n_max + 1), np.nan)
    for j in range(n_levels):
        n = (j + 1) * k
        for m in range(n + 1):
            p = prune_prob(measure, m, n, t, alpha, beta)
            p_ge[j, m] = p
            shat[j, m] = map_estimate(measure, m, n, alpha, beta)
            if p >= epsilon:
                survive[j, m] = 1
                if with_concentration:
                    c = concentration(measure, m, n, delta, alpha, beta)
                    conc[j, m] = c
                    if c >= 1.0 - gamma:
                        accept[j, m] = 1
    for a in (survive, accept, shat, p_ge, conc):
        a.setflags(write=False)
    return dict(survive=survive, accept=accept, shat=shat, p_ge=p_ge, conc=conc)
