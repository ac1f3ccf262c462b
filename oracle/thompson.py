"""Oracle (test infrastructure only: imported by tests/, never by the product
path): the latency belief of the Thompson-sampling scheduler that chooses
among rasterisation-backward implementations (Sec. 4.2: a latency belief per
implementation, kept as a distribution, updated from measured latencies).

The paper does not name the distribution; the reading taken is the conjugate
Normal-Gamma model: latencies x_1..x_n of one implementation are
Normal(mu, 1/tau), with prior mu | tau ~ Normal(mu0, 1/(kappa0 tau)) and
tau ~ Gamma(alpha0, rate beta0).  The posterior is Normal-Gamma with

    kappa_n = kappa0 + n
    mu_n    = (kappa0 mu0 + n xbar) / kappa_n
    alpha_n = alpha0 + n / 2
    beta_n  = beta0 + (1/2) sum (x_i - xbar)^2 + kappa0 n (xbar - mu0)^2 / (2 kappa_n)

(the standard result for this prior; DeGroot, Optimal Statistical Decisions,
1970).  Written here in batch form from the whole list of observations, in
float64.  The marginal posterior of mu is Student-t with 2 alpha_n degrees of
freedom, location mu_n and squared scale beta_n / (alpha_n kappa_n).
"""
import numpy as np


def posterior(xs, mu0, kappa0, alpha0, beta0):
    """(mu_n, kappa_n, alpha_n, beta_n) after the observations xs."""
    x = np.asarray(xs, np.float64)
    n = x.size
    xbar = x.mean() if n else 0.0
    ss = float(((x - xbar) ** 2).sum()) if n else 0.0
    kappa_n = kappa0 + n
    mu_n = (kappa0 * mu0 + n * xbar) / kappa_n
    alpha_n = alpha0 + n / 2.0
    beta_n = beta0 + 0.5 * ss + kappa0 * n * (xbar - mu0) ** 2 / (2.0 * kappa_n)
    return mu_n, kappa_n, alpha_n, beta_n


def mean_marginal(mu_n, kappa_n, alpha_n, beta_n):
    """Student-t marginal of mu: (degrees of freedom, location, scale)."""
    return 2.0 * alpha_n, mu_n, float(np.sqrt(beta_n / (alpha_n * kappa_n)))
