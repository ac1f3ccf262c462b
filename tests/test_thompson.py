"""Thompson-sampling scheduler of the backward variants (gs_ts_*, host code):
the oracle's Normal-Gamma posterior pinned by numerical integration of prior x
likelihood; the library's posterior against the oracle; the sampler's draws
against the Student-t marginal; determinism, convergence to the fastest arm,
and argument errors."""
import ctypes as C

import numpy as np
import pytest
from scipy import stats

from oracle import thompson as O

PRIOR = dict(mu0=0.3, kappa0=0.5, alpha0=2.0, beta0=0.01)


def _lib():
    from paper_2605_00219_amd import _lib as G
    return G


def _state(n_arms=3, seed=1, prior=PRIOR):
    G = _lib()
    st = G.GsTsState()
    assert G.lib.gs_ts_init(C.byref(st), n_arms, seed, prior["mu0"], prior["kappa0"], prior["alpha0"],
                            prior["beta0"]) == 0
    return G, st


def test_oracle_posterior_against_numerical_integration():
    """E[mu] and E[tau] of prior x likelihood on a (mu, tau) grid equal mu_n and
    alpha_n / beta_n of the closed form."""
    rng = np.random.default_rng(5)
    xs = rng.normal(0.27, 0.02, size=7)
    mu_n, kappa_n, alpha_n, beta_n = O.posterior(xs, **PRIOR)
    mu = np.linspace(0.1, 0.45, 1401)[:, None]
    tau = np.linspace(1.0, 6000.0, 3001)[None, :]
    logp = (stats.norm.logpdf(mu, PRIOR["mu0"], 1.0 / np.sqrt(PRIOR["kappa0"] * tau))
            + stats.gamma.logpdf(tau, PRIOR["alpha0"], scale=1.0 / PRIOR["beta0"]))
    for x in xs:
        logp = logp + stats.norm.logpdf(x, mu, 1.0 / np.sqrt(tau))
    w = np.exp(logp - logp.max())
    w /= w.sum()
    assert (w * mu).sum() == pytest.approx(mu_n, rel=1e-4)
    assert (w * tau).sum() == pytest.approx(alpha_n / beta_n, rel=2e-3)


def test_oracle_prior_only_and_one_observation():
    assert O.posterior([], **PRIOR) == (PRIOR["mu0"], PRIOR["kappa0"], PRIOR["alpha0"], PRIOR["beta0"])
    mu_n, kappa_n, alpha_n, beta_n = O.posterior([0.5], **PRIOR)
    k0 = PRIOR["kappa0"]
    assert mu_n == pytest.approx((k0 * 0.3 + 0.5) / (k0 + 1))
    assert beta_n == pytest.approx(PRIOR["beta0"] + k0 * 0.2 ** 2 / (2 * (k0 + 1)))


def test_library_posterior_matches_oracle():
    G, st = _state()
    rng = np.random.default_rng(9)
    obs = {0: [], 1: [], 2: []}
    for i in range(60):
        a = int(rng.integers(0, 3))
        x = float(rng.normal(0.3 + 0.05 * a, 0.01 + 0.01 * a))
        obs[a].append(x)
        assert G.lib.gs_ts_update(C.byref(st), a, x) == 0
    out = (C.c_double * 4)()
    for a in range(3):
        assert G.lib.gs_ts_posterior(C.byref(st), a, out) == 0
        np.testing.assert_allclose(list(out), O.posterior(obs[a], **PRIOR), rtol=1e-12)


def test_sampler_draws_follow_the_student_t_marginal():
    G, st = _state(n_arms=1, seed=123)
    for x in (0.31, 0.29, 0.33, 0.30, 0.28):
        G.lib.gs_ts_update(C.byref(st), 0, x)
    out = (C.c_double * 4)()
    G.lib.gs_ts_posterior(C.byref(st), 0, out)
    df, loc, scale = O.mean_marginal(*list(out))
    draws = np.array([G.lib.gs_ts_sample(C.byref(st), 0) for _ in range(20000)])
    assert stats.kstest(draws, stats.t(df, loc, scale).cdf).pvalue > 1e-3
    assert draws.mean() == pytest.approx(loc, abs=5 * scale / np.sqrt(20000) * np.sqrt(df / (df - 2)))


def test_selection_is_deterministic_per_seed():
    seqs = []
    for seed in (4, 4, 5):
        G, st = _state(seed=seed)
        seq = []
        for i in range(40):
            a = G.lib.gs_ts_select(C.byref(st))
            seq.append(a)
            G.lib.gs_ts_update(C.byref(st), a, 0.3 + 0.01 * a + 0.001 * (i % 3))
        seqs.append(seq)
    assert seqs[0] == seqs[1]
    assert seqs[0] != seqs[2]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_converges_to_the_fastest_arm(seed):
    true = [0.30, 0.26, 0.33, 0.29]
    G, st = _state(n_arms=4, seed=seed, prior=dict(mu0=0.3, kappa0=1e-3, alpha0=1.0, beta0=0.03 ** 2))
    rng = np.random.default_rng(seed)
    picks = []
    for _ in range(400):
        a = G.lib.gs_ts_select(C.byref(st))
        picks.append(a)
        G.lib.gs_ts_update(C.byref(st), a, true[a] + rng.normal(0, 0.01))
    assert set(picks) == {0, 1, 2, 3}                 # every arm explored
    assert np.mean(np.array(picks[200:]) == 1) > 0.9


def test_argument_errors():
    G = _lib()
    st = G.GsTsState()
    assert G.lib.gs_ts_init(C.byref(st), 0, 1, 0.3, 1.0, 1.0, 0.01) < 0
    assert G.lib.gs_ts_init(C.byref(st), 9, 1, 0.3, 1.0, 1.0, 0.01) < 0
    assert G.lib.gs_ts_init(C.byref(st), 2, 1, 0.3, 0.0, 1.0, 0.01) < 0
    assert G.lib.gs_ts_init(C.byref(st), 2, 1, 0.3, 1.0, 0.5, 0.01) < 0
    assert G.lib.gs_ts_init(C.byref(st), 2, 1, 0.3, 1.0, 1.0, 0.01) == 0
    assert G.lib.gs_ts_update(C.byref(st), 2, 0.3) < 0
    assert G.lib.gs_ts_update(C.byref(st), 0, float("nan")) < 0
    assert np.isnan(G.lib.gs_ts_sample(C.byref(st), 5))
