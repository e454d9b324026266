"""Thermodynamic estimators (<E>, C_V/N, <R_gyr^2>, <R_ee^2> per temperature,
with binned and jackknife errors): the oracle's, pinned to closed forms of
Gaussian statistics, and the package's, checked against the oracle's."""
import math

import numpy as np

from oracle import thermo as OT
from paper_1107_3490_amd import thermo as PT


def _gauss_series(sweeps, slots, mu, sigma, seed):
    rng = np.random.default_rng(seed)
    s = np.zeros((sweeps, slots, 3))
    s[:, :, 0] = mu + sigma * rng.standard_normal((sweeps, slots))
    s[:, :, 1] = 2.0 + rng.random((sweeps, slots))
    s[:, :, 2] = 1.0 + 0.5 * rng.random((sweeps, slots))
    return s


def test_oracle_estimates_gaussian_closed_forms():
    """For independent normal energies the mean has standard error sigma/sqrt(n)
    and the sample variance sigma^2 sqrt(2/n); C_V/N = beta^2 sigma^2 / N."""
    n, mu, sigma, beta, nb = 64000, -3.0, 1.7, 0.8, 20
    s = _gauss_series(n, 1, mu, sigma, 11)
    est = OT.estimates(s, [beta], [nb], burn_in=0.0, m=32)[0]
    se = sigma / math.sqrt(n)
    assert abs(est["E"] - mu) < 3 * se
    assert 0.7 < est["dE"] / se < 1.3
    cv_exact = beta * beta * sigma * sigma / nb
    cv_se = cv_exact * math.sqrt(2.0 / n)
    assert abs(est["Cv"] - cv_exact) < 3 * cv_se
    assert 0.7 < est["dCv"] / cv_se < 1.3
    # uniform R^2 columns: means 2.5 and 1.25, standard errors from their variances
    assert abs(est["Ree2"] - 2.5) < 3 * math.sqrt(1 / 12 / n)
    assert abs(est["Rg2"] - 1.25) < 3 * 0.5 * math.sqrt(1 / 12 / n)


def test_oracle_jackknife_of_a_mean_is_the_binned_error():
    """The jackknife over bins of a linear statistic reproduces the standard
    error of the bin means exactly (an identity of the method)."""
    rng = np.random.default_rng(3)
    xs = list(rng.standard_normal(32 * 50))
    mu, err = OT.mean_and_error(xs, 32)
    sums, size = OT._bin_sums(xs, 32)
    loo = [(sum(sums) - sums[b]) / (len(xs) - size) for b in range(32)]
    lbar = sum(loo) / 32
    jk = math.sqrt(31 / 32 * sum((v - lbar) ** 2 for v in loo))
    assert abs(jk - err) <= 1e-12 * err


def test_package_estimates_match_oracle_estimates():
    """Correlated series (an AR(1) process per slot): the package's vectorised
    estimates equal the oracle's loops to rounding."""
    rng = np.random.default_rng(7)
    sweeps, slots = 5000, 6
    s = np.zeros((sweeps, slots, 3))
    x = np.zeros(slots)
    for t in range(sweeps):
        x = 0.9 * x + rng.standard_normal(slots)
        s[t, :, 0] = -10 + x
        s[t, :, 1] = 4 + 0.3 * x + rng.random(slots)
        s[t, :, 2] = 2 - 0.1 * x + rng.random(slots)
    betas = np.linspace(0.5, 3.0, slots)
    nb = np.full(slots, 30)
    o = OT.estimates(s, betas, nb, burn_in=0.2, m=32)
    p = PT.estimates(s, betas, nb, burn_in=0.2, n_bins=32)
    for g in range(slots):
        for k in ("E", "dE", "Cv", "dCv", "Rg2", "dRg2", "Ree2", "dRee2", "dRg2dT", "ddRg2dT"):
            assert abs(p[k][g] - o[g][k]) <= 1e-9 * max(1.0, abs(o[g][k])), (g, k, p[k][g], o[g][k])


def test_accumulator_summary_matches_series_means():
    s = _gauss_series(1000, 3, -2.0, 0.5, 5)
    acc = np.zeros((3, 5))
    acc[:, 0] = 1000
    acc[:, 1] = s[:, :, 0].sum(axis=0)
    acc[:, 2] = (s[:, :, 0] ** 2).sum(axis=0)
    acc[:, 3] = s[:, :, 2].sum(axis=0)
    acc[:, 4] = s[:, :, 1].sum(axis=0)
    a = PT.from_accumulators(acc, [1.0, 2.0, 3.0], [10, 10, 10])
    p = PT.estimates(s, [1.0, 2.0, 3.0], [10, 10, 10], burn_in=0.0, n_bins=10)
    for k in ("E", "Cv", "Rg2", "Ree2"):
        assert np.allclose(a[k], p[k], rtol=1e-12, atol=0)


def test_oracle_rg2_derivative_bivariate_normal_closed_form():
    """d<R_gyr^2>/dT = beta^2 Cov(R_gyr^2, E).  For jointly normal (R_gyr^2, E)
    with standard deviations s_a, s_e and correlation rho the covariance is
    rho s_a s_e, and the sample covariance of n independent draws has the
    standard error sqrt((s_a^2 s_e^2 + (rho s_a s_e)^2) / n) (Isserlis'
    theorem for the fourth moment of normals)."""
    n, beta = 64000, 1.3
    s_a, s_e = 0.8, 2.5
    for rho in (0.6, -0.35, 0.0):
        rng = np.random.default_rng(int(100 + 100 * rho))
        z1, z2 = rng.standard_normal(n), rng.standard_normal(n)
        a = 3.0 + s_a * z1
        e = -40.0 + s_e * (rho * z1 + math.sqrt(1 - rho * rho) * z2)
        d, err = OT.rg2_temperature_derivative(list(a), list(e), beta, m=32)
        cov = rho * s_a * s_e
        se = beta * beta * math.sqrt((s_a * s_a * s_e * s_e + cov * cov) / n)
        assert abs(d - beta * beta * cov) < 3.5 * se, (rho, d, beta * beta * cov, se)
        assert 0.7 < err / se < 1.3, (rho, err, se)


def test_oracle_rg2_derivative_of_a_function_of_energy():
    """If R_gyr^2 = c E + k exactly, the covariance is c Var(E): the estimate
    is beta^2 c times the (biased, 1/n) sample variance of E, to rounding."""
    rng = np.random.default_rng(9)
    es = list(-20 + 1.5 * rng.standard_normal(32 * 100))
    c, k, beta = -0.25, 7.0, 0.9
    d, _ = OT.rg2_temperature_derivative([c * x + k for x in es], es, beta, m=32)
    mu = sum(es) / len(es)
    var = sum((x - mu) ** 2 for x in es) / len(es)
    assert abs(d - beta * beta * c * var) <= 1e-9 * abs(beta * beta * c * var)
