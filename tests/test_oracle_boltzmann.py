"""Statistical pins of the oracle's sampler (Metropolis, Eq. 5, plus exchange,
Eq. 6) against exact canonical averages of tiny chains.

For N = 2 the energy depends on the bond length r alone, and the canonical
density of r is proportional to r^2 exp(-beta [E_mod(r) + E_FENE(r)]) on
(r0 - R, r0 + R) (Eqs. 1-4).  For N = 3 the weight is
r12^2 r23^2 exp(-beta [u(r12) + u(r23) + E_mod(r13)]) over the two bond
lengths and the cosine of the bond angle, u = E_mod + E_FENE.  The averages
come from numerical quadrature written here from Eqs. (1)-(3), independent
of the oracle's code; the Monte Carlo averages must agree within 4 binned
standard errors at every temperature of the ladder.
"""
import math

import numpy as np
from scipy import integrate, special

from oracle import oracle as O
from oracle import thermo as OT
from paper_1107_3490_amd import inputs as I

M = I.model_params()
SIG, RC, R0, R, K = M["sigma"], M["r_cut"], M["fene_r0"], M["fene_R"], M["fene_k"]


def e_mod(r):
    r = np.minimum(r, RC)
    return 4 * ((SIG / r) ** 12 - (SIG / r) ** 6) - 4 * ((SIG / RC) ** 12 - (SIG / RC) ** 6)


def e_fene(r):
    x = (r - R0) / R
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.where(np.abs(x) < 1, -0.5 * K * R * R * np.log1p(-x * x), np.inf)


def u_bond(r):
    return e_mod(r) + e_fene(r)


def exact_n2(beta):
    lo, hi = R0 - R, R0 + R
    emin = float(u_bond(np.array(R0)))
    w = lambda r: r * r * math.exp(-beta * (float(u_bond(np.array(r))) - emin))
    z = integrate.quad(w, lo, hi, points=[R0], limit=400, epsabs=0, epsrel=1e-12)[0]
    m1 = integrate.quad(lambda r: w(r) * float(u_bond(np.array(r))), lo, hi, points=[R0],
                        limit=400, epsabs=0, epsrel=1e-12)[0]
    m2 = integrate.quad(lambda r: w(r) * float(u_bond(np.array(r))) ** 2, lo, hi, points=[R0],
                        limit=400, epsabs=0, epsrel=1e-12)[0]
    return m1 / z, m2 / z - (m1 / z) ** 2


def _bond_nodes(beta, nr):
    """Nodes and weights for integrals over a bond length on (r0 - R, r0 + R)
    carrying the FENE Boltzmann factor exp(-beta E_FENE) = (1 - x^2)^(beta K R^2 / 2),
    x = (r - r0)/R: Gauss-Jacobi in x absorbs the endpoint power law exactly."""
    a = beta * 0.5 * K * R * R
    x, wx = special.roots_jacobi(nr, a, a)
    return R0 + R * x, R * wx


def exact_n3(beta, nr=64, nc=48):
    r, wr = _bond_nodes(beta, nr)
    xc, wc = np.polynomial.legendre.leggauss(nc)
    r1, r2 = np.meshgrid(r, r, indexing="ij")
    w12 = np.outer(wr, wr)
    # Split the angle integral where r13 crosses the cutoff (kink of E_mod).
    cstar = np.clip((r1 ** 2 + r2 ** 2 - RC ** 2) / (2 * r1 * r2), -1.0, 1.0)
    tot = [0.0, 0.0, 0.0]
    base = e_mod(r1) + e_mod(r2)          # FENE factors sit in the Jacobi weights
    fene = e_fene(r1) + e_fene(r2)
    for a, b in ((-np.ones_like(cstar), cstar), (cstar, np.ones_like(cstar))):
        c = 0.5 * (b - a)[..., None] * xc + 0.5 * (b + a)[..., None]
        wc_ = 0.5 * (b - a)[..., None] * wc
        r13 = np.sqrt(np.maximum(r1[..., None] ** 2 + r2[..., None] ** 2
                                 - 2 * r1[..., None] * r2[..., None] * c, 1e-300))
        e_nb = base[..., None] + e_mod(r13)
        e = e_nb + fene[..., None]
        wt = (r1 ** 2 * r2 ** 2 * w12)[..., None] * wc_ * np.exp(-beta * (e_nb + 3.0))
        tot[0] += wt.sum()
        tot[1] += (wt * e).sum()
        tot[2] += (wt * e * e).sum()
    mean = tot[1] / tot[0]
    return mean, tot[2] / tot[0] - mean ** 2


def binned(x, nbins=50):
    x = x[: len(x) // nbins * nbins].reshape(nbins, -1).mean(axis=1)
    return x.mean(), x.std(ddof=1) / math.sqrt(nbins)


def _check(n, exact, seed, sweeps=300000, temps=(0.3, 2.5), slots=4):
    w = I.make_workload([n], [slots], [temps], "straight", seed, sweeps, "fp64")
    s = O.Simulation(w)
    e = s.run(sweeps, series=True)["series"][sweeps // 10:, :, 0]
    for g, beta in enumerate(w.betas):
        want, var = exact(beta)
        m, err = binned(e[:, g])
        assert abs(m - want) < 4 * err, (n, g, beta, m, want, err)
        # second moment <E^2> = var + <E>^2 (specific heat, Eq. 7)
        m2, err2 = binned(e[:, g] ** 2)
        assert abs(m2 - (var + want * want)) < 4 * err2, (n, g, beta, m2, var + want * want)
        # C_V/N = beta^2 var / N with its jackknife error (the oracle's estimator)
        cv, dcv = OT.specific_heat(list(e[:, g]), beta, n, 50)
        assert abs(cv - beta * beta * var / n) < 4 * dcv, (n, g, beta, cv, beta * beta * var / n, dcv)


def test_two_bead_chain_matches_quadrature():
    _check(2, exact_n2, 104)


def test_three_bead_chain_matches_quadrature():
    _check(3, exact_n3, 104)
