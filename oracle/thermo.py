"""Thermodynamic estimates from the oracle's per-sweep series -- test
infrastructure, like the rest of oracle/ (only tests, the smoke check and the
CPU baseline of the benchmark use it).

Per slot (one temperature each), over the sweeps after a burn-in fraction:
  <E>, <R_gyr^2>, <R_ee^2>        plain means (Eqs. 7-8),
  C_V/N = beta^2 (<E^2> - <E>^2) / N   specific heat per monomer (Sec. 4,
                                       k_B = 1),
  d<R_gyr^2>/dT = beta^2 (<R_gyr^2 E> - <R_gyr^2><E>)
                                       the temperature derivative of the
                                       canonical mean of R_gyr^2 (k_B = 1),
                                       the reading taken of the paper's
                                       "fluctuation of r_gyr^2" (Sec. 4.1),
with errors from M equal consecutive bins: the standard error of the bin
means for the plain averages, the jackknife over the same bins for C_V/N and
d<R_gyr^2>/dT.
Written as plain loops so that it can be read against these definitions.
"""
import math


def _bin_sums(xs, m):
    size = len(xs) // m
    return [sum(xs[b * size:(b + 1) * size]) for b in range(m)], size


def mean_and_error(xs, m=32):
    """Mean of xs over m equal bins (a tail that does not fill a bin is
    dropped) and the standard error of that mean from the spread of the bin
    means."""
    sums, size = _bin_sums(xs, m)
    means = [s / size for s in sums]
    mu = sum(means) / m
    var = sum((b - mu) ** 2 for b in means) / (m - 1)
    return mu, math.sqrt(var / m)


def specific_heat(es, beta, n_beads, m=32):
    """C_V/N and its jackknife error over m bins."""
    sums, size = _bin_sums(es, m)
    sums2, _ = _bin_sums([e * e for e in es], m)
    tot, tot2, cnt = sum(sums), sum(sums2), size * m
    cv = beta * beta * (tot2 / cnt - (tot / cnt) ** 2) / n_beads
    loo = []
    for b in range(m):
        e1 = (tot - sums[b]) / (cnt - size)
        e2 = (tot2 - sums2[b]) / (cnt - size)
        loo.append(beta * beta * (e2 - e1 * e1) / n_beads)
    lbar = sum(loo) / m
    err = math.sqrt((m - 1) / m * sum((c - lbar) ** 2 for c in loo))
    return cv, err


def rg2_temperature_derivative(rgs, es, beta, m=32):
    """d<R_gyr^2>/dT and its jackknife error over m bins.  In the canonical
    ensemble <A> = sum A exp(-beta E) / Z, so d<A>/dbeta = -(<A E> - <A><E>)
    and, with beta = 1/T, d<A>/dT = beta^2 (<A E> - <A><E>)."""
    sa, size = _bin_sums(rgs, m)
    se, _ = _bin_sums(es, m)
    sae, _ = _bin_sums([a * e for a, e in zip(rgs, es)], m)
    ta, te, tae, cnt = sum(sa), sum(se), sum(sae), size * m
    d = beta * beta * (tae / cnt - (ta / cnt) * (te / cnt))
    loo = []
    for b in range(m):
        k = cnt - size
        a1, e1, ae1 = (ta - sa[b]) / k, (te - se[b]) / k, (tae - sae[b]) / k
        loo.append(beta * beta * (ae1 - a1 * e1))
    lbar = sum(loo) / m
    err = math.sqrt((m - 1) / m * sum((c - lbar) ** 2 for c in loo))
    return d, err


def estimates(series, betas, n_beads, burn_in=0.2, m=32):
    """series: [sweeps][slots][3] of (E, R_ee^2, R_gyr^2); betas and n_beads
    per slot.  Returns a list of dicts, one per slot."""
    sweeps = len(series)
    start = int(burn_in * sweeps)
    out = []
    for g in range(len(betas)):
        es = [float(series[t][g][0]) for t in range(start, sweeps)]
        ree = [float(series[t][g][1]) for t in range(start, sweeps)]
        rg = [float(series[t][g][2]) for t in range(start, sweeps)]
        e, de = mean_and_error(es, m)
        cv, dcv = specific_heat(es, float(betas[g]), int(n_beads[g]), m)
        r2, dr2 = mean_and_error(rg, m)
        q2, dq2 = mean_and_error(ree, m)
        dt, ddt = rg2_temperature_derivative(rg, es, float(betas[g]), m)
        out.append(dict(E=e, dE=de, Cv=cv, dCv=dcv, Rg2=r2, dRg2=dr2, Ree2=q2, dRee2=dq2,
                        dRg2dT=dt, ddRg2dT=ddt))
    return out
