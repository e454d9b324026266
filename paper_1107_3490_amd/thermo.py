"""Per-temperature thermodynamics from the per-sweep series of a run
(pt_get_series: [sweeps, slots, 3] of E, R_ee^2, R_gyr^2, recorded after each
sweep and before the exchange step).

For every slot, over the sweeps after a burn-in fraction, with errors from M
equal consecutive bins (standard error of the bin means; jackknife over the
bins for the non-linear estimates):

  E      <E>
  Cv     C_V / N = beta^2 (<E^2> - <E>^2) / N        (Sec. 4, k_B = 1)
  Rg2    <R_gyr^2>,  Ree2  <R_ee^2>                  (Eqs. 7-8)
  dRg2dT d<R_gyr^2>/dT = beta^2 (<R_gyr^2 E> - <R_gyr^2><E>)

Host-side post-processing of what the device recorded; no device work.
"""
from __future__ import annotations

import numpy as np


def _bins(x: np.ndarray, m: int) -> np.ndarray:
    """[m, slots] bin sums of x [sweeps, slots] (the tail past m full bins is dropped)."""
    size = x.shape[0] // m
    if size == 0:
        raise ValueError(f"{x.shape[0]} sweeps cannot fill {m} bins")
    return x[: size * m].reshape(m, size, -1).sum(axis=1), size


def estimates(series: np.ndarray, betas, n_beads, burn_in: float = 0.2, n_bins: int = 32) -> dict:
    """Arrays over slots: E, dE, Cv, dCv, Rg2, dRg2, Ree2, dRee2, dRg2dT, ddRg2dT."""
    s = np.asarray(series, dtype=np.float64)
    s = s[int(burn_in * s.shape[0]):]
    beta = np.asarray(betas, dtype=np.float64)
    nb = np.asarray(n_beads, dtype=np.float64)
    e, ree, rg = s[:, :, 0], s[:, :, 1], s[:, :, 2]
    m = n_bins
    cols = {"e": e, "e2": e * e, "rg": rg, "ree": ree, "rge": rg * e}
    sums, size = {}, 0
    for k, v in cols.items():
        sums[k], size = _bins(v, m)
    tot = {k: v.sum(axis=0) for k, v in sums.items()}
    cnt = size * m
    mean = {k: v / cnt for k, v in tot.items()}
    # leave-one-bin-out means [m, slots]
    loo = {k: (tot[k][None, :] - sums[k]) / (cnt - size) for k in sums}

    def jack(f_all, f_loo):
        fb = f_loo.mean(axis=0)
        return f_all, np.sqrt((m - 1) / m * ((f_loo - fb) ** 2).sum(axis=0))

    def plain(k):
        bm = sums[k] / size
        return mean[k], bm.std(axis=0, ddof=1) / np.sqrt(m)

    out = {}
    out["E"], out["dE"] = plain("e")
    out["Rg2"], out["dRg2"] = plain("rg")
    out["Ree2"], out["dRee2"] = plain("ree")
    b2 = beta * beta
    out["Cv"], out["dCv"] = jack(b2 * (mean["e2"] - mean["e"] ** 2) / nb,
                                 b2 * (loo["e2"] - loo["e"] ** 2) / nb)
    out["dRg2dT"], out["ddRg2dT"] = jack(b2 * (mean["rge"] - mean["rg"] * mean["e"]),
                                         b2 * (loo["rge"] - loo["rg"] * loo["e"]))
    out["beta"] = beta
    return out


def from_accumulators(acc: np.ndarray, betas, n_beads) -> dict:
    """<E>, C_V/N, <R_gyr^2>, <R_ee^2> from the device accumulators of
    pt_observables ([slots, 5]: n, sum E, sum E^2, sum R_gyr^2, sum R_ee^2);
    no error bars (those need the series)."""
    a = np.asarray(acc, dtype=np.float64)
    n = a[:, 0]
    beta = np.asarray(betas, dtype=np.float64)
    e = a[:, 1] / n
    return {"E": e, "Cv": beta * beta * (a[:, 2] / n - e * e) / np.asarray(n_beads, dtype=np.float64),
            "Rg2": a[:, 3] / n, "Ree2": a[:, 4] / n, "n": n}
