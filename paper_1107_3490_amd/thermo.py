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


def scan(n_beads: int, t_min: float, t_max: float, slots: int, sweeps: int, seed: int = 1,
         precision: str = "mixed", start: str = "straight", burn_in: float = 0.2, n_bins: int = 32,
         step_edge: float = 0.2, chunk: int = 100000) -> dict:
    """Parallel-tempering run of one chain on the GPU (geometric ladder
    [t_min, t_max], exchange after every sweep) and its per-temperature
    estimates; adds T = 1/beta.  The series is kept on the device for all
    sweeps (sweeps x slots x 24 bytes)."""
    from . import inputs as I
    from . import pt

    w = I.make_workload([n_beads], [slots], [(t_min, t_max)], start, seed, sweeps, precision,
                        step_edge=step_edge)
    sim = pt.Simulation(w, precision=precision, series_capacity=sweeps)
    done = 0
    while done < sweeps:
        n = min(chunk, sweeps - done)
        sim.sweep(n)
        done += n
    ser = sim.series()
    sim.close()
    out = estimates(ser, w.betas, [n_beads] * slots, burn_in=burn_in, n_bins=n_bins)
    out["T"] = 1.0 / np.asarray(w.betas)
    return out


def main(argv=None):
    """python -m paper_1107_3490_amd.thermo --n 13 --tmin 0.1 --tmax 2.5 --slots 64 --sweeps 200000"""
    import argparse
    import json

    ap = argparse.ArgumentParser(description="per-temperature thermodynamics of one chain (GPU)")
    ap.add_argument("--n", type=int, default=13)
    ap.add_argument("--tmin", type=float, default=0.1)
    ap.add_argument("--tmax", type=float, default=2.5)
    ap.add_argument("--slots", type=int, default=64)
    ap.add_argument("--sweeps", type=int, default=200000)
    ap.add_argument("--seed", type=int, default=7)
    ap.add_argument("--burn-in", type=float, default=0.2)
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    a = ap.parse_args(argv)
    r = scan(a.n, a.tmin, a.tmax, a.slots, a.sweeps, seed=a.seed, precision=a.precision, burn_in=a.burn_in)
    i = int(np.argmax(r["Cv"]))
    # d<R_gyr^2>/dT peaks at freezing too; report the peak above twice the C_V peak.
    hot = np.nonzero(r["T"] > 2 * r["T"][i])[0]
    j = int(hot[np.argmax(r["dRg2dT"][hot])]) if hot.size else int(np.argmax(r["dRg2dT"]))
    print(json.dumps({"N": a.n, "Cv_peak_T": float(r["T"][i]), "dRg2dT_peak_T_above_freezing": float(r["T"][j])}))
    for k in range(len(r["T"])):
        print(f"T={r['T'][k]:.4f}  E={r['E'][k]:.4f}+-{r['dE'][k]:.4f}  Cv/N={r['Cv'][k]:.4f}+-{r['dCv'][k]:.4f}"
              f"  Rg2={r['Rg2'][k]:.4f}  dRg2/dT={r['dRg2dT'][k]:.4f}+-{r['ddRg2dT'][k]:.4f}")


if __name__ == "__main__":
    main()
