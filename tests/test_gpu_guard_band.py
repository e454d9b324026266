"""The guard band of the mixed-precision path, at scale.

The mixed path scores a move with FP32 Lennard-Jones brackets (Eqs. 1-2) from
FP64 separations and relies on a rigorous bound on the error of that score:
every decision whose score lies within the bound of the Metropolis threshold
(Eq. 5) is re-scored in the FP64 order.  These tests check the bound against
the exact values, computed in 64-bit-mantissa long double from the same FP64
inputs (relative error ~1e-19, far below the bounds checked):

* one pair term at a time (the old separation on the cutoff), 10^8 random
  geometries from near contact to beyond the cutoff;
* the whole pair sum of a move, on random chains (random walks, compact
  globules, chains with near-contacts) and random moves, through the same
  device code the sweep kernel uses (8 beads per lane, one wavefront).
The largest observed error over bound is printed; the design margin is a
factor two, so it must stay at or below 0.5.
"""
import math

import numpy as np
import pytest

from paper_1107_3490_amd import inputs as I

pytestmark = pytest.mark.gpu

L = np.longdouble


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1107_3490_amd import pt
    pt.lib()  # raises if the HIP library is missing: no fallback
    yield


def _emod(r2, m):
    """Eqs. (1)-(2) in long double from a long-double r^2: truncated at rc and
    shifted by E_LJ(rc)."""
    sig2 = L(m["sigma"]) ** 2
    rc2 = L(m["r_cut"]) ** 2
    four_eps = 4 * L(m["epsilon"])
    with np.errstate(over="ignore", divide="ignore", invalid="ignore"):
        s6 = (sig2 / r2) ** 3
        s6c = (sig2 / rc2) ** 3
        e = four_eps * (s6 * s6 - s6) - four_eps * (s6c * s6c - s6c)
    return np.where(r2 < rc2, e, L(0))


def test_fp32_term_bound_is_sound_on_1e8_geometries():
    from paper_1107_3490_amd import pt
    m = I.model_params()
    rc = m["r_cut"]
    chunk, chunks = 1 << 21, 48          # 1.007e8 geometries
    worst, n_tot = 0.0, 0
    for c in range(chunks):
        rng = np.random.default_rng(7000 + c)
        q = chunk // 8
        r = np.concatenate([
            rng.uniform(0.3, 3.0, 3 * q),                      # everything
            rc * (1 + rng.uniform(-1e-6, 1e-6, q)),            # on the cutoff
            rc * (1 + rng.uniform(-1e-3, 1e-3, q)),            # near the cutoff
            rng.uniform(0.2, 0.5, q),                          # near contact
            rng.uniform(0.69, 0.71, q),                        # around the minimum
            np.exp(rng.uniform(math.log(0.05), math.log(rc), q)),  # log-uniform, deep contact
        ])
        phi = rng.uniform(0, 2 * math.pi, r.size)
        dx, dy = r * np.cos(phi), r * np.sin(phi)
        if c == 0:
            print(f"\n[case] single-term bound, {chunks} chunks of {r.size}", flush=True)
        out = pt.pt_selftest(m, pt.OP_LJ32, dx, dy).reshape(-1, 2)
        exact = _emod(dx.astype(L) ** 2 + dy.astype(L) ** 2, m)
        bound = out[:, 1]
        ok = np.isfinite(bound)            # an infinite bound sends the move to FP64
        err = np.abs(out[ok, 0].astype(L) - exact[ok]).astype(np.float64)
        bad = np.flatnonzero(err > bound[ok])
        assert bad.size == 0, f"bound exceeded at r = {r[ok][bad[:5]]!r}"
        worst = max(worst, float(np.max(err / np.maximum(bound[ok], 1e-300))))
        n_tot += int(ok.sum())
    print(f"  FP32 term: {n_tot} geometries, max observed/bound = {worst:.3f}", flush=True)
    assert worst <= 0.5


def _globule(n, rng, dmin=0.62):
    """A compact conformation: beads placed one after another within reach of
    the previous one, at least dmin from all others when possible (random
    sequential placement in a ball)."""
    rad = 0.62 * n ** (1.0 / 3.0) + 0.5
    xyz = np.zeros((n, 3))
    for j in range(1, n):
        for _ in range(200):
            v = rng.standard_normal(3)
            p = xyz[j - 1] + rng.uniform(0.6, 0.8) * v / np.linalg.norm(v)
            if np.linalg.norm(p) > rad:
                continue
            if j < 2 or np.min(np.linalg.norm(xyz[:j - 1] - p, axis=1)) >= dmin:
                break
        xyz[j] = p
    return xyz


def _chain(kind, n, rng):
    if kind == "walk":
        return I.random_walk(n, rng)
    if kind == "globule":
        return _globule(n, rng)
    # near contacts: a walk with shorter bonds, folded back onto itself
    xyz = I.random_walk(n, rng, bond=0.45)
    return xyz * rng.uniform(0.5, 1.0)


def test_mixed_move_bound_is_sound_on_random_moves():
    """The bound on the whole FP32 pair sum of a move (what the decision band
    is made of), on 1.5x10^5 moves: chain lengths 2..512, three kinds of
    conformation, displacements of edge 0.02, 0.2 and 0.6."""
    from paper_1107_3490_amd import pt
    m = I.model_params()
    item = pt.MOVE_ITEM
    per_call, calls = 1000, 150
    worst, n_ok, n_inf = 0.0, 0, 0
    for c in range(calls):
        rng = np.random.default_rng(9100 + c)
        kind = ("walk", "globule", "contact")[c % 3]
        edge = (0.02, 0.2, 0.6)[(c // 3) % 3]
        ns = rng.integers(2, 513, size=per_call) if c % 5 else np.full(per_call, 512)
        x = np.zeros((per_call, item))
        x[:, 0:3 * 512:3] = 1.0e30       # padding beads far away, as in the kernels
        confs = []
        base = _chain(kind, 512, rng)    # one conformation per call, cut to each N
        for i, nb in enumerate(ns):
            xyz = base[:nb] + rng.uniform(-1e-3, 1e-3, (nb, 3)) * (kind != "contact")
            x[i, :3 * nb] = xyz.ravel()
            k = int(rng.integers(0, nb))
            d = (rng.random(3) - 0.5) * edge
            x[i, 3 * 512:3 * 512 + 5] = [nb, k, d[0], d[1], d[2]]
            confs.append((xyz, k, d))
        if c == 0:
            print(f"\n[case] move bound, {calls} calls of {per_call} moves", flush=True)
        out = pt.pt_selftest(m, pt.OP_MOVE32, x.ravel()).reshape(-1, 2)
        for i, (xyz, k, d) in enumerate(confs):
            if not np.isfinite(out[i, 1]) or not np.isfinite(out[i, 0]):
                n_inf += 1               # the sweep re-scores such a move in FP64
                continue
            xo = xyz[k]
            xn = xo + d                  # FP64, as the kernel forms r'_k
            others = np.delete(xyz, k, axis=0).astype(L)
            r2n = np.sum((others - xn.astype(L)) ** 2, axis=1)
            r2o = np.sum((others - xo.astype(L)) ** 2, axis=1)
            exact = np.sum(_emod(r2n, m) - _emod(r2o, m))
            err = float(abs(L(out[i, 0]) - exact))
            assert err <= out[i, 1], (c, i, len(xyz), k, err, out[i, 1])
            worst = max(worst, err / max(out[i, 1], 1e-300))
            n_ok += 1
    print(f"  FP32 move sum: {n_ok} moves, {n_inf} with a non-finite score or bound, "
          f"max observed/bound = {worst:.3g}", flush=True)
    assert n_ok > 0.9 * per_call * calls
    assert worst <= 0.5
