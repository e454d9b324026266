"""Pins of the CPU oracle against what the paper and mathematics fix.

None of these compares the oracle with itself: each checks a closed form of
Eqs. (1)-(3) at the paper's parameters (Sec. 3.1), an invariant of Eq. (4),
a library routine (mpmath's log, rocRAND's Philox4x32-10), exact integer
identities of the draw maps, or the limiting behaviour of Eqs. (5)-(6).
"""
import ctypes as C
import json
import math
import os
import shutil
import subprocess

import mpmath as mp
import numpy as np
import pytest

from oracle import oracle as O
from paper_1107_3490_amd import inputs as I

M = I.model_params()
GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_parameters.json")

# E_LJ(r_c) with sigma/r_c = 2/5 exactly: 4 (0.4^12 - 0.4^6)   (Eq. 2, Sec. 3.1)
E_RC = 4.0 * (0.4 ** 12 - 0.4 ** 6)


def test_parameters_match_paper():
    g = json.load(open(GOLD))
    assert M["epsilon"] == g["lennard_jones"]["epsilon"]
    assert M["fene_r0"] == g["lennard_jones"]["r0"] == g["fene"]["r0"]
    assert M["fene_k"] == g["fene"]["K"] and M["fene_R"] == g["fene"]["R"]
    assert abs(M["sigma"] - 0.7 * 2 ** (-1 / 6)) < 1e-16
    assert abs(M["r_cut"] / M["sigma"] - g["lennard_jones"]["r_cut_over_sigma"]) < 1e-15


def test_lj_closed_forms():
    r0 = 0.7
    # Minimum of E_LJ at 2^(1/6) sigma = r0 with depth -epsilon, shifted by -E_LJ(rc).
    assert abs(O.lj(M, r0 * r0) - (-1.0 - E_RC)) < 1e-15
    # E_LJ(sigma) = 0, so E_mod(sigma) = -E_LJ(rc) = +0.016316891136.
    s = M["sigma"]
    assert abs(O.lj(M, s * s) - 0.016316891136) < 1e-14
    # At r = sqrt(2) r0: (sigma/r)^6 = 1/16, E_LJ = 4 (1/256 - 1/16) = -0.234375.
    assert abs(O.lj(M, 2 * r0 * r0) - (-0.234375 - E_RC)) < 1e-14
    # At r = 2 r0: (sigma/r)^6 = 1/128.
    assert abs(O.lj(M, 4 * r0 * r0) - (4 * (1 / 128 ** 2 - 1 / 128) - E_RC)) < 1e-14
    # Truncation (Eq. 1): exactly zero at and beyond the cutoff.
    rc2 = M["r_cut"] ** 2
    assert O.lj(M, rc2) == 0.0
    assert O.lj(M, 9 * r0 * r0) == 0.0 and O.lj(M, 1e6) == 0.0
    # Continuity at the cutoff: just inside, |E_mod| is of order (dE/dr2) * dr2.
    assert abs(O.lj(M, rc2 * (1 - 1e-9))) < 1e-9
    # Coincident beads: +inf, never NaN.
    assert O.lj(M, 0.0) == math.inf
    assert O.lj(M, 1e-300) == math.inf


def test_lj_curvature_at_minimum():
    # d^2 E_LJ/dr^2 at the minimum r_m = 2^(1/6) sigma is 72 epsilon / r_m^2.
    r0, h = 0.7, 1e-4
    f = lambda r: O.lj(M, r * r)
    d2 = (f(r0 + h) - 2 * f(r0) + f(r0 - h)) / h ** 2
    assert abs(d2 - 72.0 / r0 ** 2) / (72.0 / r0 ** 2) < 1e-5


def test_fene_closed_forms():
    K, R = 40.0, 0.3
    assert O.fene(M, 0.49) == 0.0               # minimum at r0 (Eq. 3)
    # |r - r0| = 0.1: -(K/2) R^2 log(1 - 1/9) = 1.8 log(9/8)
    want = 1.8 * math.log(9 / 8)
    assert abs(O.fene(M, 0.6 ** 2) - want) < 2e-16 * 4 * want + 1e-16
    assert abs(O.fene(M, 0.8 ** 2) - want) < 1e-15
    assert abs(want - 0.212009464181490218) < 1e-16
    # |r - r0| = 0.2: 1.8 log(9/5)
    assert abs(O.fene(M, 0.25) - 1.8 * math.log(9 / 5)) < 1e-15
    # Divergence at r0 +- R: huge just inside, +inf from there on.
    assert O.fene(M, 0.40001 ** 2) > 10.0 and O.fene(M, 0.99999 ** 2) > 10.0
    for r in (0.39999, 1.00001, 0.39, 1.2, 0.0):
        assert O.fene(M, r * r) == math.inf
    # Curvature at the minimum equals K.
    h = 1e-4
    f = lambda r: O.fene(M, r * r)
    d2 = (f(0.7 + h) - 2 * f(0.7) + f(0.7 - h)) / h ** 2
    assert abs(d2 - K) / K < 1e-6


def _ulps(a: float, b) -> float:
    b = float(b)
    return abs(a - b) / math.ulp(b) if b != 0 else abs(a) / 5e-324


def test_plog_against_mpmath():
    mp.mp.prec = 120
    rng = np.random.default_rng(7)
    xs = list(rng.random(4000))                                 # acceptance draws
    xs += list(1.0 - rng.random(2000) * 1e-3)                   # FENE y near 1
    xs += list(np.exp(rng.uniform(-700, 700, 2000)))            # wide range
    xs += [2.0 ** k for k in range(-60, 61)] + [0.5 + 1e-16, 1 + 2 ** -52, 1 - 2 ** -53,
                                                 math.sqrt(0.5), math.sqrt(2.0), 5e-324, 1e-310]
    worst = 0.0
    for x in xs:
        got = O.plog(float(x))
        want = mp.log(mp.mpf(float(x)))
        if float(want) == 0.0:
            assert got == 0.0
            continue
        worst = max(worst, _ulps(got, want))
    assert worst <= 2.0, worst
    assert O.plog(1.0) == 0.0
    assert O.plog(0.0) == -math.inf
    assert O.plog(math.inf) == math.inf
    assert math.isnan(O.plog(-1.0))


def _rocrand_reference():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    hdr = "/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"
    if not (os.path.exists(hipcc) and os.path.exists(hdr)):
        return None
    src = os.path.join(os.path.dirname(__file__), "rocrand_philox_ref.cpp")
    out = os.path.join(os.environ.get("TMPDIR", "/tmp"), f"pt_rocrand_ref_{os.getpid()}.so")
    subprocess.run([hipcc, "-fPIC", "-shared", "-O1", src, "-o", out], check=True,
                   stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    L = C.CDLL(out)
    L.ref_philox.argtypes = [C.POINTER(C.c_uint32), C.c_uint64, C.POINTER(C.c_uint32)]
    return L


def test_philox_matches_rocrand():
    L = _rocrand_reference()
    if L is None:
        pytest.skip("rocRAND headers / hipcc not available")
    rng = np.random.default_rng(11)
    for i in range(3000):
        ctr = [int(v) for v in rng.integers(0, 2 ** 32, size=4)]
        if i < 8:
            ctr = [i, 0, 0, 0]
        seed = int(rng.integers(0, 2 ** 63)) if i % 3 else i
        c = (C.c_uint32 * 4)(*ctr)
        o = (C.c_uint32 * 4)()
        L.ref_philox(c, C.c_uint64(seed), o)
        assert list(o) == [int(v) for v in O.philox(ctr, seed)], (ctr, seed)


def test_move_draw_maps_are_exact():
    rng = np.random.default_rng(3)
    edge = 0.2
    for _ in range(500):
        m, t, g = (int(v) for v in rng.integers(0, 2 ** 20, size=3))
        n = int(rng.integers(2, 5000))
        seed = int(rng.integers(0, 2 ** 62))
        k, d, u = O.move_draws(seed, m, t, g, n, edge)
        w = O.philox([m, t, g, 0], seed)
        v = O.philox([m, t, g, 1], seed)
        assert k == (int(w[0]) * n) >> 32 and 0 <= k < n
        for a in range(3):
            # ((w + 1/2) 2^-32 - 1/2) is exact in FP64; one rounding in the product.
            exact = (mp.mpf(int(w[a + 1])) + mp.mpf(0.5)) / 2 ** 32 - mp.mpf(0.5)
            assert float(exact) == float(exact * 1)  # representable
            assert d[a] == float(exact) * edge
            assert -edge / 2 < d[a] < edge / 2
        assert u == (int(v[0]) + 0.5) / 2 ** 32 and 0.0 < u < 1.0


def test_straight_chain_energy_closed_form():
    # 2 r0 = 1.4 < r_c < 2.1 = 3 r0: only nearest and next-nearest pairs interact,
    # every bond sits at the FENE minimum.  E = (N-1) E_mod(r0) + (N-2) E_mod(2 r0).
    e1 = -1.0 - E_RC
    e2 = 4 * (1 / 128 ** 2 - 1 / 128) - E_RC
    for n in (2, 3, 13, 30, 55, 100, 129):
        want = (n - 1) * e1 + (n - 2) * e2
        got = O.energy(M, I.straight_chain(n))
        assert abs(got - want) <= 1e-12 * abs(want), (n, got, want)


def _brute_energy(xyz):
    """Eq. (4) in 50-digit arithmetic, both orders of every pair, halved."""
    mp.mp.dps = 50
    sig, rc, eps, K, R, r0 = (mp.mpf(M[k]) for k in
                              ("sigma", "r_cut", "epsilon", "fene_k", "fene_R", "fene_r0"))
    def elj(r):
        return 4 * eps * ((sig / r) ** 12 - (sig / r) ** 6)
    n = len(xyz)
    pts = [[mp.mpf(float(v)) for v in p] for p in xyz]
    tot = mp.mpf(0)
    for i in range(n):
        for j in range(n):
            if i != j:
                r = mp.sqrt(sum((pts[i][a] - pts[j][a]) ** 2 for a in range(3)))
                tot += (elj(min(r, rc)) - elj(rc)) / 2
    for i in range(n - 1):
        r = mp.sqrt(sum((pts[i][a] - pts[i + 1][a]) ** 2 for a in range(3)))
        tot += -K / 2 * R ** 2 * mp.log(1 - ((r - r0) / R) ** 2)
    return tot


def test_energy_matches_high_precision_sum():
    rng = np.random.default_rng(5)
    for n in (2, 3, 4, 5, 7, 9):
        xyz = I.random_walk(n, rng)
        xyz += rng.uniform(-0.05, 0.05, xyz.shape)  # break exact bond lengths
        got = O.energy(M, xyz)
        want = _brute_energy(xyz)
        assert abs(got - float(want)) <= 1e-13 * max(1.0, abs(float(want))), (n, got, want)


def test_delta_e_equals_full_recompute():
    rng = np.random.default_rng(9)
    for n in (2, 3, 13, 30, 64, 65, 100):
        for trial in range(12):
            xyz = I.random_walk(n, rng) + rng.uniform(-0.03, 0.03, (n, 3))
            k = [0, n - 1, int(rng.integers(0, n))][trial % 3]
            rn = xyz[k] + rng.uniform(-0.1, 0.1, 3)
            e0 = O.energy(M, xyz)
            x1 = xyz.copy()
            x1[k] = rn
            e1 = O.energy(M, x1)
            de = O.delta_e(M, xyz, k, rn)
            if not math.isfinite(e1):
                assert de == math.inf
                continue
            scale = 1.0 + abs(e0) + abs(e1)
            assert abs(de - (e1 - e0)) <= 1e-12 * scale, (n, k, de, e1 - e0)


def test_energy_translation_and_reflection_invariant():
    rng = np.random.default_rng(13)
    xyz = I.random_walk(40, rng)
    e = O.energy(M, xyz)
    assert abs(O.energy(M, xyz + np.array([0.25, -0.5, 1.0])) - e) < 1e-12 * abs(e)
    # A mirror image flips every coordinate difference sign: bitwise the same.
    assert O.energy(M, -xyz) == e
    # An axis swap changes the fma order of the squared distance: equal to rounding.
    assert abs(O.energy(M, xyz[:, [1, 0, 2]]) - e) <= 1e-12 * abs(e)


def test_shape_closed_forms():
    for n in (2, 5, 30, 100):
        ree2, rg2 = O.shape(I.straight_chain(n))
        b = 0.7
        assert abs(ree2 - (b * (n - 1)) ** 2) < 1e-12 * ree2
        assert abs(rg2 - b * b * (n * n - 1) / 12.0) < 1e-12 * rg2


def test_metropolis_rule_and_limits():
    rng = np.random.default_rng(17)
    us = (np.arange(20000) + 0.5) / 20000
    for x in (0.05, 0.7, 2.0, 5.0):
        acc = sum(O.metropolis(1.0, x, u) for u in us)
        assert abs(acc / len(us) - math.exp(-x)) < 2e-4
    for u in rng.random(200):
        assert O.metropolis(3.0, -1e-3, u) == 1       # downhill always
        assert O.metropolis(0.0, 1e6, u) == 1          # beta = 0 accepts finite moves
        assert O.metropolis(0.0, math.inf, u) == 0     # broken bond never accepted
        assert O.metropolis(1e9, 1e-3, u) == 0         # frozen: uphill never


def test_exchange_rule_and_limits():
    us = (np.arange(20000) + 0.5) / 20000
    for d in (0.1, 1.0, 3.0):
        # (beta_i - beta_j)(E_i - E_j) = -d
        acc = sum(O.exchange_accept(2.0, 1.0, 0.0, d, u) for u in us)
        assert abs(acc / len(us) - math.exp(-d)) < 2e-4
    for u in (1e-9, 0.5, 1 - 1e-9):
        assert O.exchange_accept(2.0, 1.0, -5.0, -5.0, u) == 1   # equal energies
        assert O.exchange_accept(1.5, 1.5, -1.0, 7.0, u) == 1    # equal temperatures
        assert O.exchange_accept(2.0, 1.0, 4.0, -1.0, u) == 1    # cold slot holds the higher E


def test_beta_zero_accepts_every_finite_move():
    w = I.make_workload([12], [1], [(1e300, 1e300)], "walk", 21, 0, "fp64")
    w.betas[:] = 0.0
    s = O.Simulation(w)
    xyz0 = s.coords.copy().reshape(-1, 3)
    log = s.run(30, accept_log=True)["accept_log"]
    # Replay the draws on a copy: accepted iff the move keeps both bonds finite.
    xyz = xyz0.copy()
    for t in range(30):
        for m in range(12):
            k, d, u = O.move_draws(w.seed, m, t, 0, 12, M["step_edge"])
            de = O.delta_e(M, xyz, k, xyz[k] + d)
            bit = (int(log[t, 0]) >> m) & 1
            assert bit == (1 if math.isfinite(de) else 0)
            if bit:
                xyz[k] = xyz[k] + d
    assert np.array_equal(xyz.ravel(), s.coords)


def test_frozen_chain_energy_never_increases():
    w = I.make_workload([20], [1], [(1e-9, 1e-9)], "walk", 23, 0, "fp64")
    s = O.Simulation(w)
    ser = s.run(200, series=True)["series"][:, 0, 0]
    assert np.all(np.diff(ser) <= 1e-12 * np.abs(ser[1:]))


def test_identical_replicas_always_exchange():
    w = I.make_workload([15], [6], [(0.2, 1.0)], "walk", 29, 0, "fp64")
    first = w.coords[:45].copy()
    w.coords = np.tile(first, 6)
    s = O.Simulation(w)
    row = s.exchange()
    assert list(row[:5]) == [1, 255, 1, 255, 1]
    assert list(s.perm) == [1, 0, 3, 2, 5, 4]


def test_resume_and_subset_reproduce_streams():
    w = I.named("c1", sweeps=0)
    a = O.Simulation(w)
    la = a.run(40, accept_log=True, exch_log=True)
    b = O.Simulation(w)
    lb1 = b.run(15, accept_log=True, exch_log=True)
    lb2 = b.run(25, accept_log=True, exch_log=True)
    assert np.array_equal(a.coords, b.coords) and np.array_equal(a.perm, b.perm)
    assert np.array_equal(la["accept_log"], np.concatenate([lb1["accept_log"], lb2["accept_log"]]))
    assert np.array_equal(la["exch_log"], np.concatenate([lb1["exch_log"], lb2["exch_log"]]))
    # A two-chain batch and its second chain alone draw the same streams.
    big = I.make_workload([13, 21], [4, 5], [(0.2, 1.0), (0.3, 2.0)], "walk", 31, 0, "fp64")
    sub = I.subset(big, [1])
    sb, ss = O.Simulation(big), O.Simulation(sub)
    lbig = sb.run(10, accept_log=True)["accept_log"]
    lsub = ss.run(10, accept_log=True)["accept_log"]
    assert np.array_equal(lbig[:, 4:], lsub)
    assert np.array_equal(sb.coords[4 * 13 * 3:], ss.coords)
