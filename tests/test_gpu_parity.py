"""GPU parity of libpt.so against the CPU oracle.

The contract (include/pt.h): accept/reject and exchange decisions are
bit-identical to the oracle's on the same Philox streams, so coordinates,
slot permutations and the FP64-order energies (pt_energy) are bit-identical
too; the running energies the kernels carry stay within their own rigorous
bound of the FP64-order energy, and for the plain FP64 path within 1e-9
relative of it.  Every case runs the oracle on the same seeded inputs.
"""
import math
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_1107_3490_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1107_3490_amd import pt
    pt.lib()  # raises if the HIP library is missing: no fallback
    yield


def _pt():
    from paper_1107_3490_amd import pt
    return pt


def run_gpu(w, sweeps, precision, schedule=0, chunks=None, mapping=None, guard=None):
    """Runs the library; returns every observable state.  chunks splits the
    sweeps over several pt_sweep calls; guard widens the guard bands."""
    pt = _pt()
    sim = pt.Simulation(w, precision=precision, series_capacity=sweeps, log_capacity=sweeps,
                        schedule=schedule, mapping=mapping)
    if guard is not None:
        sim.set_guard_scale(guard)
    for n in (chunks or [sweeps]):
        sim.sweep(n)
    g = dict(coords=sim.coords(), energy=sim.energy(), obs=sim.observables(), series=sim.series())
    g["alog"], g["elog"] = sim.logs()
    g["e_run"], g["b_run"] = sim.running()
    g["persistent"] = sim.mapping()[2]
    sim.close()
    return g


def run_both(w, sweeps, precision, label, schedule=0):
    print(f"\n[case] {label}: chains={len(w.n_beads)} N={sorted(set(w.n_beads))} "
          f"slots={w.total_slots} sweeps={sweeps} precision={precision} schedule={schedule}", flush=True)
    g = run_gpu(w, sweeps, precision, schedule)
    orc = O.Simulation(w)
    r = orc.run(sweeps, accept_log=True, exch_log=True, series=True)
    o = dict(coords=orc.coords, energy=orc.energy, perm=orc.perm, alog=r["accept_log"],
             elog=r["exch_log"], series=r["series"], accepts=orc.accepts,
             exch_accepts=orc.exch_accepts, exch_tries=orc.exch_tries)
    return g, o


def assert_parity(g, o, precision):
    # decisions: bit-identical logs
    assert g["alog"].shape == o["alog"].shape
    bad = np.argwhere(g["alog"] != o["alog"])
    assert bad.size == 0, f"accept logs differ first at (sweep, word) {bad[0]}"
    assert np.array_equal(g["elog"], o["elog"]), "exchange logs differ"
    assert np.array_equal(g["obs"]["perm"], o["perm"])
    assert np.array_equal(g["obs"]["counts"][:, 0], o["accepts"])
    assert np.array_equal(g["obs"]["counts"][:, 1], o["exch_tries"])
    assert np.array_equal(g["obs"]["counts"][:, 2], o["exch_accepts"])
    # state: bit-identical coordinates and FP64-order energies
    assert np.array_equal(g["coords"], o["coords"])
    assert np.array_equal(g["energy"], o["energy"])
    # per-sweep shape observables are FP64-order trees: bit-identical
    assert np.array_equal(g["series"][:, :, 1:], o["series"][:, :, 1:])
    # running energies: within their rigorous bound of the FP64-order energy
    perm = g["obs"]["perm"]
    e_slot, b_slot = g["e_run"][perm], g["b_run"][perm]
    err = np.abs(e_slot - o["energy"])
    assert np.all(err <= b_slot * (1 + 1e-6) + 1e-300), (err, b_slot)
    ser_err = np.abs(g["series"][:, :, 0] - o["series"][:, :, 0])
    rel = ser_err / np.maximum(1.0, np.abs(o["series"][:, :, 0]))
    print(f"  running-energy error vs FP64 order: max abs {ser_err.max():.3e}, "
          f"max rel {rel.max():.3e}; rescored moves {int(g['obs']['counts'][:, 3].sum())} of "
          f"{int(g['obs']['counts'][:, 5].sum())}; exchange recomputes {int(g['obs']['counts'][:, 4].sum())}",
          flush=True)
    if precision == "fp64":
        assert rel.max() <= 1e-9


def test_device_arithmetic_matches_host():
    pt = _pt()
    m = I.model_params()
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.random(200000) * 4, np.exp(rng.uniform(-700, 700, 100000)),
                        [0.0, 1.0, 2.0, 0.25, 5e-324, 1e-310, 1e300]])
    assert np.array_equal(pt.pt_selftest(m, pt.OP_SQRT, x), np.sqrt(x)), "FP64 sqrt not IEEE"
    y = np.exp(rng.uniform(-300, 300, x.size))
    with np.errstate(over="ignore"):
        keep = np.isfinite(x / y)
    x, y = x[keep], y[keep]
    assert np.array_equal(pt.pt_selftest(m, pt.OP_DIV, x, y), x / y), "FP64 division not IEEE"
    xs = np.concatenate([rng.random(20000), 1 - rng.random(5000) * 1e-3, np.exp(rng.uniform(-700, 700, 5000))])
    got = pt.pt_selftest(m, pt.OP_LOG, xs)
    want = np.array([O.plog(v) for v in xs])
    assert np.array_equal(got, want), "device log differs from the oracle's"
    r2 = np.concatenate([rng.uniform(0.1, 3.0, 20000), rng.uniform(0.16, 1.0, 20000),
                         [0.49, 0.36, 0.64, m["r_cut"] ** 2, 0.0]])
    c = O.consts(m)
    assert np.array_equal(pt.pt_selftest(m, pt.OP_LJ, r2), np.array([O.lib().orc_lj(c, v) for v in r2]))
    assert np.array_equal(pt.pt_selftest(m, pt.OP_FENE, r2), np.array([O.lib().orc_fene(c, v) for v in r2]))
    ctr = rng.integers(0, 2 ** 32, size=(4000, 4)).astype(np.float64)
    seed = 0x0123456789ABCDEF
    out = pt.pt_selftest(m, pt.OP_PHILOX, ctr.ravel(), [seed & 0xFFFFFFFF, seed >> 32]).reshape(-1, 4)
    want = np.array([O.philox([int(v) for v in row], seed) for row in ctr], dtype=np.float64)
    assert np.array_equal(out, want)


def test_fp64_sqrt_and_division_are_correctly_rounded_on_1e8_inputs():
    """The FP64 square root and division the kernels compile to (the bond
    length of Eq. 3, sigma^2/r^2 of Eq. 1, the log's s = f/(2+f)) are bitwise
    the host's IEEE results on 10^8 inputs each: half uniform bit patterns over
    all positive finite doubles (subnormals, overflow and underflow of the
    quotient included), half in the range of squared separations."""
    pt = _pt()
    m = I.model_params()
    for chunk in range(10):
        rng = np.random.default_rng(1000 + chunk)
        half = 5_000_000
        x = np.concatenate([rng.integers(1, 0x7FF0000000000000, size=half, dtype=np.int64).view(np.float64),
                            rng.random(half) * 10.0])
        y = np.concatenate([rng.integers(1, 0x7FF0000000000000, size=half, dtype=np.int64).view(np.float64),
                            rng.random(half) * 10.0 + 1e-3])
        print(f"\n[case] sqrt/div chunk {chunk}", flush=True)
        got = pt.pt_selftest(m, pt.OP_SQRT, x)
        bad = np.flatnonzero(got != np.sqrt(x))
        assert bad.size == 0, f"sqrt differs at x = {x[bad[:5]]!r}"
        with np.errstate(over="ignore", under="ignore"):
            want = x / y
        got = pt.pt_selftest(m, pt.OP_DIV, x, y)
        bad = np.flatnonzero(got != want)
        assert bad.size == 0, f"division differs at {list(zip(x[bad[:5]], y[bad[:5]]))!r}"


def _pairwise(v):
    while len(v) > 1:
        v = [v[i] + v[i + 1] for i in range(0, len(v), 2)]
    return v[0]


def test_wavefront_reduction_is_the_pairwise_tree():
    """The kernels' 64-lane reduction equals the pairwise tree over lanes, bit
    for bit, in FP64 and FP32 (values spanning many magnitudes and signs, so a
    different association order would show)."""
    pt = _pt()
    rng = np.random.default_rng(5)
    x = rng.standard_normal(64 * 200) * np.exp(rng.uniform(-30, 30, 64 * 200))
    got = pt.pt_selftest(I.model_params(), pt.OP_WAVE64, x).reshape(-1, 64)
    for grp, row in zip(x.reshape(-1, 64), got):
        want = _pairwise(list(grp))
        assert np.all(row == want)
    got32 = pt.pt_selftest(I.model_params(), pt.OP_WAVE32, x).reshape(-1, 64)
    for grp, row in zip(x.reshape(-1, 64), got32):
        want = _pairwise([np.float32(v) for v in grp])
        assert np.all(row == np.float64(want))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_c1_full_run(precision):
    w = I.named("c1")
    g, o = run_both(w, w.sweeps, precision, "c1 full")
    assert_parity(g, o, precision)


@pytest.mark.parametrize("n", [2, 3, 63, 64, 65, 129, 512, 513, 1024, 1025, 2048])
def test_edge_lengths(n):
    """Ragged and exact tile sizes of every (beads per lane, wavefronts) class,
    including the longest chain the kernels take."""
    w = I.make_workload([n], [5], [(0.2, 2.0)], "walk", 40 + n, 0, "fp64")
    sweeps = 25 if n < 500 else 3
    for prec in ("fp64", "mixed"):
        g, o = run_both(w, sweeps, prec, f"N={n}")
        assert_parity(g, o, prec)


def test_mapping_classes():
    pt = _pt()
    w = I.make_workload([13, 100, 300, 500, 600, 2000], [2] * 6, [(0.3, 1.0)] * 6, "walk", 5, 0, "mixed")
    sim = pt.Simulation(w)
    bpl, wpr, _ = sim.mapping()
    sim.close()
    assert list(bpl) == [1, 2, 8, 8, 8, 8] and list(wpr) == [1, 1, 1, 1, 2, 4]


def test_single_slot_and_no_exchange():
    w = I.make_workload([40, 17], [1, 3], [(0.5, 0.5), (0.3, 1.0)], "walk", 77, 0, "fp64",
                        exchange_every=0)
    g, o = run_both(w, 20, "mixed", "no exchange")
    assert_parity(g, o, "mixed")
    assert np.all(g["elog"] == 255)


def test_segment_split_and_explicit_exchange_are_deterministic():
    pt = _pt()
    w = I.make_workload([50, 30], [6, 4], [(0.2, 1.5), (0.3, 1.0)], "walk", 91, 0, "mixed",
                        exchange_every=3)
    a = pt.Simulation(w, log_capacity=40)
    a.sweep(33)
    b = pt.Simulation(w, log_capacity=40)
    for _ in range(33):
        b.sweep(1)
    assert np.array_equal(a.coords(), b.coords())
    assert np.array_equal(a.logs()[0], b.logs()[0])
    assert np.array_equal(a.observables()["perm"], b.observables()["perm"])
    # explicit exchange steps match the oracle's
    a.exchange()
    orc = O.Simulation(w)
    orc.run(33)
    orc.energy = orc.slot_energies()
    orc.exchange()
    assert np.array_equal(a.observables()["perm"], orc.perm)
    assert a.observables()["e"] == orc.e
    # and the run goes on from there alike
    a.sweep(10)
    orc.run(10)
    assert np.array_equal(a.observables()["perm"], orc.perm)
    assert np.array_equal(a.coords(), orc.coords)


def _assert_same_decisions(a, b):
    """Decisions, conformations, FP64-order energies and shape observables
    identical; the running energies may be rounded differently (each side
    within its own bound of the FP64-order energy)."""
    for key in ("coords", "energy", "alog", "elog"):
        assert np.array_equal(a[key], b[key]), key
    assert np.array_equal(a["series"][:, :, 1:], b["series"][:, :, 1:]), "series"
    assert np.array_equal(a["obs"]["perm"], b["obs"]["perm"]), "perm"
    assert np.array_equal(a["obs"]["counts"][:, :3], b["obs"]["counts"][:, :3]), "counts"
    for g in (a, b):
        perm = g["obs"]["perm"]
        assert np.all(np.abs(g["e_run"][perm] - g["energy"]) <= g["b_run"][perm] * (1 + 1e-6) + 1e-300)
    assert a["obs"]["t"] == b["obs"]["t"] and a["obs"]["e"] == b["obs"]["e"]


def _assert_same_state(a, b):
    for key in ("coords", "energy", "series", "alog", "elog", "e_run", "b_run"):
        assert np.array_equal(a[key], b[key]), key
    for key in ("perm", "counts", "acc"):
        assert np.array_equal(a["obs"][key], b["obs"][key]), key
    assert a["obs"]["t"] == b["obs"]["t"] and a["obs"]["e"] == b["obs"]["e"]


@pytest.mark.parametrize("schedule", [2, 3])
@pytest.mark.parametrize("case", ["c1", "c4", "uneven_every3", "n2048", "n700_odd", "two_widths",
                                  "two_widths_fp64"])
def test_persistent_schedule_equals_per_sweep(case, schedule):
    """The persistent kernel (one launch, pairwise exchange synchronisation)
    and the task flow (one launch, tasks taken in order, the later of a pair
    deciding) leave every output bit-identical to one sweep launch plus one
    exchange launch per sweep, also when the run is split over several calls.
    two_widths, two_widths_fp64: chains mapped to two and to one wavefront(s),
    two persistent launches per call (one per wavefront count, each block taking
    its chain's bead count per lane: 1, 2 and 4 at both widths in the FP64
    case), checked against the oracle too."""
    mapping = None
    if case == "two_widths":
        w = I.make_workload([300, 40, 250, 61], [6, 5, 4, 3], [(0.2, 1.5), (0.3, 1.0), (0.2, 2.0), (0.5, 0.9)],
                            "walk", 94, 0, "mixed")
        sweeps, prec, chunks, mapping = 30, "mixed", [7, 23], [0x42, 0x11, 0x42, 0x11]
    elif case == "two_widths_fp64":
        w = I.make_workload([100, 30, 200, 90, 13, 250], [4, 3, 5, 2, 4, 3],
                            [(0.2, 1.5), (0.3, 1.0), (0.2, 2.0), (0.5, 0.9), (0.3, 2.0), (0.25, 1.2)],
                            "walk", 95, 0, "fp64")
        sweeps, prec, chunks, mapping = 20, "fp64", [9, 11], [0x22, 0x12, 0x41, 0x21, 0x11, 0x42]
    elif case == "c1":
        w, sweeps, prec, chunks = I.named("c1"), 400, "mixed", [1, 150, 249]
    elif case == "c4":
        w, sweeps, prec, chunks = I.named("c4"), 6, "mixed", [2, 4]
    elif case == "uneven_every3":
        w = I.make_workload([50, 30, 9], [7, 4, 1], [(0.2, 1.5), (0.3, 1.0), (0.5, 0.5)], "walk", 93, 0,
                            "fp64", exchange_every=3)
        sweeps, prec, chunks = 40, "fp64", [5, 35]
    elif case == "n2048":
        w = I.make_workload([2048], [6], [(0.2, 2.0)], "walk", 17, 0, "mixed")
        sweeps, prec, chunks = 3, "mixed", [1, 2]
    else:
        w = I.make_workload([700], [9], [(0.2, 2.0)], "walk", 18, 0, "fp64")
        sweeps, prec, chunks = 4, "fp64", [4]
    print(f"\n[case] schedules {case} ({schedule}): slots={w.total_slots} sweeps={sweeps} {prec}", flush=True)
    a = run_gpu(w, sweeps, prec, schedule=1, mapping=mapping)
    b = run_gpu(w, sweeps, prec, schedule=schedule, chunks=chunks, mapping=mapping)
    assert np.all(a["persistent"] == 0) and np.all(b["persistent"] == (1 if schedule == 2 else 2))
    _assert_same_state(a, b)
    if case in ("two_widths", "two_widths_fp64"):
        o = O.Simulation(w)
        o.run(sweeps)
        assert np.array_equal(b["coords"], o.coords) and np.array_equal(b["obs"]["perm"], o.perm)
        if schedule == 2:
            sim = _pt().Simulation(w, precision=prec, schedule=schedule, mapping=mapping)
            launches = sim.time_sweeps(2)[2]
            sim.close()
            assert launches == 2


def test_flow_runs_classes_that_do_not_fit():
    """1024 replicas of N = 2000 do not fit on the device at once: the default
    schedule runs them as a task flow, with outputs bit-identical to one launch
    per sweep (the uneven start of the flow's tasks across sweeps included)."""
    w = I.make_workload([2000], [1024], [(0.3, 2.5)], "walk", 21, 0, "mixed")
    print(f"\n[case] task flow, 1024 replicas of N = 2000, 3 sweeps", flush=True)
    a = run_gpu(w, 3, "mixed", schedule=1)
    b = run_gpu(w, 3, "mixed", schedule=0, chunks=[1, 2])
    assert np.all(a["persistent"] == 0) and np.all(b["persistent"] == 2)
    _assert_same_state(a, b)


def test_thermodynamics_agree_with_oracle():
    """Per-temperature <E>, C_V/N, <R_gyr^2> and d<R_gyr^2>/dT of the mixed GPU
    run (from its running energies) lie within 2 sigma of the oracle's
    estimates, sigma being the oracle's binned / jackknife error, on the full
    small-chain run; the device accumulators agree with the series."""
    from oracle import thermo as OT
    from paper_1107_3490_amd import thermo as TH
    pt = _pt()
    w = I.named("c1")
    print(f"\n[case] thermodynamics c1: slots={w.total_slots} sweeps={w.sweeps}", flush=True)
    sim = pt.Simulation(w, precision="mixed", series_capacity=w.sweeps)
    sim.sweep(w.sweeps)
    ser, acc = sim.series(), sim.observables()["acc"]
    sim.close()
    orc = O.Simulation(w)
    r = orc.run(w.sweeps, series=True)
    nb = np.repeat(w.n_beads, w.n_slots)
    p = TH.estimates(ser, w.betas, nb)
    o = OT.estimates(r["series"], w.betas, nb)
    for g in range(w.total_slots):
        assert abs(p["E"][g] - o[g]["E"]) <= 2 * o[g]["dE"], (g, p["E"][g], o[g])
        assert abs(p["Cv"][g] - o[g]["Cv"]) <= 2 * o[g]["dCv"], (g, p["Cv"][g], o[g])
        assert abs(p["Rg2"][g] - o[g]["Rg2"]) <= 2 * o[g]["dRg2"], (g, p["Rg2"][g], o[g])
        # d<R_gyr^2>/dT (the paper's fluctuation of r_gyr^2, Eq. 8): the
        # package's estimate against the oracle's plain-loop estimator
        assert abs(p["dRg2dT"][g] - o[g]["dRg2dT"]) <= 2 * o[g]["ddRg2dT"], (g, p["dRg2dT"][g], o[g])
    a = TH.from_accumulators(acc, w.betas, nb)
    whole = TH.estimates(ser, w.betas, nb, burn_in=0.0, n_bins=25)
    assert np.all(a["n"] == w.sweeps)
    for k in ("E", "Rg2", "Ree2"):
        assert np.allclose(a[k], whole[k], rtol=1e-10, atol=1e-12), k


def _mix64(z):
    m = (1 << 64) - 1
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & m
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & m
    return z ^ (z >> 31)


def _digests_from_logs(w, alog, elog, e0=0):
    """Per-slot digests written out from the decision logs (independent of the
    library): accept words in order, then exchange outcomes of lower slots."""
    S = w.total_slots
    n_of = np.repeat(w.n_beads, w.n_slots)
    words = (n_of + 63) // 64
    off = np.concatenate([[0], np.cumsum(words)[:-1]])
    d = np.zeros((S, 2), dtype=object)
    d[:, :] = 0
    for g in range(S):
        for t in range(alog.shape[0]):
            for j in range(words[g]):
                d[g, 0] = _mix64(d[g, 0] ^ int(alog[t, off[g] + j]))
        for e in range(elog.shape[0]):
            if elog[e, g] != 255:
                d[g, 1] = _mix64(d[g, 1] ^ (((e0 + e) << 1) | int(elog[e, g])))
    return d.astype(np.uint64)


def test_digests_fold_the_oracle_decisions():
    """The device digests equal those folded from the oracle's logs, also for a
    run that keeps no logs on the device."""
    pt = _pt()
    w = I.make_workload([40, 130], [6, 5], [(0.2, 1.5), (0.3, 1.0)], "walk", 61, 0, "mixed")
    sweeps = 120
    print(f"\n[case] digests: slots={w.total_slots} sweeps={sweeps}", flush=True)
    orc = O.Simulation(w)
    r = orc.run(sweeps, accept_log=True, exch_log=True)
    want = _digests_from_logs(w, r["accept_log"], r["exch_log"])
    for sched in (1, 2):
        sim = pt.Simulation(w, precision="mixed", schedule=sched)
        sim.sweep(sweeps)
        got = sim.digests()
        sim.close()
        assert np.array_equal(got, want), sched


@pytest.mark.parametrize("scheds", [(2, 1), (3, 2), (1, 3)])
def test_checkpoint_resume_is_exact(scheds):
    """Save after 37 sweeps, restore into a new handle (other schedule and
    precision), run 23 more: everything equals the uninterrupted run."""
    pt = _pt()
    w = I.make_workload([70, 33], [7, 4], [(0.2, 1.5), (0.3, 1.0)], "walk", 62, 0, "mixed",
                        exchange_every=2)
    print(f"\n[case] checkpoint: slots={w.total_slots}, schedules {scheds}", flush=True)
    a = pt.Simulation(w, precision="mixed", schedule=scheds[0])
    a.sweep(37)
    st = a.state()
    a.sweep(23)
    b = pt.Simulation(w, precision="fp64", schedule=scheds[1])
    b.sweep(5)
    b.set_state(st)
    b.sweep(23)
    oa, ob = a.observables(), b.observables()
    assert np.array_equal(a.coords(), b.coords())
    assert np.array_equal(a.digests(), b.digests())
    assert np.array_equal(oa["perm"], ob["perm"])
    assert (oa["t"], oa["e"]) == (ob["t"], ob["e"]) == (60, 30)
    assert np.array_equal(oa["counts"][:, :3], ob["counts"][:, :3])
    assert np.array_equal(a.energy(), b.energy())
    # and the same decisions as the oracle
    orc = O.Simulation(w)
    orc.run(60)
    assert np.array_equal(a.coords(), orc.coords) and np.array_equal(oa["perm"], orc.perm)
    # a state of another batch is refused
    w2 = I.make_workload([70, 33], [7, 4], [(0.2, 1.5), (0.3, 1.0)], "walk", 62, 0, "mixed")
    w2.seed = w.seed + 1
    c = pt.Simulation(w2)
    with pytest.raises(pt.PtError) as ei:
        c.set_state(st)
    assert ei.value.code == pt.PT_EINVAL
    with pytest.raises(pt.PtError):
        b.set_state(b"\0" * len(st))
    for s in (a, b, c):
        s.close()


@pytest.mark.parametrize("n,codes", [(100, [0x21, 0x12, 0x41, 0x22, 0x14]),
                                     (300, [0x81, 0x42, 0x24, 0x44]),
                                     (700, [0x82, 0x44, 0x84])])
def test_results_do_not_depend_on_mapping(n, codes):
    """Every (beads per lane, wavefronts) mapping of a chain, under both
    schedules, gives bit-identical results (and the oracle's)."""
    w = I.make_workload([n], [5], [(0.2, 2.0)], "walk", 70 + n, 0, "mixed")
    sweeps = 12 if n < 500 else 4
    print(f"\n[case] mappings N={n}: {[hex(c) for c in codes]}", flush=True)
    ref = None
    for code in codes:
        for sched in (1, 2):
            g = run_gpu(w, sweeps, "mixed", schedule=sched, mapping=[code])
            if ref is None:
                ref = g
                o = O.Simulation(w)
                o.run(sweeps)
                assert np.array_equal(g["coords"], o.coords)
            else:
                _assert_same_state(ref, g)


def test_autotune_picks_valid_mappings():
    pt = _pt()
    w = I.subset(I.named("c4"), [0, 1, 2, 3, 4, 5, 6, 7], slots=8)
    print(f"\n[case] autotune: N={list(w.n_beads)}", flush=True)
    codes = pt.autotune(w, "mixed", trial_sweeps=5)
    print("  mapping", [hex(int(c)) for c in codes], flush=True)
    for n, c in zip(w.n_beads, codes):
        b, wv = int(c) >> 4, int(c) & 15
        assert b in (1, 2, 4, 8) and wv in (1, 2, 4) and n <= 64 * b * wv  # merged classes may be wider
    a = run_gpu(w, 6, "mixed", mapping=codes)
    d = run_gpu(w, 6, "mixed")
    _assert_same_state(a, d)


def test_thirteen_bead_transitions_where_the_paper_has_them():
    """Whole-path physics check (qualitative, no closed form): a parallel-
    tempering run of N = 13 puts the specific-heat peak (freezing) near
    T = 0.33 and the peak of d<R_gyr^2>/dT (collapse) near T = 1.0, as the
    paper reports for this chain (Sec. 4)."""
    from paper_1107_3490_amd import thermo as TH
    print("\n[case] N=13 thermodynamics, 64 slots, 100000 sweeps", flush=True)
    r = TH.scan(13, 0.1, 2.5, 64, 100000, seed=7)
    t_cv = r["T"][int(np.argmax(r["Cv"]))]
    # d<R_gyr^2>/dT also peaks at the freezing transition; the collapse peak is
    # the one above T = 0.5.
    hot = r["T"] > 0.5
    t_rg = r["T"][hot][int(np.argmax(r["dRg2dT"][hot]))]
    print(f"  C_V peak at T={t_cv:.3f}, d<Rg2>/dT peak at T={t_rg:.3f}", flush=True)
    assert 0.26 <= t_cv <= 0.40
    assert 0.75 <= t_rg <= 1.25


def test_fifty_five_bead_transitions_where_the_paper_has_them():
    """The paper's second chain (Sec. 4.1): for N = 55 the collapse peak of
    d<R_gyr^2>/dT lies near T = 1.5, and the specific heat peaks on the
    low-temperature (freezing) side, well below the collapse.  4x10^5 sweeps
    on 64 slots settle the collapse peak; the coldest slots of so short a run
    have not relaxed (the freezing peak reaches the paper's T = 0.32 only
    after some 3x10^6 sweeps), so for the specific heat only the side is
    checked."""
    from paper_1107_3490_amd import thermo as TH
    print("\n[case] N=55 thermodynamics, 64 slots, 400000 sweeps", flush=True)
    r = TH.scan(55, 0.15, 3.0, 64, 400000, seed=55)
    t_cv = r["T"][int(np.argmax(r["Cv"]))]
    hot = r["T"] > 0.6
    t_rg = r["T"][hot][int(np.argmax(r["dRg2dT"][hot]))]
    print(f"  C_V peak at T={t_cv:.3f}, d<Rg2>/dT peak above T=0.6 at T={t_rg:.3f}", flush=True)
    assert t_cv <= 0.45
    assert 1.25 <= t_rg <= 1.8


@pytest.mark.parametrize("schedule", [2, 3])
def test_persistent_wait_timeout_fails_cleanly_and_recovers(schedule):
    """A persistent or task-flow run whose waits give up after one poll: every
    block still exits, the next synchronising call reports PT_EHIP, further
    sweeps PT_ESTATE, and loading a saved state restores a run that goes on
    exactly like an undisturbed one."""
    pt = _pt()
    w = I.make_workload([60], [16], [(0.2, 1.5)], "walk", 63, 0, "mixed")
    print(f"\n[case] timeout of schedule {schedule}, 16 slots, spin limit 1", flush=True)
    ref = pt.Simulation(w, schedule=schedule)
    ref.sweep(30)
    a = pt.Simulation(w, schedule=schedule)
    a.sweep(10)
    st = a.state()
    a.set_spin_limit(1)
    a.sweep(20)
    with pytest.raises(pt.PtError) as ei:
        a.energy()
    assert ei.value.code == pt.PT_EHIP
    with pytest.raises(pt.PtError) as ei:
        a.sweep(1)
    assert ei.value.code == pt.PT_ESTATE
    a.set_spin_limit(1 << 24)
    a.set_state(st)
    a.sweep(20)
    assert np.array_equal(a.coords(), ref.coords())
    assert np.array_equal(a.digests(), ref.digests())
    a.close()
    ref.close()
