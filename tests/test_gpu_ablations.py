"""The paper's alternative designs, run through the same C-ABI and checked to
the same bar as the main path: one lane per replica (the first GPU design of
Sec. 4.2) and the full energy recomputed after every sweep (Sec. 3.4).  Both
must leave every decision, coordinate and FP64-order energy bit-identical to
the oracle's; with the full recomputation the recorded per-sweep energy is the
FP64-order energy itself, so the whole series is bit-identical too."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1107_3490_amd import inputs as I

from test_gpu_parity import _assert_same_decisions, _assert_same_state, _pt, assert_parity, run_both, run_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    _pt().lib()  # raises if the HIP library is missing: no fallback
    yield


def _default_code(n):
    b = 1
    while b < 8 and 64 * b < n:
        b *= 2
    w = 1
    while 64 * w * b < n:
        w *= 2
    return 16 * b + w


def _oracle(w, sweeps):
    orc = O.Simulation(w)
    r = orc.run(sweeps, accept_log=True, exch_log=True, series=True)
    return dict(coords=orc.coords, energy=orc.energy, perm=orc.perm, alog=r["accept_log"],
                elog=r["exch_log"], series=r["series"], accepts=orc.accepts,
                exch_accepts=orc.exch_accepts, exch_tries=orc.exch_tries)


@pytest.mark.parametrize("case", ["uneven", "layouts", "n700", "n2048"])
def test_lane_per_replica_matches_oracle_and_wavefront_path(case):
    pt = _pt()
    if case == "uneven":
        # ragged lengths over several storage classes, 70 replicas: a partial
        # second wavefront of lanes
        w = I.make_workload([2, 13, 30, 64, 65, 100, 129], [10] * 7, [(0.2, 1.5)] * 7, "walk", 11, 0, "fp64")
        codes = [pt.PT_MAP_LANE | _default_code(n) for n in w.n_beads]
        sweeps = 15
    elif case == "layouts":
        # the same chain stored in wider (B, W) layouts than its default
        w = I.make_workload([100, 100, 100], [4, 4, 4], [(0.2, 1.5)] * 3, "walk", 12, 0, "fp64")
        codes = [pt.PT_MAP_LANE | 0x24, pt.PT_MAP_LANE | 0x42, pt.PT_MAP_LANE | 0x81]
        sweeps = 10
    elif case == "n700":
        w = I.make_workload([700], [4], [(0.3, 1.2)], "walk", 13, 0, "fp64")
        codes = [pt.PT_MAP_LANE | 0x82]
        sweeps = 3
    else:
        # the longest chain, in the widest layout
        w = I.make_workload([2048], [2], [(0.3, 1.2)], "walk", 18, 0, "fp64")
        codes = [pt.PT_MAP_LANE | 0x84]
        sweeps = 1
    print(f"\n[case] lane per replica {case}: N={list(w.n_beads)} codes={[hex(c) for c in codes]} "
          f"sweeps={sweeps}", flush=True)
    g = run_gpu(w, sweeps, "fp64", schedule=pt.PT_SCHED_AUTO, mapping=codes)
    assert np.all(g["persistent"] == 0)
    assert_parity(g, _oracle(w, sweeps), "fp64")
    # the wavefront kernels take the same sums: everything bit-identical,
    # running energies and bounds included
    _assert_same_state(g, run_gpu(w, sweeps, "fp64", schedule=pt.PT_SCHED_PER_SWEEP))


def test_lane_per_replica_is_fp64_only():
    pt = _pt()
    w = I.make_workload([30], [4], [(0.2, 1.5)], "walk", 14, 0, "mixed")
    with pytest.raises(pt.PtError) as ex:
        pt.Simulation(w, precision="mixed", mapping=[pt.PT_MAP_LANE | 0x11])
    assert "PT_MAP_LANE" in str(ex.value)


@pytest.mark.parametrize("variant", ["fp64-per-sweep", "fp64-persistent", "mixed-per-sweep",
                                     "mixed-persistent", "lane", "mixed-persistent-n2000"])
def test_full_energy_each_sweep_records_the_fp64_order_energy(variant):
    pt = _pt()
    prec = "mixed" if variant.startswith("mixed") else "fp64"
    sched = pt.PT_SCHED_PERSISTENT if "persistent" in variant else pt.PT_SCHED_PER_SWEEP
    if variant.endswith("n2000"):
        # four wavefronts share every FP64 energy (8 beads per lane)
        w = I.make_workload([2000], [4], [(0.3, 1.5)], "walk", 19, 0, prec)
        sweeps = 2
    else:
        w = I.make_workload([13, 55, 100, 300], [6, 6, 6, 4], [(0.2, 1.5)] * 4, "walk", 15, 0, prec)
        sweeps = 8
    mapping = [pt.PT_MAP_LANE | _default_code(n) for n in w.n_beads] if variant == "lane" else None
    print(f"\n[case] full energy each sweep, {variant}", flush=True)
    g = run_gpu(w, sweeps, prec, schedule=sched | pt.PT_SCHED_FULL_ENERGY, mapping=mapping)
    o = _oracle(w, sweeps)
    assert_parity(g, o, prec)
    assert np.array_equal(g["series"], o["series"]), "recorded energies are not the FP64-order energies"
    assert np.all(g["obs"]["counts"][:, 6] == sweeps)
    perm = g["obs"]["perm"]
    assert np.array_equal(g["e_run"][perm], o["energy"])
    # decisions and states equal those of the running-energy bookkeeping
    r = run_gpu(w, sweeps, prec, schedule=sched, mapping=mapping)
    for key in ("coords", "energy", "alog", "elog"):
        assert np.array_equal(g[key], r[key]), key
    assert np.array_equal(g["obs"]["perm"], r["obs"]["perm"])


@pytest.mark.parametrize("schedule", [1, 2, 3])
def test_fp64_on_accept_gives_fp64_accurate_running_energies(schedule):
    """Mixed precision with every accepted move re-scored in the FP64 order:
    the oracle's decisions and state, the same decisions as plain mixed, and
    running energies within 1e-9 of the FP64-order energy (the FP64 path's
    bar); every accepted move counts as re-scored."""
    pt = _pt()
    w = I.make_workload([13, 100, 300], [6, 6, 4], [(0.2, 2.0)] * 3, "walk", 23, 0, "mixed")
    sweeps = 10
    print(f"\n[case] FP64 on accept, schedule {schedule}", flush=True)
    g = run_gpu(w, sweeps, "mixed", schedule=schedule | pt.PT_SCHED_FP64_ON_ACCEPT)
    assert_parity(g, _oracle(w, sweeps), "fp64")
    counts = g["obs"]["counts"]
    assert np.all(counts[:, 3] >= counts[:, 0])
    _assert_same_decisions(g, run_gpu(w, sweeps, "mixed", schedule=schedule))


def test_autotune_considers_one_lane_per_replica_for_fp64():
    pt = _pt()
    w = I.make_workload([13, 30], [256, 64], [(0.2, 1.5)] * 2, "walk", 16, 0, "fp64")
    codes = pt.autotune(w, "fp64", trial_sweeps=3)
    print(f"\n[case] autotune fp64: {[hex(int(c)) for c in codes]}", flush=True)
    for n, c in zip(w.n_beads, codes):
        c = int(c)
        assert c & ~(0xFF | pt.PT_MAP_LANE | pt.PT_MAP_PACK2 | pt.PT_MAP_PACK4) == 0
        b, wv = (c >> 4) & 15, c & 15
        assert b in (1, 2, 4, 8) and wv in (1, 2, 4) and n <= 64 * b * wv
    _assert_same_state(run_gpu(w, 5, "fp64", mapping=codes), run_gpu(w, 5, "fp64"))


@pytest.mark.parametrize("n", [2, 3, 4, 13, 54, 55, 64, 65, 100, 129, 700, 2048])
def test_pair_per_thread_energy_is_within_its_bound(n):
    """The paper's one-pair-per-thread energy (even N with the middle round
    taken once) against the oracle's FP64-order energy: within the sum of the
    two rigorous bounds, and 1e-12 relative.  A dropped or doubled row (the
    printed enumeration's even-N round) is many orders above the bound."""
    pt = _pt()
    w = I.make_workload([n], [6], [(0.2, 1.5)], "walk", 17 + n, 0, "fp64")
    s = pt.Simulation(w, precision="fp64")
    s.sweep(3)
    e0, b0, _ = s.energy_method(pt.PT_ENERGY_FP64_ORDER)
    e1, b1, ms = s.energy_method(pt.PT_ENERGY_PAIR_PER_THREAD)
    exact = s.energy()
    s.close()
    orc = O.Simulation(w)
    orc.run(3)
    want = orc.slot_energies()
    print(f"\n[case] pair-per-thread energy N={n}: max |diff| {np.max(np.abs(e1 - want)):.3e}, "
          f"bound {b1.max():.3e}, kernel {ms:.3f} ms", flush=True)
    assert np.array_equal(e0, want) and np.array_equal(exact, want)
    assert np.all(b0 > 0) and np.all(b1 > 0)
    assert np.all(np.abs(e1 - want) <= b1 + b0)
    assert np.all(np.abs(e1 - want) <= 1e-12 * np.maximum(1.0, np.abs(want)))
