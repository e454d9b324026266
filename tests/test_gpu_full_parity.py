"""GPU parity against the CPU oracle at the full sizes of the workloads.

Each case runs the oracle once on the seeded input (accept and exchange logs,
per-sweep series) and compares several GPU runs with it: both precisions,
the schedules that apply (one launch per sweep, persistent, task flow), and a
mixed run whose guard bands are widened (pt_set_guard_scale) so that many
moves are re-scored in the FP64 order and many exchange decisions need the
FP64-order energies; every decision must stay identical.  The oracle takes
the longest here (a minute or so for the N = 500 and batched workloads on
16 host cores).

  c2  1 chain, N = 100, 64 slots, all 10^4 sweeps
  c3  1 chain, N = 500, 128 slots, all 2000 sweeps
  c4  48 uneven chains x 32 slots, 500 of its 5000 sweeps
  c5  one N = 2000 chain with all 256 slots, 20 sweeps, under the task flow
  paper protocol: N = 55, 64 slots, displacement edge 0.02 (Sec. 3.2),
      an exchange step every 1000 sweeps (Sec. 4.2), 2000 sweeps
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1107_3490_amd import inputs as I
from test_gpu_parity import assert_parity, run_gpu

pytestmark = pytest.mark.gpu

# Widening of the guard bands in the exercising runs: about 1 in 10^3 .. 10^2
# moves lands in the band, and exchange decisions need FP64 energies.
GUARD = 2.0 ** 14


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1107_3490_amd import pt
    pt.lib()  # raises if the HIP library is missing: no fallback
    yield


def oracle_run(w, sweeps):
    orc = O.Simulation(w)
    r = orc.run(sweeps, accept_log=True, exch_log=True, series=True)
    return dict(coords=orc.coords, energy=orc.energy, perm=orc.perm, alog=r["accept_log"],
                elog=r["exch_log"], series=r["series"], accepts=orc.accepts,
                exch_accepts=orc.exch_accepts, exch_tries=orc.exch_tries)


def check(w, sweeps, o, precision, label, schedule=0, mapping=None, guard=None, expect_mode=None):
    print(f"\n[case] {label}: precision={precision} schedule={schedule} guard={guard} "
          f"mapping={None if mapping is None else [hex(int(c)) for c in mapping]}", flush=True)
    g = run_gpu(w, sweeps, precision, schedule=schedule, mapping=mapping, guard=guard)
    assert_parity(g, o, precision)
    counts = g["obs"]["counts"]
    rescored, exch_fp64 = int(counts[:, 3].sum()), int(counts[:, 4].sum())
    if precision == "mixed":
        assert rescored > 0, "no move was re-scored in the FP64 order"
    if guard is not None:
        assert rescored > 0 and exch_fp64 > 0, (rescored, exch_fp64)
    if expect_mode is not None:
        assert np.all(g["persistent"] == expect_mode), g["persistent"]
    return g


@pytest.fixture(scope="module")
def c2():
    w = I.named("c2")
    print(f"\n[oracle] c2: {w.sweeps} sweeps", flush=True)
    return w, oracle_run(w, w.sweeps)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("schedule,mode", [(2, 1), (1, 0)])
@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_c2_all_sweeps(c2, precision, schedule, mode):
    w, o = c2
    check(w, w.sweeps, o, precision, "c2 full", schedule=schedule, expect_mode=mode)


@pytest.mark.timeout(900)
def test_c2_all_sweeps_wide_band(c2):
    w, o = c2
    check(w, w.sweeps, o, "mixed", "c2 full, widened band", guard=GUARD)


@pytest.fixture(scope="module")
def c3():
    w = I.named("c3")
    print(f"\n[oracle] c3: {w.sweeps} sweeps", flush=True)
    return w, oracle_run(w, w.sweeps)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("precision,guard", [("mixed", None), ("fp64", None), ("mixed", GUARD)])
def test_c3_all_sweeps(c3, precision, guard):
    w, o = c3
    check(w, w.sweeps, o, precision, "c3 full", guard=guard, expect_mode=1)


C4_SWEEPS = 500


@pytest.fixture(scope="module")
def c4():
    w = I.named("c4")
    print(f"\n[oracle] c4: {C4_SWEEPS} sweeps", flush=True)
    return w, oracle_run(w, C4_SWEEPS)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("variant", ["default", "uniform_w2", "fp64", "wide_band"])
def test_c4_batched_500_sweeps(c4, variant):
    """All 48 chains in persistent launches (one per wavefront count), also with
    every chain at two wavefronts per replica (one launch for all bead counts)."""
    w, o = c4
    mapping = None
    if variant == "uniform_w2":
        mapping = []
        for n in w.n_beads:
            b = 1
            while 128 * b < n:
                b *= 2
            mapping.append(16 * b + 2)
    prec = "fp64" if variant == "fp64" else "mixed"
    guard = GUARD if variant == "wide_band" else None
    check(w, C4_SWEEPS, o, prec, f"c4 {variant}", mapping=mapping, guard=guard, expect_mode=1)


C5_SWEEPS = 20


@pytest.fixture(scope="module")
def c5():
    w = I.subset(I.named("c5"), [7])  # chain 7: all 256 slots, its own streams
    print(f"\n[oracle] c5 chain 7, 256 slots: {C5_SWEEPS} sweeps", flush=True)
    return w, oracle_run(w, C5_SWEEPS)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("precision,schedule,mode", [("mixed", 3, 2), ("fp64", 3, 2), ("mixed", 0, 1)])
def test_c5_chain_all_slots(c5, precision, schedule, mode):
    """The task-flow kernel of the large workload (PT_SCHED_FLOW) and the
    persistent one, each against the oracle on a full-size chain."""
    w, o = c5
    check(w, C5_SWEEPS, o, precision, "c5 chain 7", schedule=schedule, expect_mode=mode)


@pytest.fixture(scope="module")
def protocol():
    w = I.make_workload([55], [64], [(0.1, 1.5)], "straight", 55, 2000, "mixed",
                        name="paper-protocol", step_edge=0.02, exchange_every=1000)
    print(f"\n[oracle] paper protocol: {w.sweeps} sweeps", flush=True)
    return w, oracle_run(w, w.sweeps)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_paper_protocol_n55(protocol, precision):
    w, o = protocol
    g = check(w, w.sweeps, o, precision, "N=55 edge 0.02 exchange every 1000")
    assert g["elog"].shape[0] == 2  # exchange steps after sweeps 999 and 1999
