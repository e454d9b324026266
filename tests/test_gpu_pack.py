"""Several replicas per wavefront (PT_MAP_PACK2 / PT_MAP_PACK4): two or four
replicas of a short chain share a wavefront, 32 or 16 lanes each.  Decisions,
coordinates, FP64-order energies, shape series, running energies and their
bounds must equal the oracle's and those of the unpacked layout (16 B + 1)
bit for bit, for both precisions, with padded groups (slot counts that are
not multiples of the packing), with many mixed-path decisions sent to the
FP64 order (widened guard band), and with the full FP64-order energy every
sweep (which then makes the energy series equal the oracle's)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1107_3490_amd import inputs as I

from test_gpu_parity import _assert_same_state, _pt, assert_parity, run_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    _pt().lib()  # raises if the HIP library is missing: no fallback
    yield


def _oracle(w, sweeps):
    orc = O.Simulation(w)
    r = orc.run(sweeps, accept_log=True, exch_log=True, series=True)
    return dict(coords=orc.coords, energy=orc.energy, perm=orc.perm, alog=r["accept_log"],
                elog=r["exch_log"], series=r["series"], accepts=orc.accepts,
                exch_accepts=orc.exch_accepts, exch_tries=orc.exch_tries)


def _case(case, prec):
    if case == "n64":
        # every length of the 64-bead layout, slot counts 3..7 (padded groups)
        w = I.make_workload([2, 13, 30, 55, 64], [5, 6, 7, 3, 4], [(0.2, 1.5), (0.15, 1.0), (0.3, 2.0),
                                                                   (0.2, 1.2), (0.25, 1.5)],
                            "walk", 41, 0, prec)
        return w, [0x11] * 5, 24
    if case == "n128":
        w = I.make_workload([65, 100, 128, 90], [5, 3, 6, 2], [(0.2, 1.5), (0.3, 1.0), (0.2, 2.0), (0.4, 0.9)],
                            "walk", 42, 0, prec)
        return w, [0x21] * 4, 16
    # short chains stored in the wider layout (eight beads per lane at PACK4)
    w = I.make_workload([13, 40], [6, 5], [(0.2, 1.5), (0.3, 1.2)], "walk", 43, 0, prec)
    return w, [0x21, 0x21], 20


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
@pytest.mark.parametrize("pack", [2, 4])
@pytest.mark.parametrize("case", ["n64", "n128", "wide_layout"])
def test_packed_replicas_match_oracle_and_unpacked(case, pack, prec):
    pt = _pt()
    w, base, sweeps = _case(case, prec)
    flag = pt.PT_MAP_PACK2 if pack == 2 else pt.PT_MAP_PACK4
    codes = [flag | c for c in base]
    print(f"\n[case] packed {case} x{pack} {prec}: N={list(w.n_beads)} slots={list(w.n_slots)} "
          f"codes={[hex(c) for c in codes]} sweeps={sweeps}", flush=True)
    g = run_gpu(w, sweeps, prec, schedule=pt.PT_SCHED_AUTO, chunks=[sweeps // 3, sweeps - sweeps // 3],
                mapping=codes)
    assert np.all(g["persistent"] == 0)
    assert_parity(g, _oracle(w, sweeps), prec)
    _assert_same_state(g, run_gpu(w, sweeps, prec, schedule=pt.PT_SCHED_PER_SWEEP, mapping=base))


@pytest.mark.parametrize("pack", [2, 4])
def test_packed_mixed_rescoring_per_group(pack):
    """A widened guard band sends many moves of some replicas of a wavefront to
    the FP64 order while the other replicas keep their FP32 decisions."""
    pt = _pt()
    w = I.make_workload([30, 55], [7, 6], [(0.2, 1.5), (0.3, 1.0)], "walk", 44, 0, "mixed")
    sweeps = 12
    flag = pt.PT_MAP_PACK2 if pack == 2 else pt.PT_MAP_PACK4
    print(f"\n[case] packed x{pack} mixed, guard band x2^12", flush=True)
    g = run_gpu(w, sweeps, "mixed", mapping=[flag | 0x11] * 2, guard=2.0 ** 12)
    counts = g["obs"]["counts"]
    assert counts[:, 3].sum() > 0 and np.any(counts[:, 3] < counts[:, 5])
    assert_parity(g, _oracle(w, sweeps), "mixed")
    _assert_same_state(g, run_gpu(w, sweeps, "mixed", schedule=pt.PT_SCHED_PER_SWEEP, mapping=[0x11] * 2,
                                  guard=2.0 ** 12))


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_packed_full_energy_each_sweep(prec):
    """The FP64-order energy of a packed replica (each lane G rows of every
    64-row block) is the oracle's, bit for bit, after every sweep."""
    pt = _pt()
    w = I.make_workload([13, 55, 100], [5, 6, 3], [(0.2, 1.5)] * 3, "walk", 45, 0, prec)
    sweeps = 8
    codes = [pt.PT_MAP_PACK4 | 0x11, pt.PT_MAP_PACK2 | 0x11, pt.PT_MAP_PACK4 | 0x21]
    print(f"\n[case] packed full energy {prec}", flush=True)
    g = run_gpu(w, sweeps, prec, schedule=pt.PT_SCHED_PER_SWEEP | pt.PT_SCHED_FULL_ENERGY, mapping=codes)
    o = _oracle(w, sweeps)
    assert_parity(g, o, prec)
    assert np.array_equal(g["series"], o["series"])
    assert np.all(g["obs"]["counts"][:, 6] == sweeps)


def test_packing_rejects_other_layouts():
    pt = _pt()
    w = I.make_workload([100], [4], [(0.2, 1.5)], "walk", 46, 0, "mixed")
    for code in (pt.PT_MAP_PACK2 | 0x12, pt.PT_MAP_PACK4 | 0x41):
        with pytest.raises(pt.PtError) as ex:
            pt.Simulation(w, precision="mixed", mapping=[code])
        assert "PT_MAP_PACK" in str(ex.value)
