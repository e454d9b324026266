"""Host-side checks of libpt.so that need no GPU: the library loads, exports
every entry point that include/pt.h declares, and rejects bad models,
configurations and workspaces before touching the device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1107_3490_amd import inputs as I
from paper_1107_3490_amd import pt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "pt.h")).read()
    return sorted(set(re.findall(r"PT_API\s+[\w\s\*]+?\b(pt_\w+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(pt.LIB_PATH):
        from paper_1107_3490_amd import build
        build.build()
    return pt.lib()


def test_exports_match_header(L):
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(pt.EXPORTS)


def _cfg(w, precision=pt.PT_FP64):
    keep = dict(n_beads=np.array(w.n_beads, dtype=np.int32), n_slots=np.array(w.n_slots, dtype=np.int32),
                beta=np.ascontiguousarray(w.betas), coords=np.ascontiguousarray(w.coords))
    cfg = pt.PtConfig(n_chains=len(w.n_beads), n_beads=pt._ptr(keep["n_beads"], C.c_int32),
                      n_slots=pt._ptr(keep["n_slots"], C.c_int32), beta=pt._ptr(keep["beta"], C.c_double),
                      coords=pt._ptr(keep["coords"], C.c_double), stream_chain=None, stream_slot0=None,
                      seed=1, precision=precision, exchange_every=1, series_capacity=0, log_capacity=0,
                      schedule=0)
    return cfg, keep


def _init_rc(model, cfg, ws=0x100000, nbytes=1 << 40):
    h = C.c_void_p()
    rc = pt.lib().pt_init(C.byref(model), C.byref(cfg), C.c_void_p(ws), nbytes, None, C.byref(h))
    return rc, pt.lib().pt_last_error().decode()


def test_workspace_bytes_scales_with_config(L):
    m = pt.model_struct(I.model_params())
    w1 = I.make_workload([30], [16], [(0.1, 1.5)], "straight", 1, 0, "fp64")
    w2 = I.make_workload([30], [64], [(0.1, 1.5)], "straight", 1, 0, "fp64")
    c1, k1 = _cfg(w1)
    c2, k2 = _cfg(w2)
    b1, b2 = pt.pt_workspace_bytes(m, c1), pt.pt_workspace_bytes(m, c2)
    assert 0 < b1 < b2
    c1.log_capacity = 100
    assert pt.pt_workspace_bytes(m, c1) > b1


def test_rejects_bad_model_and_config(L):
    w = I.make_workload([30], [4], [(0.1, 1.5)], "straight", 1, 0, "fp64")
    cfg, keep = _cfg(w)
    for field, bad in (("sigma", 0.0), ("r_cut", float("nan")), ("fene_R", -1.0), ("step_edge", 0.0)):
        m = I.model_params()
        m[field] = bad
        rc, msg = _init_rc(pt.model_struct(m), cfg)
        assert rc == pt.PT_EINVAL and field in msg
    m = pt.model_struct(I.model_params())
    keep["beta"][2] = float("inf")
    rc, _ = _init_rc(m, cfg)
    assert rc == pt.PT_EINVAL
    keep["beta"][2] = 1.0
    keep["coords"][7] = float("nan")
    rc, msg = _init_rc(m, cfg)
    assert rc == pt.PT_EINVAL and "non-finite" in msg
    keep["coords"][7] = 0.0
    cfg.precision = 7
    assert _init_rc(m, cfg)[0] == pt.PT_EINVAL


def test_broken_starting_bond_is_a_domain_error(L):
    w = I.make_workload([10], [2], [(0.1, 1.5)], "straight", 1, 0, "fp64")
    w.coords[3 * 5:] += 0.31  # bond (4,5) stretched to 0.7 + 0.31*sqrt(3) > r0 + R
    cfg, keep = _cfg(w)
    rc, msg = _init_rc(pt.model_struct(w.model), cfg)
    assert rc == pt.PT_EDOMAIN and "bond (4,5)" in msg


def test_too_long_chain_and_small_workspace(L):
    m = pt.model_struct(I.model_params())
    w = I.make_workload([2049], [1], [(0.1, 1.5)], "straight", 1, 0, "fp64")
    cfg, keep = _cfg(w)
    assert _init_rc(m, cfg)[0] == pt.PT_EUNSUPPORTED
    w = I.make_workload([100], [3], [(0.1, 1.5)], "straight", 1, 0, "fp64")
    cfg, keep = _cfg(w)
    need = pt.pt_workspace_bytes(m, cfg)
    rc, msg = _init_rc(m, cfg, nbytes=need - 1)
    assert rc == pt.PT_ENOMEM
    rc, msg = _init_rc(m, cfg, ws=0x100010, nbytes=need)
    assert rc == pt.PT_EINVAL and "aligned" in msg


def test_mapping_override_is_validated(L):
    m = pt.model_struct(I.model_params())
    w = I.make_workload([100], [2], [(0.1, 1.5)], "straight", 1, 0, "fp64")
    cfg, keep = _cfg(w)
    base = pt.pt_workspace_bytes(m, cfg)
    assert base > 0
    for code, ok in ((0x21, True), (0x12, True), (0x14, True), (0x84, True), (0x11, False),
                     (0x31, False), (0x23, False), (0x121, True), (0x111, False), (0x221, True), (0x821, False),
                     (-1, False)):
        mp = np.array([code], dtype=np.int32)
        cfg.mapping = pt._ptr(mp, C.c_int32)
        n = L.pt_workspace_bytes(C.byref(m), C.byref(cfg))
        assert (n > 0) == ok, (hex(code), n, L.pt_last_error())
        if not ok:
            assert "mapping" in L.pt_last_error().decode()
    # a wider mapping pads the replica further: more workspace
    mp = np.array([0x84], dtype=np.int32)
    cfg.mapping = pt._ptr(mp, C.c_int32)
    assert L.pt_workspace_bytes(C.byref(m), C.byref(cfg)) > base


def test_packing_flags_are_validated(L):
    """Two or four replicas per wavefront take the layouts 16 B + 1 with B = 1
    or 2 (both precisions), one packing flag at a time, not with one lane per
    replica."""
    m = pt.model_struct(I.model_params())
    w = I.make_workload([60], [3], [(0.1, 1.5)], "straight", 1, 0, "mixed")
    cfg, keep = _cfg(w, precision=pt.PT_MIXED)
    for code, ok in ((pt.PT_MAP_PACK2 | 0x11, True), (pt.PT_MAP_PACK4 | 0x11, True), (pt.PT_MAP_PACK2 | 0x21, True),
                     (pt.PT_MAP_PACK4 | 0x21, True), (pt.PT_MAP_PACK2 | 0x12, False), (pt.PT_MAP_PACK4 | 0x41, False),
                     (pt.PT_MAP_PACK2 | pt.PT_MAP_PACK4 | 0x11, False), (pt.PT_MAP_LANE | pt.PT_MAP_PACK2 | 0x11, False),
                     (0x800 | 0x11, False)):
        mp = np.array([code], dtype=np.int32)
        cfg.mapping = pt._ptr(mp, C.c_int32)
        assert (L.pt_workspace_bytes(C.byref(m), C.byref(cfg)) > 0) == ok, hex(code)
        if not ok:
            assert "PT_MAP_PACK" in L.pt_last_error().decode()


def test_ablation_flags_are_validated(L):
    """One lane per replica runs the FP64 order only; the schedule is one of
    the four, the full-energy flag the only flag it takes."""
    m = pt.model_struct(I.model_params())
    w = I.make_workload([100], [2], [(0.1, 1.5)], "straight", 1, 0, "fp64")
    cfg, keep = _cfg(w, precision=pt.PT_MIXED)
    mp = np.array([pt.PT_MAP_LANE | 0x21], dtype=np.int32)
    cfg.mapping = pt._ptr(mp, C.c_int32)
    assert L.pt_workspace_bytes(C.byref(m), C.byref(cfg)) == 0
    assert "PT_MAP_LANE" in L.pt_last_error().decode()
    cfg.precision = pt.PT_FP64
    assert L.pt_workspace_bytes(C.byref(m), C.byref(cfg)) > 0
    cfg.mapping = None
    for sched, ok in ((pt.PT_SCHED_FULL_ENERGY, True), (pt.PT_SCHED_PER_SWEEP | pt.PT_SCHED_FULL_ENERGY, True),
                      (pt.PT_SCHED_PERSISTENT | pt.PT_SCHED_FULL_ENERGY, True), (pt.PT_SCHED_FLOW, True),
                      (pt.PT_SCHED_FLOW | pt.PT_SCHED_FULL_ENERGY, True), (4, False), (64, False),
                      (pt.PT_SCHED_FP64_ON_ACCEPT, True),
                      (pt.PT_SCHED_FLOW | pt.PT_SCHED_FP64_ON_ACCEPT | pt.PT_SCHED_FULL_ENERGY, True),
                      (pt.PT_SCHED_FULL_ENERGY | 4, False), (-1, False)):
        cfg.schedule = sched
        n = L.pt_workspace_bytes(C.byref(m), C.byref(cfg))
        assert (n > 0) == ok, (sched, n)
        if not ok:
            assert "schedule" in L.pt_last_error().decode()


def test_selftest_move_items_are_validated_on_the_host(L):
    """The move diagnostic (op 9) rejects a chain length outside 2..512 or a
    moved bead outside the chain before any device work."""
    m = pt.model_struct(I.model_params())
    x = np.zeros(pt.MOVE_ITEM)
    out = np.zeros(2)
    for nb, k in ((1, 0), (513, 0), (10, 10), (10, -1), (10.5, 1)):
        x[3 * 512:3 * 512 + 2] = [nb, k]
        rc = L.pt_selftest(C.byref(m), pt.OP_MOVE32, pt._ptr(x, C.c_double), None, pt._ptr(out, C.c_double), 1)
        assert rc == pt.PT_EINVAL and "op 9" in L.pt_last_error().decode()
    rc = L.pt_selftest(C.byref(m), 10, pt._ptr(x, C.c_double), None, pt._ptr(out, C.c_double), 1)
    assert rc == pt.PT_EINVAL
