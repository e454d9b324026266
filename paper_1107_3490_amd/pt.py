"""Python binding of libpt.so (C ABI in include/pt.h).

Argument marshalling only: every step of the simulation runs in the HIP
library.  PyTorch provides the device workspace and the stream.  The module
refuses to work without the built library (``python -m
paper_1107_3490_amd.build``); there is no fallback path.

The functions ``pt_workspace_bytes``, ``pt_init``, ``pt_sweep``,
``pt_exchange``, ``pt_energy``, ``pt_observables`` ... mirror the C calls
one to one; :class:`Simulation` bundles them for a
:class:`paper_1107_3490_amd.inputs.Workload`.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpt.so")

PT_OK, PT_EINVAL, PT_EDOMAIN, PT_ENOMEM, PT_EHIP, PT_ESTATE, PT_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
PT_FP64, PT_MIXED = 0, 1
PT_SCHED_AUTO, PT_SCHED_PER_SWEEP, PT_SCHED_PERSISTENT, PT_SCHED_FLOW = 0, 1, 2, 3
# The paper's alternative designs (see include/pt.h): or-ed into the schedule
# (full energy after every sweep) or into a chain's mapping code (one lane per
# replica, FP64 only).
PT_SCHED_FULL_ENERGY, PT_SCHED_FP64_ON_ACCEPT, PT_MAP_LANE = 16, 32, 0x100
PT_MAP_PACK2, PT_MAP_PACK4 = 0x200, 0x400
PT_ENERGY_FP64_ORDER, PT_ENERGY_PAIR_PER_THREAD = 0, 1

# Diagnostic ops of pt_selftest.
OP_SQRT, OP_DIV, OP_LOG, OP_FENE, OP_LJ, OP_LJ32, OP_PHILOX, OP_WAVE64, OP_WAVE32, OP_MOVE32 = range(10)
MOVE_ITEM = 3 * 512 + 8  # doubles per OP_MOVE32 item

EXPORTS = ("pt_workspace_bytes", "pt_init", "pt_autotune", "pt_sweep", "pt_exchange", "pt_energy",
           "pt_energy_method",
           "pt_observables", "pt_reset_observables", "pt_get_coords", "pt_get_running",
           "pt_get_series", "pt_get_logs", "pt_get_digests", "pt_state_bytes", "pt_get_state",
           "pt_set_state", "pt_set_spin_limit", "pt_set_guard_scale", "pt_time_sweeps", "pt_get_mapping", "pt_selftest", "pt_selftest_noalloc", "pt_destroy",
           "pt_last_error")


class PtError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"pt error {code}: {msg}")
        self.code = code


class PtModel(C.Structure):
    _fields_ = [(n, C.c_double) for n in
                ("epsilon", "sigma", "r_cut", "fene_k", "fene_R", "fene_r0", "step_edge")]


class PtConfig(C.Structure):
    _fields_ = [("n_chains", C.c_int32), ("n_beads", C.POINTER(C.c_int32)),
                ("n_slots", C.POINTER(C.c_int32)), ("beta", C.POINTER(C.c_double)),
                ("coords", C.POINTER(C.c_double)), ("stream_chain", C.POINTER(C.c_uint32)),
                ("stream_slot0", C.POINTER(C.c_uint32)), ("seed", C.c_uint64),
                ("precision", C.c_int32), ("exchange_every", C.c_int32),
                ("series_capacity", C.c_int64), ("log_capacity", C.c_int64),
                ("schedule", C.c_int32), ("mapping", C.POINTER(C.c_int32))]


_lib = None


def lib():
    """The loaded libpt.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1107_3490_amd.build`")
        L = C.CDLL(LIB_PATH)
        P = C.POINTER
        L.pt_workspace_bytes.argtypes = [P(PtModel), P(PtConfig)]
        L.pt_workspace_bytes.restype = C.c_size_t
        L.pt_init.argtypes = [P(PtModel), P(PtConfig), C.c_void_p, C.c_size_t, C.c_void_p, P(C.c_void_p)]
        L.pt_sweep.argtypes = [C.c_void_p, C.c_int64]
        L.pt_exchange.argtypes = [C.c_void_p]
        L.pt_energy.argtypes = [C.c_void_p, P(C.c_double)]
        L.pt_observables.argtypes = [C.c_void_p, P(C.c_double), P(C.c_int64), P(C.c_int32), P(C.c_int64)]
        L.pt_reset_observables.argtypes = [C.c_void_p]
        L.pt_get_coords.argtypes = [C.c_void_p, P(C.c_double)]
        L.pt_get_running.argtypes = [C.c_void_p, P(C.c_double), P(C.c_double)]
        L.pt_get_series.argtypes = [C.c_void_p, P(C.c_double), P(C.c_int64)]
        L.pt_get_logs.argtypes = [C.c_void_p, P(C.c_uint64), P(C.c_int64), P(C.c_uint8), P(C.c_int64)]
        L.pt_time_sweeps.argtypes = [C.c_void_p, C.c_int64, P(C.c_double), P(C.c_double), P(C.c_int64)]
        L.pt_get_mapping.argtypes = [C.c_void_p, P(C.c_int32), P(C.c_int32), P(C.c_int32)]
        L.pt_get_digests.argtypes = [C.c_void_p, P(C.c_uint64)]
        L.pt_autotune.argtypes = [P(PtModel), P(PtConfig), C.c_int32, C.c_void_p, P(C.c_int32)]
        L.pt_state_bytes.argtypes = [C.c_void_p]
        L.pt_state_bytes.restype = C.c_size_t
        L.pt_get_state.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t]
        L.pt_set_state.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t]
        L.pt_set_spin_limit.argtypes = [C.c_void_p, C.c_uint32]
        L.pt_set_guard_scale.argtypes = [C.c_void_p, C.c_double]
        L.pt_selftest.argtypes = [P(PtModel), C.c_int, P(C.c_double), P(C.c_double), P(C.c_double), C.c_int64]
        L.pt_selftest_noalloc.argtypes = [P(PtModel), C.c_int, P(C.c_double), P(C.c_double), P(C.c_double),
                                          C.c_int64]
        L.pt_destroy.argtypes = [C.c_void_p]
        L.pt_destroy.restype = None
        L.pt_last_error.argtypes = []
        L.pt_last_error.restype = C.c_char_p
        for name in EXPORTS:
            if name not in ("pt_workspace_bytes", "pt_state_bytes", "pt_destroy", "pt_last_error"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(rc: int) -> None:
    if rc != PT_OK:
        raise PtError(rc, lib().pt_last_error().decode())


def _ptr(a: np.ndarray, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def model_struct(model: dict) -> PtModel:
    return PtModel(**{k: float(model[k]) for k in
                      ("epsilon", "sigma", "r_cut", "fene_k", "fene_R", "fene_r0", "step_edge")})


# ----------------------------------------------------------- C-ABI mirrors --

def pt_workspace_bytes(model: PtModel, cfg: PtConfig) -> int:
    return int(lib().pt_workspace_bytes(C.byref(model), C.byref(cfg)))


def pt_init(model: PtModel, cfg: PtConfig, d_workspace: int, ws_bytes: int, stream: int) -> int:
    h = C.c_void_p()
    _check(lib().pt_init(C.byref(model), C.byref(cfg), C.c_void_p(d_workspace), ws_bytes,
                         C.c_void_p(stream), C.byref(h)))
    return h.value


def pt_sweep(h: int, n: int) -> None:
    _check(lib().pt_sweep(C.c_void_p(h), int(n)))


def pt_exchange(h: int) -> None:
    _check(lib().pt_exchange(C.c_void_p(h)))


def pt_energy(h: int, out: np.ndarray) -> None:
    _check(lib().pt_energy(C.c_void_p(h), _ptr(out, C.c_double)))


def pt_energy_method(h: int, method: int, out: np.ndarray, bound: np.ndarray) -> float:
    ms = C.c_double(0.0)
    _check(lib().pt_energy_method(C.c_void_p(h), int(method), _ptr(out, C.c_double),
                                  _ptr(bound, C.c_double), C.byref(ms)))
    return ms.value


def pt_observables(h: int, acc, counts, perm, te) -> None:
    _check(lib().pt_observables(C.c_void_p(h),
                                _ptr(acc, C.c_double) if acc is not None else None,
                                _ptr(counts, C.c_int64) if counts is not None else None,
                                _ptr(perm, C.c_int32) if perm is not None else None,
                                _ptr(te, C.c_int64) if te is not None else None))


def pt_reset_observables(h: int) -> None:
    _check(lib().pt_reset_observables(C.c_void_p(h)))


def pt_get_coords(h: int, out: np.ndarray) -> None:
    _check(lib().pt_get_coords(C.c_void_p(h), _ptr(out, C.c_double)))


def pt_get_running(h: int, e: np.ndarray, b: np.ndarray) -> None:
    _check(lib().pt_get_running(C.c_void_p(h), _ptr(e, C.c_double), _ptr(b, C.c_double)))


def pt_get_series(h: int, out: Optional[np.ndarray]) -> int:
    rows = C.c_int64()
    _check(lib().pt_get_series(C.c_void_p(h), _ptr(out, C.c_double) if out is not None else None,
                               C.byref(rows)))
    return rows.value


def pt_get_logs(h: int, alog: Optional[np.ndarray], elog: Optional[np.ndarray]):
    ra, re = C.c_int64(), C.c_int64()
    _check(lib().pt_get_logs(C.c_void_p(h), _ptr(alog, C.c_uint64) if alog is not None else None,
                             C.byref(ra), _ptr(elog, C.c_uint8) if elog is not None else None,
                             C.byref(re)))
    return ra.value, re.value


def pt_time_sweeps(h: int, n: int):
    sw, tot, la = C.c_double(), C.c_double(), C.c_int64()
    _check(lib().pt_time_sweeps(C.c_void_p(h), int(n), C.byref(sw), C.byref(tot), C.byref(la)))
    return sw.value, tot.value, la.value


def pt_get_mapping(h: int, n_chains: int):
    bpl = np.zeros(n_chains, dtype=np.int32)
    wpr = np.zeros(n_chains, dtype=np.int32)
    per = np.zeros(n_chains, dtype=np.int32)
    _check(lib().pt_get_mapping(C.c_void_p(h), _ptr(bpl, C.c_int32), _ptr(wpr, C.c_int32),
                                _ptr(per, C.c_int32)))
    return bpl, wpr, per


def pt_get_digests(h: int, n_slots: int) -> np.ndarray:
    out = np.zeros((n_slots, 2), dtype=np.uint64)
    _check(lib().pt_get_digests(C.c_void_p(h), _ptr(out, C.c_uint64)))
    return out


def pt_get_state(h: int) -> bytes:
    n = lib().pt_state_bytes(C.c_void_p(h))
    if n == 0:
        _check(PT_EINVAL)
    buf = C.create_string_buffer(n)
    _check(lib().pt_get_state(C.c_void_p(h), buf, n))
    return buf.raw


def pt_set_state(h: int, state: bytes) -> None:
    buf = C.create_string_buffer(bytes(state), len(state))
    _check(lib().pt_set_state(C.c_void_p(h), buf, len(state)))


def pt_selftest(model: dict, op: int, x, y=None) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64)
    n = x.size // 4 if op == OP_PHILOX else (x.size // MOVE_ITEM if op == OP_MOVE32 else x.size)
    yy = np.ascontiguousarray(y, dtype=np.float64) if y is not None else None
    nout = 2 * n if op in (OP_LJ32, OP_MOVE32) else (4 * n if op == OP_PHILOX else n)
    out = np.zeros(nout)
    _check(lib().pt_selftest(C.byref(model_struct(model)), op, _ptr(x, C.c_double),
                             _ptr(yy, C.c_double) if yy is not None else None,
                             _ptr(out, C.c_double), n))
    return out


def pt_selftest_noalloc(model: dict, op: int, x, y=None) -> np.ndarray:
    """pt_selftest through the entry point that allocates no device memory."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    n = x.size // 4 if op == OP_PHILOX else (x.size // MOVE_ITEM if op == OP_MOVE32 else x.size)
    yy = np.ascontiguousarray(y, dtype=np.float64) if y is not None else None
    nout = 2 * n if op in (OP_LJ32, OP_MOVE32) else (4 * n if op == OP_PHILOX else n)
    out = np.zeros(nout)
    _check(lib().pt_selftest_noalloc(C.byref(model_struct(model)), op, _ptr(x, C.c_double),
                                     _ptr(yy, C.c_double) if yy is not None else None,
                                     _ptr(out, C.c_double), n))
    return out


def pt_destroy(h: int) -> None:
    lib().pt_destroy(C.c_void_p(h))


def autotune(w, precision: Optional[str] = None, schedule: int = PT_SCHED_AUTO,
             trial_sweeps: int = 20) -> np.ndarray:
    """pt_autotune on workload w: one mapping code (16 B + W, possibly
    | PT_MAP_PACK2 or PT_MAP_PACK4, or | PT_MAP_LANE for FP64) per chain."""
    import torch

    prec = precision or w.precision
    nb = np.array(w.n_beads, dtype=np.int32)
    ns = np.array(w.n_slots, dtype=np.int32)
    beta = np.ascontiguousarray(w.betas, dtype=np.float64)
    xyz = np.ascontiguousarray(w.coords, dtype=np.float64)
    sc = np.array(w.stream_chain, dtype=np.uint32) if w.stream_chain is not None else None
    ss = np.array(w.stream_slot0, dtype=np.uint32) if w.stream_slot0 is not None else None
    cfg = PtConfig(n_chains=len(w.n_beads), n_beads=_ptr(nb, C.c_int32), n_slots=_ptr(ns, C.c_int32),
                   beta=_ptr(beta, C.c_double), coords=_ptr(xyz, C.c_double),
                   stream_chain=_ptr(sc, C.c_uint32) if sc is not None else None,
                   stream_slot0=_ptr(ss, C.c_uint32) if ss is not None else None,
                   seed=int(w.seed), precision=PT_MIXED if prec == "mixed" else PT_FP64,
                   exchange_every=int(w.exchange_every), series_capacity=0, log_capacity=0,
                   schedule=int(schedule))
    out = np.zeros(len(w.n_beads), dtype=np.int32)
    stream = torch.cuda.current_stream()
    _check(lib().pt_autotune(C.byref(model_struct(w.model)), C.byref(cfg), int(trial_sweeps),
                             C.c_void_p(stream.cuda_stream), _ptr(out, C.c_int32)))
    return out


# ------------------------------------------------------------ convenience --

class Simulation:
    """A workload on the GPU: workspace, handle and typed read-backs."""

    def __init__(self, w, precision: Optional[str] = None, series_capacity: int = 0,
                 log_capacity: int = 0, device: str = "cuda", schedule: int = PT_SCHED_AUTO,
                 mapping=None):
        import torch

        self.w = w
        prec = precision or w.precision
        self.n_beads = np.array(w.n_beads, dtype=np.int32)
        self.n_slots = np.array(w.n_slots, dtype=np.int32)
        self.beta = np.ascontiguousarray(w.betas, dtype=np.float64)
        self.coords0 = np.ascontiguousarray(w.coords, dtype=np.float64)
        self.total = int(self.n_slots.sum())
        self.words = int(sum(((n + 63) // 64) * r for n, r in zip(w.n_beads, w.n_slots)))
        self._sc = (np.array(w.stream_chain, dtype=np.uint32) if w.stream_chain is not None else None)
        self._ss = (np.array(w.stream_slot0, dtype=np.uint32) if w.stream_slot0 is not None else None)
        self.model = model_struct(w.model)
        self.cfg = PtConfig(
            n_chains=len(w.n_beads), n_beads=_ptr(self.n_beads, C.c_int32),
            n_slots=_ptr(self.n_slots, C.c_int32), beta=_ptr(self.beta, C.c_double),
            coords=_ptr(self.coords0, C.c_double),
            stream_chain=_ptr(self._sc, C.c_uint32) if self._sc is not None else None,
            stream_slot0=_ptr(self._ss, C.c_uint32) if self._ss is not None else None,
            seed=int(w.seed), precision=PT_MIXED if prec == "mixed" else PT_FP64,
            exchange_every=int(w.exchange_every), series_capacity=int(series_capacity),
            log_capacity=int(log_capacity), schedule=int(schedule))
        self._map = None
        if mapping is not None:
            self._map = np.ascontiguousarray(mapping, dtype=np.int32)
            if self._map.shape != (len(w.n_beads),):
                raise ValueError("mapping needs one code per chain")
            self.cfg.mapping = _ptr(self._map, C.c_int32)
        nbytes = pt_workspace_bytes(self.model, self.cfg)
        if nbytes == 0:
            _check(PT_EINVAL)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.stream = torch.cuda.current_stream(self.ws.device)
        self.series_capacity = int(series_capacity)
        self.log_capacity = int(log_capacity)
        self.h = pt_init(self.model, self.cfg, self.ws.data_ptr(), nbytes, self.stream.cuda_stream)

    def close(self):
        if getattr(self, "h", None):
            pt_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sweep(self, n: int = 1):
        pt_sweep(self.h, n)

    def exchange(self):
        pt_exchange(self.h)

    def energy(self) -> np.ndarray:
        out = np.zeros(self.total)
        pt_energy(self.h, out)
        return out

    def energy_method(self, method: int):
        """(energies, error bounds, kernel ms) per slot by PT_ENERGY_FP64_ORDER
        or PT_ENERGY_PAIR_PER_THREAD."""
        out, bound = np.zeros(self.total), np.zeros(self.total)
        ms = pt_energy_method(self.h, method, out, bound)
        return out, bound, ms

    def observables(self) -> dict:
        acc = np.zeros((self.total, 5))
        counts = np.zeros((self.total, 7), dtype=np.int64)
        perm = np.zeros(self.total, dtype=np.int32)
        te = np.zeros(2, dtype=np.int64)
        pt_observables(self.h, acc, counts, perm, te)
        return dict(acc=acc, counts=counts, perm=perm, t=int(te[0]), e=int(te[1]))

    def reset_observables(self):
        pt_reset_observables(self.h)

    def coords(self) -> np.ndarray:
        out = np.zeros_like(self.coords0)
        pt_get_coords(self.h, out)
        return out

    def running(self):
        e, b = np.zeros(self.total), np.zeros(self.total)
        pt_get_running(self.h, e, b)
        return e, b

    def series(self) -> np.ndarray:
        rows = pt_get_series(self.h, None)
        out = np.zeros((max(rows, 0), self.total, 3))
        if rows:
            pt_get_series(self.h, out)
        return out

    def logs(self):
        ra, re = pt_get_logs(self.h, None, None)
        alog = np.zeros((ra, self.words), dtype=np.uint64)
        elog = np.zeros((re, self.total), dtype=np.uint8)
        pt_get_logs(self.h, alog if ra else None, elog if re else None)
        return alog, elog

    def time_sweeps(self, n: int):
        return pt_time_sweeps(self.h, n)

    def mapping(self):
        """(beads per lane, wavefronts per replica, schedule: 1 persistent, 2 task flow,
        0 per sweep) per chain."""
        return pt_get_mapping(self.h, len(self.w.n_beads))

    def digests(self) -> np.ndarray:
        """[slots, 2] uint64 decision digests (accept words, exchange outcomes)."""
        return pt_get_digests(self.h, self.total)

    def state(self) -> bytes:
        """A checkpoint of the run (see pt_get_state)."""
        return pt_get_state(self.h)

    def set_state(self, state: bytes) -> None:
        pt_set_state(self.h, state)

    def set_spin_limit(self, polls: int) -> None:
        """Test hook for the bounded waits of the persistent and task-flow schedules."""
        _check(lib().pt_set_spin_limit(C.c_void_p(self.h), int(polls)))

    def set_guard_scale(self, factor: float) -> None:
        """Test hook: widen the guard bands by factor >= 1 (decisions unchanged;
        more of them go to the FP64 order)."""
        _check(lib().pt_set_guard_scale(C.c_void_p(self.h), float(factor)))
