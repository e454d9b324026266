"""Seeded synthetic inputs for the replica-exchange polymer workloads.

This module only *generates inputs*: model parameters, temperature ladders,
chain lengths and starting conformations.  It holds none of the method's
arithmetic (no energies, no Metropolis or exchange rule, no Philox stream),
so that both the HIP library and the CPU oracle can be fed from it without
sharing any of the computation they are checked on.

Model parameters follow the paper's Sec. 3.1 (Eqs. 1-3): epsilon = 1,
sigma = 2^(-1/6) r0, r0 = 0.7, r_c = 2.5 sigma, K = 40, R = 0.3.  The
displacement cube edge is a workload parameter; the paper's Sec. 3.2 uses
components in [-0.01, 0.01] (edge 0.02), the named workloads below use 0.2.

Starting conformations are built with numpy's PCG64 generator from the
workload seed (straight chains need no randomness).  Coordinates are
returned per conformation, bead-major, xyz-minor (AoS), in float64.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

BOND = 0.7  # starting bond length (= r0, the FENE / LJ minimum)


def model_params(step_edge: float = 0.2) -> dict:
    """Paper Sec. 3.1 parameters plus the displacement cube edge (Sec. 3.2)."""
    r0 = 0.7
    sigma = r0 * 2.0 ** (-1.0 / 6.0)
    return dict(epsilon=1.0, sigma=sigma, r_cut=2.5 * sigma, fene_k=40.0,
                fene_R=0.3, fene_r0=r0, step_edge=float(step_edge))


def geometric_ladder(n_slots: int, t_min: float, t_max: float) -> np.ndarray:
    """Inverse temperatures beta_i = 1/T_i, T_i geometric in [t_min, t_max].

    Slot 0 is the coldest (largest beta).  k_B = 1.
    """
    if n_slots == 1:
        return np.array([1.0 / t_min])
    i = np.arange(n_slots, dtype=np.float64)
    temps = t_min * (t_max / t_min) ** (i / (n_slots - 1))
    return 1.0 / temps


def straight_chain(n_beads: int, bond: float = BOND) -> np.ndarray:
    """r_i = (bond * i, 0, 0)."""
    xyz = np.zeros((n_beads, 3))
    xyz[:, 0] = bond * np.arange(n_beads, dtype=np.float64)
    return xyz


def random_walk(n_beads: int, rng: np.random.Generator, bond: float = BOND) -> np.ndarray:
    """Free random walk: r_0 = 0, r_i = r_{i-1} + bond * n_i, n_i uniform on S^2."""
    u = rng.random((n_beads - 1, 2))
    cz = 2.0 * u[:, 0] - 1.0
    phi = 2.0 * math.pi * u[:, 1]
    sz = np.sqrt(np.maximum(0.0, 1.0 - cz * cz))
    steps = np.stack([sz * np.cos(phi), sz * np.sin(phi), cz], axis=1) * bond
    xyz = np.zeros((n_beads, 3))
    xyz[1:] = np.cumsum(steps, axis=0)
    return xyz


@dataclasses.dataclass
class Workload:
    """A batch of independent chains, each with its own temperature ladder.

    ``coords`` is the concatenation over chains c and slots s (chain-major)
    of each starting conformation, AoS [bead][xyz], float64.
    """
    name: str
    n_beads: List[int]
    n_slots: List[int]
    betas: np.ndarray          # [sum R_c], per chain slot 0 coldest
    coords: np.ndarray         # [sum_c R_c * N_c * 3]
    seed: int
    sweeps: int
    precision: str             # "fp64" | "mixed"
    model: dict
    exchange_every: int = 1
    # Random-stream identities (the chain number and the first global slot
    # number that the counters of the method's random draws use).  None means
    # "this chain's position in the batch" / "running slot offset".  A subset of
    # a bigger workload keeps the ids of the chains it was cut from, so both
    # draw the same streams.
    stream_chain: Optional[List[int]] = None
    stream_slot0: Optional[List[int]] = None

    @property
    def n_chains(self) -> int:
        return len(self.n_beads)

    @property
    def total_slots(self) -> int:
        return int(sum(self.n_slots))

    def pair_interactions_per_sweep(self) -> int:
        """Sum over replicas of N (N - 1): N moves, each against N - 1 beads."""
        return int(sum(r * n * (n - 1) for n, r in zip(self.n_beads, self.n_slots)))

    def conformation(self, conf: int) -> np.ndarray:
        off = 0
        g = 0
        for n, r in zip(self.n_beads, self.n_slots):
            if conf < g + r:
                off += (conf - g) * n * 3
                return self.coords[off:off + n * 3].reshape(n, 3)
            off += r * n * 3
            g += r
        raise IndexError(conf)


def make_workload(n_beads, n_slots, ladders, start: str, seed: int, sweeps: int,
                  precision: str, name: str = "custom", step_edge: float = 0.2,
                  exchange_every: int = 1) -> Workload:
    """Build a workload from per-chain lengths, slot counts and (t_min, t_max) ladders."""
    rng = np.random.Generator(np.random.PCG64(seed))
    betas, coords = [], []
    for n, r, (tmin, tmax) in zip(n_beads, n_slots, ladders):
        betas.append(geometric_ladder(r, tmin, tmax))
        for _ in range(r):
            if start == "straight":
                coords.append(straight_chain(n).ravel())
            elif start == "walk":
                coords.append(random_walk(n, rng).ravel())
            else:
                raise ValueError(start)
    return Workload(name=name, n_beads=[int(v) for v in n_beads],
                    n_slots=[int(v) for v in n_slots], betas=np.concatenate(betas),
                    coords=np.concatenate(coords), seed=seed, sweeps=sweeps,
                    precision=precision, model=model_params(step_edge),
                    exchange_every=exchange_every)


C4_LENGTHS = (13, 30, 55, 100, 200, 500)


def named(name: str, sweeps: Optional[int] = None, precision: Optional[str] = None) -> Workload:
    """The five named workloads.

    c1: 1 chain, N=30, 16 slots, T in [0.1, 1.5], straight start, 2000 sweeps, seed 1, FP64.
    c2: 1 chain, N=100, 64 slots, T in [0.1, 1.5], random-walk start, 10^4 sweeps, seed 2.
    c3: 1 chain, N=500, 128 slots, T in [0.2, 2.0], random walk, 2000 sweeps, seed 3, mixed.
    c4: 48 chains, N uniform over {13,30,55,100,200,500}, 32 slots each, T in [0.1, 1.5],
        random walks, 5000 sweeps, seed 4, mixed.
    c5: 16 chains, N=2000, 256 slots each, T in [0.3, 2.5], random walks, 1000 sweeps,
        seed 5, mixed.
    """
    if name == "c1":
        w = make_workload([30], [16], [(0.1, 1.5)], "straight", 1, 2000, "fp64", name)
    elif name == "c2":
        w = make_workload([100], [64], [(0.1, 1.5)], "walk", 2, 10000, "mixed", name)
    elif name == "c3":
        w = make_workload([500], [128], [(0.2, 2.0)], "walk", 3, 2000, "mixed", name)
    elif name == "c4":
        rng = np.random.Generator(np.random.PCG64(4))
        lengths = [C4_LENGTHS[i] for i in rng.integers(0, len(C4_LENGTHS), size=48)]
        w = make_workload(lengths, [32] * 48, [(0.1, 1.5)] * 48, "walk", 4, 5000, "mixed", name)
    elif name == "c5":
        w = make_workload([2000] * 16, [256] * 16, [(0.3, 2.5)] * 16, "walk", 5, 1000, "mixed", name)
    else:
        raise KeyError(name)
    if sweeps is not None:
        w.sweeps = int(sweeps)
    if precision is not None:
        w.precision = precision
    return w


def subset(w: Workload, chains, slots: Optional[int] = None) -> Workload:
    """A workload restricted to some chains (and optionally their first ``slots`` slots)."""
    n_beads, n_slots, betas, coords, sc, ss = [], [], [], [], [], []
    boff = 0
    coff = 0
    src_chain = w.stream_chain or list(range(w.n_chains))
    src_slot0 = w.stream_slot0 or list(np.cumsum([0] + list(w.n_slots[:-1])))
    for c, (n, r) in enumerate(zip(w.n_beads, w.n_slots)):
        if c in chains:
            rr = r if slots is None else min(slots, r)
            n_beads.append(n)
            n_slots.append(rr)
            betas.append(w.betas[boff:boff + rr])
            coords.append(w.coords[coff:coff + rr * n * 3])
            sc.append(int(src_chain[c]))
            ss.append(int(src_slot0[c]))
        boff += r
        coff += r * n * 3
    return Workload(name=w.name + "-subset", n_beads=n_beads, n_slots=n_slots,
                    betas=np.concatenate(betas), coords=np.concatenate(coords),
                    seed=w.seed, sweeps=w.sweeps, precision=w.precision, model=dict(w.model),
                    exchange_every=w.exchange_every, stream_chain=sc, stream_slot0=ss)
