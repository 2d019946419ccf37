"""Seeded synthetic workloads shared by the tests, the smoke check and the
benchmark.  This module holds problem *parameters* and random draws only --
none of the method's arithmetic -- so that the oracle and the GPU library can
both be fed from it without sharing any code path.

The problems are the textbook ones the paper defines (half MBB beam, Sec. 3;
3D cantilever, Sec. 4) at the sizes of the paper's timing runs
(3e4 to 4.8e5 elements in 2D, 2.2e5 in 3D); no dataset is involved.
"""
from dataclasses import dataclass, field, replace
from typing import Optional, Tuple

import numpy as np


@dataclass(frozen=True)
class Config:
    name: str
    kind: str                 # 'mbb' | 'cantilever2d' | 'cantilever3d'
    nelx: int
    nely: int
    nelz: int = 0             # 0 -> 2D
    volfrac: float = 0.5
    penal: float = 3.0
    rmin: float = 2.0
    ft: int = 1               # 1 density filter, 2 projection fixed eta, 3 volume-preserving eta
    bc: str = "D"             # filter boundary rule 'D' | 'N'
    eta: float = 0.5
    beta: float = 1.0
    move: float = 0.2
    E0: float = 1.0
    Emin: float = 1e-9
    nu: float = 0.3
    iterations: int = 50
    precision: str = "f64"    # 'f64' | 'f32' (FP32 fields, FP64 solve vectors and sums)
    # continuation (istart, maxPar, isteps, delta, 'add' | 'mul'); None = off
    penal_sched: Optional[Tuple] = None
    beta_sched: Optional[Tuple] = None
    load: int = 0             # load node: MBB column / cantilever row

    @property
    def dim(self):
        return 3 if self.nelz else 2

    @property
    def m(self):
        return self.nelx * self.nely * (self.nelz or 1)


# Small FP64 case: MBB 60 x 20, density filter only, 50 iterations.
C0 = Config("mbb60x20", "mbb", 60, 20, rmin=2.0, ft=1, bc="D", iterations=50)


def c1(nelx):
    """MBB at 300x100 / 600x200 / 1200x400: rmin = 2 nelx / 60, volume-
    preserving projection with beta 1 -> 32 (x2 every 25 iterations) and
    penal 1 -> 3 (+0.25 every 25 iterations), FP32 fields, 200 iterations."""
    return Config(f"mbb{nelx}x{nelx // 3}", "mbb", nelx, nelx // 3, rmin=2.0 * nelx / 60.0,
                  penal=1.0, ft=3, bc="D", eta=0.5, beta=1.0, iterations=200,
                  precision="f32", penal_sched=(1, 3.0, 25, 0.25, "add"),
                  beta_sched=(1, 32.0, 25, 2.0, "mul"))


C1 = {n: c1(n) for n in (300, 600, 1200)}

# 3D cantilever 96 x 48 x 48, rmin = sqrt(3), mirror filter boundary.
C2 = Config("cantilever96x48x48", "cantilever3d", 96, 48, 48, volfrac=0.12, penal=3.0,
            rmin=float(np.sqrt(3.0)), ft=3, bc="N", eta=0.5, beta=2.0, iterations=100)

# A 3D case small enough for the oracle to finish in seconds.
C2_SMALL = replace(C2, name="cantilever12x6x6", nelx=12, nely=6, nelz=6, iterations=10)


# Frame reinforcement (Sec. 3.5): 900 x 900, volfrac 0.2, p = 3, rmin = 8,
# volume-preserving projection with beta = 2, no continuation, 100 steps;
# passive frame and opening, distributed loads (load = 0: the code's sign of
# the horizontal load, 1: the opposite one).  The filter boundary rule is not
# stated for this example; zero-Neumann is taken.
C4 = Config("frame900", "frame", 900, 900, volfrac=0.2, penal=3.0, rmin=8.0, ft=3, bc="N", eta=0.5, beta=2.0,
            iterations=100, precision="f64")

# The same problem small enough for the oracle.
C4_SMALL = replace(C4, name="frame100", nelx=100, nely=100, rmin=2.0, iterations=8)


# The convergence tests of Table 4 (MBB, f = 0.5, rmin = 8.75, 2,500
# iterations at most, stop when |r|_2 / sqrt(m) < 1e-6 on the physical field):
# T1 density filter alone; T2 volume-preserving projection with beta = 2;
# T3 as T2 with continuation on beta (from 250, x2 every 25, up to 16) and p
# (from 50, +0.25 every 25, 1 -> 3); T4 as T2 on 600 x 200 (rmin kept).
# The filter boundary rule of these runs is not stated; 'D' is taken.
PAE_T = {
    "T1": Config("T1", "mbb", 300, 100, volfrac=0.5, rmin=8.75, ft=1, bc="D", iterations=2500),
    "T2": Config("T2", "mbb", 300, 100, volfrac=0.5, rmin=8.75, ft=3, bc="D", beta=2.0, iterations=2500),
    "T3": Config("T3", "mbb", 300, 100, volfrac=0.5, rmin=8.75, ft=3, bc="D", beta=2.0, penal=1.0,
                 iterations=2500, beta_sched=(250, 16.0, 25, 2.0, "mul"), penal_sched=(50, 3.0, 25, 0.25, "add")),
    "T4": Config("T4", "mbb", 600, 200, volfrac=0.5, rmin=8.75, ft=3, bc="D", beta=2.0, iterations=2500),
}
PAE_Q0 = {"T1": 20, "T2": 20, "T3": 500, "T4": 20}


def batch_configs(count=64, seed=0):
    """Ragged batch: per instance (drawn in this order) the problem type
    (cantilever or MBB, 1/2 each), nelx uniform over even integers in
    [100, 400] with nely = nelx / 2, the load position on the free edge,
    volfrac ~ U[0.3, 0.5], rmin ~ U[1.5, 4]; ft = 3, beta = 2, p = 3, 'D'."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        kind = "cantilever2d" if rng.random() < 0.5 else "mbb"
        nelx = 2 * int(rng.integers(50, 201))
        nely = nelx // 2
        load = int(rng.integers(0, nely + 1)) if kind == "cantilever2d" else int(rng.integers(0, nelx))
        vf = float(rng.uniform(0.3, 0.5))
        rmin = float(rng.uniform(1.5, 4.0))
        out.append(Config(f"batch{i}", kind, nelx, nely, volfrac=vf, rmin=rmin, ft=3, bc="D",
                          beta=2.0, penal=3.0, iterations=100, precision="f32", load=load))
    return out


# --- random fields for kernel-level parity and microbenchmarks ---------------
def design_field(m, seed, lo=0.0, hi=1.0):
    return np.random.default_rng(seed).uniform(lo, hi, m)


def smooth_design(cfg, seed):
    """A smooth design in [0.02, 0.98] on the element grid (a few random
    Fourier modes): closer to mid-run designs than white noise."""
    rng = np.random.default_rng(seed)
    shape = (cfg.nely, cfg.nelz, cfg.nelx) if cfg.nelz else (cfg.nely, cfg.nelx)
    grids = np.meshgrid(*[np.linspace(0, 1, s) for s in shape], indexing="ij")
    v = np.full(shape, cfg.volfrac)
    for _ in range(6):
        k = rng.integers(1, 5, len(shape))
        ph = rng.uniform(0, 2 * np.pi, len(shape))
        term = np.ones(shape)
        for g, kk, p in zip(grids, k, ph):
            term = term * np.cos(np.pi * kk * g + p)
        v = v + 0.15 * term
    return np.clip(v, 0.02, 0.98).reshape(-1, order="F")


def displacement_field(n, seed):
    return np.random.default_rng(seed).standard_normal(n)


def sensitivity_field(m, seed):
    return -np.random.default_rng(seed).uniform(0.0, 1.0, m)


# --- the learned warm start --------------------------------------------------
def network_params(layers, seed, taps=9):
    """Initial network parameters, flat, per layer W[taps][c_out][c_in] then
    b[c_out]: He-normal weights (standard deviation sqrt(2 / (taps c_in)))
    and small normal biases.  `layers` lists (c_in, c_out); taps is 9 for
    the 2D network, 27 for the 3D one."""
    rng = np.random.default_rng(seed)
    out = []
    for ci, co in layers:
        out.append(rng.standard_normal(taps * co * ci) * np.sqrt(2.0 / (taps * ci)))
        out.append(rng.standard_normal(co) * 0.05)
    return np.concatenate(out)


def warm_start_instances3(count, nelx, nely, nelz, seed):
    """Training / held-out instances for the 3D learned warm start: the 3D
    cantilever with its sine line load moved to a random height iz on the
    free end (drawn uniformly, `load`) and volfrac uniform in [0.08, 0.2];
    rmin sqrt(3), 'N', projection with beta 2, FP32 fields."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        out.append(Config(f"ws3_{seed}_{i}", "cantilever3d", nelx, nely, nelz, volfrac=float(rng.uniform(0.08, 0.2)),
                          rmin=float(np.sqrt(3.0)), ft=3, bc="N", eta=0.5, beta=2.0, penal=3.0, iterations=100,
                          precision="f32", load=int(rng.integers(0, nelz + 1))))
    return out


def warm_start_instances(count, nelx, nely, seed):
    """Training / held-out instances for the learned warm start: the MBB beam
    with the load node drawn uniformly on the top edge and volfrac uniform in
    [0.3, 0.5]; density filter radius as in the MBB configurations, projection
    with beta 2, FP32 fields."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        out.append(Config(f"ws{seed}_{i}", "mbb", nelx, nely, volfrac=float(rng.uniform(0.3, 0.5)),
                          rmin=max(1.5, 2.0 * nelx / 60.0), ft=3, bc="D", beta=2.0, penal=3.0,
                          iterations=100, precision="f32", load=int(rng.integers(0, nelx))))
    return out
