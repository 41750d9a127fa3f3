"""Seeded synthetic inputs shared by the GPU path's tests/benchmark and the oracle.

This module only draws numbers: water boxes, jitter streams, lattices and
request streams.  It holds none of the SPME arithmetic.

The paper measures a 65,536-atom system on a 64^3 grid without stating its
composition (§V.E); TIP3P-like water boxes of the same size stand in for it:
oxygen uniform in the box, two hydrogens at 0.9572 A with a 104.52 degree
H-O-H angle in a uniformly random orientation, charges -0.834 / +0.417 (net
zero), atom order O, H, H per molecule.
"""
from dataclasses import dataclass, field
import math

import numpy as np

R_OH = 0.9572                 # A
ANGLE_HOH = 104.52            # degrees
Q_O, Q_H = -0.834, 0.417      # e
WATER_DENSITY = 0.0334        # molecules / A^3


def random_rotations(rng, n):
    """n uniformly random rotation matrices (normalised Gaussian 4-vectors as quaternions)."""
    qv = rng.standard_normal((n, 4))
    qv /= np.linalg.norm(qv, axis=1, keepdims=True)
    w, x, y, z = qv.T
    R = np.empty((n, 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - z * w)
    R[:, 0, 2] = 2 * (x * z + y * w)
    R[:, 1, 0] = 2 * (x * y + z * w)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - x * w)
    R[:, 2, 0] = 2 * (x * z - y * w)
    R[:, 2, 1] = 2 * (y * z + x * w)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def water_box(n_waters, L, seed):
    """(pos [3n,3] float64, q [3n] float64, box [3,3]) for n waters in a cubic box of edge L."""
    rng = np.random.default_rng(seed)
    O = rng.uniform(0.0, L, size=(n_waters, 3))
    half = math.radians(ANGLE_HOH / 2.0)
    body = np.array([[R_OH * math.sin(half), 0.0, R_OH * math.cos(half)],
                     [-R_OH * math.sin(half), 0.0, R_OH * math.cos(half)]])
    R = random_rotations(rng, n_waters)
    H = np.einsum("nij,hj->nhi", R, body) + O[:, None, :]
    pos = np.empty((n_waters, 3, 3))
    pos[:, 0] = O
    pos[:, 1:] = H
    q = np.tile(np.array([Q_O, Q_H, Q_H]), n_waters)
    return pos.reshape(-1, 3), q, np.diag([float(L)] * 3)


def jitter_stream(pos0, n_frames, sigma, seed):
    """Random walk x_t = x_{t-1} + N(0, sigma^2) per coordinate; frame 0 is pos0 itself."""
    rng = np.random.default_rng(seed)
    frames = np.empty((n_frames,) + pos0.shape)
    frames[0] = pos0
    for t in range(1, n_frames):
        frames[t] = frames[t - 1] + rng.normal(0.0, sigma, size=pos0.shape)
    return frames


def grid_for_edge(L, choices=(32, 48, 64)):
    """Grid size with spacing closest to 1 A among the supported choices."""
    return min(choices, key=lambda K: (abs(L / K - 1.0), K))


@dataclass
class Workload:
    name: str
    n_waters: int
    L: float
    K: int
    order: int
    beta: float
    seed: int
    note: str = ""

    @property
    def n_atoms(self):
        return 3 * self.n_waters

    def make(self):
        return water_box(self.n_waters, self.L, self.seed)


# The four single-system workloads (plain FP64 check, the 65k/64^3 headline
# system, and the 128^3 system at two spline orders).
SMALL_32 = Workload("water_4095_k32", 1365, 32.0, 32, 4, 0.35, 1,
                    "4,095 atoms, 32 A box, 32^3 grid, p=4")
HEADLINE_64 = Workload("water_65535_k64", 21845, 86.8, 64, 4, 0.34, 2,
                       "65,535 atoms, 86.8 A box, 64^3 grid, p=4")
LARGE_128_P4 = Workload("water_209715_k128_p4", 69905, 128.0, 128, 4, 0.32, 3,
                        "209,715 atoms, 128 A box, 128^3 grid, p=4")
LARGE_128_P6 = Workload("water_209715_k128_p6", 69905, 128.0, 128, 6, 0.32, 3,
                        "209,715 atoms, 128 A box, 128^3 grid, p=6")
HEADLINE_JITTER_SEED = 1002
HEADLINE_JITTER_SIGMA = 0.01


@dataclass
class BatchMember:
    index: int
    n_waters: int
    L: float
    K: int
    seed: int

    @property
    def n_atoms(self):
        return 3 * self.n_waters

    def make(self):
        return water_box(self.n_waters, self.L, self.seed)


def batch_mix(n_systems=64, seed=4, lo=3000, hi=65000, beta=0.34):
    """Uneven batch: atom counts log-uniform in [lo, hi], edge from water density,
    grid by ~1 A spacing over {32, 48, 64}."""
    rng = np.random.default_rng(seed)
    n_atoms = np.exp(rng.uniform(math.log(lo), math.log(hi), size=n_systems))
    out = []
    for i, na in enumerate(n_atoms):
        nw = int(round(na / 3.0))
        L = (nw / WATER_DENSITY) ** (1.0 / 3.0)
        out.append(BatchMember(i, nw, L, grid_for_edge(L), seed * 1000 + i))
    return out


def serving_pool(seed_large=5000, n_large=4):
    """The batch mix plus four 128^3 / 209,715-atom boxes."""
    pool = batch_mix()
    for j in range(n_large):
        pool.append(BatchMember(len(pool), 69905, 128.0, 128, seed_large + j))
    return pool


def poisson_requests(n_requests=20000, rate=2000.0, seed=5, p_large=0.1, n_small=64, n_large=4):
    """Open-loop arrivals: (arrival times [s], pool index) with exponential gaps."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=n_requests)
    t = np.cumsum(gaps)
    large = rng.uniform(size=n_requests) < p_large
    idx = np.where(large, n_small + rng.integers(0, n_large, size=n_requests),
                   rng.integers(0, n_small, size=n_requests))
    return t, idx


def rock_salt(M, r0, offset=(0.0, 0.0, 0.0)):
    """M^3 ions of charge (-1)^(i+j+k) at spacing r0 in a cubic box of edge M r0."""
    idx = np.arange(M)
    i, j, k = np.meshgrid(idx, idx, idx, indexing="ij")
    pos = np.stack([i, j, k], axis=-1).reshape(-1, 3).astype(np.float64) * r0
    pos += np.asarray(offset, dtype=np.float64)
    q = np.where(((i + j + k) % 2 == 0).reshape(-1), 1.0, -1.0)
    return pos, q, np.diag([M * r0] * 3)


def random_neutral(n, L, seed, qscale=1.0):
    """n random charges in a cubic box with zero net charge (last charge balances)."""
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0.0, L, size=(n, 3))
    q = rng.uniform(-qscale, qscale, size=n)
    q[-1] = -q[:-1].sum()
    return pos, q, np.diag([float(L)] * 3)


def water_exclusions(n_atoms):
    """Symmetric exclusion lists (CSR offsets [n+1], partners) that exclude
    every pair inside a water molecule, atoms ordered O, H, H."""
    off, idx = [0], []
    for i in range(n_atoms):
        m = i // 3
        idx += [3 * m + k for k in range(3) if 3 * m + k != i and 3 * m + k < n_atoms]
        off.append(len(idx))
    return np.array(off, dtype=np.int32), np.array(idx, dtype=np.int32)
