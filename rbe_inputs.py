"""Seeded synthetic charge systems for the RBE k-space path.

This module only generates inputs (positions, charges, box sizes, upstream
gradients).  It holds none of the method's arithmetic and is shared by the
tests, the benchmark and the smoke check; both the HIP library and the CPU
oracle receive its arrays unchanged.

All generators use ``numpy.random.Generator(PCG64(seed))`` and return float64
structure-of-arrays ``x, y, z, q`` plus the box edge ``L``.

Workload recipes (the paper's own systems are self-generated, Sec. 4):
  * uniform +-1 charges in a cube (primitive electrolyte, Sec. 4.1/4.2);
  * SPC/E-like rigid water (O -0.8476 e, two H +0.4238 e, O-H 1.0 A,
    H-O-H 109.47 deg) with uniform random centres and uniformly random
    orientations, wrapped into [0, L) (Sec. 4.1, water benchmark);
  * water with 1 mol/L NaCl ions replacing randomly chosen molecule slots;
  * rock-salt lattices (Madelung checks);
  * batches of independent replicas.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

WATER_DENSITY = 0.0334          # molecules per A^3 (liquid water)
Q_O = -0.8476
Q_H = 0.4238
R_OH = 1.0                      # A
HOH_DEG = 109.47


@dataclasses.dataclass
class System:
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    q: np.ndarray
    L: float
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.q.shape[0])


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform_pm1(n: int, L: float, seed: int) -> System:
    """n point charges, n/2 at +1 and n/2 at -1 (shuffled), uniform in [0, L)^3."""
    if n % 2:
        raise ValueError("n must be even for a neutral +-1 system")
    g = _rng(seed)
    pos = g.random((3, n)) * L
    q = np.concatenate([np.ones(n // 2), -np.ones(n // 2)])
    g.shuffle(q)
    return System(pos[0].copy(), pos[1].copy(), pos[2].copy(), q, float(L), f"uniform_pm1_{n}")


def random_charges(n: int, L: float, seed: int) -> System:
    """n charges with N(0,1) values made exactly neutral by removing the mean; tiny-N checks."""
    g = _rng(seed)
    pos = g.random((3, n)) * L
    q = g.standard_normal(n)
    q -= q.mean()
    return System(pos[0].copy(), pos[1].copy(), pos[2].copy(), q, float(L), f"random_{n}")


def _random_rotations(g: np.random.Generator, n: int) -> np.ndarray:
    """n uniformly random rotation matrices from normalised Gaussian quaternions, shape (n, 3, 3)."""
    quat = g.standard_normal((n, 4))
    quat /= np.linalg.norm(quat, axis=1, keepdims=True)
    w, a, b, c = quat.T
    rot = np.empty((n, 3, 3))
    rot[:, 0, 0] = 1 - 2 * (b * b + c * c)
    rot[:, 0, 1] = 2 * (a * b - c * w)
    rot[:, 0, 2] = 2 * (a * c + b * w)
    rot[:, 1, 0] = 2 * (a * b + c * w)
    rot[:, 1, 1] = 1 - 2 * (a * a + c * c)
    rot[:, 1, 2] = 2 * (b * c - a * w)
    rot[:, 2, 0] = 2 * (a * c - b * w)
    rot[:, 2, 1] = 2 * (b * c + a * w)
    rot[:, 2, 2] = 1 - 2 * (a * a + b * b)
    return rot


def water_box(n_slots: int, seed: int, n_ion_pairs: int = 0, density: float = WATER_DENSITY,
              L: float | None = None) -> System:
    """SPC/E-like water with optional Na+/Cl- ions replacing molecule slots.

    Each slot has a uniform random centre in [0, L)^3.  A water slot puts O at
    the centre and the two H atoms at R_OH from O, at +-HOH/2 about the
    molecular bisector, in a uniformly random orientation.  An ion slot puts a
    single +1 (Na) or -1 (Cl) charge at the centre.  Coordinates are wrapped
    into [0, L).  Atoms are ordered: all waters (O, H, H per molecule), then
    the Na ions, then the Cl ions.
    """
    if L is None:
        L = (n_slots / density) ** (1.0 / 3.0)
    g = _rng(seed)
    centres = g.random((n_slots, 3)) * L
    ion_slots = np.zeros(n_slots, dtype=bool)
    if n_ion_pairs:
        ion_idx = g.choice(n_slots, size=2 * n_ion_pairs, replace=False)
        ion_slots[ion_idx] = True
    else:
        ion_idx = np.empty(0, dtype=np.int64)
    wat = centres[~ion_slots]
    n_w = wat.shape[0]
    half = math.radians(HOH_DEG) / 2.0
    h_local = np.array([[R_OH * math.sin(half), 0.0, R_OH * math.cos(half)],
                        [-R_OH * math.sin(half), 0.0, R_OH * math.cos(half)]])
    rot = _random_rotations(g, n_w)
    h1 = wat + rot @ h_local[0]
    h2 = wat + rot @ h_local[1]
    atoms = np.stack([wat, h1, h2], axis=1).reshape(-1, 3)
    q_w = np.tile(np.array([Q_O, Q_H, Q_H]), n_w)
    na = centres[ion_idx[:n_ion_pairs]] if n_ion_pairs else np.empty((0, 3))
    cl = centres[ion_idx[n_ion_pairs:]] if n_ion_pairs else np.empty((0, 3))
    pos = np.concatenate([atoms, na, cl], axis=0)
    pos = np.mod(pos, L)
    pos[pos >= L] -= L          # np.mod can round up to L for tiny negatives
    q = np.concatenate([q_w, np.ones(n_ion_pairs), -np.ones(n_ion_pairs)])
    return System(pos[:, 0].copy(), pos[:, 1].copy(), pos[:, 2].copy(), q, float(L),
                  f"water_{n_slots}_ions_{n_ion_pairs}")


def nacl_lattice(cells: int, r0: float = 1.0) -> System:
    """Perfect rock-salt crystal of cells^3 conventional cells, nearest-neighbour distance r0.

    Sites on the simple-cubic grid of spacing r0, charge (-1)^(i+j+k); box L = 2 r0 cells.
    """
    n_side = 2 * cells
    idx = np.arange(n_side)
    i, j, k = np.meshgrid(idx, idx, idx, indexing="ij")
    i, j, k = i.ravel(), j.ravel(), k.ravel()
    q = np.where((i + j + k) % 2 == 0, 1.0, -1.0)
    return System(i * r0 + 0.0, j * r0 + 0.0, k * r0 + 0.0, q, float(n_side * r0), f"nacl_{cells}")


def gaussian_vectors(n: int, seed: int) -> np.ndarray:
    """(3, n) N(0,1) array, e.g. reference forces F_ref for the differentiable workload."""
    return _rng(seed).standard_normal((3, n))


# --------------------------------------------------------------------------------------
# Named workloads (sizes of the benchmark and parity cases)
# --------------------------------------------------------------------------------------

def c1_small() -> tuple[System, float, int]:
    """3,000 +-1 charges, L = 31 A, alpha = 0.1 A^-2, P = 100."""
    return uniform_pm1(3000, 31.0, 1001), 0.1, 100


def c2_water() -> tuple[System, float, int]:
    """300,000-atom SPC/E-like water (100,000 molecules), alpha = 0.08, P = 100."""
    return water_box(100_000, 1002), 0.08, 100


# 1 mol/L NaCl in water at 0.0334 slots/A^3: 341,544 slots -> 329,228 waters + 6,158 + 6,158 ions
C3A_SLOTS, C3A_PAIRS = 341_544, 6_158
C3B_SLOTS, C3B_PAIRS = 3_415_440, 61_580


def c3a_electrolyte() -> tuple[System, float, int]:
    """1,000,000-atom water + 1 mol/L NaCl, alpha = 0.06 (P = 100 or 200)."""
    return water_box(C3A_SLOTS, 1003, C3A_PAIRS), 0.06, 100


def c3b_electrolyte() -> tuple[System, float, int]:
    """10,000,000-atom water + 1 mol/L NaCl, alpha = 0.06 (P = 100 or 200)."""
    return water_box(C3B_SLOTS, 1004, C3B_PAIRS), 0.06, 100


def c4_differentiable() -> tuple[System, float, int]:
    """200,000 +-1 charges in L = 126 A, alpha = 0.08, P = 100."""
    return uniform_pm1(200_000, 126.0, 1005), 0.08, 100


def e3_electrolyte() -> tuple[System, float, int]:
    """Primitive 1:1 electrolyte, 500 + 500 ions, L = 10, alpha = 0.362, P = 100 (reduced units)."""
    return uniform_pm1(1000, 10.0, 1006), 0.362, 100


def e4_water() -> tuple[System, float, int]:
    """1,000 SPC/E-like molecules in L = 66.9 A, alpha = 0.048, P = 100."""
    return water_box(1000, 1007, L=66.9), 0.048, 100


@dataclasses.dataclass
class Replicas:
    systems: list
    alphas: list
    P: int


def c5_replicas(B: int = 128, seed_base: int = 5000, P: int = 100) -> Replicas:
    """B neutral +-1 systems, N_b = 2 n_b with n_b uniform in [2500, 75000], density 0.1 /A^3,
    L_b = (N_b / 0.1)^(1/3), alpha_b uniform in [0.05, 0.12]."""
    systems, alphas = [], []
    for b in range(B):
        g = _rng(seed_base + b)
        n_half = int(g.integers(2500, 75001))
        alpha = float(g.uniform(0.05, 0.12))
        n = 2 * n_half
        L = (n / 0.1) ** (1.0 / 3.0)
        systems.append(uniform_pm1(n, L, seed_base + 100_000 + b))
        alphas.append(alpha)
    return Replicas(systems, alphas, P)


# ---------------------------------------------------------------- short-range (RBL) systems

@dataclasses.dataclass
class LJSystem:
    """Charged Lennard-Jones particles: positions, charges and per-particle LJ eps, sigma."""
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    q: np.ndarray
    eps: np.ndarray
    sig: np.ndarray
    L: float

    @property
    def n(self) -> int:
        return int(self.q.shape[0])


def primitive_electrolyte(n: int, density: float, seed: int, jitter: float = 0.25) -> LJSystem:
    """The paper's primitive-model 1:1 electrolyte (Sec. 4): n/2 cations (+1) and n/2 anions
    (-1), LJ eps = sigma = 1 (reduced units), at `density` particles per sigma^3.  Positions:
    a simple cubic lattice of spacing a = L / ceil(n^(1/3)) filled in random order, each
    site moved by a uniform random offset of up to jitter * a per axis (no overlaps, a
    liquid-like spread of distances)."""
    g = _rng(seed)
    L = (n / density) ** (1.0 / 3.0)
    side = int(math.ceil(n ** (1.0 / 3.0)))
    a = L / side
    sites = np.stack(np.meshgrid(*(np.arange(side),) * 3, indexing="ij"), axis=-1).reshape(-1, 3)
    pick = g.permutation(sites.shape[0])[:n]
    pos = (sites[pick] + 0.5 + g.uniform(-jitter, jitter, size=(n, 3))) * a
    q = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    g.shuffle(q)
    return LJSystem(pos[:, 0].copy(), pos[:, 1].copy(), pos[:, 2].copy(), q, np.ones(n), np.ones(n), float(L))
