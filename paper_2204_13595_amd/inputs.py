"""Seeded synthetic inputs: SPC/E-like rigid water in a cubic periodic box.

This module only builds inputs (positions, charges, atom types, molecule ids and
the Lennard-Jones tables). It holds none of the force method's arithmetic, so
that both the HIP path and the CPU oracle can be fed from it.

Recipe (the paper's water runs use equilibrated SPC/E water, which is not
available; these are stand-ins of the same density and composition):

* oxygen sites on a cubic lattice of spacing a = L / n_side, each jittered by
  U(-0.1 a, 0.1 a) per axis; when the molecule count is not a perfect cube the
  smallest lattice that holds it is used and randomly chosen sites stay empty;
* each molecule gets a uniformly random orientation (a normalised 4-D Gaussian
  quaternion) of the rigid geometry OH = 0.1 nm, HOH = 109.47 degrees;
* atoms are ordered O, H, H per molecule; type 0 = O, type 1 = H; the molecule id
  marks the intramolecular pairs that the force method excludes;
* charges q_O = -0.8476 e, q_H = +0.4238 e; Lennard-Jones acts on O-O only with
  sigma = 0.3166 nm, epsilon = 0.650 kJ/mol.

Positions are not wrapped into the box: the force method must handle that.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

Q_O = -0.8476
Q_H = 0.4238
SIGMA_OO = 0.3166
EPS_OO = 0.650
R_OH = 0.1
THETA_HOH_DEG = 109.47
COULOMB_K = 138.935458  # kJ mol^-1 nm e^-2


@dataclasses.dataclass
class WaterSystem:
    n_waters: int
    box: float
    pos: np.ndarray        # [N, 3] float64, nm
    charge: np.ndarray     # [N] float64, e
    atom_type: np.ndarray  # [N] int32
    molecule: np.ndarray   # [N] int32
    lj_sigma: np.ndarray   # [n_types * n_types] float64
    lj_eps: np.ndarray     # [n_types * n_types] float64

    @property
    def n_atoms(self) -> int:
        return int(self.pos.shape[0])

    n_types = 2


def _random_rotations(rng: np.random.Generator, n: int) -> np.ndarray:
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    rot = np.empty((n, 3, 3))
    rot[:, 0, 0] = 1 - 2 * (y * y + z * z)
    rot[:, 0, 1] = 2 * (x * y - z * w)
    rot[:, 0, 2] = 2 * (x * z + y * w)
    rot[:, 1, 0] = 2 * (x * y + z * w)
    rot[:, 1, 1] = 1 - 2 * (x * x + z * z)
    rot[:, 1, 2] = 2 * (y * z - x * w)
    rot[:, 2, 0] = 2 * (x * z - y * w)
    rot[:, 2, 1] = 2 * (y * z + x * w)
    rot[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return rot


def lj_tables(sigma_oo: float = SIGMA_OO, eps_oo: float = EPS_OO):
    sigma = np.zeros(4)
    eps = np.zeros(4)
    sigma[0] = sigma_oo
    eps[0] = eps_oo
    return sigma, eps


def make_water(n_waters: int, box: float, seed: int = 2204, *, q_o: float = Q_O,
               sigma_oo: float = SIGMA_OO, eps_oo: float = EPS_OO) -> WaterSystem:
    rng = np.random.default_rng(seed)
    n_side = int(math.ceil(round(n_waters ** (1.0 / 3.0), 9)))
    while n_side ** 3 < n_waters:
        n_side += 1
    a = box / n_side
    n_sites = n_side ** 3
    if n_sites == n_waters:
        sites = np.arange(n_sites)
    else:
        sites = np.sort(rng.choice(n_sites, size=n_waters, replace=False))
    iz, rem = np.divmod(sites, n_side * n_side)
    iy, ix = np.divmod(rem, n_side)
    centre = (np.stack([ix, iy, iz], axis=1) + 0.5) * a
    centre += rng.uniform(-0.1 * a, 0.1 * a, size=centre.shape)
    half = math.radians(THETA_HOH_DEG) / 2.0
    body = np.array([[0.0, 0.0, 0.0],
                     [R_OH * math.sin(half), 0.0, R_OH * math.cos(half)],
                     [-R_OH * math.sin(half), 0.0, R_OH * math.cos(half)]])
    rot = _random_rotations(rng, n_waters)
    pos = centre[:, None, :] + np.einsum("nab,kb->nka", rot, body)
    pos = pos.reshape(-1, 3).copy()
    q_h = -q_o / 2.0
    charge = np.tile(np.array([q_o, q_h, q_h]), n_waters)
    atom_type = np.tile(np.array([0, 1, 1], dtype=np.int32), n_waters)
    molecule = np.repeat(np.arange(n_waters, dtype=np.int32), 3)
    sigma, eps = lj_tables(sigma_oo, eps_oo)
    return WaterSystem(n_waters, float(box), pos, charge, atom_type, molecule, sigma, eps)


# Workloads: (waters, box edge in nm). Density is 33.4-33.5 waters per nm^3.
WORKLOADS = {
    "water512": (512, 2.4834),
    "water32k": (32768, 9.93),
    "water1M": (1048576, 31.5),
    "water4k": (4096, 4.97),
    "water2M": (2097152, 39.7),
}


def workload(name: str, seed: int = 2204) -> WaterSystem:
    n, box = WORKLOADS[name]
    return make_water(n, box, seed)


def perturbed_parameters(seed: int = 4):
    """q_O, sigma_OO, eps_OO each scaled by U(0.95, 1.05) (force-matching target set)."""
    rng = np.random.default_rng(seed)
    f = rng.uniform(0.95, 1.05, size=3)
    return Q_O * f[0], SIGMA_OO * f[1], EPS_OO * f[2]


@dataclasses.dataclass
class IonSystem:
    box: float
    pos: np.ndarray        # [N, 3]
    charge: np.ndarray     # [N]
    atom_type: np.ndarray  # [N] 0 = cation, 1 = anion
    molecule: np.ndarray   # [N] all -1: no excluded pairs
    lj_sigma: np.ndarray   # [4]
    lj_eps: np.ndarray     # [4]

    @property
    def n_atoms(self) -> int:
        return int(self.pos.shape[0])


def electrolyte(valence: int = 1, seed: int = 2204, box: float = 80.0, n_anions: int = 2560) -> IonSystem:
    """Primitive-model electrolyte in reduced units (sigma = 1), the paper's
    electrolyte sizes: 2560 monovalent cations and 2560 anions (valence 1), or
    1280 divalent cations and 2560 monovalent anions (valence 2), L = 80 sigma
    (other sizes: `n_anions` anions and the neutralising cations in `box`).
    Ions sit on the sites of the smallest cubic lattice that holds them (random
    vacancies), jittered by U(-0.1 a, 0.1 a), in random species order. LJ with
    sigma = eps = 1 for every pair (plain, truncated at the shell cutoff)."""
    rng = np.random.default_rng(seed)
    n_an = int(n_anions)
    n_cat = n_an if valence == 1 else n_an // 2
    n = n_cat + n_an
    n_side = 1
    while n_side ** 3 < n:
        n_side += 1
    a = box / n_side
    sites = np.sort(rng.choice(n_side ** 3, size=n, replace=False))
    iz, rem = np.divmod(sites, n_side * n_side)
    iy, ix = np.divmod(rem, n_side)
    pos = (np.stack([ix, iy, iz], axis=1) + 0.5) * a + rng.uniform(-0.1 * a, 0.1 * a, size=(n, 3))
    species = rng.permutation(np.r_[np.zeros(n_cat, np.int32), np.ones(n_an, np.int32)])
    charge = np.where(species == 0, float(valence), -1.0)
    return IonSystem(float(box), pos, charge, species.astype(np.int32), np.full(n, -1, np.int32),
                     np.ones(4), np.ones(4))


def nacl_crystal(n_cells: int, d: float = 0.5, q: float = 1.0):
    """Rock-salt lattice of (2 n_cells)^3 ions, nearest-neighbour distance d."""
    m = 2 * n_cells
    idx = np.stack(np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij"), -1)
    idx = idx.reshape(-1, 3)
    pos = idx * d + 0.5 * d
    sign = np.where(idx.sum(axis=1) % 2 == 0, 1.0, -1.0)
    return pos.astype(np.float64), (q * sign).astype(np.float64), float(m * d)
