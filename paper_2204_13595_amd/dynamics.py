"""Python binding of the Langevin integrator and observables of ``libirbe.so``
(argument marshalling only), and the rigid-water topology they need.

The integrator (``irbe_dyn_*`` in ``include/irbe.h``) advances FP64 positions
and velocities by one step of the underdamped Langevin equations with rigid
bond lengths per group of at most three atoms; ``rdf`` and ``msd`` accumulate
the oxygen-oxygen radial distribution and the mean-squared displacement. There
is no fallback: without the library or a GPU the calls raise.
"""
from __future__ import annotations

import ctypes
import math

import numpy as np
import torch

from . import inputs
from .irbe import IRBE_ABI_VERSION, IRBE_FP64, IRBE_MIXED_FP32, DynConfig, IRBEError, load_library

M_O = 15.9994  # g/mol
M_H = 1.008
KB = 0.0083144626  # kJ/mol/K
THERMOSTAT = {"langevin": 0, "nose_hoover": 1}


def water_topology(n_waters: int):
    """Constraint groups (O, H, H) with the rigid geometry of the inputs
    (OH = 0.1 nm, HOH = 109.47 degrees) and inverse masses, atoms ordered
    O, H, H per molecule."""
    groups = np.arange(3 * n_waters, dtype=np.int32).reshape(n_waters, 3)
    d_hh = 2.0 * inputs.R_OH * math.sin(math.radians(inputs.THETA_HOH_DEG) / 2.0)
    lengths = np.tile(np.array([inputs.R_OH, inputs.R_OH, d_hh]), (n_waters, 1))
    inv_mass = np.tile(np.array([1.0 / M_O, 1.0 / M_H, 1.0 / M_H]), n_waters)
    return groups, lengths, inv_mass


class Langevin:
    """One integrator on the current HIP stream of ``device``."""

    def __init__(self, inv_mass, groups, lengths, *, dt: float, gamma: float, kT: float, seed: int = 1,
                 precision: str = "mixed", thermostat: str = "langevin", tau: float = 0.0, device=None):
        self.lib = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("the IRBE HIP library needs a GPU")
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.force_dtype = torch.float64 if precision == "fp64" else torch.float32
        inv_mass = torch.as_tensor(np.asarray(inv_mass, dtype=np.float64), device=self.device).contiguous()
        groups = torch.as_tensor(np.asarray(groups, dtype=np.int32), device=self.device).contiguous()
        lengths = torch.as_tensor(np.asarray(lengths, dtype=np.float64), device=self.device).contiguous()
        self.n_atoms = int(inv_mass.shape[0])
        self.inv_mass = inv_mass
        cfg = DynConfig(IRBE_ABI_VERSION, IRBE_FP64 if precision == "fp64" else IRBE_MIXED_FP32, self.n_atoms,
                        int(groups.shape[0]), float(dt), float(gamma), float(kT), int(seed), THERMOSTAT[thermostat], 0,
                        float(tau))
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
            h = ctypes.c_void_p()
            st = self.lib.irbe_dyn_create(ctypes.byref(cfg), ctypes.c_void_p(self.stream.cuda_stream),
                                          ctypes.byref(h))
        if st != 0:
            raise IRBEError(st, self.lib.irbe_dyn_last_error(None).decode())
        self.h = h
        self._check(self.lib.irbe_dyn_set_system(self.h, _p(inv_mass), _p(groups), _p(lengths)))
        self.n_dof = int(self.lib.irbe_dyn_degrees_of_freedom(self.h))

    def _check(self, st: int):
        if st != 0:
            raise IRBEError(st, self.lib.irbe_dyn_last_error(self.h).decode())

    def _arr(self, t, shape, dtype):
        if not isinstance(t, torch.Tensor) or t.device != self.device or t.dtype != dtype or not t.is_contiguous() \
                or tuple(t.shape) != tuple(shape):
            raise ValueError(f"expected a contiguous {dtype} tensor of shape {shape} on {self.device}")
        return t

    def step(self, pos: torch.Tensor, vel: torch.Tensor, force: torch.Tensor, step: int,
             pos_copy: torch.Tensor | None = None):
        """Advances pos and vel (FP64, [N, 3]) in place; pos_copy (force dtype) receives the new positions."""
        n = self.n_atoms
        self._arr(pos, (n, 3), torch.float64)
        self._arr(vel, (n, 3), torch.float64)
        self._arr(force, (n, 3), self.force_dtype)
        if pos_copy is not None:
            self._arr(pos_copy, (n, 3), self.force_dtype)
        self._check(self.lib.irbe_dyn_step(self.h, _p(pos), _p(vel), _p(force), int(step), _p(pos_copy)))

    def kinetic(self, vel: torch.Tensor) -> torch.Tensor:
        """Kinetic energy (kJ/mol) as a 1-element device tensor (not synchronised)."""
        self._arr(vel, (self.n_atoms, 3), torch.float64)
        out = torch.empty(1, dtype=torch.float64, device=self.device)
        self._check(self.lib.irbe_dyn_kinetic(self.h, _p(vel), _p(out)))
        return out

    def msd(self, pos: torch.Tensor, ref: torch.Tensor, sel: torch.Tensor) -> torch.Tensor:
        self._arr(pos, (self.n_atoms, 3), torch.float64)
        self._arr(ref, (self.n_atoms, 3), torch.float64)
        self._arr(sel, (sel.shape[0],), torch.int32)
        out = torch.empty(1, dtype=torch.float64, device=self.device)
        self._check(self.lib.irbe_dyn_msd(self.h, _p(pos), _p(ref), _p(sel), int(sel.shape[0]), _p(out)))
        return out

    def rdf(self, pos: torch.Tensor, sel: torch.Tensor, box: float, r_max: float, hist: torch.Tensor,
            sel_b: torch.Tensor | None = None):
        """Adds to hist (int64, [n_bins]) the pair-distance counts of the selected
        atoms (pairs within sel, or between sel and sel_b)."""
        self._arr(pos, (self.n_atoms, 3), torch.float64)
        self._arr(sel, (sel.shape[0],), torch.int32)
        if sel_b is not None:
            self._arr(sel_b, (sel_b.shape[0],), torch.int32)
        self._arr(hist, (hist.shape[0],), torch.int64)
        self._check(self.lib.irbe_dyn_rdf(self.h, _p(pos), _p(sel), int(sel.shape[0]), _p(sel_b),
                                          0 if sel_b is None else int(sel_b.shape[0]), float(box), float(r_max),
                                          int(hist.shape[0]), _p(hist)))

    def thermostat_state(self) -> torch.Tensor:
        """Nose-Hoover {xi, sum of h xi} as a 2-element device tensor (zeros for Langevin)."""
        out = torch.empty(2, dtype=torch.float64, device=self.device)
        self._check(self.lib.irbe_dyn_thermostat_state(self.h, _p(out)))
        return out

    def check(self):
        """Waits and raises on a non-finite state or a constraint iteration that did not converge."""
        self._check(self.lib.irbe_dyn_check(self.h))

    def close(self):
        if getattr(self, "h", None):
            self.lib.irbe_dyn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def rdf_normalise(counts: np.ndarray, m: int, box: float, r_max: float, frames: int,
                  m_b: int | None = None) -> tuple[np.ndarray, np.ndarray]:
    """g(r) at the bin centres from pair counts summed over `frames` frames: pairs
    within m atoms, or between m and m_b atoms of distinct species."""
    n_bins = counts.shape[0]
    edges = np.linspace(0.0, r_max, n_bins + 1)
    pairs = 0.5 * m * (m - 1) if m_b is None else float(m) * m_b
    ideal = pairs / box ** 3 * 4.0 / 3.0 * math.pi * (edges[1:] ** 3 - edges[:-1] ** 3) * frames
    return 0.5 * (edges[1:] + edges[:-1]), counts / ideal
