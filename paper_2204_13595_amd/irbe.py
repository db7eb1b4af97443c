"""Python binding of ``libirbe.so`` (argument marshalling only).

Every step of the force evaluation runs in the HIP kernels of the library; this
module only checks tensors, passes device pointers and the current HIP stream,
and wraps the forward/backward pair in a ``torch.autograd.Function``. There is
no fallback: if the library or a GPU is missing, the calls raise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libirbe.so")

IRBE_ABI_VERSION = 3
IRBE_MIXED_FP32 = 0
IRBE_FP64 = 1
IRBE_ENERGY = 1
IRBE_VIRIAL = 2
SHELL_SOURCE = {"list": 0, "stencil": 1}

DBG = {
    "cell_start": 1, "cell_atoms": 2, "core_off": 3, "core_idx": 4, "shell_off": 5, "shell_idx": 6,
    "batch_off": 7, "batch_rank": 8, "kvec": 9, "rho": 10, "fcorr": 11, "scalars": 12, "counts": 13,
    "batch_atoms": 14, "adj_atomics": 15, "adj_batch": 16, "shell_bits": 17,
}
_DBG_DTYPE = {1: np.int64, 2: np.int64, 3: np.int64, 4: np.int32, 5: np.int64, 6: np.int32, 7: np.int64,
              8: np.int32, 9: np.int32, 10: np.float64, 11: np.float64, 12: np.float64, 13: np.int64, 14: np.int32,
              15: np.int64, 16: np.int64, 17: np.int64}

STATUS = {0: "IRBE_OK", -1: "IRBE_EINVAL", -2: "IRBE_ENOMEM", -3: "IRBE_EHIP", -4: "IRBE_ECAPACITY",
          -5: "IRBE_ESTATE", -6: "IRBE_EUNSUPPORTED", -7: "IRBE_ENONFINITE", -8: "IRBE_ECONVERGENCE"}

EXPORTED = ("irbe_probe_rates", "irbe_create", "irbe_set_system", "irbe_update_parameters", "irbe_build_lists", "irbe_compute_forces",
            "irbe_compute_forces_backward", "irbe_compute_forces_noalloc", "irbe_sync", "irbe_enable_timing", "irbe_get_timing", "irbe_get_debug",
            "irbe_get_debug_rows", "irbe_last_error", "irbe_destroy", "irbe_dyn_create", "irbe_dyn_set_system",
            "irbe_dyn_step", "irbe_dyn_kinetic", "irbe_dyn_msd", "irbe_dyn_rdf", "irbe_dyn_thermostat_state",
            "irbe_dyn_degrees_of_freedom", "irbe_dyn_check", "irbe_dyn_last_error", "irbe_dyn_destroy")

STAGES = ("bin", "lists", "quantize", "ksample", "rho", "pair", "pair_reduce", "kspace", "energy", "grad_gather",
          "rho_adj", "pair_adj", "kspace_adj")


class DynConfig(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_int32), ("force_precision", ctypes.c_int32), ("n_atoms", ctypes.c_int64),
        ("n_groups", ctypes.c_int64), ("dt", ctypes.c_double), ("gamma", ctypes.c_double), ("kT", ctypes.c_double),
        ("seed", ctypes.c_uint64), ("thermostat", ctypes.c_int32), ("reserved", ctypes.c_int32),
        ("tau", ctypes.c_double),
    ]


class IRBEError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class Config(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_int32), ("precision", ctypes.c_int32), ("n_atoms", ctypes.c_int64),
        ("box_length", ctypes.c_double), ("ewald_beta", ctypes.c_double), ("coulomb_k", ctypes.c_double),
        ("r_core", ctypes.c_double), ("r_shell", ctypes.c_double), ("p_shell", ctypes.c_int32),
        ("p_kspace", ctypes.c_int32), ("n_types", ctypes.c_int32), ("shell_source", ctypes.c_int32),
        ("seed", ctypes.c_uint64), ("capacity_hint", ctypes.c_double), ("skin", ctypes.c_double),
        ("lj_cut", ctypes.c_double), ("shell_entries", ctypes.c_int32),
    ]


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libirbe.so (built by ``python -m paper_2204_13595_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(f"{path} is missing: build it with `python -m paper_2204_13595_amd.build`")
    L = ctypes.CDLL(path)
    vp = ctypes.c_void_p
    L.irbe_probe_rates.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    L.irbe_create.argtypes = [ctypes.POINTER(Config), vp, ctypes.POINTER(vp)]
    L.irbe_set_system.argtypes = [vp, vp, vp, vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    L.irbe_update_parameters.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    L.irbe_build_lists.argtypes = [vp, vp, ctypes.c_uint64]
    L.irbe_compute_forces.argtypes = [vp, vp, ctypes.c_uint64, vp, ctypes.c_uint32, vp]
    L.irbe_compute_forces_backward.argtypes = [vp, vp, ctypes.c_uint64, vp, vp, vp, vp]
    L.irbe_compute_forces_noalloc.argtypes = [vp, vp, ctypes.c_uint64, vp, ctypes.c_uint32, vp]
    L.irbe_sync.argtypes = [vp]
    L.irbe_enable_timing.argtypes = [vp, ctypes.c_int32]
    L.irbe_get_timing.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]
    L.irbe_get_debug.argtypes = [vp, ctypes.c_int32, vp, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]
    L.irbe_get_debug_rows.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64), ctypes.c_int64, vp,
                                      ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]
    L.irbe_last_error.argtypes = [vp]
    L.irbe_last_error.restype = ctypes.c_char_p
    L.irbe_destroy.argtypes = [vp]
    L.irbe_dyn_create.argtypes = [ctypes.POINTER(DynConfig), vp, ctypes.POINTER(vp)]
    L.irbe_dyn_set_system.argtypes = [vp, vp, vp, vp]
    L.irbe_dyn_step.argtypes = [vp, vp, vp, vp, ctypes.c_uint64, vp]
    L.irbe_dyn_kinetic.argtypes = [vp, vp, vp]
    L.irbe_dyn_msd.argtypes = [vp, vp, vp, vp, ctypes.c_int64, vp]
    L.irbe_dyn_rdf.argtypes = [vp, vp, vp, ctypes.c_int64, vp, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                               ctypes.c_int32, vp]
    L.irbe_dyn_thermostat_state.argtypes = [vp, vp]
    L.irbe_dyn_degrees_of_freedom.argtypes = [vp]
    L.irbe_dyn_check.argtypes = [vp]
    L.irbe_dyn_last_error.argtypes = [vp]
    L.irbe_dyn_last_error.restype = ctypes.c_char_p
    L.irbe_dyn_destroy.argtypes = [vp]
    L.irbe_dyn_degrees_of_freedom.restype = ctypes.c_int64
    for name in EXPORTED:
        if name not in ("irbe_last_error", "irbe_dyn_last_error", "irbe_dyn_degrees_of_freedom"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def probe_rates(stream=None) -> dict:
    """Measured VALU lane-operation rate and streaming-copy bandwidth of the
    current device (irbe_probe_rates), on `stream` (default: torch's current)."""
    L = load_library()
    s = stream if stream is not None else torch.cuda.current_stream()
    valu, copy = ctypes.c_double(), ctypes.c_double()
    st = L.irbe_probe_rates(ctypes.c_void_p(s.cuda_stream), ctypes.byref(valu), ctypes.byref(copy))
    if st != 0:
        raise IRBEError(st, L.irbe_last_error(None).decode())
    return {"valu_lane_ops_per_s": valu.value, "copy_bytes_per_s": copy.value}


def _ptr(t: torch.Tensor | None):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _dbl(a):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Handle:
    """One system size and parameter set on the current HIP stream."""

    def __init__(self, n_atoms: int, box: float, *, beta: float = 3.0, r_core: float = 0.5, r_shell: float = 1.2,
                 p_shell: int = 100, p_kspace: int = 100, seed: int = 13595, n_types: int = 2,
                 precision: str = "mixed", coulomb_k: float = 138.935458, capacity_hint: float = 0.0,
                 shell_source: str = "list", skin: float = 0.0, lj_cut: float = 0.0,
                 shell_entries: int = 0, device: torch.device | str | None = None):
        self.lib = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("the IRBE HIP library needs a GPU")
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.dtype = torch.float64 if precision == "fp64" else torch.float32
        self.n_atoms = int(n_atoms)
        self.n_types = int(n_types)
        self.cfg = Config(IRBE_ABI_VERSION, IRBE_FP64 if precision == "fp64" else IRBE_MIXED_FP32, self.n_atoms,
                          float(box), float(beta), float(coulomb_k), float(r_core), float(r_shell), int(p_shell),
                          int(p_kspace), self.n_types, SHELL_SOURCE[shell_source], int(seed), float(capacity_hint),
                          float(skin), float(lj_cut), int(shell_entries))
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
            h = ctypes.c_void_p()
            st = self.lib.irbe_create(ctypes.byref(self.cfg), ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if st != 0:
            raise IRBEError(st, self.lib.irbe_last_error(None).decode())
        self.h = h

    # -- helpers -----------------------------------------------------------
    def _check(self, st: int):
        if st != 0:
            raise IRBEError(st, self.lib.irbe_last_error(self.h).decode())

    def _vec(self, t: torch.Tensor, shape, dtype) -> torch.Tensor:
        if not isinstance(t, torch.Tensor) or t.device != self.device:
            raise ValueError(f"expected a tensor on {self.device}")
        if t.dtype != dtype:
            raise ValueError(f"expected {dtype}, got {t.dtype}")
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"expected shape {tuple(shape)}, got {tuple(t.shape)}")
        return t.contiguous()

    # -- C ABI -------------------------------------------------------------
    def set_system(self, atom_type: torch.Tensor, charge: torch.Tensor, molecule: torch.Tensor, lj_sigma, lj_eps):
        n = self.n_atoms
        t = self._vec(atom_type, (n,), torch.int32)
        q = self._vec(charge, (n,), self.dtype)
        m = self._vec(molecule, (n,), torch.int32)
        s, sp = _dbl(lj_sigma)
        e, ep = _dbl(lj_eps)
        if s.size != self.n_types ** 2 or e.size != self.n_types ** 2:
            raise ValueError("LJ tables must have n_types^2 entries")
        self._check(self.lib.irbe_set_system(self.h, _ptr(t), _ptr(q), _ptr(m), sp, ep))

    def update_parameters(self, charge: torch.Tensor | None = None, lj_sigma=None, lj_eps=None):
        q = None if charge is None else self._vec(charge, (self.n_atoms,), self.dtype)
        sp = ep = None
        if lj_sigma is not None:
            s, sp = _dbl(lj_sigma)
            e, ep = _dbl(lj_eps)
        self._check(self.lib.irbe_update_parameters(self.h, _ptr(q), sp, ep))
        self._keep = (q,)

    def build_lists(self, pos: torch.Tensor, step: int = 0):
        p = self._vec(pos, (self.n_atoms, 3), self.dtype)
        self._check(self.lib.irbe_build_lists(self.h, _ptr(p), int(step)))

    def compute_forces(self, pos: torch.Tensor, step: int = 0, out: torch.Tensor | None = None,
                       energy: bool = False):
        p = self._vec(pos, (self.n_atoms, 3), self.dtype)
        f = out if out is not None else torch.empty((self.n_atoms, 3), dtype=self.dtype, device=self.device)
        ev = torch.empty(11, dtype=torch.float64, device=self.device) if energy else None
        flags = (IRBE_ENERGY | IRBE_VIRIAL) if energy else 0
        self._check(self.lib.irbe_compute_forces(self.h, _ptr(p), int(step), _ptr(f), flags, _ptr(ev)))
        return (f, ev) if energy else f

    def compute_forces_noalloc(self, pos: torch.Tensor, step: int, out: torch.Tensor,
                               energy_out: torch.Tensor | None = None):
        """irbe_compute_forces_noalloc: the caller passes the output buffers (the
        library allocates nothing during the call)."""
        p = self._vec(pos, (self.n_atoms, 3), self.dtype)
        f = self._vec(out, (self.n_atoms, 3), self.dtype)
        ev = None if energy_out is None else self._vec(energy_out, (11,), torch.float64)
        flags = 0 if ev is None else (IRBE_ENERGY | IRBE_VIRIAL)
        self._check(self.lib.irbe_compute_forces_noalloc(self.h, _ptr(p), int(step), _ptr(f), flags, _ptr(ev)))
        return f

    def compute_forces_backward(self, pos: torch.Tensor, step: int, grad_force: torch.Tensor, want_charge=True,
                                want_lj=True):
        n = self.n_atoms
        p = self._vec(pos, (n, 3), self.dtype)
        g = self._vec(grad_force, (n, 3), self.dtype)
        gp = torch.empty((n, 3), dtype=self.dtype, device=self.device)
        gq = torch.empty(n, dtype=self.dtype, device=self.device) if want_charge else None
        gl = torch.empty(2 * self.n_types ** 2, dtype=torch.float64, device=self.device) if want_lj else None
        self._check(self.lib.irbe_compute_forces_backward(self.h, _ptr(p), int(step), _ptr(g), _ptr(gp), _ptr(gq),
                                                          _ptr(gl)))
        return gp, gq, gl

    def sync(self):
        self._check(self.lib.irbe_sync(self.h))

    def enable_timing(self, on: bool = True):
        self._check(self.lib.irbe_enable_timing(self.h, 1 if on else 0))

    def timing(self) -> dict:
        """{stage: (total ms, launches)} since timing was enabled."""
        buf = (ctypes.c_double * (2 * len(STAGES)))()
        written = ctypes.c_int64()
        self._check(self.lib.irbe_get_timing(self.h, buf, len(buf), ctypes.byref(written)))
        return {name: (buf[2 * s], int(buf[2 * s + 1])) for s, name in enumerate(STAGES)}

    def debug(self, what: str) -> np.ndarray:
        sel = DBG[what]
        written = ctypes.c_int64()
        self._check(self.lib.irbe_get_debug(self.h, sel, None, 0, ctypes.byref(written)))
        out = np.empty(max(written.value, 1), dtype=_DBG_DTYPE[sel])
        self._check(self.lib.irbe_get_debug(self.h, sel, out.ctypes.data_as(ctypes.c_void_p), written.value,
                                            ctypes.byref(written)))
        return out[:written.value]

    def debug_rows(self, what: str, rows) -> np.ndarray:
        """Per-atom read-back (core/shell lists, batch ranks) of the caller ids in rows."""
        sel = DBG[what]
        rows = np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
        rp = rows.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        written = ctypes.c_int64()
        self._check(self.lib.irbe_get_debug_rows(self.h, sel, rp, rows.size, None, 0, ctypes.byref(written)))
        out = np.empty(max(written.value, 1), dtype=_DBG_DTYPE[sel])
        self._check(self.lib.irbe_get_debug_rows(self.h, sel, rp, rows.size, out.ctypes.data_as(ctypes.c_void_p),
                                                 written.value, ctypes.byref(written)))
        return out[:written.value]

    def close(self):
        if getattr(self, "h", None):
            self.lib.irbe_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class IRBEForce(torch.autograd.Function):
    """F = IRBE force(pos, charge, LJ tables) at the samples of ``step`` and the
    lists of the handle's last build; backward gives dL/dpos, dL/dcharge and
    dL/dsigma, dL/deps of the LJ tables (n_types^2 each)."""

    @staticmethod
    def forward(ctx, pos, charge, lj_sigma, lj_eps, handle: Handle, step: int):
        handle.update_parameters(charge=charge.detach().contiguous(), lj_sigma=lj_sigma.detach().cpu().numpy(),
                                 lj_eps=lj_eps.detach().cpu().numpy())
        f = handle.compute_forces(pos.detach().contiguous(), step)
        ctx.handle = handle
        ctx.step = step
        ctx.save_for_backward(pos, charge, lj_sigma, lj_eps)
        return f

    @staticmethod
    def backward(ctx, grad_f):
        pos, charge, lj_sigma, lj_eps = ctx.saved_tensors
        h: Handle = ctx.handle
        h.update_parameters(charge=charge.detach().contiguous(), lj_sigma=lj_sigma.detach().cpu().numpy(),
                            lj_eps=lj_eps.detach().cpu().numpy())
        gp, gq, gl = h.compute_forces_backward(pos.detach().contiguous(), ctx.step, grad_f.contiguous(),
                                               want_charge=True, want_lj=True)
        nt2 = h.n_types ** 2
        g_sig = gl[:nt2].to(lj_sigma.dtype).reshape(lj_sigma.shape).to(lj_sigma.device)
        g_eps = gl[nt2:].to(lj_eps.dtype).reshape(lj_eps.shape).to(lj_eps.device)
        return gp, gq, g_sig, g_eps, None, None
