"""Python front end of the FP64 CPU oracle (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this module. It loads ``liborc.so`` built from ``irbe_oracle.c`` (plain
C, compiled with gcc) and runs the steps of one force evaluation of the
improved random batch Ewald method in the order of Algorithm 1 of
Liang, Xu, Zhao, arXiv:2204.13595:

  cells and core/shell lists -> shell batches -> core + rescaled shell forces
  -> momentum correction -> k samples -> structure factor -> long-range force.

Modes: ``rbl`` (random batch list + random batch Ewald, the IRBE force),
``stencil`` (the same, with the shell batch drawn from the atoms of the
stencil's cells instead of from the shell list: weight = candidate count / p~,
a drawn atom counts only when it is a shell member), ``full`` (every pair
within r_shell + random batch Ewald: the paper's "RBE" comparator) and
``ewald`` (every pair within r_shell + the full reciprocal sum: the
deterministic Ewald reference whose expectation the estimators match).
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "irbe_oracle.c")
_SO = os.path.join(_HERE, "liborc.so")

_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_f64p = ctypes.POINTER(ctypes.c_double)
_u8p = ctypes.POINTER(ctypes.c_uint8)


class _System(ctypes.Structure):
    _fields_ = [("L", ctypes.c_double), ("beta", ctypes.c_double), ("ke", ctypes.c_double),
                ("n_types", ctypes.c_int32), ("lj_cut", ctypes.c_double)]


def build_library() -> str:
    """Compile the oracle with gcc (FP64, no FMA contraction, OpenMP)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off", "-o", _SO, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build_library()
        L = ctypes.CDLL(_SO)
        L.orc_quantize.argtypes = [ctypes.c_int64, ctypes.c_double, _f64p, _u32p]
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_num_threads.argtypes = []
        L.orc_n_cells.restype = ctypes.c_int32
        L.orc_n_cells.argtypes = [ctypes.c_double, ctypes.c_double]
        L.orc_shell_reach.restype = ctypes.c_int32
        L.orc_shell_reach.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int32]
        L.orc_threshold.restype = ctypes.c_uint64
        L.orc_threshold.argtypes = [ctypes.c_double, ctypes.c_double]
        L.orc_cell_lists.argtypes = [ctypes.c_int64, ctypes.c_int32, _u32p, _i64p, _i64p]
        L.orc_build_lists.argtypes = [ctypes.c_int64, _u32p, _i32p, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_double, ctypes.c_int, _i64p, ctypes.c_int64,
                                      _i64p, _i32p, _i64p, _i32p]
        L.orc_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
        L.orc_noise_words.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64, _u32p]
        L.orc_shell_ranks.restype = ctypes.c_int32
        L.orc_shell_ranks.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32,
                                      ctypes.c_int32, _i32p]
        L.orc_ktable.restype = ctypes.c_int32
        L.orc_ktable.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int32, _u64p, _f64p, _f64p]
        L.orc_kdraw.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32, _u64p, _i32p]
        L.orc_shell_batches.argtypes = [ctypes.c_uint64, ctypes.c_uint64, _i64p, ctypes.c_int64, _i64p,
                                        ctypes.c_int32, _i64p, _i32p, _f64p]
        L.orc_exclusion_rows.argtypes = [ctypes.c_int64, _i32p, _i64p, ctypes.c_int64, _i64p, _i64p, ctypes.c_int64,
                                         _i64p, _i64p]
        L.orc_short_range.argtypes = [ctypes.POINTER(_System), ctypes.c_int64, _u32p, _f64p, _i32p, _f64p, _f64p,
                                      _i64p, ctypes.c_int64, _i64p, _i32p, _i64p, _i32p, _i64p, _i32p, _f64p,
                                      _u8p, _u8p, _f64p, _f64p]
        L.orc_batch_accept.argtypes = [_u32p, _i32p, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                       _i64p, ctypes.c_int64, _i64p, _i32p, _i64p, _i32p, _u8p]
        L.orc_exclusions.argtypes = [ctypes.POINTER(_System), _u32p, _f64p, _i64p, ctypes.c_int64, _i64p, _i64p,
                                     _f64p, _f64p]
        L.orc_structure_factor.argtypes = [_u32p, _f64p, _i64p, ctypes.c_int64, ctypes.c_int32, _i32p, _f64p]
        L.orc_kspace_force.argtypes = [ctypes.POINTER(_System), _u32p, _f64p, _i64p, ctypes.c_int64,
                                       ctypes.c_int32, _i32p, _f64p, _f64p, _f64p]
        L.orc_kspace_energy.argtypes = [ctypes.POINTER(_System), ctypes.c_int32, _i32p, _f64p, _f64p, _f64p]
        L.orc_short_range_adjoint.argtypes = [ctypes.POINTER(_System), ctypes.c_int64, _u32p, _f64p, _i32p,
                                              _f64p, _f64p, _i64p, ctypes.c_int64, _i64p, _i32p, _i64p, _i32p,
                                              _i64p, _i32p, _f64p, _u8p, _u8p, ctypes.c_int, _f64p, _f64p, _f64p,
                                              _f64p, _f64p]
        L.orc_exclusions_adjoint.argtypes = [ctypes.POINTER(_System), _u32p, _f64p, _i64p, ctypes.c_int64, _i64p,
                                             _i64p, _f64p, _f64p, _f64p]
        L.orc_kspace_adjoint.argtypes = [ctypes.POINTER(_System), _u32p, _f64p, _i64p, ctypes.c_int64,
                                         ctypes.c_int32, _i32p, _f64p, _f64p, _f64p, _f64p, _f64p]
        _lib = L
    return _lib


def _p(a, t):
    if a is None:
        return None
    return a.ctypes.data_as(t)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


COULOMB_K = 138.935458


@dataclasses.dataclass
class Params:
    box: float
    beta: float = 3.0
    r_core: float = 0.5
    r_shell: float = 1.2
    p_shell: int = 100
    p_kspace: int = 100
    seed: int = 13595
    ke: float = COULOMB_K
    n_types: int = 2
    skin: float = 0.0      # lists kept over steps: cells and list radii enlarged by the skin
    lj_cut: float = 0.0    # > 0: LJ truncated at lj_cut * sigma_ij and shifted to zero there

    @property
    def alpha(self) -> float:
        return self.beta * self.beta

    def system(self) -> _System:
        return _System(self.box, self.beta, self.ke, self.n_types, self.lj_cut)


# --------------------------------------------------------------------------- geometry

def quantize(pos: np.ndarray, box: float) -> np.ndarray:
    pos = _c(pos, np.float64)
    s = np.empty(pos.shape, dtype=np.uint32)
    rc = lib().orc_quantize(pos.shape[0], box, _p(pos, _f64p), _p(s, _u32p))
    if rc != 0:
        raise ValueError(f"quantize failed ({rc})")
    return s


def n_cells(box: float, r_core: float) -> int:
    return int(lib().orc_n_cells(box, r_core))


def shell_reach(box: float, r_shell: float, n_c: int) -> int:
    return int(lib().orc_shell_reach(box, r_shell, n_c))


def threshold(radius: float, box: float) -> int:
    return int(lib().orc_threshold(radius, box))


def cell_lists(s: np.ndarray, n_c: int):
    s = _c(s, np.uint32)
    n = s.shape[0]
    start = np.empty(n_c ** 3 + 1, dtype=np.int64)
    atoms = np.empty(max(n, 1), dtype=np.int64)
    lib().orc_cell_lists(n, n_c, _p(s, _u32p), _p(start, _i64p), _p(atoms, _i64p))
    return start, atoms[:n]


@dataclasses.dataclass
class Lists:
    core_off: np.ndarray
    core_idx: np.ndarray
    shell_off: np.ndarray
    shell_idx: np.ndarray
    rows: np.ndarray | None


def build_lists(s, mol, box, r_core, r_shell, full=False, rows=None, stencil=False, skin=0.0) -> Lists:
    """C(i) and S(i) per row (Sec. 2.3); ``full``: one list C(i) u S(i);
    ``stencil``: C(i) and, in place of S(i), the stencil candidates K(i);
    ``skin``: the radii (and the cell edge) enlarged for lists kept over steps."""
    kind = 2 if stencil else (1 if full else 0)
    s = _c(s, np.uint32)
    mol = _c(mol, np.int32)
    n = s.shape[0]
    rows_a = None if rows is None else _c(rows, np.int64)
    nr = n if rows is None else rows_a.shape[0]
    core_off = np.zeros(nr + 1, dtype=np.int64)
    shell_off = np.zeros(nr + 1, dtype=np.int64)
    L = lib()
    rc = L.orc_build_lists(n, _p(s, _u32p), _p(mol, _i32p), box, r_core, r_shell, skin, kind, _p(rows_a, _i64p),
                           nr, _p(core_off, _i64p), None, _p(shell_off, _i64p), None)
    if rc != 0:
        raise ValueError(f"build_lists: invalid geometry ({rc})")
    core_idx = np.empty(max(int(core_off[-1]), 1), dtype=np.int32)
    shell_idx = np.empty(max(int(shell_off[-1]), 1), dtype=np.int32)
    L.orc_build_lists(n, _p(s, _u32p), _p(mol, _i32p), box, r_core, r_shell, skin, kind, _p(rows_a, _i64p), nr,
                      _p(core_off, _i64p), _p(core_idx, _i32p), _p(shell_off, _i64p), _p(shell_idx, _i32p))
    return Lists(core_off, core_idx[:core_off[-1]], shell_off, shell_idx[:shell_off[-1]], rows_a)


def exclusion_lists(mol: np.ndarray, rows=None):
    """Partners of each (row) atom: the other atoms with the same molecule id >= 0, in id order."""
    mol = _c(mol, np.int32)
    n = mol.shape[0]
    ids = np.arange(n, dtype=np.int64)
    valid = ids[mol >= 0]
    order = _c(valid[np.lexsort((valid, mol[valid]))], np.int64)
    pos_in = np.full(n, -1, dtype=np.int64)
    pos_in[order] = np.arange(order.shape[0])
    rows_a = None if rows is None else _c(rows, np.int64)
    nr = n if rows is None else rows_a.shape[0]
    off = np.zeros(nr + 1, dtype=np.int64)
    L = lib()
    L.orc_exclusion_rows(n, _p(mol, _i32p), _p(order, _i64p), order.shape[0], _p(pos_in, _i64p), _p(rows_a, _i64p),
                         nr, _p(off, _i64p), None)
    idx = np.empty(max(int(off[-1]), 1), dtype=np.int64)
    L.orc_exclusion_rows(n, _p(mol, _i32p), _p(order, _i64p), order.shape[0], _p(pos_in, _i64p), _p(rows_a, _i64p),
                         nr, _p(off, _i64p), _p(idx, _i64p))
    return off, idx[:off[-1]]


# --------------------------------------------------------------------------- randomness

def philox4x32_10(ctr, key) -> np.ndarray:
    c = _c(ctr, np.uint32)
    k = _c(key, np.uint32)
    out = np.empty(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_p(c, _u32p), _p(k, _u32p), _p(out, _u32p))
    return out


def shell_ranks(seed: int, step: int, atom_id: int, n_s: int, p_s: int) -> np.ndarray:
    out = np.empty(max(min(n_s, p_s), 1), dtype=np.int32)
    cnt = lib().orc_shell_ranks(seed, step, atom_id, n_s, p_s, _p(out, _i32p))
    return out[:cnt]


def shell_batches(seed: int, step: int, lists: Lists, p_s: int):
    """Per-row batch ranks (CSR) and weights N_S / p_s (1 when N_S <= p_s)."""
    n_rows = lists.shell_off.shape[0] - 1
    rows = None if lists.rows is None else _c(lists.rows, np.int64)
    off = np.zeros(n_rows + 1, dtype=np.int64)
    L = lib()
    L.orc_shell_batches(seed, step, _p(rows, _i64p), n_rows, _p(lists.shell_off, _i64p), p_s, _p(off, _i64p), None,
                        None)
    rank = np.empty(max(int(off[-1]), 1), dtype=np.int32)
    w = np.ones(n_rows)
    L.orc_shell_batches(seed, step, _p(rows, _i64p), n_rows, _p(lists.shell_off, _i64p), p_s, _p(off, _i64p),
                        _p(rank, _i32p), _p(w, _f64p))
    return off, rank[:off[-1]], w


def batch_accept(s, mol, box, r_core, r_shell, lists: Lists, batches, kind: int = 1) -> np.ndarray:
    """Per batch entry (``batches`` = (off, rank, w)), or per list entry when
    ``batches`` is None: 1 when the atom is a member at the positions ``s`` of
    C(i) (kind 0, tested on the core list), S(i) (kind 1) or the full list
    (kind 2, on the shell arrays)."""
    s = _c(s, np.uint32)
    mol = _c(mol, np.int32)
    rows = None if lists.rows is None else _c(lists.rows, np.int64)
    if kind == 0:
        off, idx = lists.core_off, lists.core_idx
    else:
        off, idx = lists.shell_off, lists.shell_idx
    n_rows = off.shape[0] - 1
    if batches is not None:
        b_off, b_rank = _c(batches[0], np.int64), _c(batches[1], np.int32)
        total = int(b_off[-1])
    else:
        b_off = b_rank = None
        total = int(off[-1])
    out = np.zeros(max(total, 1), dtype=np.uint8)
    lib().orc_batch_accept(_p(s, _u32p), _p(mol, _i32p), box, r_core, r_shell, kind, _p(rows, _i64p), n_rows,
                           _p(_c(off, np.int64), _i64p), _p(_c(idx, np.int32), _i32p), _p(b_off, _i64p),
                           _p(b_rank, _i32p), _p(out, _u8p))
    return out


def ktable(beta: float, box: float, max_m: int = 1 << 16):
    L = lib()
    H = ctypes.c_double()
    S = ctypes.c_double()
    M = L.orc_ktable(beta, box, max_m, None, ctypes.byref(H), ctypes.byref(S))
    if M < 0:
        raise ValueError("k table too large")
    U = np.empty(2 * M + 1, dtype=np.uint64)
    L.orc_ktable(beta, box, max_m, _p(U, _u64p), None, None)
    return M, U, H.value, S.value


def kdraw(seed: int, step: int, P: int, M: int, U: np.ndarray) -> np.ndarray:
    U = _c(U, np.uint64)
    out = np.empty((P, 3), dtype=np.int32)
    lib().orc_kdraw(seed, step, P, M, _p(U, _u64p), _p(out, _i32p))
    return out


def ewald_kvectors(beta: float, box: float):
    """Half of k-space (m != 0, one of each +-m pair) with per-k weight
    exp(-k^2/(4 alpha)) >= 2^-64; weights are doubled for the missing half."""
    M, _, _, _ = ktable(beta, box)
    a = math.pi / (beta * box)
    r = np.arange(-M, M + 1)
    mz, my, mx = np.meshgrid(r, r, r, indexing="ij")
    m = np.stack([mx.ravel(), my.ravel(), mz.ravel()], axis=1)
    half = (m[:, 2] > 0) | ((m[:, 2] == 0) & (m[:, 1] > 0)) | ((m[:, 2] == 0) & (m[:, 1] == 0) & (m[:, 0] > 0))
    m = m[half]
    wgt = np.exp(-(a * a) * (m.astype(np.float64) ** 2).sum(axis=1))
    keep = wgt >= 2.0 ** -64
    return _c(m[keep], np.int32), 2.0 * wgt[keep]


# --------------------------------------------------------------------------- forces

@dataclasses.dataclass
class Result:
    force: np.ndarray          # [rows, 3]
    energy: np.ndarray         # [11]: U_coul, U_lj, U_long, U_self, U_excl, W_xx W_yy W_zz W_xy W_xz W_yz
    f_short: np.ndarray        # short-range force before the momentum correction
    f_excl: np.ndarray
    f_long: np.ndarray
    fcorr: np.ndarray
    rho: np.ndarray            # [n_k, 2]
    kvec: np.ndarray           # [n_k, 3]
    wk: np.ndarray
    lists: Lists
    batch_off: np.ndarray | None
    batch_rank: np.ndarray | None
    weight: np.ndarray | None
    s: np.ndarray
    S: float
    accept: np.ndarray | None = None
    core_accept: np.ndarray | None = None


def sample_kspace(params: Params, step: int):
    M, U, H, S = ktable(params.beta, params.box)
    m = kdraw(params.seed, step, params.p_kspace, M, U)
    return m, np.full(params.p_kspace, S / params.p_kspace), S


def structure_factor(s, q, kvec, rows=None) -> np.ndarray:
    """rho(k_l) = sum_j q_j e^{i k_l.r_j} (Eq. 2.4) over all atoms (or the rows): [n_k, 2]."""
    s = _c(s, np.uint32)
    q = _c(q, np.float64)
    m = _c(kvec, np.int32)
    rows_a = None if rows is None else _c(rows, np.int64)
    n_rows = s.shape[0] if rows is None else rows_a.shape[0]
    rho = np.zeros((m.shape[0], 2))
    lib().orc_structure_factor(_p(s, _u32p), _p(q, _f64p), _p(rows_a, _i64p), n_rows, m.shape[0], _p(m, _i32p),
                               _p(rho, _f64p))
    return rho


def forward(pos, q, atom_type, mol, lj_sigma, lj_eps, params: Params, step: int = 0, mode: str = "rbl",
            rows=None, s=None, lists: Lists | None = None, batches=None, kspace=None, rho=None,
            accept=None, core_accept=None) -> Result:
    """One force evaluation. ``s`` (quantized positions), ``lists``, ``batches``
    ((off, rank, w)), ``kspace`` ((m, W, S)) and ``accept`` / ``core_accept``
    (which drawn candidates and core entries count: stencil sampling, skin
    lists) may be given to freeze them.
    With ``rows`` only those atoms are evaluated; ``rho`` (from
    :func:`structure_factor` over all atoms) then gives their exact long-range
    force, otherwise rho is summed over the rows only."""
    q = _c(q, np.float64)
    atom_type = _c(atom_type, np.int32)
    mol = _c(mol, np.int32)
    lj_sigma = _c(lj_sigma, np.float64)
    lj_eps = _c(lj_eps, np.float64)
    if s is None:
        s = quantize(pos, params.box)
    n = s.shape[0]
    rows_a = None if rows is None else _c(rows, np.int64)
    n_rows = n if rows is None else rows_a.shape[0]
    full = mode in ("full", "ewald")
    sampled = mode in ("rbl", "stencil")
    if lists is None:
        lists = build_lists(s, mol, params.box, params.r_core, params.r_shell, full=full, rows=rows_a,
                            stencil=mode == "stencil", skin=params.skin)
    # stencil draws are always tested at these positions; list entries only when
    # the lists were built with a skin (without one they count as built)
    masked = mode == "stencil" or params.skin > 0
    if not masked:
        accept = None
    if params.skin <= 0:
        core_accept = None
    if sampled:
        if batches is None:
            batches = shell_batches(params.seed, step, lists, params.p_shell)
        b_off, b_rank, w = batches
    else:
        b_off = b_rank = w = None
    if masked:
        # entries count only when members at these positions
        if accept is None:
            accept = batch_accept(s, mol, params.box, params.r_core, params.r_shell, lists,
                                  batches if sampled else None, kind=1 if sampled else 2)
        if core_accept is None and not full and params.skin > 0:
            core_accept = batch_accept(s, mol, params.box, params.r_core, params.r_shell, lists, None, kind=0)
    if kspace is None:
        if mode == "ewald":
            m, W = ewald_kvectors(params.beta, params.box)
            S = float("nan")
        else:
            m, W, S = sample_kspace(params, step)
    else:
        m, W, S = kspace
    m = _c(m, np.int32)
    W = _c(W, np.float64)
    sy = params.system()
    L = lib()
    e8 = np.zeros(8)
    f_sr = np.zeros((n_rows, 3))
    L.orc_short_range(ctypes.byref(sy), n, _p(s, _u32p), _p(q, _f64p), _p(atom_type, _i32p), _p(lj_sigma, _f64p),
                      _p(lj_eps, _f64p), _p(rows_a, _i64p), n_rows, _p(lists.core_off, _i64p),
                      _p(_c(lists.core_idx, np.int32), _i32p), _p(lists.shell_off, _i64p),
                      _p(_c(lists.shell_idx, np.int32), _i32p), _p(b_off, _i64p),
                      _p(None if b_rank is None else _c(b_rank, np.int32), _i32p),
                      _p(None if w is None else _c(w, np.float64), _f64p), _p(core_accept, _u8p), _p(accept, _u8p),
                      _p(f_sr, _f64p), _p(e8, _f64p))
    fcorr = f_sr.mean(axis=0) if (sampled and n_rows > 0) else np.zeros(3)
    x_off, x_idx = exclusion_lists(mol, rows_a)
    e7x = np.zeros(7)
    f_x = np.zeros((n_rows, 3))
    L.orc_exclusions(ctypes.byref(sy), _p(s, _u32p), _p(q, _f64p), _p(rows_a, _i64p), n_rows, _p(x_off, _i64p),
                     _p(x_idx, _i64p), _p(f_x, _f64p), _p(e7x, _f64p))
    n_k = m.shape[0]
    if rho is None:
        rho = np.zeros((n_k, 2))
        L.orc_structure_factor(_p(s, _u32p), _p(q, _f64p), _p(rows_a, _i64p), n_rows, n_k, _p(m, _i32p),
                               _p(rho, _f64p))
    else:
        rho = _c(rho, np.float64)
    f_long = np.zeros((n_rows, 3))
    L.orc_kspace_force(ctypes.byref(sy), _p(s, _u32p), _p(q, _f64p), _p(rows_a, _i64p), n_rows, n_k,
                       _p(m, _i32p), _p(W, _f64p), _p(rho, _f64p), _p(f_long, _f64p))
    e7k = np.zeros(7)
    L.orc_kspace_energy(ctypes.byref(sy), n_k, _p(m, _i32p), _p(W, _f64p), _p(rho, _f64p), _p(e7k, _f64p))
    q_rows = q if rows_a is None else q[rows_a]
    u_self = -params.ke * params.beta / math.sqrt(math.pi) * float(np.sum(q_rows * q_rows))
    energy = np.zeros(11)
    energy[0] = e8[0]
    energy[1] = e8[1]
    energy[2] = e7k[0]
    energy[3] = u_self
    energy[4] = e7x[0]
    energy[5:11] = e8[2:8] + e7x[1:7] + e7k[1:7]
    force = f_sr - fcorr + f_x + f_long
    return Result(force, energy, f_sr, f_x, f_long, fcorr, rho, m, W, lists, b_off, b_rank, w, s, S, accept,
                  core_accept)


def backward(G, q, atom_type, mol, lj_sigma, lj_eps, params: Params, res: Result, mode: str = "rbl"):
    """Gradients of L = sum_i G_i . F_i with respect to positions, charges and the
    LJ tables, with the lists, batches and k of ``res`` frozen (all atoms)."""
    assert res.lists.rows is None
    return _adjoint(G, q, atom_type, mol, lj_sigma, lj_eps, params, res, mode, None)


def backward_rows(G, q, atom_type, mol, lj_sigma, lj_eps, params: Params, res: Result, mode: str = "rbl"):
    """The same gradients for a dL/dF = G that vanishes outside the rows of
    ``res`` (a :func:`forward` with ``rows``, its ``rho`` over all atoms) and
    sums to zero. Then G' = G - mean(G) = G (the adjoint of the momentum
    correction of Eq. (2.12) is the identity), so every short-range and
    excluded-pair term of L is a term G_i . f_ij of a row atom i with its own
    lists and batch, and A_l = sum_m q_m (G_m . k_l) e^{i k_l . r_m} runs over
    the rows: the rows' lists suffice. Returns dL/dr and dL/dq of the row atoms
    (in row order) and dL/dsigma, dL/deps (every pair's term)."""
    rows = res.lists.rows
    assert rows is not None
    G = _c(G, np.float64)
    n = res.s.shape[0]
    mask = np.zeros(n, dtype=bool)
    mask[rows] = True
    assert not np.any(G[~mask]), "dL/dF must vanish outside the rows"
    assert np.abs(G.sum(axis=0)).max() <= 1e-12 * max(np.abs(G).sum(), 1e-300), "dL/dF must sum to zero"
    g_pos, g_q, g_sig, g_eps = _adjoint(G, q, atom_type, mol, lj_sigma, lj_eps, params, res, mode, rows)
    return g_pos[rows], g_q[rows], g_sig, g_eps


def _adjoint(G, q, atom_type, mol, lj_sigma, lj_eps, params: Params, res: Result, mode, rows):
    G = _c(G, np.float64)
    q = _c(q, np.float64)
    atom_type = _c(atom_type, np.int32)
    mol = _c(mol, np.int32)
    lj_sigma = _c(lj_sigma, np.float64)
    lj_eps = _c(lj_eps, np.float64)
    s = res.s
    n = s.shape[0]
    rows_a = None if rows is None else _c(rows, np.int64)
    n_rows = n if rows is None else rows_a.shape[0]
    sy = params.system()
    L = lib()
    g_pos = np.zeros((n, 3))
    g_q = np.zeros(n)
    g_sig = np.zeros(params.n_types ** 2)
    g_eps = np.zeros(params.n_types ** 2)
    rbl = mode in ("rbl", "stencil")
    L.orc_short_range_adjoint(ctypes.byref(sy), n, _p(s, _u32p), _p(q, _f64p), _p(atom_type, _i32p),
                              _p(lj_sigma, _f64p), _p(lj_eps, _f64p), _p(rows_a, _i64p), n_rows,
                              _p(res.lists.core_off, _i64p),
                              _p(_c(res.lists.core_idx, np.int32), _i32p), _p(res.lists.shell_off, _i64p),
                              _p(_c(res.lists.shell_idx, np.int32), _i32p),
                              _p(res.batch_off if rbl else None, _i64p),
                              _p(_c(res.batch_rank, np.int32) if rbl else None, _i32p),
                              _p(_c(res.weight, np.float64) if rbl else None, _f64p),
                              _p(res.core_accept, _u8p), _p(res.accept, _u8p), int(rbl), _p(G, _f64p),
                              _p(g_pos, _f64p), _p(g_q, _f64p), _p(g_sig, _f64p), _p(g_eps, _f64p))
    x_off, x_idx = exclusion_lists(mol, rows_a)
    L.orc_exclusions_adjoint(ctypes.byref(sy), _p(s, _u32p), _p(q, _f64p), _p(rows_a, _i64p), n_rows,
                             _p(x_off, _i64p), _p(x_idx, _i64p), _p(G, _f64p), _p(g_pos, _f64p), _p(g_q, _f64p))
    L.orc_kspace_adjoint(ctypes.byref(sy), _p(s, _u32p), _p(q, _f64p), _p(rows_a, _i64p), n_rows,
                         res.kvec.shape[0], _p(res.kvec, _i32p), _p(res.wk, _f64p),
                         _p(_c(res.rho, np.float64), _f64p), _p(G, _f64p), _p(g_pos, _f64p), _p(g_q, _f64p))
    return g_pos, g_q, g_sig, g_eps


def self_energy_gradient_q(q, params: Params):
    """dU_self/dq_i (energies only; forces carry no self term)."""
    return -2.0 * params.ke * params.beta / math.sqrt(math.pi) * np.asarray(q)
