"""Lists of dilute systems (a few atoms per cell), which the library builds
with one lane per atom, against the oracle's lists bit for bit: split, full,
core-only (stencil sampling) and skin lists of the primitive-model electrolyte
(Sec. 4 parameters, R = 4), with and without excluded pairs, and a box with one
crowded cell row whose stencil rows no longer fit one LDS tile."""
import math

import numpy as np
import pytest

from paper_2204_13595_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

R_CORE, R_SHELL = 5.0, 15.0


def _crowded(w, n_extra=400, seed=3):
    """The electrolyte plus n_extra neutral pairs of ions in one cell row along x."""
    rng = np.random.default_rng(seed)
    cell = w.box / math.floor(w.box / R_CORE)
    x = rng.uniform(0.0, w.box, n_extra)
    y = rng.uniform(0.1, 0.9, n_extra) * cell + 2 * cell
    z = rng.uniform(0.1, 0.9, n_extra) * cell + 5 * cell
    pos = np.concatenate([w.pos, np.stack([x, y, z], 1)])
    q = np.concatenate([w.charge, np.where(np.arange(n_extra) % 2 == 0, 1.0, -1.0)])
    t = np.concatenate([w.atom_type, (np.arange(n_extra) % 2).astype(np.int32)])
    return pos, q, t


@pytest.mark.parametrize("kind", ["split", "full", "stencil", "skin"])
@pytest.mark.parametrize("system", ["plain", "pairs", "crowded"])
def test_dilute_lists_bit_exact(orc, kind, system):
    from paper_2204_13595_amd import irbe
    w = inputs.electrolyte(1)
    pos_np, q_np, t_np = w.pos, w.charge, w.atom_type
    if system == "crowded":
        pos_np, q_np, t_np = _crowded(w)
    n = len(pos_np)
    mol = np.full(n, -1, np.int32) if system != "pairs" else (np.arange(n) // 2).astype(np.int32)
    dev = torch.device("cuda", 0)
    skin = 0.5 if kind == "skin" else 0.0
    h = irbe.Handle(n, w.box, beta=math.sqrt(0.03), r_core=R_CORE, r_shell=R_SHELL,
                    p_shell=0 if kind == "full" else 10, p_kspace=20, coulomb_k=1.0,
                    shell_source="stencil" if kind == "stencil" else "list", skin=skin, device=dev)
    pos = torch.tensor(pos_np, dtype=torch.float32, device=dev)
    h.set_system(torch.tensor(t_np, device=dev), torch.tensor(q_np, dtype=torch.float32, device=dev),
                 torch.tensor(mol, device=dev), w.lj_sigma, w.lj_eps)
    h.build_lists(pos, 0)
    s = orc.quantize(pos.double().cpu().numpy(), w.box)
    ref = orc.build_lists(s, mol, w.box, R_CORE, R_SHELL, full=kind == "full", stencil=kind == "stencil", skin=skin)
    if kind != "full":
        assert np.array_equal(h.debug("core_off"), ref.core_off)
        assert np.array_equal(h.debug("core_idx"), ref.core_idx)
    if kind != "stencil":
        assert np.array_equal(h.debug("shell_off"), ref.shell_off)
        assert np.array_equal(h.debug("shell_idx"), ref.shell_idx)
    if system == "crowded" and kind != "skin":
        # a cell row (hence every stencil row over it) holds more candidates than one tile
        start = h.debug("cell_start")
        n_c = int(round((len(start) - 1) ** (1.0 / 3.0)))
        assert (start[n_c::n_c] - start[:-1:n_c]).max() > 256
    h.close()
