"""The two storages of the shell lists S(i) (Sec. 2.3): 16-bit codes (the
member's stencil row and its position in that row's candidate range of the
atom's list-build group) and 32-bit sorted indices. Both must give the oracle's
lists bit for bit, and the same batches, forces, energies and gradients bit for
bit; a stencil row whose candidate range does not fit the codes turns the
handle to 32-bit entries, on the first (waiting) build and on a later
asynchronous one, which reports it as a capacity error at the next check."""
import math

import numpy as np
import pytest

from paper_2204_13595_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _moved(pos, skin, seed=8):
    """Positions displaced by less than skin / 2 per atom (none without a skin)."""
    if skin == 0.0:
        return pos
    h = skin / (2.0 * math.sqrt(3.0)) * 0.999
    d = np.random.default_rng(seed).uniform(-h, h, size=tuple(pos.shape))
    return pos + torch.tensor(d, dtype=pos.dtype, device=pos.device)


def _water(w, precision, entries, skin=0.0):
    from paper_2204_13595_amd import irbe
    dt = torch.float64 if precision == "fp64" else torch.float32
    dev = torch.device("cuda", 0)
    h = irbe.Handle(w.n_atoms, w.box, p_shell=100, p_kspace=50, precision=precision, skin=skin,
                    shell_entries=entries, device=dev)
    h.set_system(torch.tensor(w.atom_type, device=dev), torch.tensor(w.charge, dtype=dt, device=dev),
                 torch.tensor(w.molecule, device=dev), w.lj_sigma, w.lj_eps)
    return h, torch.tensor(w.pos, dtype=dt, device=dev)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("skin", [0.0, 0.1])
def test_shell_entry_formats_agree(orc, precision, skin):
    """water4k (n_c = 9, or 8 with the skin; R = 3: 49 stencil rows): the default
    takes the codes, shell_entries = 32 the indices. Lists, batch atoms, forces,
    energies and gradients agree bit for bit: the backward reads the decoded batch
    (16-bit) or the ranks and shell rows (32-bit) after the first forward, the
    batch atoms the forward wrote after the second."""
    w = inputs.workload("water4k")
    G = np.random.default_rng(5).standard_normal((w.n_atoms, 3))
    out = {}
    for entries in (0, 32):
        h, pos = _water(w, precision, entries, skin)
        h.build_lists(pos, 3)
        assert int(h.debug("shell_bits")[0]) == (16 if entries == 0 else 32)
        lists = [h.debug(k) for k in ("core_off", "core_idx", "shell_off", "shell_idx")]
        pos_m = _moved(pos, skin)
        Gt = torch.tensor(G, dtype=pos.dtype, device=pos.device)
        res = []
        for step in (3, 4):
            f, ev = h.compute_forces(pos_m, step, energy=True)
            batch = torch.tensor(h.debug_rows("batch_atoms", np.arange(0, w.n_atoms, 7, dtype=np.int64)))
            res += [f, ev, batch, *h.compute_forces_backward(pos_m, step, Gt)]
        out[entries] = (lists, res)
        pos_np = pos.double().cpu().numpy()
        h.close()
    for a, b in zip(out[0][0], out[32][0]):
        assert np.array_equal(a, b)
    for a, b in zip(out[0][1], out[32][1]):
        assert torch.equal(a.cpu(), b.cpu())
    if skin == 0.0:
        # and the oracle's lists
        ref = orc.build_lists(orc.quantize(pos_np, w.box), w.molecule, w.box, 0.5, 1.2)
        assert np.array_equal(out[0][0][2], ref.shell_off)
        assert np.array_equal(out[0][0][3], ref.shell_idx)


def _cluster_system(n_bulk=4000, n_cluster=1100, box=5.0, seed=21):
    """Atoms spread over a 5 nm box (n_c = 10 at r_core = 0.5) and a cluster of
    1,100 atoms inside the cell (5, 5, 5): the cell rows through that cell hold
    more than the 1,024 candidates a 10-bit position can address."""
    rng = np.random.default_rng(seed)
    bulk = rng.uniform(0.0, box, size=(n_bulk, 3))
    clus = 2.75 + rng.uniform(-0.15, 0.15, size=(n_cluster, 3))
    spread = rng.uniform(0.0, box, size=(n_bulk + n_cluster, 3))
    return np.vstack([bulk, clus]), spread


def _plain_handle(n, box):
    from paper_2204_13595_amd import irbe
    dev = torch.device("cuda", 0)
    h = irbe.Handle(n, box, r_core=0.5, r_shell=1.2, p_shell=20, p_kspace=8, n_types=1, precision="fp64",
                    device=dev)
    h.set_system(torch.zeros(n, dtype=torch.int32, device=dev), torch.zeros(n, dtype=torch.float64, device=dev),
                 torch.arange(n, dtype=torch.int32, device=dev), np.array([[0.3]]), np.array([[0.5]]))
    return h


def _check_lists(orc, h, pos_np, box, n):
    s = orc.quantize(pos_np, box)
    ref = orc.build_lists(s, np.arange(n, dtype=np.int32), box, 0.5, 1.2)
    assert np.array_equal(h.debug("shell_off"), ref.shell_off)
    assert np.array_equal(h.debug("shell_idx"), ref.shell_idx)
    assert np.array_equal(h.debug("core_off"), ref.core_off)
    assert np.array_equal(h.debug("core_idx"), ref.core_idx)


def test_long_row_range_falls_back_on_first_build(orc):
    clustered, _ = _cluster_system()
    n, box = clustered.shape[0], 5.0
    h = _plain_handle(n, box)
    pos = torch.tensor(clustered, dtype=torch.float64, device="cuda")
    h.build_lists(pos, 0)
    h.sync()
    assert int(h.debug("shell_bits")[0]) == 32
    _check_lists(orc, h, clustered, box, n)
    h.close()


def test_long_row_range_falls_back_on_async_build(orc):
    from paper_2204_13595_amd import irbe
    clustered, spread = _cluster_system()
    n, box = clustered.shape[0], 5.0
    h = _plain_handle(n, box)
    pos_s = torch.tensor(spread, dtype=torch.float64, device="cuda")
    pos_c = torch.tensor(clustered, dtype=torch.float64, device="cuda")
    h.build_lists(pos_s, 0)
    assert int(h.debug("shell_bits")[0]) == 16
    _check_lists(orc, h, spread, box, n)
    # an asynchronous build whose codes (and rows) overflow: reported at the check
    h.build_lists(pos_c, 1)
    with pytest.raises(irbe.IRBEError):
        h.sync()
    h.build_lists(pos_c, 2)
    h.sync()
    assert int(h.debug("shell_bits")[0]) == 32
    _check_lists(orc, h, clustered, box, n)
    h.close()
