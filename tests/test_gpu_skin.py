"""Lists built with a skin and kept while the atoms move (Sec. 2.3: cells
slightly larger than r_core), on the GPU against the FP64 oracle.

The lists (cells of edge >= r_core + skin, C(i) within r_core + skin, S(i)
within (r_core - skin, r_shell + skin]) are compared bit-exactly; forces,
energies and gradients at positions moved by less than skin / 2 after the
build, where each entry counts only when it is a member at the new positions,
within the tolerances of the other parity tests.
"""
import math

import numpy as np
import pytest

from paper_2204_13595_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# (workload, skin): water4k narrow stencils (n_c = 8, R = 3); water512 a stencil
# that wraps the box (n_c = 4, R = 2) with r_shell + skin just under L/2
CASES = [("water4k", 0.1), ("water512", 0.03)]
MODES = {"rbl": dict(p_shell=100), "full": dict(p_shell=0), "stencil": dict(p_shell=100, shell_source="stencil")}


def _rms_rel(a, b):
    return float(np.sqrt(((a - b) ** 2).sum() / (b ** 2).sum()))


def _max_atom(a, b):
    """Largest per-atom error |a_i - b_i| in units of the RMS per-atom magnitude
    of b. With ~10^4 atoms whose errors scatter normally, the largest is about
    4.5 times their RMS, so a bound of 20 times the RMS tolerance holds with a
    margin while a single atom with a wrong or missing term (orders of magnitude
    above the rounding) fails it."""
    a = np.asarray(a).reshape(len(a), -1)
    b = np.asarray(b).reshape(len(b), -1)
    return float(np.sqrt(((a - b) ** 2).sum(1)).max() / np.sqrt((b ** 2).sum(1).mean()))


def _moved(pos_np, skin, seed=8):
    """Positions displaced by less than skin / 2 per atom."""
    h = skin / (2.0 * math.sqrt(3.0)) * 0.999
    return pos_np + np.random.default_rng(seed).uniform(-h, h, size=pos_np.shape)


def _setup(w, precision, skin, mode, seed=13595):
    from paper_2204_13595_amd import irbe
    dt = torch.float64 if precision == "fp64" else torch.float32
    dev = torch.device("cuda", 0)
    h = irbe.Handle(w.n_atoms, w.box, p_kspace=100, seed=seed, precision=precision, skin=skin, device=dev,
                    **MODES[mode])
    pos = torch.tensor(w.pos, dtype=dt, device=dev)
    q = torch.tensor(w.charge, dtype=dt, device=dev)
    h.set_system(torch.tensor(w.atom_type, device=dev), q, torch.tensor(w.molecule, device=dev), w.lj_sigma, w.lj_eps)
    return h, pos, q, pos.double().cpu().numpy(), q.double().cpu().numpy()


def _oracle_lists(orc, w, pos_np, skin, mode):
    return orc.build_lists(orc.quantize(pos_np, w.box), w.molecule, w.box, 0.5, 1.2, full=mode == "full",
                           stencil=mode == "stencil", skin=skin)


@pytest.mark.parametrize("mode", ["rbl", "full", "stencil"])
@pytest.mark.parametrize("name,skin", CASES)
def test_skin_lists_bit_exact(orc, name, skin, mode):
    w = inputs.workload(name)
    h, pos, q, pos_np, q_np = _setup(w, "mixed", skin, mode)
    h.build_lists(pos, 0)
    s = orc.quantize(pos_np, w.box)
    n_c = orc.n_cells(w.box, 0.5 + skin)
    start, atoms = orc.cell_lists(s, n_c)
    assert np.array_equal(h.debug("cell_start"), start)
    assert np.array_equal(h.debug("cell_atoms"), atoms)
    lists = _oracle_lists(orc, w, pos_np, skin, mode)
    if mode != "stencil":
        assert np.array_equal(h.debug("shell_off"), lists.shell_off)
        assert np.array_equal(h.debug("shell_idx"), lists.shell_idx)
    if mode != "full":
        assert np.array_equal(h.debug("core_off"), lists.core_off)
        assert np.array_equal(h.debug("core_idx"), lists.core_idx)
    if mode == "rbl":
        # the lists overlap: r_core - skin < r <= r_core + skin is in both
        both = 0
        for i in range(0, w.n_atoms, 97):
            c = lists.core_idx[lists.core_off[i]:lists.core_off[i + 1]]
            sh = lists.shell_idx[lists.shell_off[i]:lists.shell_off[i + 1]]
            both += np.intersect1d(c, sh).size
        assert both > 0
    h.close()


@pytest.mark.parametrize("precision,tol_f,tol_e", [("fp64", 1e-11, 1e-10), ("mixed", 1e-5, 2e-5)])
@pytest.mark.parametrize("mode", ["rbl", "full", "stencil"])
@pytest.mark.parametrize("name,skin", CASES)
def test_skin_forces_energies_after_moves(orc, name, skin, mode, precision, tol_f, tol_e):
    w = inputs.workload(name)
    step = 6
    h, pos, q, pos_np, q_np = _setup(w, precision, skin, mode)
    h.build_lists(pos, step)
    lists = _oracle_lists(orc, w, pos_np, skin, mode)
    pos = torch.tensor(_moved(pos_np, skin), dtype=pos.dtype, device=pos.device)
    pos_np = pos.double().cpu().numpy()
    f, ev = h.compute_forces(pos, step, energy=True)
    f = f.double().cpu().numpy()
    ev = ev.cpu().numpy()
    p = orc.Params(box=w.box, skin=skin, p_shell=MODES[mode]["p_shell"])
    ref = orc.forward(None, q_np, w.atom_type, w.molecule, w.lj_sigma, w.lj_eps, p, step=step, mode=mode,
                      s=orc.quantize(pos_np, w.box), lists=lists)
    assert _rms_rel(f, ref.force) < tol_f
    assert _max_atom(f, ref.force) < 20 * tol_f
    scale = np.abs(ref.energy[:5]).max()
    for c in range(11):
        assert abs(ev[c] - ref.energy[c]) < tol_e * scale, (c, ev[c], ref.energy[c])
    h.close()


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("mixed", 2e-5)])
@pytest.mark.parametrize("mode", ["rbl", "full", "stencil"])
def test_skin_backward_after_moves(orc, mode, precision, tol):
    w = inputs.workload("water4k")
    skin = 0.1
    step = 5
    h, pos, q, pos_np, q_np = _setup(w, precision, skin, mode)
    h.build_lists(pos, step)
    lists = _oracle_lists(orc, w, pos_np, skin, mode)
    pos = torch.tensor(_moved(pos_np, skin), dtype=pos.dtype, device=pos.device)
    pos_np = pos.double().cpu().numpy()
    G = np.random.default_rng(11).standard_normal((w.n_atoms, 3))
    Gt = torch.tensor(G, dtype=pos.dtype, device=pos.device)
    gp, gq, gl = h.compute_forces_backward(pos, step, Gt)
    if mode == "rbl":
        # the shell terms' bucket keys use the cells of the build, so atoms that
        # moved since keep to their buckets: no record takes the atomic fallback
        assert int(h.debug("adj_atomics")[0]) == 0
    gp = gp.double().cpu().numpy()
    gq = gq.double().cpu().numpy()
    gl = gl.cpu().numpy()
    p = orc.Params(box=w.box, skin=skin, p_shell=MODES[mode]["p_shell"])
    ref = orc.forward(None, q_np, w.atom_type, w.molecule, w.lj_sigma, w.lj_eps, p, step=step, mode=mode,
                      s=orc.quantize(pos_np, w.box), lists=lists)
    G_used = Gt.double().cpu().numpy()
    r_pos, r_q, r_sig, r_eps = orc.backward(G_used, q_np, w.atom_type, w.molecule, w.lj_sigma, w.lj_eps, p, ref,
                                            mode=mode)
    assert _rms_rel(gp, r_pos) < tol
    assert _max_atom(gp, r_pos) < 20 * tol
    assert _rms_rel(gq, r_q) < tol
    assert abs(gl[0] - r_sig[0]) < tol * max(abs(r_sig[0]), 1.0) * 10
    assert abs(gl[4] - r_eps[0]) < tol * max(abs(r_eps[0]), 1.0) * 10
    h.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_skin_backward_reads_forward_batch(precision):
    """Skin lists kept over steps at moved positions: after a forward and a
    backward, the forward of the next step writes its batch atoms and the backward
    reads them (with the membership test at the moved positions); its gradients
    equal bit for bit those of a handle that reads the ranks."""
    w = inputs.workload("water4k")
    skin = 0.1
    ha, pos, q, pos_np, q_np = _setup(w, precision, skin, "rbl")
    hb, *_ = _setup(w, precision, skin, "rbl")
    ha.build_lists(pos, 5)
    hb.build_lists(pos, 5)
    pos_m = torch.tensor(_moved(pos_np, skin), dtype=pos.dtype, device=pos.device)
    G = torch.tensor(np.random.default_rng(12).standard_normal((w.n_atoms, 3)), dtype=pos.dtype, device=pos.device)
    for step in (6, 7):
        ha.compute_forces(pos_m, step)
        got = ha.compute_forces_backward(pos_m, step, G)
    assert int(ha.debug("adj_batch")[0]) == 1
    hb.compute_forces(pos_m, 7)
    ref = hb.compute_forces_backward(pos_m, 7, G)
    assert int(hb.debug("adj_batch")[0]) == 0
    for x, y in zip(got, ref):
        assert torch.equal(x, y)
    ha.close()
    hb.close()


def test_skin_lists_with_all_members_equal_fresh_lists():
    """With p~ above every list length, skin lists at moved positions give the
    forces of skin-free lists built at those positions (GPU against GPU; the
    summation order differs, so FP64 agreement to rounding)."""
    from paper_2204_13595_amd import irbe
    w = inputs.workload("water4k")
    dev = torch.device("cuda", 0)
    pos0 = torch.tensor(w.pos, dtype=torch.float64, device=dev)
    pos1 = torch.tensor(_moved(w.pos, 0.1), dtype=torch.float64, device=dev)
    out = []
    for skin, build_pos in ((0.1, pos0), (0.0, pos1)):
        h = irbe.Handle(w.n_atoms, w.box, p_shell=4000, p_kspace=100, precision="fp64", skin=skin, device=dev)
        h.set_system(torch.tensor(w.atom_type, device=dev), torch.tensor(w.charge, device=dev),
                     torch.tensor(w.molecule, device=dev), w.lj_sigma, w.lj_eps)
        h.build_lists(build_pos, 3)
        out.append(h.compute_forces(pos1, 3).cpu().numpy())
        h.close()
    assert _rms_rel(out[0], out[1]) < 1e-12


def test_skin_invalid_arguments_rejected():
    from paper_2204_13595_amd import irbe
    with pytest.raises(irbe.IRBEError):
        irbe.Handle(1536, 2.4834, skin=-0.01)
    with pytest.raises(irbe.IRBEError):
        irbe.Handle(1536, 2.4834, skin=0.05)  # r_shell + skin >= L/2
    with pytest.raises(irbe.IRBEError):
        irbe.Handle(1536, 2.4834, r_core=0.7, r_shell=1.0, skin=0.2)  # floor(L / (r_core + skin)) < 3
    with pytest.raises(irbe.IRBEError):
        irbe.Handle(1536, 2.4834, skin=float("nan"))
