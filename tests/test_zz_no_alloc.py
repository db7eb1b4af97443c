"""irbe_compute_forces_noalloc (per-call scratch in a static device array)
against irbe_compute_forces on the same handle, through the C ABI.

Both run the same kernels with the same launch shapes, so forces and energies
must agree bit for bit. Two calls in a row, the second on a smaller system, so
that the second reuses the array the first one filled."""
import numpy as np
import pytest

from paper_2204_13595_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _handle(w, precision, p_shell=100, p_kspace=100, shell_entries=0):
    from paper_2204_13595_amd import irbe
    dt = torch.float64 if precision == "fp64" else torch.float32
    dev = torch.device("cuda", 0)
    h = irbe.Handle(w.n_atoms, w.box, p_shell=p_shell, p_kspace=p_kspace, precision=precision,
                    shell_entries=shell_entries, device=dev)
    pos = torch.tensor(w.pos, dtype=dt, device=dev)
    q = torch.tensor(w.charge, dtype=dt, device=dev)
    h.set_system(torch.tensor(w.atom_type, device=dev), q, torch.tensor(w.molecule, device=dev), w.lj_sigma, w.lj_eps)
    return h, pos


def _compare(h, pos, step):
    f_ref, ev_ref = h.compute_forces(pos, step, energy=True)
    f = torch.full_like(f_ref, float("nan"))
    ev = torch.full((11,), float("nan"), dtype=torch.float64, device=pos.device)
    h.compute_forces_noalloc(pos, step, f, ev)
    h.sync()
    assert torch.equal(f, f_ref)
    assert torch.equal(ev, ev_ref)
    # forces without energies (a kernel variant of its own), into a fresh buffer
    f_ref2 = h.compute_forces(pos, step)
    f2 = torch.full_like(f_ref, float("nan"))
    h.compute_forces_noalloc(pos, step, f2)
    h.sync()
    assert torch.equal(f2, f_ref2)


@pytest.mark.parametrize("precision,p_shell,entries", [("mixed", 100, 0), ("fp64", 100, 0), ("mixed", 0, 0),
                                                       ("mixed", 100, 32)])
def test_noalloc_matches_compute_forces_large_then_small(precision, p_shell, entries):
    """water4k takes 16-bit shell entries by default (entries = 32: indices);
    water512, whose stencil wraps the box, 32-bit ones."""
    for name, step in (("water4k", 3), ("water512", 7)):
        w = inputs.workload(name)
        h, pos = _handle(w, precision, p_shell=p_shell, shell_entries=entries)
        h.build_lists(pos, step)
        _compare(h, pos, step)
        # the handle keeps working as before: the normal path after the no-alloc one
        g = torch.ones_like(pos)
        gp_a, gq_a, _ = h.compute_forces_backward(pos, step, g)
        f_b = h.compute_forces(pos, step)
        gp_b, gq_b, _ = h.compute_forces_backward(pos, step, g)
        h.sync()
        assert torch.equal(gp_a, gp_b) and torch.equal(gq_a, gq_b)
        assert torch.isfinite(f_b).all()
        h.close()


def test_noalloc_moved_positions_and_new_step():
    w = inputs.workload("water4k")
    h, pos = _handle(w, "mixed")
    h.build_lists(pos, 0)
    rng = np.random.default_rng(5)
    moved = pos + torch.tensor(rng.uniform(-1e-3, 1e-3, size=tuple(pos.shape)), dtype=pos.dtype, device=pos.device)
    _compare(h, moved, 11)
    h.close()


def test_noalloc_rejects_system_beyond_scratch():
    from paper_2204_13595_amd import irbe
    w = inputs.workload("water32k")
    h, pos = _handle(w, "mixed", p_shell=1000)  # 2 kB of batch ranks per atom: ~200 MB
    h.build_lists(pos, 0)
    f = torch.empty_like(pos)
    with pytest.raises(irbe.IRBEError) as ei:
        h.compute_forces_noalloc(pos, 0, f)
    assert ei.value.status == -4 and "scratch" in str(ei.value)
    # the handle is unchanged: the normal path still runs
    h.compute_forces(pos, 0, out=f)
    h.sync()
    assert torch.isfinite(f).all()
    h.close()
