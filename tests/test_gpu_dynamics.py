"""The Langevin integrator and the observables on the GPU (through the C ABI)
against the FP64 dynamics oracle, and a short coupled run with the IRBE force.

Steps: positions and velocities within 1e-12 (relative to their scale) of the
oracle's after one step and after 20 chained steps, in both force precisions;
kinetic energy and mean-squared displacement to rounding; radial distribution
counts bit-exact (the distance and bin arithmetic is the plain definition's,
without fused operations, on both sides).
"""
import math

import numpy as np
import pytest

from paper_2204_13595_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dyn_orc():
    from oracle import dynamics
    return dynamics


def _state(n_waters=4096, box=4.97, seed=3):
    from paper_2204_13595_amd import dynamics
    w = inputs.make_water(n_waters, box, seed=seed)
    groups, lengths, inv_mass = dynamics.water_topology(n_waters)
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(w.pos.shape) * np.sqrt(2.5 * inv_mass)[:, None]
    f = rng.standard_normal(w.pos.shape) * 800.0
    return w, groups, lengths, inv_mass, v, f


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_langevin_steps_match_oracle(dyn_orc, precision):
    from paper_2204_13595_amd import dynamics
    w, groups, lengths, inv_mass, v0, f0 = _state()
    dev = torch.device("cuda", 0)
    fdt = torch.float64 if precision == "fp64" else torch.float32
    d = dynamics.Langevin(inv_mass, groups, lengths, dt=0.002, gamma=1.0, kT=2.4777, seed=77, precision=precision,
                          device=dev)
    pos = torch.tensor(w.pos, device=dev)
    vel = torch.tensor(v0, device=dev)
    x, v = w.pos.copy(), v0.copy()
    rng = np.random.default_rng(5)
    copy = torch.empty((w.n_atoms, 3), dtype=fdt, device=dev)
    for s in range(20):
        f = f0 if s == 0 else rng.standard_normal(x.shape) * 800.0
        ft = torch.tensor(f, dtype=fdt, device=dev)
        d.step(pos, vel, ft, 1000 + s, pos_copy=copy)
        x, v = dyn_orc.langevin_step(x, v, ft.double().cpu().numpy(), inv_mass, groups, lengths, 0.002, 1.0, 2.4777,
                                     77, 1000 + s)
        if s == 0 or s == 19:
            gx, gv = pos.cpu().numpy(), vel.cpu().numpy()
            assert np.abs(gx - x).max() < 1e-12 * np.abs(x).max(), s
            assert np.abs(gv - v).max() < 1e-11 * np.abs(v).max(), s
            assert np.array_equal(copy.cpu().numpy(), gx.astype(copy.cpu().numpy().dtype))
    d.check()
    d.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_nose_hoover_steps_match_oracle(dyn_orc, precision):
    from paper_2204_13595_amd import dynamics
    w, groups, lengths, inv_mass, v0, f0 = _state()
    dev = torch.device("cuda", 0)
    fdt = torch.float64 if precision == "fp64" else torch.float32
    kT, tau, h = 2.4777, 0.1, 0.002
    d = dynamics.Langevin(inv_mass, groups, lengths, dt=h, gamma=0.0, kT=kT, precision=precision,
                          thermostat="nose_hoover", tau=tau, device=dev)
    n_dof = dyn_orc.degrees_of_freedom(groups, lengths, w.n_atoms)
    assert d.n_dof == n_dof
    pos = torch.tensor(w.pos, device=dev)
    vel = torch.tensor(v0, device=dev)
    x, v, nh = w.pos.copy(), v0.copy(), (0.0, 0.0)
    rng = np.random.default_rng(9)
    for s in range(20):
        ft = torch.tensor(f0 if s == 0 else rng.standard_normal(x.shape) * 800.0, dtype=fdt, device=dev)
        d.step(pos, vel, ft, s)
        x, v, nh = dyn_orc.nose_hoover_step(x, v, ft.double().cpu().numpy(), inv_mass, groups, lengths, h, kT, tau,
                                            n_dof, nh)
    state = d.thermostat_state().cpu().numpy()
    assert abs(state[0] - nh[0]) < 1e-11 * max(abs(nh[0]), 1.0)
    assert abs(state[1] - nh[1]) < 1e-11 * max(abs(nh[1]), 1.0)
    assert np.abs(pos.cpu().numpy() - x).max() < 1e-12 * np.abs(x).max()
    assert np.abs(vel.cpu().numpy() - v).max() < 1e-11 * np.abs(v).max()
    d.check()
    d.close()


def test_kinetic_msd_rdf_match_oracle(dyn_orc):
    from paper_2204_13595_amd import dynamics
    w, groups, lengths, inv_mass, v0, _ = _state()
    dev = torch.device("cuda", 0)
    d = dynamics.Langevin(inv_mass, groups, lengths, dt=0.002, gamma=1.0, kT=2.4777, device=dev)
    pos = torch.tensor(w.pos, device=dev)
    vel = torch.tensor(v0, device=dev)
    ke = d.kinetic(vel).item()
    assert abs(ke - dyn_orc.kinetic_energy(v0, inv_mass)) < 1e-12 * ke
    ref = pos + 0.05 * torch.tensor(np.random.default_rng(2).standard_normal(w.pos.shape), device=dev)
    sel = torch.arange(0, w.n_atoms, 3, dtype=torch.int32, device=dev)
    m = d.msd(pos, ref, sel).item()
    assert abs(m - dyn_orc.msd(w.pos, ref.cpu().numpy(), sel.cpu().numpy())) < 1e-12 * m
    for r_max, bins in ((2.4, 480), (1.0, 7)):
        hist = torch.zeros(bins, dtype=torch.int64, device=dev)
        d.rdf(pos, sel, w.box, r_max, hist)
        d.rdf(pos, sel, w.box, r_max, hist)  # accumulates
        got = hist.cpu().numpy()
        want = dyn_orc.rdf_counts(w.pos, sel.cpu().numpy(), w.box, r_max, bins)
        assert np.array_equal(got, 2 * want)
    # between oxygens and the first hydrogens, plus three oxygens in both selections
    sel_b = torch.cat([torch.arange(1, w.n_atoms, 3, dtype=torch.int32, device=dev), sel[:3]])
    hist = torch.zeros(300, dtype=torch.int64, device=dev)
    d.rdf(pos, sel, w.box, 1.5, hist, sel_b=sel_b)
    want = dyn_orc.rdf_counts(w.pos, sel.cpu().numpy(), w.box, 1.5, 300, sel_b=sel_b.cpu().numpy())
    assert np.array_equal(hist.cpu().numpy(), want)
    d.close()


def test_free_waters_thermalize_and_keep_their_shape():
    from paper_2204_13595_amd import dynamics
    nw = 4096
    w = inputs.make_water(nw, 20.0, seed=6)
    groups, lengths, inv_mass = dynamics.water_topology(nw)
    dev = torch.device("cuda", 0)
    kT = 2.4777
    d = dynamics.Langevin(inv_mass, groups, lengths, dt=0.002, gamma=5.0, kT=kT, seed=3, precision="fp64",
                          device=dev)
    pos = torch.tensor(w.pos, device=dev)
    vel = torch.zeros_like(pos)
    zero = torch.zeros_like(pos)
    ks = []
    for s in range(2000):
        d.step(pos, vel, zero, s)
        if s >= 400 and s % 10 == 0:
            ks.append(d.kinetic(vel))
    d.check()
    ratio = torch.cat(ks).mean().item() / (3.0 * kT * nw)
    assert abs(ratio - 1.0) < 0.01, ratio
    x = pos.cpu().numpy()
    for k, (p, q) in enumerate(((0, 1), (0, 2), (1, 2))):
        dist = np.linalg.norm(x[groups[:, q]] - x[groups[:, p]], axis=1)
        assert np.abs(dist / lengths[:, k] - 1.0).max() < 1e-12
    d.close()


def test_invalid_topology_rejected():
    from paper_2204_13595_amd import dynamics, irbe
    groups, lengths, inv_mass = dynamics.water_topology(4)
    bad = groups.copy()
    bad[1, 2] = 0  # atom 0 twice
    with pytest.raises(irbe.IRBEError):
        dynamics.Langevin(inv_mass, bad, lengths, dt=0.002, gamma=1.0, kT=1.0)
    with pytest.raises(irbe.IRBEError):
        dynamics.Langevin(np.where(np.arange(12) == 5, 0.0, inv_mass), groups, lengths, dt=0.002, gamma=1.0, kT=1.0)
    with pytest.raises(irbe.IRBEError):
        dynamics.Langevin(inv_mass, groups, lengths, dt=0.0, gamma=1.0, kT=1.0)
    with pytest.raises(irbe.IRBEError):
        dynamics.Langevin(inv_mass, groups[:, ::-1].copy() * 0 - 1, lengths, dt=0.002, gamma=1.0, kT=1.0)


def test_short_water_run_with_irbe_forces():
    """901 waters, L = 3 nm, 1000 steps of RBL+RBE forces and Langevin steps
    (lists rebuilt every step) from the lattice start: no error, and the mean
    temperature of the run within 25% of the target (the lattice start is still
    releasing potential energy; the long runs settle at the target)."""
    from paper_2204_13595_amd import md
    res = md.run_water(warm_steps=1000, equil_steps=0, prod_steps=1000, sample_every=50)
    assert res["frames"] == 20
    assert abs(res["temperature"] / 298.0 - 1.0) < 0.25, res["temperature"]
    assert np.isfinite(res["u_per_molecule"])
    assert np.all(np.isfinite(res["g"]))


def test_short_electrolyte_run():
    """2:1 primitive-model electrolyte, 1,500 steps of RBL+RBE forces with the
    shifted-truncated LJ and Langevin steps: no error, finite observables."""
    from paper_2204_13595_amd import md
    res = md.run_electrolyte(2, equil_steps=500, prod_steps=1000, sample_every=50, msd_window=500,
                             msd_origin_every=250)
    assert res["frames"] == 20
    assert np.isfinite(res["u_per_atom"]) and res["u_per_atom"] < 0.0
    for k in ("g+-", "g++", "g--", "msd+", "msd-"):
        assert np.all(np.isfinite(res[k])), k


def test_selection_outside_the_system_is_flagged():
    """msd and rdf skip selection entries outside [0, N) and report them at the next check."""
    from paper_2204_13595_amd import dynamics, irbe
    groups, lengths, inv_mass = dynamics.water_topology(4)
    dev = torch.device("cuda", 0)
    d = dynamics.Langevin(inv_mass, groups, lengths, dt=0.002, gamma=1.0, kT=1.0, device=dev)
    pos = torch.tensor(inputs.make_water(4, 2.0).pos, device=dev)
    bad = torch.tensor([0, 3, 99], dtype=torch.int32, device=dev)
    m = d.msd(pos, pos, bad)
    with pytest.raises(irbe.IRBEError):
        d.check()
    assert m.item() == 0.0
    hist = torch.zeros(10, dtype=torch.int64, device=dev)
    d.rdf(pos, bad, 2.0, 1.0, hist)
    with pytest.raises(irbe.IRBEError):
        d.check()
    assert int(hist.sum().item()) == 1  # the one pair of valid atoms, (0, 3), 0.99 nm apart
    d.check()  # cleared
    d.close()
