"""Pins of the dynamics oracle (oracle/dynamics.py) against what the equations
of motion and the splitting fix, independently of the oracle's own formulas.

* the thermostat noise is standard normal (moments, independence);
* for a harmonic potential the kick-drift-noise-drift splitting samples the
  exact Boltzmann distribution of the positions, kT/k per component, for any
  stable step (Leimkuhler and Matthews 2013): a step in another order or a
  wrong noise amplitude is off by (omega h / 2)^2 or more;
* free rigid water molecules thermalize to equipartition, 3 kT per molecule
  (3 translational and 3 rotational degrees of freedom);
* constraint lengths hold to rounding and, without friction or forces, the
  total momentum is conserved;
* without friction the total energy of a cluster of rigid waters under a
  conservative potential written here does not drift;
* with the Nose-Hoover thermostat the extended energy U + K + n_dof kT
  (tau^2 xi^2 / 2 + integral of xi) of that cluster does not drift, and the mean
  kinetic energy settles at n_dof kT / 2.
"""
import math

import numpy as np
import pytest

from paper_2204_13595_amd import inputs

M_O, M_H = 15.9994, 1.008


@pytest.fixture(scope="module")
def dyn():
    from oracle import dynamics
    return dynamics


def _water_groups(n_waters):
    groups = np.arange(3 * n_waters, dtype=np.int32).reshape(n_waters, 3)
    d_hh = 2.0 * inputs.R_OH * math.sin(math.radians(inputs.THETA_HOH_DEG) / 2.0)
    lengths = np.tile(np.array([inputs.R_OH, inputs.R_OH, d_hh]), (n_waters, 1))
    inv_mass = np.tile(np.array([1.0 / M_O, 1.0 / M_H, 1.0 / M_H]), n_waters)
    return groups, lengths, inv_mass


def _singles(n):
    groups = np.stack([np.arange(n), -np.ones(n, np.int64), -np.ones(n, np.int64)], axis=1).astype(np.int32)
    return groups, np.zeros((n, 3))


def test_noise_is_standard_normal(dyn):
    n = 200000
    z = dyn.noise(2204, 77, n)
    assert z.shape == (n, 3)
    se = 1.0 / math.sqrt(n)
    assert np.all(np.abs(z.mean(axis=0)) < 5 * se)
    assert np.all(np.abs(z.var(axis=0) - 1.0) < 5 * math.sqrt(2.0) * se)
    assert np.all(np.abs((z ** 4).mean(axis=0) - 3.0) < 5 * math.sqrt(96.0) * se)
    c = np.corrcoef(z.T)
    assert np.all(np.abs(c[np.triu_indices(3, 1)]) < 5 * se)
    z2 = dyn.noise(2204, 78, n)
    assert abs(np.mean(z * z2)) < 5 * se  # another step: independent
    assert not np.array_equal(z, dyn.noise(2205, 77, n))


@pytest.mark.parametrize("omega_h", [1.0, 1.5])
def test_harmonic_positions_exact_for_any_step(dyn, omega_h):
    n, k, m, kT, gamma = 3000, 1.0, 1.0, 1.0, 1.0
    h = omega_h / math.sqrt(k / m)
    groups, lengths = _singles(n)
    inv = np.full(n, 1.0 / m)
    x = np.zeros((n, 3))
    v = np.zeros((n, 3))
    xx, vv = [], []
    for s in range(1300):
        x, v = dyn.langevin_step(x, v, -k * x, inv, groups, lengths, h, gamma, kT, 11, s)
        if s >= 100:
            xx.append((x * x).mean())
            vv.append((v * v).mean())
    # independent-sample error ~ sqrt(2/(3 n)) per step, correlated over ~1/(gamma h) steps
    tol = 6.0 * math.sqrt(2.0 / (3 * n)) * math.sqrt(2.0 / (gamma * h) / len(xx))
    assert abs(np.mean(xx) - kT / k) < tol
    assert abs(np.mean(vv) - kT / m) < tol


def test_free_rigid_waters_equipartition(dyn):
    nw = 1000
    groups, lengths, inv = _water_groups(nw)
    w = inputs.make_water(nw, 10.0, seed=3)
    x = w.pos
    v = np.zeros_like(x)
    kT, gamma, h = 2.478957, 5.0, 0.002
    ks = []
    for s in range(1500):
        x, v = dyn.langevin_step(x, v, np.zeros_like(x), inv, groups, lengths, h, gamma, kT, 5, s)
        if s >= 300:
            ks.append(dyn.kinetic_energy(v, inv))
    ratio = np.mean(ks) / (3.0 * kT * nw)
    assert abs(ratio - 1.0) < 0.02, ratio


def test_constraints_hold_and_momentum_is_conserved(dyn):
    nw = 64
    groups, lengths, inv = _water_groups(nw)
    w = inputs.make_water(nw, 2.0, seed=9)
    rng = np.random.default_rng(1)
    x = w.pos
    v = dyn.constrain_velocities(x, rng.standard_normal(x.shape), inv, groups, lengths)
    r = np.stack([x[groups[:, q]] - x[groups[:, p]] for p, q in dyn.PAIRS], axis=1)
    vr = np.stack([v[groups[:, q]] - v[groups[:, p]] for p, q in dyn.PAIRS], axis=1)
    assert np.abs((r * vr).sum(axis=2)).max() < 1e-12 * np.abs(vr).max()
    mass = 1.0 / inv
    p0 = (mass[:, None] * v).sum(axis=0)
    for s in range(50):
        x, v = dyn.langevin_step(x, v, np.zeros_like(x), inv, groups, lengths, 0.002, 0.0, 0.0, 1, s)
        d = np.stack([np.linalg.norm(x[groups[:, q]] - x[groups[:, p]], axis=1) for p, q in dyn.PAIRS], axis=1)
        assert np.abs(d / lengths - 1.0).max() < 1e-12
    p1 = (mass[:, None] * v).sum(axis=0)
    assert np.abs(p1 - p0).max() < 1e-10 * np.abs(mass[:, None] * v).sum()


def _cluster_force(x, mol, A=20.0, s=0.25, k_trap=50.0):
    """U = sum over atom pairs of different molecules of A exp(-r^2 / (2 s^2))
    + sum_i k_trap |x_i|^2 / 2, and F = -grad U."""
    d = x[None, :, :] - x[:, None, :]  # d[i, j] = x_j - x_i
    r2 = (d * d).sum(axis=2)
    other = mol[:, None] != mol[None, :]
    e = np.where(other, A * np.exp(-r2 / (2.0 * s * s)), 0.0)
    U = 0.5 * e.sum() + 0.5 * k_trap * (x * x).sum()
    # dU/dx_i = sum_j e_ij (x_j - x_i) / s^2 (repulsion pushes i away from j)
    F = -(e[:, :, None] * d).sum(axis=1) / (s * s) - k_trap * x
    return U, F


def test_energy_is_conserved_without_friction(dyn):
    nw = 27
    groups, lengths, inv = _water_groups(nw)
    w = inputs.make_water(nw, 1.2, seed=4)
    x = w.pos - w.pos.mean(axis=0)
    mol = w.molecule
    rng = np.random.default_rng(2)
    v = dyn.constrain_velocities(x, rng.standard_normal(x.shape) * np.sqrt(2.5 * inv)[:, None], inv, groups,
                                 lengths)
    h = 0.001
    U, F = _cluster_force(x, mol)
    k_prev = dyn.kinetic_energy(v, inv)
    energies = []
    for s in range(3000):
        x, v = dyn.langevin_step(x, v, F, inv, groups, lengths, h, 0.0, 0.0, 1, s)
        k_next = dyn.kinetic_energy(v, inv)
        energies.append(U + 0.5 * (k_prev + k_next))  # U at x_n, K at n -/+ 1/2
        U, F = _cluster_force(x, mol)
        k_prev = k_next
    e = np.array(energies)
    k_scale = 3.0 * 2.5 * nw
    assert np.abs(e - e[0]).max() < 0.02 * k_scale
    # no drift: the mean of the last third against the first third
    assert abs(e[-1000:].mean() - e[:1000].mean()) < 0.002 * k_scale


def test_rdf_counts_brute_force(dyn):
    rng = np.random.default_rng(3)
    box = 2.0
    pos = rng.uniform(-1.0, 3.0, size=(60, 3))
    sel = np.arange(0, 60, 2)
    r_max, n_bins = 0.9, 30
    got = dyn.rdf_counts(pos, sel, box, r_max, n_bins)
    ref = np.zeros(n_bins, dtype=np.int64)
    for a in range(len(sel)):
        for b in range(a + 1, len(sel)):
            best = min(np.linalg.norm(pos[sel[b]] - pos[sel[a]] + box * np.array([i, j, k]))
                       for i in range(-3, 4) for j in range(-3, 4) for k in range(-3, 4))
            if best < r_max:
                ref[min(int(best / (r_max / n_bins)), n_bins - 1)] += 1
    assert np.array_equal(got, ref)
    # between two selections (sharing atoms 0 and 2): every pair of distinct atoms
    sel_b = np.r_[np.arange(1, 60, 2), [0, 2]]
    got = dyn.rdf_counts(pos, sel, box, r_max, n_bins, sel_b=sel_b)
    ref = np.zeros(n_bins, dtype=np.int64)
    for a in sel:
        for b in sel_b:
            if a == b:
                continue
            best = min(np.linalg.norm(pos[b] - pos[a] + box * np.array([i, j, k]))
                       for i in range(-3, 4) for j in range(-3, 4) for k in range(-3, 4))
            if best < r_max:
                ref[min(int(best / (r_max / n_bins)), n_bins - 1)] += 1
    assert np.array_equal(got, ref)


def test_rdf_of_uniform_points_is_one(dyn):
    rng = np.random.default_rng(8)
    box, n = 3.0, 2000
    pos = rng.uniform(0.0, box, size=(n, 3))
    r_max, n_bins = 1.2, 12
    c = dyn.rdf_counts(pos, np.arange(n), box, r_max, n_bins)
    edges = np.linspace(0.0, r_max, n_bins + 1)
    ideal = 0.5 * n * (n - 1) / box ** 3 * 4.0 / 3.0 * math.pi * (edges[1:] ** 3 - edges[:-1] ** 3)
    g = c / ideal
    assert np.all(np.abs(g[3:] - 1.0) < 5.0 / np.sqrt(ideal[3:]))


def test_msd_of_a_translation(dyn):
    rng = np.random.default_rng(4)
    pos = rng.standard_normal((50, 3))
    t = np.array([0.3, -0.2, 0.7])
    assert abs(dyn.msd(pos + t, pos, np.arange(0, 50, 3)) - float(t @ t)) < 1e-14


def test_nose_hoover_extended_energy_is_conserved(dyn):
    nw = 27
    groups, lengths, inv = _water_groups(nw)
    w = inputs.make_water(nw, 1.2, seed=4)
    x = w.pos - w.pos.mean(axis=0)
    mol = w.molecule
    n_dof = dyn.degrees_of_freedom(groups, lengths, x.shape[0])
    assert n_dof == 6 * nw - 3
    kT, tau, h = 2.5, 0.05, 0.001
    v = np.zeros_like(x)
    nh = (0.0, 0.0)
    U, F = _cluster_force(x, mol)
    k_prev = dyn.kinetic_energy(v, inv)
    ext, kin = [], []
    for s in range(4000):
        xi0 = nh[0]
        x, v, nh = dyn.nose_hoover_step(x, v, F, inv, groups, lengths, h, kT, tau, n_dof, nh)
        k_next = dyn.kinetic_energy(v, inv)
        # U and xi at step n, K at n -/+ 1/2, the integral of xi up to step n
        ext.append(U + 0.5 * (k_prev + k_next) + n_dof * kT * (0.5 * tau * tau * xi0 * xi0 + nh[1] - 0.5 * h * xi0))
        kin.append(k_next)
        U, F = _cluster_force(x, mol)
        k_prev = k_next
    e = np.array(ext)
    k_scale = 0.5 * n_dof * kT
    # after the start-up transient (velocities start at zero): no drift, small excursions
    assert abs(e[-1000:].mean() - e[1000:2000].mean()) < 0.01 * k_scale
    assert np.abs(e[500:] - e[500]).max() < 0.05 * k_scale
    assert abs(np.mean(kin[1000:]) / k_scale - 1.0) < 0.05
