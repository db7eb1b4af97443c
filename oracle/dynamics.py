"""FP64 CPU oracle of the Langevin dynamics step and its observables (test
infrastructure only: only the test suite may import this module).

The equations of motion are the underdamped Langevin equations of the paper's
convergence analysis (Sec. 3): dr = v dt, m dv = (F - gamma m v) dt +
sqrt(2 gamma m kT) dW, here with gamma a rate (1/ps) so that the friction is
gamma m v, integrated with the splitting kick-drift-noise-drift (B A O A) in its
leapfrog form with one force evaluation per step, and rigid bond-length
constraints per group of at most three atoms (rigid water). One step, with
forces F(x) of the constrained positions x and w = 1/m:

  1. v <- v + h w F
  2. v <- v + w sum_k mu_k g_k             (relative velocity along each
                                             constraint vector r_k(x) made zero)
  3. y <- x + (h/2) v
  4. v <- a v + sqrt((1 - a^2) kT w) xi,   a = exp(-gamma h)
  5. y <- y + (h/2) v
  6. x' <- y + w sum_k lambda_k g_k        (|x'_q - x'_p| = d_k for every
                                             constraint (p, q); directions r_k(x))
  7. v <- v + (x' - y) / h                 (the constraint displacement as a
                                             velocity change)

g_k moves atom p by -r_k and atom q by +r_k. Step 6 is solved by Newton's
method on the squared-length conditions, step 2 is linear. xi comes from the
Philox4x32-10 block of counter (atom, 2^31, step low, 2 step high) under the
key seed, turned into three normals by the Box-Muller transform (Box and
Muller 1958) of the word pairs (w0, w1) and (w2, w3) with u = (w + 1) 2^-32 and
angle 2 pi w 2^-32.

Nose-Hoover (the thermostat of the paper's water runs, Sec. 4): step 4 is
v <- exp(-xi h) v instead, and after step 7 xi <- xi + h (2 K / (n_dof kT) - 1)
/ tau^2 with K the kinetic energy of the new velocities and n_dof = 3 N -
(constraints) - 3; U + K + n_dof kT (tau^2 xi^2 / 2 + sum h xi) is the
quantity the Nose-Hoover equations conserve.

Groups: int32 [G, 3] atom indices, -1 for an empty slot; lengths [G, 3] for
the slot pairs (0, 1), (0, 2), (1, 2), a constraint where both slots are used
and the length is > 0.
"""
from __future__ import annotations

import ctypes
import math

import numpy as np

from . import oracle as _orc

PAIRS = ((0, 1), (0, 2), (1, 2))
# G[s, k]: +1 when slot s is the second atom of pair k, -1 when it is the first
_G = np.array([[-1, -1, 0], [1, 0, -1], [0, 1, 1]], dtype=np.float64)


def noise(seed: int, step: int, n: int) -> np.ndarray:
    """[n, 3] standard normals of the thermostat for atoms 0 .. n-1."""
    w = np.empty((n, 4), dtype=np.uint32)
    _orc.lib().orc_noise_words(seed, step, n, w.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)))
    w = w.astype(np.float64)
    u1 = (w[:, 0] + 1.0) * 2.0 ** -32
    u2 = (w[:, 2] + 1.0) * 2.0 ** -32
    r1 = np.sqrt(-2.0 * np.log(u1))
    r2 = np.sqrt(-2.0 * np.log(u2))
    t1 = 2.0 * math.pi * (w[:, 1] * 2.0 ** -32)
    t2 = 2.0 * math.pi * (w[:, 3] * 2.0 ** -32)
    return np.stack([r1 * np.cos(t1), r1 * np.sin(t1), r2 * np.cos(t2)], axis=1)


def _gather(a: np.ndarray, groups: np.ndarray) -> np.ndarray:
    """[G, 3, ...] values of the group slots (zero for empty slots)."""
    out = a[np.maximum(groups, 0)]
    return np.where((groups >= 0).reshape(groups.shape + (1,) * (a.ndim - 1)), out, 0.0)


def _scatter_add(a: np.ndarray, groups: np.ndarray, delta: np.ndarray) -> np.ndarray:
    out = a.copy()
    for s in range(3):
        m = groups[:, s] >= 0
        out[groups[m, s]] += delta[m, s]
    return out


def _setup(groups, lengths, inv_mass):
    groups = np.asarray(groups, dtype=np.int64)
    lengths = np.asarray(lengths, dtype=np.float64)
    w = _gather(np.asarray(inv_mass, dtype=np.float64), groups)  # [G, 3]
    active = np.stack([(groups[:, p] >= 0) & (groups[:, q] >= 0) & (lengths[:, k] > 0)
                       for k, (p, q) in enumerate(PAIRS)], axis=1)  # [G, 3]
    # C[g, k, j] = w_q(k) G[q(k), j] - w_p(k) G[p(k), j], zero for inactive j
    C = np.zeros((groups.shape[0], 3, 3))
    for k, (p, q) in enumerate(PAIRS):
        C[:, k, :] = w[:, q, None] * _G[q][None, :] - w[:, p, None] * _G[p][None, :]
    C *= active[:, None, :]
    return groups, lengths, w, active, C


def _pair_vectors(xg):
    """[G, 3, 3] vector (second - first) of each slot pair."""
    return np.stack([xg[:, q] - xg[:, p] for p, q in PAIRS], axis=1)


def constrain_velocities(x, v, inv_mass, groups, lengths):
    """Step 2: v + w sum_k mu_k g_k with (v'_q - v'_p) . r_k = 0 for every constraint."""
    groups, lengths, w, active, C = _setup(groups, lengths, inv_mass)
    r = _pair_vectors(_gather(x, groups))
    vr = _pair_vectors(_gather(v, groups))
    M = np.einsum("gkj,gjd,gkd->gkj", C, r, r)
    b = -np.einsum("gkd,gkd->gk", vr, r)
    idle = ~active
    M[idle] = 0.0
    gi, ki = np.nonzero(idle)
    M[gi, ki, ki] = 1.0
    b[idle] = 0.0
    mu = np.linalg.solve(M, b[..., None])[..., 0]
    dv = w[:, :, None] * np.einsum("sj,gj,gjd->gsd", _G, mu * active, r)
    return _scatter_add(v, groups, dv)


def shake(x_ref, y, inv_mass, groups, lengths, tol=1e-14, max_iter=50):
    """Step 6: y + w sum_k lambda_k g_k (directions r_k of x_ref) with every
    constraint length exact, by Newton's method on |s_k|^2 - d_k^2 = 0."""
    groups, lengths, w, active, C = _setup(groups, lengths, inv_mass)
    r = _pair_vectors(_gather(x_ref, groups))
    s0 = _pair_vectors(_gather(y, groups))
    d2 = np.where(active, lengths, 1.0) ** 2
    lam = np.zeros(active.shape)
    idle = ~active
    for _ in range(max_iter):
        s = s0 + np.einsum("gkj,gjd->gkd", C, lam[..., None] * r)
        f = np.where(active, np.einsum("gkd,gkd->gk", s, s) - d2, lam)
        if np.all(np.abs(np.where(active, f / d2, 0.0)) < tol):
            break
        J = 2.0 * np.einsum("gkj,gkd,gjd->gkj", C, s, r)
        J[idle] = 0.0
        gi, ki = np.nonzero(idle)
        J[gi, ki, ki] = 1.0
        lam = lam - np.linalg.solve(J, f[..., None])[..., 0]
    else:
        raise RuntimeError("constraint iteration did not converge")
    dx = w[:, :, None] * np.einsum("sj,gj,gjd->gsd", _G, lam * active, r)
    return _scatter_add(y, groups, dx)


def langevin_step(x, v, f, inv_mass, groups, lengths, dt, gamma, kT, seed, step):
    """One step (1-7 above); returns the new positions and velocities."""
    x = np.asarray(x, dtype=np.float64)
    w = np.asarray(inv_mass, dtype=np.float64)[:, None]
    v = np.asarray(v, dtype=np.float64) + dt * w * np.asarray(f, dtype=np.float64)
    v = constrain_velocities(x, v, inv_mass, groups, lengths)
    y = x + 0.5 * dt * v
    a = math.exp(-gamma * dt)
    v = a * v + np.sqrt((1.0 - a * a) * kT * w) * noise(seed, step, x.shape[0])
    y = y + 0.5 * dt * v
    x_new = shake(x, y, inv_mass, groups, lengths)
    return x_new, v + (x_new - y) / dt


def degrees_of_freedom(groups, lengths, n_atoms: int) -> int:
    """3 N - (active constraints) - 3."""
    _, _, _, active, _ = _setup(groups, lengths, np.ones(n_atoms))
    return 3 * n_atoms - int(active.sum()) - 3


def nose_hoover_step(x, v, f, inv_mass, groups, lengths, dt, kT, tau, n_dof, nh):
    """One Nose-Hoover step; nh = (xi, sum of h xi). Returns x', v', nh'."""
    x = np.asarray(x, dtype=np.float64)
    w = np.asarray(inv_mass, dtype=np.float64)[:, None]
    v = np.asarray(v, dtype=np.float64) + dt * w * np.asarray(f, dtype=np.float64)
    v = constrain_velocities(x, v, inv_mass, groups, lengths)
    y = x + 0.5 * dt * v
    xi, integral = nh
    v = math.exp(-xi * dt) * v
    y = y + 0.5 * dt * v
    x_new = shake(x, y, inv_mass, groups, lengths)
    v = v + (x_new - y) / dt
    K = kinetic_energy(v, inv_mass)
    return x_new, v, (xi + dt * (2.0 * K / (n_dof * kT) - 1.0) / (tau * tau), integral + dt * xi)


def kinetic_energy(v, inv_mass) -> float:
    m = 1.0 / np.asarray(inv_mass, dtype=np.float64)
    return float(0.5 * np.sum(m[:, None] * np.asarray(v) ** 2))


def rdf_counts(pos, sel, box, r_max, n_bins, sel_b=None) -> np.ndarray:
    """Pairs i < j of the selected atoms (or every pair of an atom of sel and a
    different atom of sel_b) by minimum-image distance r (FP64,
    d = r_j - r_i - L rint((r_j - r_i) / L) per axis, r = sqrt(d.d) without
    fused operations), in n_bins equal bins of [0, r_max): bin floor(r / (r_max /
    n_bins)), clamped to the last; distances >= r_max are not counted."""
    sel = np.asarray(sel)
    p = np.asarray(pos, dtype=np.float64)[sel]
    out = np.zeros(n_bins, dtype=np.int64)
    width = r_max / n_bins
    for i in range(p.shape[0]):
        if sel_b is None:
            d = p[i + 1:] - p[i]
        else:
            other = np.asarray(sel_b)
            other = other[other != sel[i]]
            d = np.asarray(pos, dtype=np.float64)[other] - p[i]
        d -= box * np.rint(d / box)
        r = np.sqrt((d * d).sum(axis=1))
        b = np.minimum(np.floor(r / width).astype(np.int64), n_bins - 1)
        np.add.at(out, b[r < r_max], 1)
    return out


def msd(pos, ref, sel) -> float:
    """Mean over the selected atoms of |r - r_ref|^2 (unwrapped positions)."""
    sel = np.asarray(sel)
    d = np.asarray(pos, dtype=np.float64)[sel] - np.asarray(ref, dtype=np.float64)[sel]
    return float((d * d).sum(axis=1).mean())
