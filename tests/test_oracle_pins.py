"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

Every test here runs on the CPU. Each pins a part of the oracle against
something other than itself: published known-answer vectors, closed forms,
textbook constants, brute force on small inputs, invariants of the method, or
finite differences.
"""
import math
import os

import numpy as np
import pytest
from scipy import special, stats

from paper_2204_13595_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _water(name="water512"):
    return inputs.workload(name)


def _args(w):
    return (w.pos, w.charge, w.atom_type, w.molecule, w.lj_sigma, w.lj_eps)


# --------------------------------------------------------------------------- randomness

def test_philox_known_answers(orc):
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) if not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = orc.philox4x32_10(v[0:4], v[4:6])
        assert [int(x) for x in out] == v[6:10]


def test_floyd_subsets_equiprobable(orc):
    # N_S = 6, p = 3: all C(6,3) = 20 subsets must be equally likely.
    counts = {}
    n_draw = 20000
    for t in range(n_draw):
        r = tuple(sorted(orc.shell_ranks(7, t // 1000, t % 1000, 6, 3).tolist()))
        assert len(set(r)) == 3 and all(0 <= x < 6 for x in r)
        counts[r] = counts.get(r, 0) + 1
    assert len(counts) == 20
    obs = np.array(list(counts.values()))
    chi2 = ((obs - n_draw / 20) ** 2 / (n_draw / 20)).sum()
    assert stats.chi2.sf(chi2, 19) > 1e-4


def test_floyd_inclusion_probability(orc):
    n_s, p = 57, 11
    hits = np.zeros(n_s)
    n_draw = 6000
    for t in range(n_draw):
        r = orc.shell_ranks(99, 3, t, n_s, p)
        assert len(np.unique(r)) == p
        hits[r] += 1
    exp = n_draw * p / n_s
    chi2 = ((hits - exp) ** 2 / (exp * (1 - p / n_s))).sum()
    assert stats.chi2.sf(chi2, n_s - 1) > 1e-4
    # all members taken when N_S <= p (Algorithm 1)
    assert orc.shell_ranks(1, 1, 1, 5, 8).tolist() == [0, 1, 2, 3, 4]


# --------------------------------------------------------------------------- k sampling

@pytest.mark.parametrize("beta,box", [(3.0, 2.4834), (3.0, 9.93), (3.0, 31.5), (3.0, 39.7), (5.0, 2.0)])
def test_ktable_poisson_closed_form(orc, beta, box):
    """S = H^3 - 1 with H given by the Poisson-summation form (Eqs. 2.6-2.7)."""
    M, U, H, S = orc.ktable(beta, box)
    alpha = beta * beta
    m = np.arange(-4, 5)
    h_poisson = math.sqrt(alpha * box * box / math.pi) * np.exp(-alpha * m * m * box * box).sum()
    assert abs(H - h_poisson) <= 1e-14 * h_poisson
    assert abs(S - (H ** 3 - 1)) <= 1e-12 * S
    assert U[-1] == np.iinfo(np.uint64).max
    assert np.all(np.diff(U.astype(np.float64)) >= 0)
    # the weight just beyond the table is below 2^-64 (of the peak)
    assert math.exp(-(math.pi * (M + 1) / (beta * box)) ** 2) < 2.0 ** -64


def test_kdraw_marginals_and_no_zero(orc):
    beta, box = 3.0, 2.4834
    M, U, H, S = orc.ktable(beta, box)
    draws = np.concatenate([orc.kdraw(5, step, 500, M, U) for step in range(80)])
    assert not np.any(np.all(draws == 0, axis=1))
    assert np.all(np.abs(draws) <= M)
    a = math.pi / (beta * box)
    w = np.exp(-(a * np.arange(-M, M + 1)) ** 2) / H
    p0 = w[M] ** 3
    # marginal of one axis given that the triple is not (0,0,0)
    marg = w.copy()
    marg[M] -= p0
    marg /= 1.0 - p0
    for axis in range(3):
        obs = np.bincount(draws[:, axis] + M, minlength=2 * M + 1).astype(np.float64)
        exp = marg * draws.shape[0]
        keep = exp > 20
        rest_o = obs[~keep].sum()
        rest_e = exp[~keep].sum()
        o = np.append(obs[keep], rest_o)
        e = np.append(exp[keep], rest_e)
        chi2 = ((o - e) ** 2 / e).sum()
        assert stats.chi2.sf(chi2, len(o) - 1) > 1e-4


# --------------------------------------------------------------------------- geometry

def test_quantize_closed_forms(orc):
    L = 2.5
    pos = np.array([[0.0, 0.5 * L, 0.25 * L], [-0.25 * L, L, 1.75 * L], [1e-300, -1e-300, 3 * L]])
    s = orc.quantize(pos, L)
    assert s[0].tolist() == [0, 2 ** 31, 2 ** 30]
    assert s[1].tolist() == [3 * 2 ** 30, 0, 3 * 2 ** 30]
    assert s[2].tolist() == [0, 0, 0]
    with pytest.raises(ValueError):
        orc.quantize(np.array([[np.nan, 0, 0]]), L)


def _brute_lists(s, mol, box, r_core, r_shell, rows, full=False):
    """O(N^2) reference for C(i), S(i) and their canonical order."""
    n_c = int(math.floor(box / r_core))
    R = int(math.floor(r_shell * n_c / box)) + 1
    t_c = math.floor((r_core * 2 ** 32 / box) ** 2)
    t_s = math.floor((r_shell * 2 ** 32 / box) ** 2)
    d = (s[None, :, :].astype(np.int64) - s[rows, None, :].astype(np.int64))
    d = (d + 2 ** 31) % 2 ** 32 - 2 ** 31
    d2 = (d.astype(object) ** 2).sum(axis=2) if False else (d * d).sum(axis=2).astype(np.uint64)
    cell = (s.astype(np.uint64) * n_c) >> np.uint64(32)
    cell = cell.astype(np.int64)
    out = []
    for k, i in enumerate(rows):
        same = (mol == mol[i]) & (mol[i] >= 0)
        same[i] = True
        core = np.flatnonzero((d2[k] <= t_c) & ~same)
        if full:
            shell = np.flatnonzero((d2[k] <= t_s) & ~same)
        else:
            shell = np.flatnonzero((d2[k] > t_c) & (d2[k] <= t_s) & ~same)

        def order(js, reach):
            off = (cell[js] - cell[i]) % n_c
            if 2 * reach + 1 <= n_c:
                off = np.where(off > reach, off - n_c, off)
            else:
                h = (n_c - 1) // 2
                off = (off + h) % n_c - h
            key = np.lexsort((js, s[js, 0], off[:, 0], off[:, 1], off[:, 2]))
            return js[key]

        out.append((order(core, 1), order(shell, R)))
    return out


@pytest.mark.parametrize("name,nrows", [("water512", 1536), ("water4k", 400)])
def test_lists_match_brute_force(orc, name, nrows):
    w = _water(name)
    s = orc.quantize(w.pos, w.box)
    rng = np.random.default_rng(1)
    rows = np.sort(rng.choice(w.n_atoms, size=nrows, replace=False))
    lists = orc.build_lists(s, w.molecule, w.box, 0.5, 1.2, rows=rows)
    ref = _brute_lists(s, w.molecule, w.box, 0.5, 1.2, rows)
    for k in range(nrows):
        c = lists.core_idx[lists.core_off[k]:lists.core_off[k + 1]]
        sh = lists.shell_idx[lists.shell_off[k]:lists.shell_off[k + 1]]
        assert np.array_equal(c, ref[k][0])
        assert np.array_equal(sh, ref[k][1])
    full = orc.build_lists(s, w.molecule, w.box, 0.5, 1.2, full=True, rows=rows[:50])
    ref_full = _brute_lists(s, w.molecule, w.box, 0.5, 1.2, rows[:50], full=True)
    for k in range(50):
        assert np.array_equal(full.shell_idx[full.shell_off[k]:full.shell_off[k + 1]], ref_full[k][1])


@pytest.mark.parametrize("name,nrows", [("water512", 200), ("water4k", 120)])
def test_stencil_candidates_are_the_stencil_cells(orc, name, nrows):
    """K(i) = every atom of the shell stencil's cells (brute force over all atoms,
    canonical order), and it holds S(i) and C(i)."""
    w = _water(name)
    s = orc.quantize(w.pos, w.box)
    rng = np.random.default_rng(2)
    rows = np.sort(rng.choice(w.n_atoms, size=nrows, replace=False))
    st = orc.build_lists(s, w.molecule, w.box, 0.5, 1.2, rows=rows, stencil=True)
    split = orc.build_lists(s, w.molecule, w.box, 0.5, 1.2, rows=rows)
    n_c = int(math.floor(w.box / 0.5))
    R_ = int(math.floor(1.2 * n_c / w.box)) + 1
    cell = ((s.astype(np.uint64) * n_c) >> np.uint64(32)).astype(np.int64)
    for k, i in enumerate(rows):
        off = (cell - cell[i]) % n_c
        if 2 * R_ + 1 <= n_c:
            off = np.where(off > R_, off - n_c, off)
            inside = np.all(np.abs(off) <= R_, axis=1)
        else:
            h = (n_c - 1) // 2
            off = (off + h) % n_c - h
            inside = np.ones(len(s), bool)
        js = np.flatnonzero(inside)
        key = np.lexsort((js, s[js, 0], off[js, 0], off[js, 1], off[js, 2]))
        ref = js[key]
        got = st.shell_idx[st.shell_off[k]:st.shell_off[k + 1]]
        assert np.array_equal(got, ref)
        assert np.array_equal(st.core_idx[st.core_off[k]:st.core_off[k + 1]],
                              split.core_idx[split.core_off[k]:split.core_off[k + 1]])
        members = set(split.shell_idx[split.shell_off[k]:split.shell_off[k + 1]].tolist())
        assert members <= set(got.tolist())


def test_skin_lists_match_brute_force(orc):
    """Lists with a skin: cells of edge >= r_core + skin, C(i) within r_core + skin,
    S(i) within (r_core - skin, r_shell + skin], canonical order (brute force)."""
    w = _water("water4k")
    skin = 0.1
    s = orc.quantize(w.pos, w.box)
    rows = np.sort(np.random.default_rng(5).choice(w.n_atoms, size=150, replace=False))
    lists = orc.build_lists(s, w.molecule, w.box, 0.5, 1.2, rows=rows, skin=skin)
    n_c = int(math.floor(w.box / (0.5 + skin)))
    R_ = int(math.floor((1.2 + skin) * n_c / w.box)) + 1
    t = lambda r: math.floor((r * 2 ** 32 / w.box) ** 2)
    d = (s[None, :, :].astype(np.int64) - s[rows, None, :].astype(np.int64))
    d = (d + 2 ** 31) % 2 ** 32 - 2 ** 31
    d2 = (d * d).sum(axis=2).astype(np.uint64)
    cell = ((s.astype(np.uint64) * n_c) >> np.uint64(32)).astype(np.int64)
    for k, i in enumerate(rows):
        same = (w.molecule == w.molecule[i]) & (w.molecule[i] >= 0)
        same[i] = True

        def order(js, reach):
            off = (cell[js] - cell[i]) % n_c
            off = np.where(off > reach, off - n_c, off)
            return js[np.lexsort((js, s[js, 0], off[:, 0], off[:, 1], off[:, 2]))]

        core = order(np.flatnonzero((d2[k] <= t(0.5 + skin)) & ~same), 1)
        shell = order(np.flatnonzero((d2[k] > t(0.5 - skin)) & (d2[k] <= t(1.2 + skin)) & ~same), R_)
        assert np.array_equal(lists.core_idx[lists.core_off[k]:lists.core_off[k + 1]], core)
        assert np.array_equal(lists.shell_idx[lists.shell_off[k]:lists.shell_off[k + 1]], shell)


def _moved(w, skin, seed=8):
    """Positions displaced by less than skin / 2 per atom."""
    h = skin / (2.0 * math.sqrt(3.0)) * 0.999
    return w.pos + np.random.default_rng(seed).uniform(-h, h, size=w.pos.shape)


def test_list_sizes_match_density(orc):
    """Mean list sizes against (4/3) pi r^3 rho (water: the paper's ~700 within 1.2 nm)."""
    w = _water("water4k")
    s = orc.quantize(w.pos, w.box)
    lists = orc.build_lists(s, w.molecule, w.box, 0.5, 1.2)
    rho = w.n_atoms / w.box ** 3
    core = np.diff(lists.core_off).mean() + 2.0  # + the two excluded partners
    shell = np.diff(lists.shell_off).mean()
    assert abs(core - 4 / 3 * math.pi * 0.5 ** 3 * rho) < 0.06 * core
    assert abs(core + shell - 4 / 3 * math.pi * 1.2 ** 3 * rho) < 0.02 * (core + shell)


# --------------------------------------------------------------------------- Ewald reference

def _nacl(orc, beta=5.0):
    pos, q, box = inputs.nacl_crystal(2, d=0.5)
    n = q.shape[0]
    p = orc.Params(box=box, beta=beta, r_core=0.6, r_shell=0.99, ke=1.0, n_types=1)
    res = orc.forward(pos, q, np.zeros(n, np.int32), -np.ones(n, np.int32), np.zeros(1), np.zeros(1), p,
                      mode="ewald")
    return res, n


def test_madelung_constant(orc):
    madelung = float(open(os.path.join(GOLDEN, "madelung.txt")).read().split()[-1])
    res, n = _nacl(orc)
    u = res.energy[:5].sum()
    d = 0.5
    # energy per ion = -M q^2 / (2 d)
    assert abs(u / n - (-madelung / (2 * d))) < 2e-6 * madelung / (2 * d)
    assert np.abs(res.force).max() < 1e-9


@pytest.mark.parametrize("beta,tol", [(3.0, 5e-6), (3.5, 1e-7), (4.0, 1e-9)])
def test_ewald_independent_of_beta(orc, beta, tol):
    """The Ewald total (Eq. 2.3) does not depend on the splitting; what is left is
    the real-space truncation at r_shell, of order erfc(beta r_shell)."""
    w = _water()
    ref = orc.forward(*_args(w), orc.Params(box=w.box, beta=4.5), mode="ewald")
    other = orc.forward(*_args(w), orc.Params(box=w.box, beta=beta), mode="ewald")
    u0, u1 = ref.energy[:5].sum(), other.energy[:5].sum()
    assert abs(u0 - u1) < tol * abs(ref.energy[3])
    err = np.sqrt(((ref.force - other.force) ** 2).sum() / (ref.force ** 2).sum())
    assert err < tol


def test_single_molecule_energy_vanishes(orc):
    """One neutral water in a growing box: every pair is intramolecular, so the
    excluded-pair correction, the self energy and the reciprocal sum must cancel
    up to the periodic images' dipole energy, which decays as L^-3."""
    base = inputs.make_water(1, 1.0, seed=3)
    us = []
    for box in (3.0, 6.0):
        pos = base.pos - base.pos[0] + box / 2
        p = orc.Params(box=box, beta=3.0, r_core=0.6, r_shell=1.2)
        r = orc.forward(pos, base.charge, base.atom_type, base.molecule, base.lj_sigma, base.lj_eps, p, mode="ewald")
        us.append(r.energy[:5].sum())
    assert abs(us[0]) < 1.0  # kJ/mol, against an excluded-pair energy of ~1e3
    assert abs(us[1]) < abs(us[0]) / 4


def test_real_space_brute_force_raw_positions(orc):
    """Full-list real-space energy and LJ (min image, r <= r_shell, same-molecule
    pairs out) by an O(N^2) sum on the raw FP64 positions: the oracle's quantized
    geometry must agree to ~1e-7."""
    w = _water()
    p = orc.Params(box=w.box)
    res = orc.forward(*_args(w), p, mode="ewald")
    pos = w.pos
    d = pos[None, :, :] - pos[:, None, :]
    d -= w.box * np.round(d / w.box)
    r = np.sqrt((d * d).sum(axis=2))
    same = w.molecule[:, None] == w.molecule[None, :]
    mask = (r <= 1.2) & ~same
    qq = w.charge[:, None] * w.charge[None, :]
    rr = np.where(mask, r, 1.0)
    u_coul = 0.5 * (p.ke * qq * special.erfc(p.beta * rr) / rr)[mask].sum()
    oo = (w.atom_type[:, None] == 0) & (w.atom_type[None, :] == 0)
    sr6 = (inputs.SIGMA_OO / rr) ** 6
    u_lj = 0.5 * (4 * inputs.EPS_OO * (sr6 * sr6 - sr6))[mask & oo].sum()
    assert abs(res.energy[0] - u_coul) < 1e-7 * abs(u_coul) + 1e-6
    assert abs(res.energy[1] - u_lj) < 1e-7 * abs(u_lj)
    # excluded pairs: -ke q_i q_j erf(beta r)/r, each pair once
    iu = np.triu(same, 1)
    u_excl = -(p.ke * qq * special.erf(p.beta * np.where(iu, r, 1.0)) / np.where(iu, r, 1.0))[iu].sum()
    assert abs(res.energy[4] - u_excl) < 1e-7 * abs(u_excl)
    u_self = -p.ke * p.beta / math.sqrt(math.pi) * (w.charge ** 2).sum()
    assert abs(res.energy[3] - u_self) < 1e-12 * abs(u_self)


def _frozen_energy(orc, w, p, res, s):
    r = orc.forward(None, w.charge, w.atom_type, w.molecule, w.lj_sigma, w.lj_eps, p, mode="ewald", s=s,
                    lists=res.lists, kspace=(res.kvec, res.wk, float("nan")))
    return r.energy[:5].sum()


def test_ewald_force_is_minus_energy_gradient(orc):
    w = _water()
    p = orc.Params(box=w.box)
    res = orc.forward(*_args(w), p, mode="ewald")
    quantum = w.box / 2 ** 32
    hq = int(round(1e-5 / quantum))
    h = hq * quantum
    for i in (0, 1, 2, 700, 1535):
        for a in range(3):
            sp = res.s.copy()
            sm = res.s.copy()
            sp[i, a] += np.uint32(hq)
            sm[i, a] -= np.uint32(hq)
            g = (_frozen_energy(orc, w, p, res, sp) - _frozen_energy(orc, w, p, res, sm)) / (2 * h)
            assert abs(-g - res.force[i, a]) < 2e-6 * max(abs(res.force[i, a]), 100.0)


def test_ewald_virial_trace_is_strain_derivative(orc):
    """trace W = -dU/d(lambda) under the homogeneous strain (1+lambda) of box and
    positions (fractional coordinates fixed)."""
    w = _water()
    p = orc.Params(box=w.box)
    res = orc.forward(*_args(w), p, mode="ewald")
    h = 1e-6
    us = []
    m2 = (res.kvec.astype(np.float64) ** 2).sum(axis=1)
    for lam in (h, -h):
        box = w.box * (1 + lam)
        pl = orc.Params(box=box)
        wk = 2.0 * np.exp(-(2 * math.pi / box) ** 2 * m2 / (4 * pl.alpha))
        r = orc.forward(None, w.charge, w.atom_type, w.molecule, w.lj_sigma, w.lj_eps, pl, mode="ewald", s=res.s,
                        lists=res.lists, kspace=(res.kvec, wk, float("nan")))
        us.append(r.energy[:5].sum())
    dudl = (us[0] - us[1]) / (2 * h)
    trace = res.energy[5:8].sum()
    assert abs(trace + dudl) < 1e-6 * abs(dudl)


# --------------------------------------------------------------------------- the estimators

def test_rbl_reduces_to_full_list(orc):
    w = _water()
    big = orc.Params(box=w.box, p_shell=100000)
    rbl = orc.forward(*_args(w), big, mode="rbl")
    full = orc.forward(*_args(w), big, mode="full")
    assert np.all(rbl.weight == 1.0)
    assert np.abs(rbl.fcorr).max() < 1e-9
    assert np.abs(rbl.force - full.force).max() < 1e-8
    assert np.allclose(rbl.energy, full.energy, rtol=1e-12, atol=1e-8)


def test_stencil_sampling_reduces_to_full_list(orc):
    """Stencil sampling with p~ above every candidate count takes all of K(i) with
    weight 1; the acceptance test then keeps exactly S(i): the full-list short range."""
    w = _water("water4k")
    big = orc.Params(box=w.box, p_shell=100000)
    st = orc.forward(*_args(w), big, mode="stencil")
    full = orc.forward(*_args(w), big, mode="full")
    assert np.all(st.weight == 1.0)
    scale = np.abs(full.f_short).max()
    assert np.abs(st.f_short - full.f_short).max() < 1e-12 * scale
    assert np.allclose(st.energy[:2], full.energy[:2], rtol=1e-12)
    # accepted entries per row = |S(i)|
    lists = orc.build_lists(orc.quantize(w.pos, w.box), w.molecule, w.box, 0.5, 1.2)
    acc = np.add.reduceat(st.accept.astype(np.int64), st.batch_off[:-1])
    assert np.array_equal(acc, np.diff(lists.shell_off))


@pytest.mark.parametrize("mode", ["rbl", "full", "stencil"])
def test_skin_lists_exact_after_moves(orc, mode):
    """Lists built with a skin, positions then moved by less than skin / 2: with
    every list entry taken (p~ above every list length) the short-range force at
    the new positions is the full-list one of lists built there without a skin."""
    w = _water("water4k")
    skin = 0.1
    big = orc.Params(box=w.box, p_shell=100000, skin=skin)
    s0 = orc.quantize(w.pos, w.box)
    s1 = orc.quantize(_moved(w, skin), w.box)
    lists = orc.build_lists(s0, w.molecule, w.box, 0.5, 1.2, full=mode == "full", stencil=mode == "stencil",
                            skin=skin)
    r = orc.forward(None, w.charge, w.atom_type, w.molecule, w.lj_sigma, w.lj_eps, big, mode=mode, s=s1,
                    lists=lists)
    ref = orc.forward(None, w.charge, w.atom_type, w.molecule, w.lj_sigma, w.lj_eps, orc.Params(box=w.box),
                      mode="full", s=s1)
    assert np.all(r.weight == 1.0) if r.weight is not None else True
    assert np.abs(r.f_short - ref.f_short).max() < 1e-12 * np.abs(ref.f_short).max()


@pytest.mark.slow
def test_skin_lists_unbiased_over_seeds(orc):
    """Random batch list over skin lists at moved positions: the mean short-range
    force over seeds is the full-list one at those positions (z-scores)."""
    w = _water("water4k")
    skin = 0.1
    s0 = orc.quantize(w.pos, w.box)
    s1 = orc.quantize(_moved(w, skin), w.box)
    rows = np.arange(0, w.n_atoms, 97)
    lists = orc.build_lists(s0, w.molecule, w.box, 0.5, 1.2, rows=rows, skin=skin)
    ref = orc.forward(None, w.charge, w.atom_type, w.molecule, w.lj_sigma, w.lj_eps, orc.Params(box=w.box),
                      mode="full", s=s1, rows=rows)
    n_seed = 300
    f = np.empty((n_seed,) + ref.f_short.shape)
    for k in range(n_seed):
        r = orc.forward(None, w.charge, w.atom_type, w.molecule, w.lj_sigma, w.lj_eps,
                        orc.Params(box=w.box, seed=7000 + k, skin=skin), mode="rbl", s=s1, rows=rows, lists=lists)
        f[k] = r.f_short
    z = (f.mean(axis=0) - ref.f_short) / (f.std(axis=0, ddof=1) / math.sqrt(n_seed))
    assert abs((z ** 2).mean() - 1.0) < 0.15
    assert np.abs(z).max() < 5.5


@pytest.mark.slow
def test_stencil_sampling_unbiased_over_seeds(orc):
    """E[w_i sum_B f_ij 1(j in S(i))] with B drawn from K(i) and w_i = |K(i)|/p~
    is the full shell sum: the mean short-range force over seeds matches the
    full-list one (per-component z-scores)."""
    w = _water("water4k")
    s = orc.quantize(w.pos, w.box)
    rows = np.arange(0, w.n_atoms, 97)
    ref = orc.forward(None, w.charge, w.atom_type, w.molecule, w.lj_sigma, w.lj_eps, orc.Params(box=w.box),
                      mode="full", s=s, rows=rows)
    lists = orc.build_lists(s, w.molecule, w.box, 0.5, 1.2, rows=rows, stencil=True)
    n_seed = 300
    f = np.empty((n_seed,) + ref.f_short.shape)
    for k in range(n_seed):
        r = orc.forward(None, w.charge, w.atom_type, w.molecule, w.lj_sigma, w.lj_eps,
                        orc.Params(box=w.box, seed=5000 + k), mode="stencil", s=s, rows=rows, lists=lists)
        f[k] = r.f_short
    z = (f.mean(axis=0) - ref.f_short) / (f.std(axis=0, ddof=1) / math.sqrt(n_seed))
    assert abs((z ** 2).mean() - 1.0) < 0.15
    assert np.abs(z).max() < 5.5


def test_momentum_conservation(orc):
    w = _water()
    for mode in ("rbl", "full", "ewald"):
        r = orc.forward(*_args(w), orc.Params(box=w.box), mode=mode)
        scale = np.abs(r.force).sum()
        assert np.abs(r.force.sum(axis=0)).max() < 1e-10 * scale
        assert np.abs(r.f_long.sum(axis=0)).max() < 1e-10 * scale


@pytest.mark.slow
def test_unbiased_over_seeds(orc):
    """E[F_RBL+RBE] = F_Ewald (Sec. 2.4), E[U*] = U and E[W*] = W, as per-component z-scores."""
    w = _water()
    ref = orc.forward(*_args(w), orc.Params(box=w.box), mode="ewald")
    n_seed = 160
    f = np.empty((n_seed,) + ref.force.shape)
    u = np.empty(n_seed)
    vir = np.empty((n_seed, 6))
    for k in range(n_seed):
        r = orc.forward(*_args(w), orc.Params(box=w.box, seed=1000 + k), mode="rbl")
        f[k] = r.force
        u[k] = r.energy[:5].sum()
        vir[k] = r.energy[5:11]
    z = (f.mean(axis=0) - ref.force) / (f.std(axis=0, ddof=1) / math.sqrt(n_seed))
    assert abs((z ** 2).mean() - 1.0) < 0.15
    assert np.abs(z).max() < 5.5
    zu = (u.mean() - ref.energy[:5].sum()) / (u.std(ddof=1) / math.sqrt(n_seed))
    assert abs(zu) < 4.0
    # the importance-sampled virial estimator is unbiased too, component by component
    zv = (vir.mean(axis=0) - ref.energy[5:11]) / (vir.std(axis=0, ddof=1) / math.sqrt(n_seed))
    assert np.abs(zv).max() < 4.5, zv


def test_rbe_variance_scales_as_one_over_p(orc):
    """Var[F_long*] is proportional to 1/p (Eq. 2.14)."""
    w = _water()
    s = orc.quantize(w.pos, w.box)
    lists = orc.build_lists(s, w.molecule, w.box, 0.5, 1.2, full=True)
    var = {}
    for P in (20, 80):
        fl = []
        for step in range(120):
            p = orc.Params(box=w.box, p_kspace=P)
            r = orc.forward(None, w.charge, w.atom_type, w.molecule, w.lj_sigma, w.lj_eps, p, step=step,
                            mode="full", s=s, lists=lists)
            fl.append(r.f_long)
        var[P] = np.var(np.array(fl), axis=0, ddof=1).sum()
    assert 3.3 < var[20] / var[80] < 4.8


def test_shell_estimator_exact_variance(orc):
    """SRSWOR: Var[w sum_B f] = N_S^2 (1 - p/N_S) s^2 / p, s^2 the member variance;
    it vanishes at p = N_S (the factor (N_S - p)/p of Theorem 2.1)."""
    w = _water()
    p = orc.Params(box=w.box, p_shell=60)
    s = orc.quantize(w.pos, w.box)
    rows = np.array([10, 500, 1201])
    lists = orc.build_lists(s, w.molecule, w.box, 0.5, 1.2, rows=rows)
    # every member's pair force, through the oracle with batches of one member
    n_s = np.diff(lists.shell_off)
    samples = []
    for step in range(400):
        b = orc.shell_batches(p.seed, step, lists, p.p_shell)
        r = orc.forward(None, w.charge, w.atom_type, w.molecule, w.lj_sigma, w.lj_eps, p, step=step, rows=rows,
                        s=s, lists=lists, batches=b, mode="rbl")
        samples.append(r.f_short)
    samples = np.array(samples)
    for k in range(len(rows)):
        members = []
        for t in range(n_s[k]):
            one = (np.array([0, 1]), np.array([t], np.int32), np.ones(1))
            sub = orc.Lists(np.array([0, 0]), np.empty(0, np.int32),
                            np.array([0, n_s[k]]), lists.shell_idx[lists.shell_off[k]:lists.shell_off[k + 1]],
                            rows[k:k + 1])
            r = orc.forward(None, w.charge, w.atom_type, w.molecule, w.lj_sigma, w.lj_eps, p, rows=rows[k:k + 1],
                            s=s, lists=sub, batches=one, mode="rbl")
            members.append(r.f_short[0])
        members = np.array(members)
        var_exact = n_s[k] ** 2 * (1 - p.p_shell / n_s[k]) * members.var(axis=0, ddof=1) / p.p_shell
        var_emp = samples[:, k, :].var(axis=0, ddof=1)
        ratio = var_emp.sum() / var_exact.sum()
        assert 0.8 < ratio < 1.25


# --------------------------------------------------------------------------- adjoint

def _loss(orc, w, p, res, G, s=None, q=None, sig=None, eps=None, mode="rbl"):
    sampled = mode in ("rbl", "stencil")
    r = orc.forward(None, w.charge if q is None else q, w.atom_type, w.molecule,
                    w.lj_sigma if sig is None else sig, w.lj_eps if eps is None else eps, p, mode=mode,
                    s=res.s if s is None else s, lists=res.lists,
                    batches=(res.batch_off, res.batch_rank, res.weight) if sampled else None,
                    kspace=(res.kvec, res.wk, res.S), accept=res.accept, core_accept=res.core_accept)
    return float((G * r.force).sum())


@pytest.mark.parametrize("mode,skin", [("rbl", 0.0), ("full", 0.0), ("stencil", 0.0), ("rbl", 0.1)])
def test_adjoint_matches_central_differences(orc, mode, skin):
    w = _water() if skin == 0.0 else _water("water4k")
    p = orc.Params(box=w.box, skin=skin)
    if skin > 0.0:
        lists = orc.build_lists(orc.quantize(w.pos, w.box), w.molecule, w.box, 0.5, 1.2, skin=skin)
        res = orc.forward(_moved(w, skin), w.charge, w.atom_type, w.molecule, w.lj_sigma, w.lj_eps, p, mode=mode,
                          lists=lists)
    else:
        res = orc.forward(*_args(w), p, mode=mode)
    G = np.random.default_rng(3).standard_normal(res.force.shape)
    g_pos, g_q, g_sig, g_eps = orc.backward(G, w.charge, w.atom_type, w.molecule, w.lj_sigma, w.lj_eps, p, res,
                                            mode=mode)
    quantum = w.box / 2 ** 32
    hq = int(round(1e-5 / quantum))
    h = hq * quantum
    for i in (0, 2, 301, 1100):
        for a in range(3):
            sp = res.s.copy()
            sm = res.s.copy()
            sp[i, a] += np.uint32(hq)
            sm[i, a] -= np.uint32(hq)
            fd = (_loss(orc, w, p, res, G, s=sp, mode=mode) - _loss(orc, w, p, res, G, s=sm, mode=mode)) / (2 * h)
            assert abs(fd - g_pos[i, a]) < 1e-5 * max(abs(g_pos[i, a]), 1e3)
    for i in (0, 1, 900):
        hq_ = 1e-4 * abs(w.charge[i])
        qp = w.charge.copy()
        qm = w.charge.copy()
        qp[i] += hq_
        qm[i] -= hq_
        fd = (_loss(orc, w, p, res, G, q=qp, mode=mode) - _loss(orc, w, p, res, G, q=qm, mode=mode)) / (2 * hq_)
        assert abs(fd - g_q[i]) < 1e-5 * max(abs(g_q[i]), 1e3)
    for tbl, grad in (("sig", g_sig), ("eps", g_eps)):
        base = w.lj_sigma if tbl == "sig" else w.lj_eps
        hh = 1e-4 * base[0]
        tp = base.copy()
        tm = base.copy()
        tp[0] += hh
        tm[0] -= hh
        kw_p = {tbl: tp}
        kw_m = {tbl: tm}
        fd = (_loss(orc, w, p, res, G, mode=mode, **kw_p) - _loss(orc, w, p, res, G, mode=mode, **kw_m)) / (2 * hh)
        assert abs(fd - grad[0]) < 1e-5 * max(abs(grad[0]), 1.0)


@pytest.mark.parametrize("mode,skin", [("rbl", 0.0), ("full", 0.0), ("stencil", 0.0), ("rbl", 0.1)])
def test_row_subset_adjoint_matches_full_adjoint(orc, mode, skin):
    """The row-subset adjoint (lists of the rows only, rho over every atom) for a
    dL/dF that vanishes outside the rows and sums to zero equals the all-atom
    adjoint (itself pinned by central differences above): positions and charges
    of the rows, and the LJ table gradients."""
    w = _water() if skin == 0.0 else _water("water4k")
    p = orc.Params(box=w.box, skin=skin)
    n = w.n_atoms
    s0 = orc.quantize(w.pos, w.box)
    pos = _moved(w, skin) if skin > 0.0 else w.pos
    lists = orc.build_lists(s0, w.molecule, w.box, 0.5, 1.2, skin=skin) if skin > 0.0 else None
    res = orc.forward(pos, w.charge, w.atom_type, w.molecule, w.lj_sigma, w.lj_eps, p, mode=mode, step=5,
                      lists=lists)
    rng = np.random.default_rng(11)
    rows = np.sort(rng.choice(n, size=300, replace=False))
    # zero-sum dL/dF on the rows: pairs of rows with opposite values
    v = rng.standard_normal((150, 3))
    G = np.zeros((n, 3))
    perm = rng.permutation(rows)
    G[perm[0::2]] = v
    G[perm[1::2]] = -v
    full = orc.backward(G, w.charge, w.atom_type, w.molecule, w.lj_sigma, w.lj_eps, p, res, mode=mode)
    lists_r = (orc.build_lists(s0, w.molecule, w.box, 0.5, 1.2, skin=skin, rows=rows) if skin > 0.0 else None)
    res_r = orc.forward(pos, w.charge, w.atom_type, w.molecule, w.lj_sigma, w.lj_eps, p, mode=mode, step=5,
                        rows=rows, lists=lists_r, kspace=(res.kvec, res.wk, res.S), rho=res.rho)
    sub = orc.backward_rows(G, w.charge, w.atom_type, w.molecule, w.lj_sigma, w.lj_eps, p, res_r, mode=mode)
    scale_p = np.abs(full[0][rows]).max()
    scale_q = np.abs(full[1][rows]).max()
    assert np.abs(sub[0] - full[0][rows]).max() < 1e-12 * scale_p
    assert np.abs(sub[1] - full[1][rows]).max() < 1e-12 * scale_q
    for a, b in ((sub[2], full[2]), (sub[3], full[3])):
        assert np.abs(a - b).max() <= 1e-12 * max(np.abs(b).max(), 1e-300)
    # the rows' gradients are not those of the rows' own terms alone: other rows'
    # batches and core lists reach them (scatter and symmetric terms)
    assert np.abs(full[0][rows]).max() > 0


# --------------------------------------------------------------------------- virial tensor

def _ewald_energy_sheared(w, frac, hmat, pairs, beta, ke, r_shell, m):
    """Plain Ewald energy of the water box in the periodic cell with edge
    vectors the columns of hmat (positions hmat @ frac), written here
    independently of the oracle: real space over the given pair set (erfc and LJ,
    minimum image in the cell), reciprocal space over the integer vectors m
    (k = 2 pi hmat^-T m; the structure factor's phases 2 pi m.frac do not depend
    on the cell), the self term and the intramolecular erf corrections."""
    V = abs(np.linalg.det(hmat))
    i, j = pairs
    df = frac[j] - frac[i]
    df -= np.round(df)
    d = df @ hmat.T
    r = np.sqrt((d * d).sum(axis=1))
    q = w.charge
    excl = w.molecule[i] == w.molecule[j]
    inr = (~excl) & (r <= r_shell)
    u_real = ke * (q[i] * q[j] * special.erfc(beta * r) / r)[inr].sum()
    nt = 2
    tp = w.atom_type[i] * nt + w.atom_type[j]
    sig, eps = w.lj_sigma[tp], w.lj_eps[tp]
    sr6 = (sig / r) ** 6
    u_lj = (4.0 * eps * (sr6 * sr6 - sr6))[inr].sum()
    u_excl = -ke * (q[i] * q[j] * special.erf(beta * r) / r)[excl].sum()
    kv = 2.0 * math.pi * m @ np.linalg.inv(hmat)  # rows: k = 2 pi h^-T m
    k2 = (kv * kv).sum(axis=1)
    rho = np.zeros(len(m), dtype=np.complex128)
    for c0 in range(0, len(m), 4096):
        ph = 2.0 * math.pi * (frac @ m[c0:c0 + 4096].T)
        rho[c0:c0 + 4096] = (q[:, None] * np.exp(1j * ph)).sum(axis=0)
    u_recip = ke * (2.0 * math.pi / V) * (np.exp(-k2 / (4.0 * beta * beta)) / k2 * np.abs(rho) ** 2).sum()
    u_self = -ke * beta / math.sqrt(math.pi) * (q * q).sum()
    return u_real + u_lj + u_recip + u_self + u_excl


@pytest.mark.slow
def test_ewald_virial_tensor_is_shear_derivative(orc):
    """Every virial component: W_ab = -dU/d(eps_ab) under the deformation
    (I + eps) of cell and positions (fractional coordinates fixed), with U from
    an independent plain Ewald sum for a general cell; also U itself at eps = 0."""
    w = _water()
    p = orc.Params(box=w.box)
    res = orc.forward(*_args(w), p, mode="ewald")
    frac = res.s.astype(np.float64) / 2.0 ** 32
    n = len(frac)
    ii, jj = np.triu_indices(n, 1)
    # the pair set is frozen at the undeformed cell (as the oracle's lists are)
    df = frac[jj] - frac[ii]
    df -= np.round(df)
    r0 = np.sqrt(((df * w.box) ** 2).sum(axis=1))
    keep = (r0 <= p.r_shell) | (w.molecule[ii] == w.molecule[jj])
    pairs = (ii[keep], jj[keep])
    M = orc.ktable(p.beta, w.box)[0]
    rr = np.arange(-M, M + 1)
    m = np.stack(np.meshgrid(rr, rr, rr, indexing="ij"), axis=-1).reshape(-1, 3).astype(np.float64)
    m = m[(m != 0).any(axis=1)]
    h0 = np.eye(3) * w.box
    u0 = _ewald_energy_sheared(w, frac, h0, pairs, p.beta, p.ke, p.r_shell, m)
    assert abs(u0 - res.energy[:5].sum()) < 1e-9 * abs(u0)
    comp = {(0, 0): 5, (1, 1): 6, (2, 2): 7, (0, 1): 8, (0, 2): 9, (1, 2): 10}
    delta = 1e-6
    for (a, b), c in comp.items():
        us = []
        for sgn in (1.0, -1.0):
            e = np.eye(3)
            e[a, b] += sgn * delta
            us.append(_ewald_energy_sheared(w, frac, e @ h0, pairs, p.beta, p.ke, p.r_shell, m))
        dudeps = (us[0] - us[1]) / (2.0 * delta)
        assert abs(res.energy[c] + dudeps) < 1e-6 * np.abs(res.energy[5:8]).max(), ((a, b), res.energy[c], dudeps)


# --------------------------------------------------------------------------- shifted-truncated LJ

WCA = 2.0 ** (1.0 / 6.0)


def test_shifted_truncated_lj_closed_form(orc):
    """Two neutral atoms (sigma = eps = 1): with the cutoff at 2^(1/6) sigma the
    LJ energy is 4((1/r)^12 - (1/r)^6) + 1 inside and 0 outside, the force
    24(2 r^-13 - r^-7) along the separation inside and 0 outside."""
    p = orc.Params(box=10.0, beta=1.0, r_core=1.5, r_shell=3.0, p_kspace=10, ke=1.0, lj_cut=WCA)
    for r in (0.9, 1.0, 1.1, WCA * (1 - 1e-6), WCA * (1 + 1e-6), 1.5, 2.5):
        pos = np.array([[5.0, 5.0, 5.0], [5.0 + r, 5.0, 5.0]])
        res = orc.forward(pos, np.zeros(2), np.zeros(2, np.int32), np.array([-1, -1], np.int32), np.ones(4),
                          np.ones(4), p, mode="full")
        rq = (orc.quantize(pos, 10.0)[1, 0] - orc.quantize(pos, 10.0)[0, 0]) * 10.0 / 2 ** 32
        u = 4.0 * (rq ** -12 - rq ** -6) + 1.0 if rq < WCA else 0.0
        f = 24.0 * (2.0 * rq ** -13 - rq ** -7) if rq < WCA else 0.0
        assert abs(res.energy[1] - u) < 1e-9 * max(1.0, abs(u)), r
        assert abs(res.force[1, 0] - f) < 1e-9 * max(1.0, abs(f)), r
        assert abs(res.force[0, 0] + f) < 1e-9 * max(1.0, abs(f)), r
    # without the cutoff the plain LJ tail acts
    res = orc.forward(np.array([[5.0, 5.0, 5.0], [6.5, 5.0, 5.0]]), np.zeros(2), np.zeros(2, np.int32),
                      np.array([-1, -1], np.int32), np.ones(4), np.ones(4),
                      orc.Params(box=10.0, beta=1.0, r_core=1.5, r_shell=3.0, p_kspace=10, ke=1.0), mode="full")
    assert res.energy[1] < 0.0


def _dense_ions(n=240, box=12.0, seed=5):
    """Random +1/-1 ions at least 0.85 sigma apart (some pairs inside 2^(1/6) sigma)."""
    import types
    rng = np.random.default_rng(seed)
    pts = []
    while len(pts) < n:
        c = rng.uniform(0.0, box, 3)
        ok = True
        for p_ in pts:
            d = c - p_
            d -= box * np.rint(d / box)
            if d @ d < 0.85 ** 2:
                ok = False
                break
        if ok:
            pts.append(c)
    charge = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    return types.SimpleNamespace(pos=np.array(pts), charge=charge, atom_type=(np.arange(n) % 2).astype(np.int32),
                                 molecule=np.full(n, -1, np.int32), lj_sigma=np.ones(4), lj_eps=np.ones(4), box=box,
                                 n_atoms=n)


def test_shifted_truncated_lj_adjoint_matches_central_differences(orc):
    w = _dense_ions()
    p = orc.Params(box=w.box, beta=0.6, r_core=2.5, r_shell=5.5, p_shell=10, p_kspace=50, ke=1.0, lj_cut=WCA)
    res = orc.forward(*_args(w), p, mode="rbl")
    s = res.s
    d = (s[None, :, :].astype(np.int64) - s[:, None, :].astype(np.int64))
    d = ((d + 2 ** 31) % 2 ** 32 - 2 ** 31) * (w.box / 2 ** 32)
    r = np.sqrt((d * d).sum(axis=2)) + np.eye(w.n_atoms) * 99
    assert (r < WCA).sum() >= 4  # some pairs feel the LJ core
    G = np.random.default_rng(3).standard_normal(res.force.shape)
    g_pos, g_q, g_sig, g_eps = orc.backward(G, *_args(w)[1:], p, res, mode="rbl")
    quantum = w.box / 2 ** 32
    hq = int(round(1e-6 / quantum))
    h = hq * quantum
    near = np.unique(np.nonzero(r < WCA)[0])[:3]
    for i in list(near) + [7]:
        for a in range(3):
            sp = res.s.copy()
            sm = res.s.copy()
            sp[i, a] += np.uint32(hq)
            sm[i, a] -= np.uint32(hq)
            fd = (_loss(orc, w, p, res, G, s=sp) - _loss(orc, w, p, res, G, s=sm)) / (2 * h)
            assert abs(fd - g_pos[i, a]) < 1e-5 * max(abs(g_pos[i, a]), 1.0)
    for tbl, grad in (("sig", g_sig), ("eps", g_eps)):
        base = w.lj_sigma if tbl == "sig" else w.lj_eps
        for k in (0, 1):
            hh = 1e-6
            tp = base.copy()
            tm = base.copy()
            tp[k] += hh
            tm[k] -= hh
            fd = (_loss(orc, w, p, res, G, **{tbl: tp}) - _loss(orc, w, p, res, G, **{tbl: tm})) / (2 * hh)
            assert abs(fd - grad[k]) < 1e-5 * max(abs(grad[k]), 1.0), (tbl, k, fd, grad[k])
