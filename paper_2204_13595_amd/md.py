"""NVT dynamics of rigid water with the IRBE force, and the observables the
paper compares between methods (oxygen-oxygen radial distribution, oxygen
mean-squared displacement, potential energy).

Every step, as Algorithm 1 writes it: build_lists, compute_forces, one
integrator step (kick - drift - thermostat - drift with rigid O-H and H-H
lengths; Nose-Hoover as in the paper's water runs, or Langevin). All three run
in the HIP library; this module only sequences the calls and reduces the
sampled observables on the host.

    python -m paper_2204_13595_amd.md --compare   # RBL+RBE against the full list

runs the water comparison of the paper's Sec. 4 on synthetic water (901
molecules, L = 3 nm, r_c = 1.2 nm, beta = 3 nm^-1 i.e. alpha = 0.09 A^-2,
p = 200, T = 298 K) for the (r_core, p~) sets of the paper's parameter table at
that alpha, and prints one JSON line;

    python -m paper_2204_13595_amd.md --electrolytes

runs the 1:1 and 2:1 primitive-model electrolytes of the same section (reduced
units, shifted-truncated LJ, Langevin thermostat) with RBL+RBE against the full
list.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np


def run_water(n_waters: int = 901, box: float = 3.0, *, p_shell: int = 100, p_kspace: int = 200,
              r_core: float = 0.7, r_shell: float = 1.2, beta: float = 3.0, T: float = 298.0, dt: float = 0.001,
              gamma: float = 1.0, warm_steps: int = 4000, equil_steps: int = 40000, prod_steps: int = 150000,
              sample_every: int = 100, rdf_bins: int = 300, rdf_rmax: float = 1.2, seed: int = 2204,
              precision: str = "mixed", thermostat: str = "nose_hoover", tau: float = 1.0,
              msd_window: int = 25000, msd_origin_every: int = 5000, log=None) -> dict:
    """One NVT run from the synthetic lattice start: `warm_steps` of Langevin
    dynamics with a small step and strong friction (the lattice start relaxes),
    `equil_steps`, then `prod_steps` sampled every `sample_every` steps, with the
    Nose-Hoover thermostat of period `tau` (ps; the paper's water runs) or
    Langevin friction `gamma` (1/ps). Returns the O-O g(r), the O mean-squared
    displacement against the time lag (averaged over time origins every
    `msd_origin_every` steps, lags up to `msd_window` steps) with the diffusion
    coefficient from its slope over the second half of the window, and the mean
    potential and kinetic energies (kJ/mol per molecule) and temperature over the
    production run."""
    import torch

    from . import dynamics, inputs, irbe
    dev = torch.device("cuda", torch.cuda.current_device())
    w = inputs.make_water(n_waters, box, seed=seed)
    n = w.n_atoms
    fdt = torch.float64 if precision == "fp64" else torch.float32
    h = irbe.Handle(n, box, beta=beta, r_core=r_core, r_shell=r_shell, p_shell=p_shell, p_kspace=p_kspace,
                    seed=seed, precision=precision, device=dev)
    h.set_system(torch.tensor(w.atom_type, device=dev), torch.tensor(w.charge, dtype=fdt, device=dev),
                 torch.tensor(w.molecule, device=dev), w.lj_sigma, w.lj_eps)
    groups, lengths, inv_mass = dynamics.water_topology(n_waters)
    kT = dynamics.KB * T
    warm = dynamics.Langevin(inv_mass, groups, lengths, dt=dt / 4.0, gamma=20.0, kT=kT, seed=seed + 1,
                             precision=precision, device=dev)
    dyn = dynamics.Langevin(inv_mass, groups, lengths, dt=dt, gamma=gamma, kT=kT, seed=seed + 2,
                            precision=precision, thermostat=thermostat, tau=tau, device=dev)
    pos = torch.tensor(w.pos, dtype=torch.float64, device=dev)
    vel = torch.zeros_like(pos)
    pos_f = pos.to(fdt).contiguous()
    force = torch.empty((n, 3), dtype=fdt, device=dev)
    sel_o = torch.arange(0, n, 3, dtype=torch.int32, device=dev)
    hist = torch.zeros(rdf_bins, dtype=torch.int64, device=dev)
    step = 0

    def advance(integ, count, sample=None):
        nonlocal step
        for k in range(count):
            h.build_lists(pos_f, step)
            want = sample is not None and k % sample_every == 0
            if want:
                _, ev = h.compute_forces(pos_f, step, out=force, energy=True)
                sample(k, ev)
            else:
                h.compute_forces(pos_f, step, out=force)
            integ.step(pos, vel, force, step, pos_copy=pos_f)
            step += 1
            if (k + 1) % 2000 == 0:
                integ.check()
                if log:
                    log(f"step {step}")
        integ.check()

    t0 = time.perf_counter()
    advance(warm, warm_steps)
    advance(dyn, equil_steps)
    u_s, k_s, xi_s = [], [], []
    origins, msd_acc = [], {}

    def sample(k, ev):
        u_s.append(ev[:5].sum().reshape(1))
        k_s.append(dyn.kinetic(vel))
        xi_s.append(dyn.thermostat_state()[:1])
        if k % msd_origin_every == 0 and k + msd_window <= prod_steps:
            origins.append((k, pos.clone()))
        for k0, ref in origins:
            if k - k0 <= msd_window:
                msd_acc.setdefault(k - k0, []).append(dyn.msd(pos, ref, sel_o))
        dyn.rdf(pos, sel_o, box, rdf_rmax, hist)

    advance(dyn, prod_steps, sample)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    frames = len(u_s)
    r, g = dynamics.rdf_normalise(hist.cpu().numpy(), n_waters, box, rdf_rmax, frames)
    u = torch.cat(u_s).cpu().numpy() / n_waters
    kin = torch.cat(k_s).cpu().numpy()
    temp = 2.0 * kin / (dyn.n_dof * dynamics.KB)
    lags = np.array(sorted(msd_acc), dtype=np.int64)
    msd = np.array([torch.cat(msd_acc[lag]).mean().item() for lag in lags])
    lag_t = lags * dt
    half = lag_t >= 0.5 * lag_t[-1] if lags.size else np.zeros(0, dtype=bool)
    diff = float(np.polyfit(lag_t[half], msd[half], 1)[0] / 6.0) if half.sum() >= 2 else float("nan")
    h.close()
    warm.close()
    dyn.close()
    xi = torch.cat(xi_s).cpu().numpy()
    return {"r": r, "g": g, "msd_t": lag_t, "msd": msd, "diffusion_nm2_per_ps": diff, "xi_mean": float(xi.mean()),
            "msd_origins": len(origins), "u_per_molecule": float(u.mean()),
            "u_sem": float(u.std(ddof=1) / math.sqrt(max(frames // 10, 1))),
            "kinetic_per_molecule": float(kin.mean() / n_waters), "temperature": float(temp.mean()),
            "frames": frames, "steps": step, "wall_s": wall, "ms_per_step": 1e3 * wall / step}


# (r_core, p~) at alpha = 0.09 A^-2 (beta = 3 nm^-1), p = 200, from the paper's parameter table
TABLE_SETS = [(0.6, 150), (0.7, 100)]


def water_sets():
    """The runs of the water comparison: name -> run_water keyword arguments."""
    sets = {"full": {"p_shell": 0}}
    for rc, ps in TABLE_SETS:
        sets[f"rbl_{rc}_{ps}"] = {"r_core": rc, "p_shell": ps}
    return sets


def compare(prod_steps: int = 150000, equil_steps: int = 40000, log=None, runs: dict | None = None) -> dict:
    """The full-list variant (every pair within r_c, RBE at p = 200) against
    RBL+RBE at the table's sets: max |g_RBL(r) - g_full(r)| over r > 0.2 nm, the
    first-peak height and position, the O mean-squared displacement at the end
    of the run, and the mean potential energy. `runs` (name -> run_water result)
    compares runs made separately instead."""
    if runs is None:
        runs = {}
        for name, kw in water_sets().items():
            runs[name] = run_water(prod_steps=prod_steps, equil_steps=equil_steps, log=log, **kw)
            if log:
                log(f"done {name}")
    ref = runs["full"]
    mask = ref["r"] > 0.2
    out = {}
    for name, res in runs.items():
        pk = int(np.argmax(res["g"]))
        out[name] = {
            "g_peak": float(res["g"][pk]), "r_peak": float(res["r"][pk]),
            "msd_end_nm2": float(res["msd"][-1]), "diffusion_1e5_cm2_per_s": 100.0 * res["diffusion_nm2_per_ps"],
            "u_per_molecule": res["u_per_molecule"], "u_sem": res["u_sem"],
            "temperature": res["temperature"], "ms_per_step": res["ms_per_step"],
            "nose_hoover_xi_mean_per_ps": res["xi_mean"],
            "max_abs_g_diff_vs_full": float(np.abs(res["g"] - ref["g"])[mask].max()),
            "rel_g_peak_diff_vs_full": float(res["g"][pk] / ref["g"].max() - 1.0),
            "rel_msd_end_diff_vs_full": float(res["msd"][-1] / ref["msd"][-1] - 1.0),
            "rel_diffusion_diff_vs_full": float(res["diffusion_nm2_per_ps"] / ref["diffusion_nm2_per_ps"] - 1.0),
            "rel_u_diff_vs_full": float(res["u_per_molecule"] / ref["u_per_molecule"] - 1.0),
        }
    out["setup"] = (f"901 rigid waters, L = 3 nm, beta = 3/nm, r_c = 1.2 nm, p = 200, T = 298 K, Nose-Hoover "
                    f"tau = 1 ps, dt = 1 fs, {ref['steps']} steps per run of which {ref['frames']} production frames "
                    f"every 100 steps, lists rebuilt every step, mixed precision; MSD over time origins every 5 ps, "
                    f"lags up to 25 ps")
    return out


def run_nve(n_waters: int = 32768, box: float = 9.93, *, p_shell: int = 100, p_kspace: int = 200,
            r_core: float = 0.5, r_shell: float = 1.2, beta: float = 3.0, T0: float = 300.0, dt: float = 0.001,
            steps: int = 1000, warm_steps: int = 2000, sample_every: int = 10, seed: int = 2204,
            precision: str = "mixed") -> dict:
    """Constant-energy run of rigid water (no thermostat: the integrator with zero
    friction is velocity Verlet with the rigid constraints) from Maxwell
    velocities at T0 (K), lists rebuilt every step. The synthetic lattice start
    first relaxes for `warm_steps` Langevin steps of h/4 with strong friction
    (untimed); the velocities are then drawn afresh. The total energy
    E_n = U(x_n) + (K_{n-1/2} + K_{n+1/2}) / 2 and the temperature
    T = 2 K / (n_dof k_B) are sampled every `sample_every` steps. A stochastic
    force heats a constant-energy run (Sec. 2.2: these methods are meant for runs
    with a thermostat): each step adds about (dt^2 / 2m) times the force
    variance per degree of freedom, and the variance of the random batch Ewald
    force scales as 1/p (Eq. (2.14)), so the initial heating rate (the slope of
    the total energy over the first 0.1 ps) scales as 1/p. (The temperature
    also moves early on as the fresh velocities equilibrate with the relaxed
    structure, so its slope is no measure of the heating.) A run that heats far
    enough for the rigid constraints to fail stops there: the state is checked
    every 100 steps, and the result then records the time of the last good check
    and keeps the samples up to it.
    Returns the traces, the initial and whole-run slopes, and ms per step (wall
    clock of the whole loop: lists, forces, integrator)."""
    import torch

    from . import dynamics, inputs, irbe
    dev = torch.device("cuda", torch.cuda.current_device())
    w = inputs.make_water(n_waters, box, seed=seed)
    n = w.n_atoms
    fdt = torch.float64 if precision == "fp64" else torch.float32
    h = irbe.Handle(n, box, beta=beta, r_core=r_core, r_shell=r_shell, p_shell=p_shell, p_kspace=p_kspace,
                    seed=seed, precision=precision, device=dev)
    h.set_system(torch.tensor(w.atom_type, device=dev), torch.tensor(w.charge, dtype=fdt, device=dev),
                 torch.tensor(w.molecule, device=dev), w.lj_sigma, w.lj_eps)
    groups, lengths, inv_mass = dynamics.water_topology(n_waters)
    dyn = dynamics.Langevin(inv_mass, groups, lengths, dt=dt, gamma=0.0, kT=0.0, precision=precision, device=dev)
    warm = dynamics.Langevin(inv_mass, groups, lengths, dt=dt / 4.0, gamma=50.0, kT=dynamics.KB * T0,
                             seed=seed + 1, precision=precision, device=dev)
    pos = torch.tensor(w.pos, dtype=torch.float64, device=dev)
    vel = torch.zeros_like(pos)
    pos_f = pos.to(fdt).contiguous()
    force = torch.empty((n, 3), dtype=fdt, device=dev)
    for step in range(warm_steps):
        h.build_lists(pos_f, step)
        h.compute_forces(pos_f, step, out=force)
        warm.step(pos, vel, force, step, pos_copy=pos_f)
    warm.check()
    warm.close()
    rng = np.random.default_rng(seed)
    v0 = rng.standard_normal((n, 3)) * np.sqrt(dynamics.KB * T0 * inv_mass)[:, None]
    v0 -= (v0 / inv_mass[:, None]).sum(axis=0) / (1.0 / inv_mass).sum()  # zero total momentum
    vel.copy_(torch.tensor(v0, device=dev))
    e_s, k_s, t_s = [], [], []
    good, done, executed, failed_at = 0, 0, 0, None  # samples and steps up to the last good check
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for step in range(warm_steps, warm_steps + steps):
        h.build_lists(pos_f, step)
        if (step - warm_steps) % sample_every == 0 and step > warm_steps:
            _, ev = h.compute_forces(pos_f, step, out=force, energy=True)
            k_prev = dyn.kinetic(vel)
            dyn.step(pos, vel, force, step, pos_copy=pos_f)
            k_mid = 0.5 * (k_prev + dyn.kinetic(vel))
            e_s.append(ev[:5].sum().reshape(1) + k_mid)
            k_s.append(k_mid.reshape(1))
            t_s.append((step - warm_steps) * dt)
        else:
            h.compute_forces(pos_f, step, out=force)
            dyn.step(pos, vel, force, step, pos_copy=pos_f)
        executed = step - warm_steps + 1
        if executed % 100 == 0 or executed == steps:
            try:
                dyn.check()
            except irbe.IRBEError:
                failed_at = executed * dt
                break
            good, done = len(e_s), executed
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    e_s, k_s, t_s = e_s[:good], k_s[:good], t_s[:good]
    if len(t_s) < 3:
        h.close()
        dyn.close()
        return {"p_kspace": p_kspace, "p_shell": p_shell, "precision": precision, "steps": done,
                "constraints_failed_by_ps": failed_at, "ms_per_step": 1e3 * wall / max(executed, 1)}
    e = torch.cat(e_s).cpu().numpy() / n_waters
    temp = 2.0 * torch.cat(k_s).cpu().numpy() / (dyn.n_dof * dynamics.KB)
    t = np.array(t_s)
    slope = float(np.polyfit(t, e, 1)[0])
    early = t <= 0.1 + 1e-9
    slope0 = float(np.polyfit(t[early], e[early], 1)[0]) if early.sum() >= 3 else float("nan")
    h.close()
    dyn.close()
    thin = max(1, len(t) // 20)
    return {"p_kspace": p_kspace, "p_shell": p_shell, "precision": precision,
            "initial_drift_kj_mol_per_ps_per_molecule": slope0,
            "drift_kj_mol_per_ps_per_molecule": slope, "energy_per_molecule_first": float(e[0]),
            "energy_per_molecule_last": float(e[-1]), "temperature_first_K": float(temp[0]),
            "temperature_last_K": float(temp[-1]),
            "trace": {"t_ps": [round(float(x), 4) for x in t[::thin]],
                      "temperature_K": [round(float(x), 2) for x in temp[::thin]],
                      "energy_per_molecule": [round(float(x), 3) for x in e[::thin]]},
            "ms_per_step": 1e3 * wall / max(executed, 1), "steps": done,
            "constraints_failed_by_ps": failed_at}


def run_electrolyte(valence: int = 1, *, p_shell: int = 10, p_kspace: int = 100, r_core: float = 5.0,
                    r_shell: float = 15.0, alpha: float = 0.03, ke: float = 1.0, dt: float = 0.002,
                    gamma: float = 1.0, equil_steps: int = 20000, prod_steps: int = 80000, sample_every: int = 100,
                    rdf_bins: int = 150, rdf_rmax: float = 15.0, msd_window: int = 20000,
                    msd_origin_every: int = 5000, seed: int = 2204, log=None) -> dict:
    """The primitive-model electrolytes of the paper's Sec. 4 in reduced units
    (sigma = m = kT = 1): 1:1 or 2:1 ions in L = 80, shifted-truncated LJ at
    2^(1/6) (soft spheres), Coulomb coupling `ke` (the Bjerrum length; not given
    in the paper), Langevin thermostat with relaxation time 1 (friction 1), time
    step 0.002. p_shell <= 0 is the full list. Returns g_{+-}, g_{++}, g_{--},
    the MSD of each species against the lag, and the potential energy per atom."""
    import torch

    from . import dynamics, inputs, irbe
    dev = torch.device("cuda", torch.cuda.current_device())
    w = inputs.electrolyte(valence, seed=seed)
    n = w.n_atoms
    h = irbe.Handle(n, w.box, beta=math.sqrt(alpha), r_core=r_core, r_shell=r_shell, p_shell=p_shell,
                    p_kspace=p_kspace, seed=seed, precision="mixed", coulomb_k=ke, lj_cut=2.0 ** (1.0 / 6.0),
                    device=dev)
    h.set_system(torch.tensor(w.atom_type, device=dev), torch.tensor(w.charge, dtype=torch.float32, device=dev),
                 torch.tensor(w.molecule, device=dev), w.lj_sigma, w.lj_eps)
    groups = np.stack([np.arange(n), -np.ones(n, np.int64), -np.ones(n, np.int64)], axis=1).astype(np.int32)
    dyn = dynamics.Langevin(np.ones(n), groups, np.zeros((n, 3)), dt=dt, gamma=gamma, kT=1.0, seed=seed + 2,
                            precision="mixed", device=dev)
    pos = torch.tensor(w.pos, dtype=torch.float64, device=dev)
    vel = torch.zeros_like(pos)
    pos_f = pos.float().contiguous()
    force = torch.empty((n, 3), dtype=torch.float32, device=dev)
    species = {"+": torch.tensor(np.nonzero(w.atom_type == 0)[0], dtype=torch.int32, device=dev),
               "-": torch.tensor(np.nonzero(w.atom_type == 1)[0], dtype=torch.int32, device=dev)}
    pairs = {"+-": ("+", "-"), "++": ("+", None), "--": ("-", None)}
    hist = {k: torch.zeros(rdf_bins, dtype=torch.int64, device=dev) for k in pairs}
    u_s, origins, msd_acc = [], [], {"+": {}, "-": {}}
    step = 0
    t0 = time.perf_counter()

    def sample(k, ev):
        u_s.append(ev[:5].sum().reshape(1))
        if k % msd_origin_every == 0 and k + msd_window <= prod_steps:
            origins.append((k, pos.clone()))
        for k0, ref in origins:
            if k - k0 <= msd_window:
                for sp, sel in species.items():
                    msd_acc[sp].setdefault(k - k0, []).append(dyn.msd(pos, ref, sel))
        for key, (a, b) in pairs.items():
            dyn.rdf(pos, species[a], w.box, rdf_rmax, hist[key], sel_b=None if b is None else species[b])

    for phase, count in (("equil", equil_steps), ("prod", prod_steps)):
        for k in range(count):
            h.build_lists(pos_f, step)
            if phase == "prod" and k % sample_every == 0:
                _, ev = h.compute_forces(pos_f, step, out=force, energy=True)
                sample(k, ev)
            else:
                h.compute_forces(pos_f, step, out=force)
            dyn.step(pos, vel, force, step, pos_copy=pos_f)
            step += 1
            if (k + 1) % 5000 == 0:
                dyn.check()
                if log:
                    log(f"step {step}")
    dyn.check()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    frames = len(u_s)
    out = {"frames": frames, "steps": step, "ms_per_step": 1e3 * wall / step}
    m = {sp: int(sel.shape[0]) for sp, sel in species.items()}
    for key, (a, b) in pairs.items():
        r, g = dynamics.rdf_normalise(hist[key].cpu().numpy(), m[a], w.box, rdf_rmax, frames,
                                      m_b=None if b is None else m[b])
        out["r"], out["g" + key] = r, g
    for sp in species:
        lags = np.array(sorted(msd_acc[sp]), dtype=np.int64)
        out["msd_t"] = lags * dt
        out["msd" + sp] = np.array([torch.cat(msd_acc[sp][lag]).mean().item() for lag in lags])
    u = torch.cat(u_s).cpu().numpy() / n
    out["u_per_atom"] = float(u.mean())
    out["u_std"] = float(u.std(ddof=1))
    h.close()
    dyn.close()
    return out


def compare_electrolytes(prod_steps: int = 80000, equil_steps: int = 20000, log=None) -> dict:
    """RBL+RBE (r_core = 5, p~ = 10) against the full list (the same RBE, p = 100)
    for the 1:1 and 2:1 electrolytes: the potential energy per atom (mean and
    standard deviation over the run), the g(r) differences and the end-of-window
    MSD of each species."""
    out = {}
    for valence in (1, 2):
        res = {m: run_electrolyte(valence, p_shell=ps, prod_steps=prod_steps, equil_steps=equil_steps, log=log)
               for m, ps in (("full", 0), ("rbl", 10))}
        f, r = res["full"], res["rbl"]
        mask = f["r"] > 1.0
        row = {}
        for m in ("full", "rbl"):
            row[m] = {"u_per_atom": res[m]["u_per_atom"], "u_std": res[m]["u_std"],
                      "ms_per_step": res[m]["ms_per_step"],
                      "msd_end": {sp: float(res[m]["msd" + sp][-1]) for sp in "+-"},
                      "g_peak_+-": float(res[m]["g+-"].max())}
        row["rel_u_diff"] = r["u_per_atom"] / f["u_per_atom"] - 1.0
        row["max_abs_g_diff"] = {k: float(np.abs(r["g" + k] - f["g" + k])[mask].max()) for k in ("+-", "++", "--")}
        row["rel_msd_end_diff"] = {sp: float(r["msd" + sp][-1] / f["msd" + sp][-1] - 1.0) for sp in "+-"}
        out[f"{valence}:1"] = row
    out["setup"] = (f"2560+2560 (1:1) or 1280+2560 (2:1) ions, L = 80, shifted-truncated LJ at 2^(1/6), ke = 1, "
                    f"alpha = 0.03, p = 100, r_c = 15, RBL r_core = 5 and p~ = 10, Langevin friction 1, dt = 0.002, "
                    f"{equil_steps} + {prod_steps} steps, lists rebuilt every step, mixed precision")
    return out


def main():
    ap = argparse.ArgumentParser(description="NVT water with the IRBE force")
    ap.add_argument("--compare", action="store_true")
    ap.add_argument("--electrolytes", action="store_true", help="the 1:1 and 2:1 primitive-model comparison")
    ap.add_argument("--elec-prod-steps", type=int, default=80000)
    ap.add_argument("--elec-equil-steps", type=int, default=20000)
    ap.add_argument("--set", help="one run of the water comparison (full, rbl_0.6_150, rbl_0.7_100), as JSON")
    ap.add_argument("--combine", nargs="+", help="compare the JSON files of separate --set runs")
    ap.add_argument("--prod-steps", type=int, default=150000)
    ap.add_argument("--equil-steps", type=int, default=40000)
    args = ap.parse_args()
    log = lambda m: print(m, file=sys.stderr, flush=True)  # noqa: E731
    if args.combine:
        runs = {}
        for path in args.combine:
            d = json.load(open(path))
            runs[d.pop("name")] = {k: (np.array(v) if isinstance(v, list) else v) for k, v in d.items()}
        print(json.dumps(compare(runs=runs)), flush=True)
    elif args.set:
        res = run_water(prod_steps=args.prod_steps, equil_steps=args.equil_steps, log=log, **water_sets()[args.set])
        res = {k: (v.tolist() if isinstance(v, np.ndarray) else v) for k, v in res.items()}
        print(json.dumps(dict(name=args.set, **res)), flush=True)
    elif args.electrolytes:
        print(json.dumps(compare_electrolytes(args.elec_prod_steps, args.elec_equil_steps, log=log)), flush=True)
    elif args.compare:
        print(json.dumps(compare(args.prod_steps, args.equil_steps, log=log)), flush=True)
    else:
        res = run_water(prod_steps=args.prod_steps, equil_steps=args.equil_steps, log=log)
        print(json.dumps({k: (v.tolist() if isinstance(v, np.ndarray) else v) for k, v in res.items()}), flush=True)


if __name__ == "__main__":
    main()
