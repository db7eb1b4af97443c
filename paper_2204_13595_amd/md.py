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
that alpha, and prints one JSON line.
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


def compare(prod_steps: int = 150000, equil_steps: int = 40000, log=None) -> dict:
    """The full-list variant (every pair within r_c, RBE at p = 200) against
    RBL+RBE at the table's sets: max |g_RBL(r) - g_full(r)| over r > 0.2 nm, the
    first-peak height and position, the O mean-squared displacement at the end
    of the run, and the mean potential energy."""
    runs = {"full": run_water(p_shell=0, prod_steps=prod_steps, equil_steps=equil_steps, log=log)}
    for rc, ps in TABLE_SETS:
        runs[f"rbl_{rc}_{ps}"] = run_water(r_core=rc, p_shell=ps, prod_steps=prod_steps, equil_steps=equil_steps,
                                           log=log)
        if log:
            log(f"done rbl {rc} {ps}")
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
                    f"tau = 1 ps, dt = 1 fs, {equil_steps} equilibration + {prod_steps} production steps, lists "
                    f"rebuilt every step, mixed precision; MSD over time origins every 5 ps, lags up to 25 ps")
    return out


def main():
    ap = argparse.ArgumentParser(description="NVT water with the IRBE force")
    ap.add_argument("--compare", action="store_true")
    ap.add_argument("--prod-steps", type=int, default=150000)
    ap.add_argument("--equil-steps", type=int, default=40000)
    args = ap.parse_args()
    log = lambda m: print(m, file=sys.stderr, flush=True)  # noqa: E731
    if args.compare:
        print(json.dumps(compare(args.prod_steps, args.equil_steps, log=log)), flush=True)
    else:
        res = run_water(prod_steps=args.prod_steps, equil_steps=args.equil_steps, log=log)
        print(json.dumps({k: (v.tolist() if isinstance(v, np.ndarray) else v) for k, v in res.items()}), flush=True)


if __name__ == "__main__":
    main()
