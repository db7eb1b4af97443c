#!/usr/bin/env python3
"""Benchmark of the IRBE non-bonded force (random batch list + random batch
Ewald) on one MI355X.

Workload: 1,048,576 synthetic SPC/E-like waters (3,145,728 atoms) in a cubic
box of 31.5 nm; beta = 3.0 nm^-1, r_core = 0.5 nm, r_shell = 1.2 nm, shell
batch p~ = 100, p = 100 sampled k-vectors; FP32 pair and k-space arithmetic with
FP64 structure-factor, momentum-correction and energy accumulation.

One step = build_lists + compute_forces (lists rebuilt every step, as in
Algorithm 1 of the paper). Printed as one JSON line: `value` is the forward
throughput in atom-steps/s; forward+backward, forces-only with reused lists, and
the full-neighbour-list variant (every pair within r_shell, same k-space) on the
same GPU are reported beside it, with the per-stage kernel times (HIP events on
the handle's stream), the roofline of the dominant kernel, and the CPU oracle
timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "atom-steps/s RBL+RBE fwd and fwd+bwd vs full-list Ewald, 3M-atom water"
HBM_PEAK_GBS = 8000.0


def log(msg: str):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="water1M")
    ap.add_argument("--p-shell", type=int, default=100)
    ap.add_argument("--p-kspace", type=int, default=100)
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="only the headline forward figure")
    ap.add_argument("--with-backward", action="store_true",
                    help="with --no-extras: also run the forward+backward steps once (for profiles)")
    ap.add_argument("--electrolyte", type=int, default=0,
                    help="only the electrolyte comparison at this many ions (one JSON line; for profiles)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one 1 GiB device copy (reference for the HBM byte counters of a profile)")
    return ap.parse_args()


def timed_steps(fn, warmup: int, steps: int, first_step: int = 0, per_step: list | None = None):
    """Mean wall-clock seconds per step over `steps` steps after `warmup` untimed
    ones, synchronized on both sides; `per_step` (if given) receives each step's
    milliseconds from events recorded between the steps on the current stream."""
    import torch
    for s in range(warmup):
        fn(first_step + s)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)] if per_step is not None else None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        if ev is not None:
            ev[s].record()
        fn(first_step + warmup + s)
    if ev is not None:
        ev[steps].record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    if ev is not None:
        per_step.extend(ev[s].elapsed_time(ev[s + 1]) for s in range(steps))
    return wall


VALU_PEAK_LANE_OPS = 256 * 64 * 2.4e9  # full-rate 32-bit VALU lane operations per second


def stage_times(h, fn, steps: int, first_step: int):
    """Average ms per launch of each stage, from HIP events on the handle's stream."""
    h.enable_timing(True)
    for s in range(steps):
        fn(first_step + s)
    t = h.timing()
    h.enable_timing(False)
    return {k: (ms / n if n else 0.0, n) for k, (ms, n) in t.items()}


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed FETCH_SIZE / WRITE_SIZE profile of
    this kernel and workload, or None when absent or taken on another version
    of the kernel's source."""
    from paper_2204_13595_amd import profiling
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    t = json.load(open(path))
    if t.get("source_sha") != profiling.source_hash(kernel):
        return None
    return t["hbm_bytes_per_launch"]


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, args):
    """The FP64 oracle (lists rebuilt, RBL+RBE forward) on the host cores: one
    full step of the benchmark workload (about 10 s of CPU work), and steps of the
    98,304-atom constant-energy workload (P = 200)."""
    from oracle import oracle as orc

    from paper_2204_13595_amd import inputs
    orc.lib()
    p = orc.Params(box=w.box, p_shell=args.p_shell, p_kspace=args.p_kspace)
    t0 = time.perf_counter()
    orc.forward(w.pos, w.charge, w.atom_type, w.molecule, w.lj_sigma, w.lj_eps, p, step=0, mode="rbl")
    t = time.perf_counter() - t0
    log(f"cpu oracle: one {w.n_atoms}-atom step in {t:.2f} s")
    w2 = inputs.workload("water32k")
    p2 = orc.Params(box=w2.box, p_shell=args.p_shell, p_kspace=200)
    k2 = 3
    t0 = time.perf_counter()
    for step in range(k2):
        orc.forward(w2.pos, w2.charge, w2.atom_type, w2.molecule, w2.lj_sigma, w2.lj_eps, p2, step=step, mode="rbl")
    t2 = (time.perf_counter() - t0) / k2
    threads = int(orc.lib().orc_num_threads())
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:
        nproc = os.cpu_count() or 1
    return {
        "value": w.n_atoms / t, "unit": "atom-steps/s", "cores": threads, "kind": "oracle",
        "sample": (f"one full step (cell lists, core/shell lists, batches, pair forces, momentum correction, "
                   f"k samples, FP64 structure factor, k-space force) of the {w.n_atoms}-atom workload by the FP64 "
                   f"oracle with OpenMP over atoms: {t:.2f} s"),
        "nproc": nproc, "cpu_model": cpu_model(),
        "water32k": {"atom_steps_per_s": w2.n_atoms / t2, "s_per_step": t2, "steps": k2,
                     "workload": "98,304 atoms (32,768 waters, L = 9.93 nm), P_s = 100, P = 200, lists rebuilt"},
    }


def rms(a):
    return float(a.double().pow(2).sum(dim=1).mean().sqrt())


def forces(make, pos, p_shell, p_kspace, seed, step=7, shell_source="list", skin=0.0, pos_eval=None):
    h = make(p_shell, p_kspace, seed, shell_source, skin)
    h.build_lists(pos, step)
    f = h.compute_forces(pos if pos_eval is None else pos_eval, step).clone()
    h.close()
    return f


def accuracy(make, pos, G, w, args, ms_rbl, timed_steps):
    """Force errors of the estimators and the full-list variant at matched error.

    Errors are RMS over atoms of |F - E[F]|, in kJ/mol/nm:
    * total error of a stochastic force from two independent seeds:
      E|F1 - F2|^2 = 2 Var, so e = RMS(F1 - F2) / sqrt(2) (the real-space
      truncation, erfc(3.6) = 3.6e-7, is negligible);
    * the RMS of the exact force follows as sqrt(E RMS(F)^2 - e^2);
    * the shell-sampling error alone: with one seed both variants draw the same
      k-vectors, so F_RBL - F_full is exactly the random batch list estimate
      minus the exact short-range force;
    * matched error: the full-list variant's error at k-space batch size p is
      e_full(p); RBL+RBE at p0 has e_full(p0)^2 + e_shell^2 (independent
      samples); the full list matches it at the smallest p with
      e_full(p)^2 <= e_full(p0)^2 + e_shell^2.
    Plus a sweep of (p_shell, p) and the FP32-vs-FP64 error of forces and gradients."""
    import math

    import torch

    from paper_2204_13595_amd import irbe
    n = w.n_atoms
    P0 = args.p_kspace
    seeds = (13595, 24681)
    f_rbl = [forces(make, pos, args.p_shell, P0, sd) for sd in seeds]
    e_rbl = rms(f_rbl[0] - f_rbl[1]) / math.sqrt(2.0)
    ms2 = 0.5 * (rms(f_rbl[0]) ** 2 + rms(f_rbl[1]) ** 2)
    f_full0 = forces(make, pos, 0, P0, seeds[0])
    e_shell = rms(f_rbl[0] - f_full0)
    del f_rbl
    e_full = {}
    for P in sorted({25, 50, 100, 200, 500, P0}):
        ff = [f_full0 if (P == P0 and sd == seeds[0]) else forces(make, pos, 0, P, sd) for sd in seeds]
        e_full[P] = rms(ff[0] - ff[1]) / math.sqrt(2.0)
    f_exact = math.sqrt(max(ms2 - e_rbl ** 2, 0.0))
    target = math.sqrt(e_full[P0] ** 2 + e_shell ** 2)
    matched = min((P for P in e_full if e_full[P] <= target), default=max(e_full))
    hf = make(0, matched)

    def fwd_full(step):
        hf.build_lists(pos, step)
        hf.compute_forces(pos, step)

    ms_full = timed_steps(fwd_full, 1, 5, 6000) * 1e3
    hf.close()
    sweep = []
    for ps in (50, 100, 200):
        for P in (100, 500):
            h = make(ps, P)

            def fwd(step):
                h.build_lists(pos, step)
                h.compute_forces(pos, step)

            ms_c = timed_steps(fwd, 1, 5, 7000) * 1e3
            h.close()
            fr, ff = forces(make, pos, ps, P, seeds[0]), forces(make, pos, 0, P, seeds[0])
            sweep.append({"p_shell": ps, "p_kspace": P, "ms_per_step": round(ms_c, 3),
                          "atom_steps_per_s": n / (ms_c * 1e-3), "shell_sampling_err": rms(fr - ff)})
    out = {
        "unit": "kJ/mol/nm, RMS over atoms",
        "exact_force_rms_estimate": f_exact,
        "rbl_rbe_err": e_rbl,
        "rbl_shell_sampling_err": e_shell,
        "full_list_err_by_p": {str(P): e for P, e in e_full.items()},
        "matched_error_full_list": {"p_kspace": matched, "err": e_full[matched], "target_err": target,
                                    "ms_per_step": ms_full, "atom_steps_per_s": n / (ms_full * 1e-3),
                                    "speedup_rbl_rbe": ms_full / ms_rbl},
        "sweep_rbl_rbe": sweep,
    }
    if args.precision == "mixed":
        # FP32 arithmetic against the FP64 path (itself within 1e-11 of the FP64 oracle)
        dev = pos.device
        q64 = torch.tensor(w.charge, device=dev).to(torch.float32).double()
        res = {}
        for prec, p_in, q_in in (("mixed", pos, q64.float()), ("fp64", pos.double(), q64)):
            h = irbe.Handle(n, w.box, p_shell=args.p_shell, p_kspace=P0, precision=prec, device=dev)
            h.set_system(torch.tensor(w.atom_type, device=dev), q_in, torch.tensor(w.molecule, device=dev),
                         w.lj_sigma, w.lj_eps)
            h.build_lists(p_in, 3)
            f = h.compute_forces(p_in, 3).double()
            gp, gq, gl = h.compute_forces_backward(p_in, 3, G.to(p_in.dtype))
            res[prec] = (f, gp.double(), gq.double(), gl.double())
            h.close()
        (f32, g32, q32, l32), (f64, g64, q64g, l64) = res["mixed"], res["fp64"]
        out["fp32_vs_fp64"] = {
            "force_rms_rel": rms(f32 - f64) / rms(f64),
            "grad_pos_rms_rel": rms(g32 - g64) / rms(g64),
            "grad_charge_rms_rel": float((q32 - q64g).pow(2).mean().sqrt() / q64g.pow(2).mean().sqrt()),
            "grad_lj_sigma_oo_rel": float(abs(l32[0] - l64[0]) / abs(l64[0])),
            "grad_lj_eps_oo_rel": float(abs(l32[4] - l64[4]) / abs(l64[4])),
        }
    return out


def stencil_sampling(make, pos, G, w, args, acc, ms_full, timed_steps):
    """The shell batch drawn from the atoms of the shell stencil's cells
    (Algorithm 1): no shell list, weight |K(i)| / p~, a drawn atom counting only
    inside the shell. Forward and forward+backward rates with lists (core only)
    rebuilt every step, the shell-sampling error against the full list at the
    same k-vectors, and the speed against the full-list variant at matched total
    error (as in the accuracy section)."""
    import math
    n = w.n_atoms
    P0 = args.p_kspace
    out = {}
    f_full0 = forces(make, pos, 0, P0, 13595)
    for ps in (args.p_shell, 4 * args.p_shell):
        h = make(ps, P0, 13595, "stencil")

        def fwd(step):
            h.build_lists(pos, step)
            h.compute_forces(pos, step)

        def fwd_bwd(step):
            fwd(step)
            h.compute_forces_backward(pos, step, G)

        ms_f = timed_steps(fwd, 2, args.steps, 8000) * 1e3
        ms_fb = timed_steps(fwd_bwd, 1, max(args.steps // 2, 2), 8500) * 1e3
        st = stage_times(h, fwd_bwd, 3, 8800)
        h.close()
        e_shell = rms(forces(make, pos, ps, P0, 13595, shell_source="stencil") - f_full0)
        e_full = acc["full_list_err_by_p"]
        target = math.sqrt(e_full[str(P0)] ** 2 + e_shell ** 2)
        matched = min((int(P) for P in e_full if e_full[P] <= target), default=max(int(P) for P in e_full))
        out[str(ps)] = {
            "atom_steps_per_s": n / (ms_f * 1e-3), "ms_per_step": ms_f,
            "fwd_bwd_atom_steps_per_s": n / (ms_fb * 1e-3), "ms_per_step_fwd_bwd": ms_fb,
            "stage_ms": {k: round(v[0], 4) for k, v in st.items() if v[1]},
            "shell_sampling_err": e_shell, "total_err": target,
            "matched_full_list_p_kspace": matched,
            "speedup_vs_full_list_equal_p": ms_full / ms_f,
        }
    out["note"] = ("p_shell -> entries; lists (core only) rebuilt every step; errors in kJ/mol/nm, RMS over atoms; "
                   "total_err combines the k-space error of the full list at the same p with the shell-sampling "
                   "error (independent samples)")
    return out


def skin_lists(make, pos, G, w, args, ms_full, timed_steps, every=10):
    """Lists built with a skin (cells of edge >= r_core + skin, core lists within
    r_core + skin, shell lists within (r_core - skin, r_shell + skin]) and
    rebuilt every `every` steps; each force evaluation counts an entry only when
    it is a member at the evaluation positions. The positions evaluated are the
    build positions displaced by just under skin / 2 per atom (the largest move
    the lists allow), so that the membership tests take effect. Per-step rates
    include the amortized list build. The same is timed for the full list with
    the same skin (the usual Verlet-list practice), and the shell-sampling error
    against the full list at the displaced positions, same k-vectors."""
    import torch
    n = w.n_atoms
    P0 = args.p_kspace
    out = {}
    gen = torch.Generator(device=pos.device).manual_seed(21)
    for skin in (0.05, 0.1):
        half = skin / (2.0 * math.sqrt(3.0)) * 0.999
        pos_m = pos + (torch.rand(pos.shape, generator=gen, device=pos.device, dtype=torch.float64) * 2.0 - 1.0
                       ).to(pos.dtype) * half
        row = {}
        for kind, ps in (("rbl", args.p_shell), ("full_list", 0)):
            h = make(ps, P0, 13595, "list", skin)

            def fwd(step):
                if step % every == 0:
                    h.build_lists(pos, step)
                h.compute_forces(pos_m, step)

            def fwd_bwd(step):
                fwd(step)
                h.compute_forces_backward(pos_m, step, G)

            ms_f = timed_steps(fwd, every, 3 * every, 9000) * 1e3
            r = {"atom_steps_per_s": n / (ms_f * 1e-3), "ms_per_step": ms_f}
            if kind == "rbl":
                ms_fb = timed_steps(fwd_bwd, every, 2 * every, 9500) * 1e3
                r.update({"fwd_bwd_atom_steps_per_s": n / (ms_fb * 1e-3), "ms_per_step_fwd_bwd": ms_fb})
                st = stage_times(h, fwd_bwd, every, 9700)
                r["stage_ms"] = {k: round(v[0], 4) for k, v in st.items() if v[1]}
                counts = h.debug("counts")
                r["list_entries_per_atom"] = {"core": int(counts[0]) / n, "shell": int(counts[1]) / n}
            h.close()
            row[kind] = r
        f_full = forces(make, pos_m, 0, P0, 13595)
        row["rbl"]["shell_sampling_err"] = rms(forces(make, pos, args.p_shell, P0, 13595, skin=skin,
                                                      pos_eval=pos_m) - f_full)
        row["rbl"]["speedup_vs_full_list_every_step"] = ms_full / row["rbl"]["ms_per_step"]
        row["rbl"]["speedup_vs_full_list_same_skin"] = row["full_list"]["ms_per_step"] / row["rbl"]["ms_per_step"]
        out[str(skin)] = row
    out["note"] = (f"skin in nm; lists rebuilt every {every} steps, forces evaluated at positions displaced by just "
                   f"under skin/2; shell_sampling_err in kJ/mol/nm, RMS over atoms, against the full list at the "
                   f"displaced positions with the same k-vectors")
    return out


def electrolyte_scaling(timed_steps, sizes=(1_000_000, 10_000_000)):
    """The 1:1 primitive-model electrolyte of the paper's scaling runs (density
    0.01 sigma^-3, reduced units, shifted-truncated LJ, alpha = 0.03, p = 100,
    r_c = 15) at 10^6 and 10^7 ions: forward step time of RBL+RBE (r_core = 5,
    p~ = 10) against the full list with the same RBE, with lists rebuilt every
    step and with a skin of 0.5 sigma and lists rebuilt every 20 steps."""
    import torch

    from paper_2204_13595_amd import inputs, irbe
    dev = torch.device("cuda", 0)
    out = {}
    for n in sizes:
        box = (n / 0.01) ** (1.0 / 3.0)
        w = inputs.electrolyte(1, n_anions=n // 2, box=box)
        pos = torch.tensor(w.pos, dtype=torch.float32, device=dev)
        row = {}
        for kind, ps, skin, every in (("rbl", 10, 0.0, 1), ("full_list", 0, 0.0, 1), ("rbl_skin", 10, 0.5, 20),
                                      ("full_list_skin", 0, 0.5, 20)):
            h = irbe.Handle(w.n_atoms, box, beta=math.sqrt(0.03), r_core=5.0, r_shell=15.0, p_shell=ps,
                            p_kspace=100, coulomb_k=1.0, lj_cut=2.0 ** (1.0 / 6.0), skin=skin, device=dev)
            h.set_system(torch.tensor(w.atom_type, device=dev), torch.tensor(w.charge, dtype=torch.float32, device=dev),
                         torch.tensor(w.molecule, device=dev), w.lj_sigma, w.lj_eps)

            def fwd(step):
                if step % every == 0:
                    h.build_lists(pos, step)
                h.compute_forces(pos, step)

            ms = timed_steps(fwd, every, max(5, 2 * every), 11000) * 1e3
            st = stage_times(h, fwd, every, 11200)
            counts = h.debug("counts")
            h.close()
            row[kind] = {"ms_per_step": ms, "atom_steps_per_s": w.n_atoms / (ms * 1e-3),
                         "stage_ms": {k: round(v[0], 3) for k, v in st.items() if v[1]},
                         "list_entries_per_atom": [int(counts[0]) / w.n_atoms, int(counts[1]) / w.n_atoms]}
        row["speedup_rbl"] = row["full_list"]["ms_per_step"] / row["rbl"]["ms_per_step"]
        row["speedup_rbl_skin"] = row["full_list_skin"]["ms_per_step"] / row["rbl_skin"]["ms_per_step"]
        out[str(w.n_atoms)] = row
        del pos
        torch.cuda.empty_cache()
    out["note"] = ("1:1 electrolyte, density 0.01, L = (N / 0.01)^(1/3); *_skin: skin 0.5 sigma, lists rebuilt every "
                   "20 steps (static positions); list_entries_per_atom = [core, shell or full]")
    return out


def precision_sweep(timed_steps):
    """FP64 against mixed precision, forward + backward, on the 6,291,456-atom box
    (2,097,152 waters, L = 39.7 nm, p_shell = 100, p = 500): atom-steps/s of
    each and the FP32-vs-FP64 error of forces and gradients (the FP64 path is
    parity-tested against the FP64 oracle)."""
    import torch

    from paper_2204_13595_amd import inputs, irbe
    w = inputs.workload("water2M")
    n = w.n_atoms
    dev = torch.device("cuda", 0)
    pos32 = torch.tensor(w.pos, dtype=torch.float32, device=dev)
    q32 = torch.tensor(w.charge, dtype=torch.float32, device=dev)
    G32 = torch.randn((n, 3), dtype=torch.float32, device=dev, generator=torch.Generator(device=dev).manual_seed(8))
    out, res = {}, {}
    for prec in ("mixed", "fp64"):
        dt = torch.float64 if prec == "fp64" else torch.float32
        pos, G = pos32.to(dt), G32.to(dt)
        h = irbe.Handle(n, w.box, p_shell=100, p_kspace=500, precision=prec, device=dev)
        h.set_system(torch.tensor(w.atom_type, device=dev), q32.to(dt), torch.tensor(w.molecule, device=dev),
                     w.lj_sigma, w.lj_eps)

        def fwd_bwd(step):
            h.build_lists(pos, step)
            h.compute_forces(pos, step)
            h.compute_forces_backward(pos, step, G)

        ms = timed_steps(fwd_bwd, 1, 3, 8000) * 1e3
        h.build_lists(pos, 5)
        f = h.compute_forces(pos, 5).double()
        gp, gq, _ = h.compute_forces_backward(pos, 5, G)
        res[prec] = (f, gp.double(), gq.double())
        h.close()
        out[prec] = {"ms_per_step_fwd_bwd": ms, "fwd_bwd_atom_steps_per_s": n / (ms * 1e-3)}
    (f32, g32, q32g), (f64, g64, q64g) = res["mixed"], res["fp64"]
    out["fp32_vs_fp64"] = {"force_rms_rel": rms(f32 - f64) / rms(f64), "grad_pos_rms_rel": rms(g32 - g64) / rms(g64),
                           "grad_charge_rms_rel": float((q32g - q64g).pow(2).mean().sqrt()
                                                        / q64g.pow(2).mean().sqrt())}
    out["workload"] = "water2M: 2097152 waters (6291456 atoms), L=39.7 nm, P_s=100, P=500"
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU decomposition is not "
              f"part of this build", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2204_13595_amd import inputs, irbe

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.electrolyte:
        log(f"electrolyte comparison at {args.electrolyte} ions")
        print(json.dumps({"electrolyte": electrolyte_scaling(timed_steps, (args.electrolyte,))}), flush=True)
        return
    log(f"generating {args.workload}")
    w = inputs.workload(args.workload)
    n = w.n_atoms
    dt = torch.float64 if args.precision == "fp64" else torch.float32
    pos = torch.tensor(w.pos, dtype=dt, device=dev)
    q = torch.tensor(w.charge, dtype=dt, device=dev)
    at = torch.tensor(w.atom_type, device=dev)
    mol = torch.tensor(w.molecule, device=dev)

    def make(p_shell, p_kspace, seed=13595, shell_source="list", skin=0.0):
        h = irbe.Handle(n, w.box, p_shell=p_shell, p_kspace=p_kspace, seed=seed, precision=args.precision,
                        shell_source=shell_source, skin=skin, device=dev)
        h.set_system(at, q, mol, w.lj_sigma, w.lj_eps)
        return h

    if args.copy_probe:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    h = make(args.p_shell, args.p_kspace)
    F = torch.empty((n, 3), dtype=dt, device=dev)
    G = torch.randn((n, 3), dtype=dt, device=dev, generator=torch.Generator(device=dev).manual_seed(5))

    def fwd(step):
        h.build_lists(pos, step)
        h.compute_forces(pos, step, out=F)

    def fwd_bwd(step):
        fwd(step)
        h.compute_forces_backward(pos, step, G)

    log("timing forward")
    per_step = []
    ms = timed_steps(fwd, args.warmup, args.steps, per_step=per_step) * 1e3
    value = n / (ms * 1e-3)
    ms_median = float(np.median(per_step))
    extras = {}
    if not args.no_extras:
        log("timing forward+backward")
        ms_fb = timed_steps(fwd_bwd, 1, max(args.steps // 2, 2), 1000) * 1e3
        h.build_lists(pos, 0)
        log("timing forces with reused lists")
        ms_f = timed_steps(lambda s: h.compute_forces(pos, s, out=F), 1, args.steps, 2000) * 1e3
        st = stage_times(h, fwd_bwd, 4, 3000)
        counts = h.debug("counts")
        shell_bits = int(h.debug("shell_bits")[0])
        h.close()
        log("timing the full-list variant")
        hf = make(0, args.p_kspace)

        def fwd_full(step):
            hf.build_lists(pos, step)
            hf.compute_forces(pos, step, out=F)

        ms_full = timed_steps(fwd_full, 1, max(args.steps // 2, 2), 4000) * 1e3
        st_full = stage_times(hf, fwd_full, 3, 5000)
        counts_full = hf.debug("counts")
        hf.close()
        # dominant kernel of the forward step and its roofline
        fwd_stages = {k: v[0] for k, v in st.items() if k in ("bin", "lists", "quantize", "ksample", "rho", "pair",
                                                              "pair_reduce", "kspace")}
        dom = max(fwd_stages, key=fwd_stages.get)
        n_core, n_shell = int(counts[0]), int(counts[1])
        # algorithmic HBM bytes of the list build: each atom's position and molecule
        # id read once (20 B), its two counts and its list entries written. The
        # "lists" stage times the whole build: the packing of the per-atom records
        # (k_pack_sorted, ~0.02 ms) and k_build_lists_tiled.
        # The count takes 4 bytes per list entry (lists as explicit CSR of indices);
        # the build stores shell entries as 16-bit codes where it can, and the bytes
        # as stored are reported beside it.
        list_bytes = 20.0 * n + 8.0 * n + 4.0 * (n_core + n_shell)
        stored_bytes = 20.0 * n + 8.0 * n + 4.0 * n_core + shell_bits / 8.0 * n_shell
        lists_ms = st["lists"][0]
        roof = {
            "kernel": "k_build_lists", "bound": "hbm", "achieved": list_bytes / (lists_ms * 1e-3) / 1e9,
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "traffic": measured_traffic("k_build_lists", args.workload),
            "algorithmic_bytes": list_bytes, "avg_launch_ms": lists_ms,
            "algorithmic_basis": "20 B read + 8 B counts + 4 B per core or shell entry",
            "shell_entry_bits": shell_bits, "stored_bytes": stored_bytes,
            "stored_frac": stored_bytes / (lists_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
        }
        roof["frac"] = roof["achieved"] / roof["peak"]
        # measured ceilings of this GPU beside the published peaks (irbe_probe_rates):
        # a streaming copy's bytes read + written per second, and the full-rate 32-bit
        # VALU lane-operation rate against 256 CUs x 64 lanes x 2.4 GHz
        probe = irbe.probe_rates()
        roof["measured_copy_gb_per_s"] = probe["copy_bytes_per_s"] / 1e9
        roof["measured_valu_lane_ops_per_s"] = probe["valu_lane_ops_per_s"]
        roof["valu_peak_lane_ops_per_s"] = VALU_PEAK_LANE_OPS
        log("accuracy: two-seed error estimates, matched-error full list, precision")
        acc = accuracy(make, pos, G, w, args, ms, timed_steps)
        log("stencil sampling")
        stencil = stencil_sampling(make, pos, G, w, args, acc, ms_full, timed_steps)
        log("skin lists")
        skin = skin_lists(make, pos, G, w, args, ms_full, timed_steps)
        del pos, q, F, G
        torch.cuda.empty_cache()
        log("precision sweep on the 6.3M-atom box")
        sweep = precision_sweep(timed_steps) if args.workload == "water1M" and args.precision == "mixed" else None
        log("electrolyte scaling")
        elec = electrolyte_scaling(timed_steps)
        log("constant-energy water32k")
        from paper_2204_13595_amd import md
        nve = {"rbl": md.run_nve(p_shell=args.p_shell), "full_list": md.run_nve(p_shell=0),
               "full_list_by_p": [md.run_nve(p_shell=0, p_kspace=pk) for pk in (800, 3200)],
               "full_list_fp64_large_p": md.run_nve(p_shell=0, p_kspace=12800, precision="fp64"),
               "note": ("32,768 rigid waters (98,304 atoms, L = 9.93 nm), 1000 velocity-Verlet steps at dt = 1 fs "
                        "from Maxwell velocities at 300 K (zero friction) after 2000 relaxation steps, lists rebuilt "
                        "every step; P = 200 unless stated; initial_* = slopes over the first 0.1 ps (the heating "
                        "by the random batch Ewald force, whose variance scales as 1/P); drift = slope over the "
                        "whole run; trace = temperature and total energy every 50 fs; ms_per_step = lists + forces "
                        "+ integrator; a run that heats until the rigid constraints fail stops at the check (every "
                        "100 steps) that found it: constraints_failed_by_ps, and the samples up to the check before")}
        extras = {
            "fwd_bwd_atom_steps_per_s": n / (ms_fb * 1e-3), "ms_per_step_fwd_bwd": ms_fb,
            "forces_only_reused_lists_atom_steps_per_s": n / (ms_f * 1e-3), "ms_per_forces_only": ms_f,
            "full_list_atom_steps_per_s": n / (ms_full * 1e-3), "ms_per_step_full_list": ms_full,
            "speedup_vs_full_list": ms_full / ms,
            "stage_ms": {k: round(v[0], 4) for k, v in st.items() if v[1]},
            "stage_ms_full_list": {k: round(v[0], 4) for k, v in st_full.items() if v[1]},
            "dominant_stage": dom,
            "list_entries_per_atom": {"core": n_core / n, "shell": n_shell / n, "full_list": counts_full[1] / n},
            "roofline": roof,
            "accuracy": acc,
            "stencil_sampling": stencil,
            "skin_lists": skin,
            "precision_sweep": sweep,
            "nve_water32k": nve,
            "electrolyte_scaling": elec,
        }
    else:
        if args.with_backward:
            for s in range(args.steps):
                fwd_bwd(9000 + s)
            torch.cuda.synchronize()
        h.close()
    out = {
        "metric": METRIC, "value": value, "unit": "atom-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "ms_per_step_median": ms_median, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if args.precision == "mixed" else "f64", "data": "synthetic",
        "config": {
            "workload": (f"{args.workload}: {w.n_waters} SPC/E-like waters ({n} atoms), L={w.box} nm, beta=3.0/nm, "
                         f"r_core=0.5 nm, r_shell=1.2 nm, P_s={args.p_shell}, P={args.p_kspace}, "
                         f"{'FP32 arithmetic with FP64 accumulation' if args.precision == 'mixed' else 'FP64'}"),
            "step": "build_lists + compute_forces (lists rebuilt every step)",
        },
    }
    if extras:
        out["roofline"] = extras.pop("roofline")
        out.update(extras)
    if not args.no_cpu_baseline:
        log("timing the CPU oracle sample")
        out["cpu_baseline"] = cpu_baseline(w, args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
