"""Parity at the full benchmark sizes, on sampled atoms.

The 3,145,728-atom water box runs in the benchmark's launch configuration
(mixed precision, p_shell = 100, p = 100); the 6,291,456-atom box in FP64 and
in mixed precision with p = 500 (errors on a 4096-atom sample). The oracle
recomputes, for a random sample of atoms, their core and
shell lists, batch ranks and uncorrected short-range, excluded-pair and
long-range forces (the structure factor over every atom). The momentum
correction is checked through a property that holds at any size: the total
force vanishes.
"""
import numpy as np
import pytest

from paper_2204_13595_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.mark.parametrize("name,precision,p_kspace,tol,n_rows", [("water1M", "mixed", 100, 1e-5, 4096),
                                                                 ("water2M", "fp64", 500, 1e-11, 4096),
                                                                 ("water2M", "mixed", 500, 1e-5, 4096)])
def test_fullsize_sampled_parity(orc, name, precision, p_kspace, tol, n_rows):
    from paper_2204_13595_amd import irbe
    w = inputs.workload(name)
    dev = torch.device("cuda", 0)
    dt = torch.float64 if precision == "fp64" else torch.float32
    step = 11
    h = irbe.Handle(w.n_atoms, w.box, p_shell=100, p_kspace=p_kspace, precision=precision, device=dev)
    pos = torch.tensor(w.pos, dtype=dt, device=dev)
    q = torch.tensor(w.charge, dtype=dt, device=dev)
    h.set_system(torch.tensor(w.atom_type, device=dev), q, torch.tensor(w.molecule, device=dev), w.lj_sigma,
                 w.lj_eps)
    h.build_lists(pos, step)
    F = h.compute_forces(pos, step)
    fcorr = h.debug("fcorr")
    rho_gpu = h.debug("rho").reshape(-1, 2)
    kvec = h.debug("kvec").reshape(-1, 3)
    Fsum = F.double().sum(dim=0).cpu().numpy()
    Fabs = F.double().abs().sum().item()
    rows = np.sort(np.random.default_rng(42).choice(w.n_atoms, size=n_rows, replace=False))
    Fr = F[torch.tensor(rows, device=dev)].double().cpu().numpy()
    core_off = h.debug_rows("core_off", rows)
    core_idx = h.debug_rows("core_idx", rows)
    shell_off = h.debug_rows("shell_off", rows)
    shell_idx = h.debug_rows("shell_idx", rows)
    b_off = h.debug_rows("batch_off", rows)
    b_rank = h.debug_rows("batch_rank", rows)
    h.close()
    del F, pos
    torch.cuda.empty_cache()

    pos_np = torch.tensor(w.pos, dtype=dt).double().numpy()
    q_np = torch.tensor(w.charge, dtype=dt).double().numpy()
    p = orc.Params(box=w.box, p_shell=100, p_kspace=p_kspace)
    s = orc.quantize(pos_np, w.box)
    lists = orc.build_lists(s, w.molecule, w.box, 0.5, 1.2, rows=rows)
    assert np.array_equal(core_off, lists.core_off) and np.array_equal(core_idx, lists.core_idx)
    assert np.array_equal(shell_off, lists.shell_off) and np.array_equal(shell_idx, lists.shell_idx)
    batches = orc.shell_batches(p.seed, step, lists, p.p_shell)
    assert np.array_equal(b_off, batches[0]) and np.array_equal(b_rank, batches[1])
    m, W, S = orc.sample_kspace(p, step)
    assert np.array_equal(kvec, m)
    rho = orc.structure_factor(s, q_np, m)
    assert np.abs(rho_gpu - rho).max() < 100 * tol * np.abs(rho).max()
    ref = orc.forward(None, q_np, w.atom_type, w.molecule, w.lj_sigma, w.lj_eps, p, step=step, mode="rbl",
                      rows=rows, s=s, lists=lists, batches=batches, kspace=(m, W, S), rho=rho)
    uncorrected = ref.f_short + ref.f_excl + ref.f_long
    err = np.sqrt(((Fr + fcorr - uncorrected) ** 2).sum() / (uncorrected ** 2).sum())
    assert err < tol, err
    # every sampled atom, in units of the RMS force (20 times the RMS bound: the
    # largest of ~4096 normally scattered errors is about 4 times their RMS)
    atom_err = np.sqrt(((Fr + fcorr - uncorrected) ** 2).sum(1)).max() / np.sqrt((uncorrected ** 2).sum(1).mean())
    assert atom_err < 20 * tol, atom_err
    # momentum: sum_i F_i = 0 (Eq. 2.12 for the short range, Im|rho|^2 = 0 for RBE)
    assert np.abs(Fsum).max() < (1e-6 if precision == "mixed" else 1e-12) * Fabs


def test_fullsize_backward_properties():
    """The adjoint at the benchmark's size and launch configuration (mixed,
    p_shell = 100, p = 100, 3,145,728 atoms), checked through identities that
    hold at any size for fixed lists and samples, with L = sum_i G_i . F_i:
      * translation invariance of every force term: sum_i dL/dr_i = 0;
      * without LJ the force is homogeneous of degree 2 in the charges:
        sum_i q_i dL/dq_i = 2 L;
      * without charges it is homogeneous of degree 1 in the LJ epsilons:
        sum_ab eps_ab dL/deps_ab = L;
    and against the FP64 path on the same inputs (FP64 arithmetic, its own
    record staging: 800 records per block against 1,200)."""
    from paper_2204_13595_amd import irbe
    w = inputs.workload("water1M")
    dev = torch.device("cuda", 0)
    step = 13
    at = torch.tensor(w.atom_type, device=dev)
    mol = torch.tensor(w.molecule, device=dev)
    # both precisions see the same (FP32-representable) positions, charges and dL/dF
    G = torch.randn((w.n_atoms, 3), dtype=torch.float32, device=dev,
                    generator=torch.Generator(device=dev).manual_seed(9)).double()
    pos32 = torch.tensor(w.pos, dtype=torch.float32, device=dev)

    def run(precision, q_scale=1.0, eps_scale=1.0):
        dt = torch.float64 if precision == "fp64" else torch.float32
        h = irbe.Handle(w.n_atoms, w.box, p_shell=100, p_kspace=100, precision=precision, device=dev)
        q = torch.tensor(w.charge * q_scale, dtype=torch.float32, device=dev).to(dt)
        h.set_system(at, q, mol, w.lj_sigma, w.lj_eps * eps_scale)
        pos = pos32.to(dt)
        h.build_lists(pos, step)
        F = h.compute_forces(pos, step)
        gp, gq, gl = h.compute_forces_backward(pos, step, G.to(dt))
        L = float((G * F.double()).sum())
        out = (L, gp.double(), gq.double(), gl.double().cpu().numpy(), q.double())
        h.close()
        return out

    L, gp, gq, gl, q = run("mixed")
    scale = float(gp.abs().sum())
    assert float(gp.sum(dim=0).abs().max()) < 1e-6 * scale
    L64, gp64, gq64, gl64, _ = run("fp64")
    assert float(((gp - gp64) ** 2).sum().sqrt() / (gp64 ** 2).sum().sqrt()) < 1e-5
    assert float(((gq - gq64) ** 2).sum().sqrt() / (gq64 ** 2).sum().sqrt()) < 1e-5
    # the LJ parameter gradients are single sums over ~10^8 FP32 pair terms of both
    # signs (dL/dF is random here), which cancel to about 1/100 of the sum of
    # their magnitudes: ~1e-7 per term becomes ~1e-5 of the result, bounded at 1e-4
    assert abs(gl[0] - gl64[0]) < 1e-4 * abs(gl64[0]) and abs(gl[4] - gl64[4]) < 1e-4 * abs(gl64[4])
    # Coulomb only (eps = 0): degree 2 in the charges
    Lc, _, gqc, _, qc = run("mixed", eps_scale=0.0)
    assert abs(float((qc * gqc).sum()) - 2.0 * Lc) < 1e-5 * float((qc * gqc).abs().sum())
    # LJ only (q = 0): degree 1 in the epsilons (only the O-O entry is non-zero)
    Ll, _, _, gll, _ = run("mixed", q_scale=0.0)
    eps = w.lj_eps
    nt2 = len(eps)
    assert abs(float((eps * gll[nt2:2 * nt2]).sum()) - Ll) < 1e-5 * abs(Ll)


def test_fullsize_backward_is_deterministic():
    """The adjoint in the benchmark's configuration (3,145,728 atoms, mixed,
    p_shell = p = 100): no shell-adjoint record takes the atomic fallback, and
    two calls agree bit for bit."""
    from paper_2204_13595_amd import irbe
    w = inputs.workload("water1M")
    dev = torch.device("cuda", 0)
    step = 3
    h = irbe.Handle(w.n_atoms, w.box, p_shell=100, p_kspace=100, device=dev)
    pos = torch.tensor(w.pos, dtype=torch.float32, device=dev)
    h.set_system(torch.tensor(w.atom_type, device=dev), torch.tensor(w.charge, dtype=torch.float32, device=dev),
                 torch.tensor(w.molecule, device=dev), w.lj_sigma, w.lj_eps)
    G = torch.randn((w.n_atoms, 3), dtype=torch.float32, device=dev,
                    generator=torch.Generator(device=dev).manual_seed(5))
    h.build_lists(pos, step)
    h.compute_forces(pos, step)
    a = h.compute_forces_backward(pos, step, G)
    assert int(h.debug("adj_atomics")[0]) == 0
    b = h.compute_forces_backward(pos, step, G)
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    h.close()


@pytest.mark.parametrize("precision,tol_f,tol_g,tol_lj", [("fp64", 1e-11, 1e-10, 1e-9), ("mixed", 1e-5, 2e-5, 1e-4)])
def test_precision_sweep_against_oracle(orc, precision, tol_f, tol_g, tol_lj):
    """The precision sweep's workload (6,291,456 atoms, L = 39.7 nm, p_shell =
    100, p = 500) in both precisions against the FP64 oracle on 4096 sampled
    atoms, for every result: forces, and the gradients with respect to the
    positions and charges of the sampled atoms and the LJ sigma and epsilon of
    L = sum_i G_i . F_i with G supported on the sample (pairs of opposite values,
    so that it sums to zero and the oracle's row-subset adjoint is exact)."""
    from paper_2204_13595_amd import irbe
    w = inputs.workload("water2M")
    dev = torch.device("cuda", 0)
    dt = torch.float64 if precision == "fp64" else torch.float32
    step, P = 17, 500
    h = irbe.Handle(w.n_atoms, w.box, p_shell=100, p_kspace=P, precision=precision, device=dev)
    pos = torch.tensor(w.pos, dtype=torch.float32, device=dev).to(dt)  # both precisions see FP32 values
    q = torch.tensor(w.charge, dtype=torch.float32, device=dev).to(dt)
    h.set_system(torch.tensor(w.atom_type, device=dev), q, torch.tensor(w.molecule, device=dev), w.lj_sigma,
                 w.lj_eps)
    rng = np.random.default_rng(23)
    rows = np.sort(rng.choice(w.n_atoms, size=4096, replace=False))
    v = rng.standard_normal((2048, 3)).astype(np.float32).astype(np.float64)
    perm = rng.permutation(rows)
    G = np.zeros((w.n_atoms, 3))
    G[perm[0::2]] = v
    G[perm[1::2]] = -v
    h.build_lists(pos, step)
    F = h.compute_forces(pos, step)
    fcorr = h.debug("fcorr")
    gp, gq, gl = h.compute_forces_backward(pos, step, torch.tensor(G, dtype=dt, device=dev))
    rows_t = torch.tensor(rows, device=dev)
    Fr = F[rows_t].double().cpu().numpy()
    gpr = gp[rows_t].double().cpu().numpy()
    gqr = gq[rows_t].double().cpu().numpy()
    gl = gl.cpu().numpy()
    h.close()
    del F, gp, gq, pos
    torch.cuda.empty_cache()

    pos_np = torch.tensor(w.pos, dtype=torch.float32).double().numpy()
    q_np = torch.tensor(w.charge, dtype=torch.float32).double().numpy()
    p = orc.Params(box=w.box, p_shell=100, p_kspace=P)
    s = orc.quantize(pos_np, w.box)
    lists = orc.build_lists(s, w.molecule, w.box, 0.5, 1.2, rows=rows)
    batches = orc.shell_batches(p.seed, step, lists, p.p_shell)
    m, W, S = orc.sample_kspace(p, step)
    rho = orc.structure_factor(s, q_np, m)
    res = orc.forward(None, q_np, w.atom_type, w.molecule, w.lj_sigma, w.lj_eps, p, step=step, mode="rbl",
                      rows=rows, s=s, lists=lists, batches=batches, kspace=(m, W, S), rho=rho)
    r_pos, r_q, r_sig, r_eps = orc.backward_rows(G, q_np, w.atom_type, w.molecule, w.lj_sigma, w.lj_eps, p, res)

    def rms(a, b):
        return float(np.sqrt(((a - b) ** 2).sum() / (b ** 2).sum()))

    def worst(a, b):
        a, b = a.reshape(len(a), -1), b.reshape(len(b), -1)
        return float(np.sqrt(((a - b) ** 2).sum(1)).max() / np.sqrt((b ** 2).sum(1).mean()))

    uncorrected = res.f_short + res.f_excl + res.f_long
    errs = {"force": rms(Fr + fcorr, uncorrected), "force_worst_atom": worst(Fr + fcorr, uncorrected),
            "grad_pos": rms(gpr, r_pos), "grad_pos_worst_atom": worst(gpr, r_pos), "grad_q": rms(gqr, r_q),
            "grad_sigma_OO": abs(gl[0] - r_sig[0]) / abs(r_sig[0]),
            "grad_eps_OO": abs(gl[4] - r_eps[0]) / abs(r_eps[0])}
    print(f"precision sweep errors against the FP64 oracle ({precision}, 4096 atoms):", errs)
    assert errs["force"] < tol_f and errs["force_worst_atom"] < 20 * tol_f
    assert errs["grad_pos"] < tol_g and errs["grad_pos_worst_atom"] < 20 * tol_g
    assert errs["grad_q"] < tol_g
    assert errs["grad_sigma_OO"] < tol_lj and errs["grad_eps_OO"] < tol_lj
