"""Host-side logic of the water comparison (no GPU): the differences that
md.compare reports for runs made separately."""
import numpy as np

from paper_2204_13595_amd import md


def _run(scale_g=1.0, u=-46.0, d=0.0023, msd_end=0.35):
    r = np.linspace(0.002, 1.198, 300)
    g = np.where(r > 0.25, 1.0 + 2.0 * np.exp(-((r - 0.28) / 0.02) ** 2), 0.0) * scale_g
    return {"r": r, "g": g, "msd_t": np.linspace(0.0, 25.0, 11), "msd": np.linspace(0.0, msd_end, 11),
            "diffusion_nm2_per_ps": d, "xi_mean": 0.05, "u_per_molecule": u, "u_sem": 0.01, "temperature": 298.0,
            "ms_per_step": 1.0, "steps": 1000, "frames": 10}


def test_compare_of_separate_runs():
    runs = {"full": _run(), "rbl_0.7_100": _run(scale_g=1.01, u=-46.46, d=0.00230, msd_end=0.3465),
            "rbl_0.6_150": _run()}
    out = md.compare(runs=runs)
    assert out["full"]["rel_u_diff_vs_full"] == 0.0
    row = out["rbl_0.7_100"]
    assert abs(row["rel_u_diff_vs_full"] - (-46.46 / -46.0 - 1.0)) < 1e-12
    assert abs(row["rel_g_peak_diff_vs_full"] - 0.01) < 1e-12
    assert abs(row["rel_msd_end_diff_vs_full"] - (0.3465 / 0.35 - 1.0)) < 1e-12
    assert abs(row["rel_diffusion_diff_vs_full"] - (0.0023 / 0.0023 - 1.0)) < 1e-12
    assert abs(row["max_abs_g_diff_vs_full"] - 0.03) < 1e-3  # 1% of the peak height 3
    assert abs(row["r_peak"] - 0.28) < 0.005
    assert "1000 steps per run" in out["setup"]
