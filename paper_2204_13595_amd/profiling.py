"""Summaries of rocprofv3 output for the kernels of this library.

    python -m paper_2204_13595_amd.profiling stats <kernel_stats.csv>
    python -m paper_2204_13595_amd.profiling traffic <fetch counter_collection.csv> <write counter_collection.csv> \
        <kernel substring> <out.json>
    python -m paper_2204_13595_amd.profiling issue <counter_collection.csv> <kernel_stats.csv>

`stats` prints the per-kernel table (calls, average and total duration) of a
`rocprofv3 --kernel-trace --stats --output-format csv` run. `traffic` turns two
`rocprofv3 --pmc FETCH_SIZE` / `--pmc WRITE_SIZE` runs into HBM bytes per launch
of one kernel: the counters (KiB per dispatch) are scaled by what they read for
the 1 GiB device-to-device copy that `bench.py --copy-probe` performs (1 GiB read,
1 GiB written), and the result records the hash of the kernel's source file so
that a later change of the kernel invalidates it. `issue` turns a run with
SQ_INSTS_VALU, SQ_INSTS_SALU and SQ_INSTS_LDS into per-dispatch instruction
counts and the VALU issue fraction of each kernel: SQ_INSTS_VALU x 4 cycles (one
wave64 instruction on a 16-lane SIMD) over the SIMD cycles of its average
duration (1,024 SIMDs at 2.4 GHz), a lower bound on VALU busy time since
quarter-rate instructions occupy the SIMD longer.
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
COPY_BYTES = 1 << 30
KERNEL_SOURCES = {"k_build_lists": "k_lists.hip", "k_pair_coop": "k_pair.hip", "k_pair_adjoint": "k_pair.hip",
                  "k_rho_partial": "k_kspace.hip", "k_kspace_forces": "k_kspace.hip", "k_draw_batches": "k_pair.hip", "k_bucket_reduce": "k_pair.hip"}


def source_hash(kernel: str) -> str | None:
    for key, fname in KERNEL_SOURCES.items():
        if key in kernel:
            data = open(os.path.join(HERE, "csrc", fname), "rb").read()
            return hashlib.sha256(data).hexdigest()[:16]
    return None


def short_name(name: str) -> str:
    name = name.replace("void ", "")
    return name.split("(")[0]


def stats_table(path: str) -> str:
    rows = list(csv.DictReader(open(path)))
    out = [f"{'kernel':58s} {'calls':>6s} {'avg_us':>10s} {'total_ms':>10s} {'pct':>6s}"]
    for r in rows:
        out.append(f"{short_name(r['Name'])[:58]:58s} {int(r['Calls']):6d} {float(r['AverageNs']) / 1e3:10.2f} "
                   f"{float(r['TotalDurationNs']) / 1e6:10.3f} {float(r['Percentage']):6.2f}")
    return "\n".join(out)


def _per_dispatch(path: str, counter: str):
    vals = {}
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        vals.setdefault(short_name(r["Kernel_Name"]), []).append(float(r["Counter_Value"]))
    return vals


def traffic(fetch_csv: str, write_csv: str, kernel: str) -> dict:
    fetch = _per_dispatch(fetch_csv, "FETCH_SIZE")
    write = _per_dispatch(write_csv, "WRITE_SIZE")

    def pick(d, key):
        names = [k for k in d if key in k]
        if not names:
            raise KeyError(f"no kernel matching {key!r}")
        v = d[names[0]]
        return sum(v) / len(v)

    copy_f = max(v for k, vals in fetch.items() if "copyBuffer" in k for v in vals)
    copy_w = max(v for k, vals in write.items() if "copyBuffer" in k for v in vals)
    f_scale = COPY_BYTES / (copy_f * 1024.0)
    w_scale = COPY_BYTES / (copy_w * 1024.0)
    kf = pick(fetch, kernel)
    kw = pick(write, kernel)
    return {
        "kernel": kernel, "fetch_kib_per_launch": kf, "write_kib_per_launch": kw,
        "copy_fetch_kib": copy_f, "copy_write_kib": copy_w, "fetch_scale": f_scale, "write_scale": w_scale,
        "hbm_bytes_per_launch": kf * 1024.0 * f_scale + kw * 1024.0 * w_scale,
        "source_sha": source_hash(kernel),
    }


N_SIMD = 1024
CLOCK_HZ = 2.4e9


def issue_table(counters_csv: str, stats_csv: str) -> str:
    dur = {short_name(r["Name"]): float(r["AverageNs"]) * 1e-9 for r in csv.DictReader(open(stats_csv))}
    cols = ("SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS")
    per = {c: _per_dispatch(counters_csv, c) for c in cols}
    out = [f"{'kernel':58s} {'avg_us':>9s} {'VALU/disp':>11s} {'SALU/disp':>11s} {'LDS/disp':>11s} {'VALU_issue':>10s}"]
    rows = []
    for k, v in per["SQ_INSTS_VALU"].items():
        if k not in dur:
            continue
        valu = sum(v) / len(v)
        salu = sum(per["SQ_INSTS_SALU"].get(k, [0.0])) / max(len(per["SQ_INSTS_SALU"].get(k, [0.0])), 1)
        lds = sum(per["SQ_INSTS_LDS"].get(k, [0.0])) / max(len(per["SQ_INSTS_LDS"].get(k, [0.0])), 1)
        frac = valu * 4.0 / (N_SIMD * CLOCK_HZ * dur[k])
        rows.append((dur[k], f"{k[:58]:58s} {dur[k] * 1e6:9.1f} {valu:11.4g} {salu:11.4g} {lds:11.4g} {frac:10.3f}"))
    out += [r for _, r in sorted(rows, reverse=True)]
    return "\n".join(out)


def main(argv):
    if argv[:1] == ["stats"]:
        print(stats_table(argv[1]))
    elif argv[:1] == ["issue"]:
        print(issue_table(argv[1], argv[2]))
    elif argv[:1] == ["traffic"]:
        t = traffic(argv[1], argv[2], argv[3])
        json.dump(t, open(argv[4], "w"), indent=1)
        print(json.dumps(t, indent=1))
    else:
        print(__doc__)
        return 2
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
