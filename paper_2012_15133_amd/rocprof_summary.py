"""Summarise rocprofv3 CSV output into the short text/JSON files kept under profiles/.

Usage:
  python -m paper_2012_15133_amd.rocprof_summary stats <kernel_stats.csv> <out.md> --command "<cmd>"
  python -m paper_2012_15133_amd.rocprof_summary traffic <fetch_dir> <write_dir> <copy_fetch_dir>
         <copy_write_dir> <copy_bytes> <workload> <F_bytes> <dim> <profiles_dir> --command "<cmd>"
  python -m paper_2012_15133_amd.rocprof_summary counters <c1_dir> <c2_dir> <label>

`traffic` turns FETCH_SIZE and WRITE_SIZE (KiB per dispatch) into HBM bytes per
launch, each scaled by the factor that makes a device copy of known size read and
write exactly that many bytes, and writes one JSON per step kernel
(traffic_<kernel>_<workload>.json) stamped with the hash of the kernel sources.
"""

from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import json
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

ROLE = {"k_spec_inv": "spec_inv", "k_real_pass": "real_pass", "k_spec_fwd": "spec_fwd",
        "k_finalize": "step_finalize", "k_update": "update"}


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2012_15133_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def _counter_means(d: str, with_counts: bool = False):
    path = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)[0]
    agg = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        agg[(r["Kernel_Name"], r["Counter_Name"])].append(float(r["Counter_Value"]))
    means = {k: sum(v) / len(v) for k, v in agg.items()}
    if with_counts:
        return means, {k: len(v) for k, v in agg.items()}
    return means


def _targs(name: str):
    """Template arguments of a kernel name, e.g. ['float', '256', '4', '3', 'true', 'false']."""
    if "<" not in name:
        return []
    return [x.strip() for x in name.split("<", 1)[1].split(">")[0].split(",")]


def _role(name: str):
    for k, v in ROLE.items():
        if k + "<" in name or k + "(" in name:
            if k == "k_real_pass" and _targs(name)[4] == "false":   # the E_1-only pass of queries
                return None
            return v
    if "k_ypass<" in name:
        return "pass_y_inv" if _targs(name)[3] == "1" else "pass_y_fwd"
    return None


def stats(src: str, out: str, command: str):
    rows = list(csv.DictReader(open(src)))
    lines = ["# rocprofv3 kernel statistics", "", f"Command: `{command}`", "",
             "| kernel | calls | average (us) | min (us) | max (us) | share (%) |", "|---|---|---|---|---|---|"]
    for r in rows:
        lines.append(f"| `{r['Name'][:90]}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                     f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | {float(r['Percentage']):.1f} |")
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def traffic(fetch_dir, write_dir, cfetch_dir, cwrite_dir, copy_bytes, workload, F, dim, outdir, command):
    fe, counts = _counter_means(fetch_dir, with_counts=True)
    wr = _counter_means(write_dir)
    cfe, cwr = _counter_means(cfetch_dir), _counter_means(cwrite_dir)
    copy_f = max(v for (k, c), v in cfe.items() if c == "FETCH_SIZE" and "copyBuffer" in k)
    copy_w = max(v for (k, c), v in cwr.items() if c == "WRITE_SIZE" and "copyBuffer" in k)
    kib = copy_bytes / 1024.0
    sf, sw = kib / copy_f, kib / copy_w
    alg = {"spec_inv": 6 * F, "real_pass": 2 * dim * F, "spec_fwd": 5 * F, "pass_y_inv": 5 * F, "pass_y_fwd": 5 * F}
    h = kernel_source_hash()
    # per role, the launch-plan variant with the most dispatches (the one the run used after
    # tuning; the tuner's trial variants appear a few times each)
    pick = {}
    for (name, c), v in fe.items():
        role = _role(name)
        if c == "FETCH_SIZE" and role in alg and (role not in pick or counts[(name, c)] > counts[(pick[role], c)]):
            pick[role] = name
    summary = []
    for (name, c), v in fe.items():
        if c != "FETCH_SIZE":
            continue
        role = _role(name)
        if role not in alg or pick.get(role) != name:
            continue
        w = wr.get((name, "WRITE_SIZE"))
        if w is None:
            continue
        fb, wb = v * 1024 * sf, w * 1024 * sw
        d = {"kernel": role, "kernel_name": name, "workload": workload, "fetch_bytes_per_launch": fb,
             "write_bytes_per_launch": wb, "hbm_bytes_per_launch": fb + wb, "algorithmic_bytes": alg[role],
             "fetch_scale": sf, "write_scale": sw, "copy_calibration_bytes": copy_bytes,
             "kernel_source_hash": h, "command": command}
        with open(os.path.join(outdir, f"traffic_{role}_{workload}.json"), "w") as fh:
            json.dump(d, fh, indent=1)
        summary.append(d)
    return summary


STEP_KERNELS = ("k_spec_inv", "k_real_pass", "k_spec_fwd", "k_ypass")


def counters(c1: str, c2: str, label: str):
    """Table rows of the SQ counter sets C1 (cycles, waits) and C2 (instructions, LDS
    conflicts, waves): per step-kernel variant the mean per dispatch.  Variants with fewer
    than 8 dispatches (start-up, energy-only passes) are left out."""
    agg = collections.defaultdict(lambda: collections.defaultdict(float))
    disp = collections.defaultdict(set)
    for k, d in ((1, c1), (2, c2)):
        for path in glob.glob(os.path.join(d, "*counter_collection.csv")):
            for row in csv.DictReader(open(path)):
                name = row["Kernel_Name"]
                if not any(x in name for x in STEP_KERNELS):
                    continue
                if "k_real_pass" in name and _targs(name)[4] == "false":
                    continue
                agg[name][row["Counter_Name"]] += float(row["Counter_Value"])
                disp[(name, k)].add(row["Dispatch_Id"])
    rows = []
    for name in sorted(agg, key=lambda n: -len(disp[(n, 1)])):
        c = agg[name]
        n1, n2 = len(disp[(name, 1)]), len(disp[(name, 2)]) or 1
        if n1 < 8:
            continue
        role = name.split("<")[0].replace("void spfc::", "")
        tmpl = [x.strip() for x in name.split("<")[1].split(">")[0].split(",")]
        if role == "k_ypass":
            role += " (" + ("inverse" if tmpl[3] == "1" else "forward") + ")"
        rows.append(f"| {label} | `{role}` | {tmpl[2]} | {c['SQ_WAVES'] / n2:.0f} | "
                    f"{c['SQ_WAVE_CYCLES'] / n1 / 1e6:.2f}M | {c['SQ_WAIT_ANY'] / n1 / 1e6:.2f}M | "
                    f"{c['SQ_WAIT_INST_LDS'] / n1 / 1e6:.2f}M | {c['SQ_INSTS_VALU'] / n2 / 1e6:.2f}M | "
                    f"{c['SQ_INSTS_LDS'] / n2 / 1e6:.3f}M | {c['SQ_LDS_BANK_CONFLICT'] / n2 / 1e6:.3f}M |")
    return rows


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd")
    s1 = sub.add_parser("stats")
    s1.add_argument("src")
    s1.add_argument("out")
    s1.add_argument("--command", default="")
    s2 = sub.add_parser("traffic")
    for a in ("fetch", "write", "cfetch", "cwrite"):
        s2.add_argument(a)
    s2.add_argument("copy_bytes", type=int)
    s2.add_argument("workload")
    s2.add_argument("F", type=float)
    s2.add_argument("dim", type=int)
    s2.add_argument("outdir")
    s2.add_argument("--command", default="")
    s3 = sub.add_parser("counters")
    s3.add_argument("c1")
    s3.add_argument("c2")
    s3.add_argument("label")
    a = ap.parse_args()
    if a.cmd == "stats":
        stats(a.src, a.out, a.command)
    elif a.cmd == "counters":
        print("\n".join(counters(a.c1, a.c2, a.label)))
    elif a.cmd == "traffic":
        for d in traffic(a.fetch, a.write, a.cfetch, a.cwrite, a.copy_bytes, a.workload, a.F, a.dim, a.outdir,
                         a.command):
            print(d["kernel"], round(d["hbm_bytes_per_launch"] / 1e6, 2), "MB vs", round(d["algorithmic_bytes"] / 1e6, 2))
