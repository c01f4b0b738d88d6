"""Summaries of rocprofv3 output for the measurement record.

* ``kernel_table``: per-kernel statistics of a ``--kernel-trace --stats`` run
  (the ``*_kernel_stats.csv`` file) as a markdown table.
* ``traffic``: HBM bytes per dispatch of one kernel from two ``--pmc`` runs
  (FETCH_SIZE, then WRITE_SIZE; both in KiB per dispatch), each scaled by what
  the same counter reads for a plain device copy of known size, written as a
  small JSON record together with a hash of the kernel sources it was taken
  on.  ``bench.py`` reports the record's traffic only while that hash still
  matches the sources.

Usage (from the repository root, on the CSV folders rocprofv3 wrote):

  python -m paper_2608_17123_amd.profiling traffic --kernel k_cgls_p2 \\
      --fetch DIR --write DIR --calib-fetch DIR --calib-write DIR \\
      --calib-bytes N --command "..." --out profiles/NAME.json
  python -m paper_2608_17123_amd.profiling table DIR "title" "command"
"""
import argparse
import csv
import glob
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
# sources that decide the CGLS phase kernels' memory traffic
TRAFFIC_SOURCES = ["kernels_solve.hip", "kernels_cgls_sep.hip", "kernels_cgls_multi.hip",
                   "cgls_sep.h", "phase.h", "stencil.h", "common.h", "launch.h"]


def source_hash(names=TRAFFIC_SOURCES):
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(HERE, "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _csv(folder, suffix):
    files = sorted(glob.glob(os.path.join(folder, "**", "*" + suffix), recursive=True))
    if not files:
        raise FileNotFoundError(f"no *{suffix} under {folder}")
    rows = []
    for f in files:
        with open(f) as fh:
            rows.extend(csv.DictReader(fh))
    return rows


def counter_per_dispatch(folder, kernel, counter):
    """Mean value of `counter` over the dispatches whose kernel name contains
    `kernel`, and the number of such dispatches."""
    vals = {}
    for r in _csv(folder, "counter_collection.csv"):
        if kernel in r["Kernel_Name"] and r["Counter_Name"] == counter:
            key = r["Dispatch_Id"]
            vals[key] = vals.get(key, 0.0) + float(r["Counter_Value"])
    if not vals:
        raise ValueError(f"no {counter} samples for kernel {kernel} in {folder}")
    return sum(vals.values()) / len(vals), len(vals)


def traffic(args):
    f_kib, nf = counter_per_dispatch(args.fetch, args.kernel, "FETCH_SIZE")
    w_kib, nw = counter_per_dispatch(args.write, args.kernel, "WRITE_SIZE")
    cf_kib, _ = counter_per_dispatch(args.calib_fetch, args.calib_kernel, "FETCH_SIZE")
    cw_kib, _ = counter_per_dispatch(args.calib_write, args.calib_kernel, "WRITE_SIZE")
    ff = cf_kib * 1024.0 / args.calib_bytes  # counter bytes per true byte read
    fw = cw_kib * 1024.0 / args.calib_bytes  # counter bytes per true byte written
    rec = {
        "kernel": args.kernel,
        "dispatches": {"fetch": nf, "write": nw},
        "fetch_kib_per_dispatch": f_kib,
        "write_kib_per_dispatch": w_kib,
        "calibration": {"kernel": args.calib_kernel, "bytes_each_way": args.calib_bytes,
                        "fetch_factor": ff, "write_factor": fw},
        "hbm_bytes_per_dispatch": f_kib * 1024.0 / ff + w_kib * 1024.0 / fw,
        "source_hash": source_hash(),
        "command": args.command,
    }
    with open(args.out, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec))


def read_traffic(path):
    """Traffic record at `path` when it was taken on the current sources."""
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_hash") != source_hash():
        return None
    return rec


def _short(name):
    return name.replace("(dbl::Job const*, unsigned int const*)", "").replace("void ", "")[:70]


def kernel_table(folder, title, command):
    """Markdown summary: per-kernel statistics, then the CGLS kernels by
    launch size (blocks per launch)."""
    rows = _csv(folder, "kernel_stats.csv")
    out = [f"# {title}", "", "Command (from the repository root on the GPU box):", "", "```",
           command, "```", "", "## Kernel statistics (rocprofv3 --kernel-trace --stats)", "",
           "| kernel | calls | total ms | avg us | min us | max us | % |",
           "|---|---|---|---|---|---|---|"]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
        out.append(f"| `{_short(r['Name'])}` | {r['Calls']} | "
                   f"{float(r['TotalDurationNs']) / 1e6:.2f} | "
                   f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['MinNs']) / 1e3:.2f} | "
                   f"{float(r['MaxNs']) / 1e3:.2f} | {float(r['Percentage']):.1f} |")
    agg = {}
    for r in _csv(folder, "kernel_trace.csv"):
        if "k_cgls" not in r["Kernel_Name"]:
            continue
        key = (_short(r["Kernel_Name"]),
               int(r["Grid_Size_X"]) // int(r["Workgroup_Size_X"]), int(r["Workgroup_Size_X"]))
        agg.setdefault(key, []).append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    out += ["", "## CGLS kernels by launch size", "",
            "| kernel | blocks per launch | threads per block | launches | avg us |",
            "|---|---|---|---|---|"]
    for k in sorted(agg):
        v = agg[k]
        out.append(f"| `{k[0]}` | {k[1]} | {k[2]} | {len(v)} | {sum(v) / len(v) / 1e3:.1f} |")
    return "\n".join(out) + "\n"


def main(argv=None):
    p = argparse.ArgumentParser()
    sub = p.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("--kernel", required=True)
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--calib-fetch", required=True)
    t.add_argument("--calib-write", required=True)
    t.add_argument("--calib-kernel", default="copy_kernel")
    t.add_argument("--calib-bytes", type=float, required=True)
    t.add_argument("--command", default="")
    t.add_argument("--out", required=True)
    k = sub.add_parser("table")
    k.add_argument("folder")
    k.add_argument("title")
    k.add_argument("command")
    a = p.parse_args(argv)
    if a.cmd == "traffic":
        traffic(a)
    else:
        sys.stdout.write(kernel_table(a.folder, a.title, a.command))


if __name__ == "__main__":
    main()
