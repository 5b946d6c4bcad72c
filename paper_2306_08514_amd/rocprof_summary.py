"""Short text summaries of rocprofv3 output (CSV format) for the kernels of
the SRP hot path, and the HBM-traffic record the benchmark reads back.

    python -m paper_2306_08514_amd.rocprof_summary trace DIR TITLE CMD... > out.md
    python -m paper_2306_08514_amd.rocprof_summary traffic FETCH_DIR WRITE_DIR TITLE CMD... > out.md

`trace` turns a `--kernel-trace --stats` run into a table of per-kernel
calls and durations.  `traffic` reads two `--pmc FETCH_SIZE` /
`--pmc WRITE_SIZE` runs of the same program, calibrates both counters with
the 1 GiB device-to-device copies that `bench.py --copy-calibration` issues
(the factor that maps the counter of a copy of known size onto its bytes),
and writes per-launch HBM bytes for every hot-path kernel, together with the
SHA-256 of the kernel source the counters were taken on.  `bench.py`
reports the traffic of its dominant kernel only while that hash still
matches the source.
"""

import csv
import glob
import hashlib
import json
import os
import re
import statistics
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCE = os.path.join(HERE, "csrc", "device.hip")
COPY_BYTES = 2 ** 30  # bench.py --copy-calibration: 2^28 float32 per copy

# short names of the hot-path kernels, matched on the (possibly mangled) name
_TAGS = [
    (r"gemm_nt_f64", "gemm_fd_f64"),
    # FD: FP32 128 x 128 tiles (also the LR fat stage), 16-bit / FP8 256 x 256;
    # the general tall GEMM: FP32 256 x 128, 16-bit / FP8 128 x 128
    (r"gemm_nt<float, 128, 128|gemm_ntIfLi128ELi128E|gemm_nt<[^,]+, 256, 256|gemm_ntI[^L]*Li256ELi256E", "gemm_fd"),
    (r"gemm_nt", "gemm_tall"),
    (r"tall_ws<.*, true>|tall_wsI.*Lb1E", "sspi_dense"),
    (r"tall_ws", "gemm_tall"),
    (r"sspi_gather", "sspi_gather"),
    (r"xi_to_frames", "xi_to_frames"),
    (r"sspi_dense_weights", "sspi_dense_weights (plan)"),
    (r"spectral_slices", "spectral_slices"),
    (r"slice_reduce", "slice_reduce"),
    (r"slri_fat", "slri_fat"),
    (r"phat_kernel", "phat"),
    (r"build_steering", "build_steering (plan)"),
    (r"gram_f64", "gram_f64 (plan)"),
    (r"slri_u_f64", "slri_u_f64 (plan)"),
    (r"sspi_windows", "sspi_windows (plan)"),
    (r"pair_absmax|scale_pairs", "scale (plan)"),
    (r"fd_gen", "gemm_fd_gen"),
    (r"gcc_fft", "gcc_fft"),
    (r"transpose_lp", "transpose_lp"),
    (r"argmax_rows", "argmax"),
    (r"convert_f32", "convert_f32 (plan)"),
    (r"transpose_xi", "transpose_xi"),
    (r"copyBuffer", "copy"),
    (r"at::native|fillBuffer", "torch (bench checks)"),
]


def source_sha256(path=KERNEL_SOURCE):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def tag(name):
    for pat, t in _TAGS:
        if re.search(pat, name):
            return t
    return name[:60]


def _find(d, suffix):
    hits = sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))
    if not hits:
        raise FileNotFoundError(f"no *{suffix} under {d}")
    return hits


def kernel_stats(d):
    """[(tag, name, calls, total_ns, avg_ns, min_ns, max_ns)] from *_kernel_stats.csv."""
    rows = []
    for path in _find(d, "kernel_stats.csv"):
        with open(path, newline="") as f:
            for r in csv.DictReader(f):
                rows.append((tag(r["Name"]), r["Name"], int(r["Calls"]), float(r["TotalDurationNs"]),
                             float(r["AverageNs"]), float(r["MinNs"]), float(r["MaxNs"])))
    rows.sort(key=lambda r: -r[3])
    return rows


def counter_values(d, counter):
    """{kernel name: [value per dispatch]} from *_counter_collection.csv; the
    value of one dispatch is the sum over its per-instance records."""
    per = {}
    for path in _find(d, "counter_collection.csv"):
        with open(path, newline="") as f:
            for r in csv.DictReader(f):
                if r["Counter_Name"] != counter:
                    continue
                key = (r["Kernel_Name"], r.get("Dispatch_Id") or r.get("Correlation_Id"))
                per[key] = per.get(key, 0.0) + float(r["Counter_Value"])
    out = {}
    for (name, _), v in per.items():
        out.setdefault(name, []).append(v)
    return out


def _calibration(vals):
    """bytes per counter unit from the largest copy dispatches (the 1 GiB copies)."""
    copies = [v for name, vs in vals.items() if tag(name) == "copy" for v in vs]
    if not copies:
        raise RuntimeError("no copy dispatch found; run the program with --copy-calibration")
    big = sorted(copies)[-3:]
    return COPY_BYTES / statistics.median(big), statistics.median(big)


def traffic(fetch_dir, write_dir):
    fv = counter_values(fetch_dir, "FETCH_SIZE")
    wv = counter_values(write_dir, "WRITE_SIZE")
    fcal, fcopy = _calibration(fv)
    wcal, wcopy = _calibration(wv)
    kernels = {}
    for name in sorted(set(fv) | set(wv)):
        t = tag(name)
        if t == "copy":
            continue
        f = statistics.median(fv[name]) if name in fv else None
        w = statistics.median(wv[name]) if name in wv else None
        kernels[t] = {"name": name, "dispatches": len(fv.get(name, [])),
                      "fetch_counter": f, "write_counter": w,
                      "fetch_bytes": f * fcal if f is not None else None,
                      "write_bytes": w * wcal if w is not None else None}
        if f is not None and w is not None:
            kernels[t]["bytes_per_launch"] = f * fcal + w * wcal
    return {"source_sha256": source_sha256(),
            "calibration": {"copy_bytes": COPY_BYTES, "fetch_counter_of_copy": fcopy,
                            "write_counter_of_copy": wcopy, "fetch_bytes_per_unit": fcal,
                            "write_bytes_per_unit": wcal},
            "kernels": kernels}


def _md_trace(d, title, cmd):
    lines = [f"# {title}", "", "Command (repository root; rocprofv3 from /tmp with TMPDIR=/tmp):", "",
             "```", cmd, "python -m paper_2306_08514_amd.rocprof_summary trace <dir> ...", "```", "",
             f"Kernel source SHA-256: `{source_sha256()}`", "",
             "| kernel | calls | total ms | avg us | min us | max us | full name |",
             "|---|---:|---:|---:|---:|---:|---|"]
    for t, name, calls, tot, avg, mn, mx in kernel_stats(d):
        lines.append(f"| {t} | {calls} | {tot / 1e6:.3f} | {avg / 1e3:.2f} | {mn / 1e3:.2f} | {mx / 1e3:.2f} | "
                     f"`{name[:110]}` |")
    return "\n".join(lines) + "\n"


def _md_traffic(fd, wd, title, cmd):
    rec = traffic(fd, wd)
    c = rec["calibration"]
    lines = [f"# {title}", "", "Commands (repository root; rocprofv3 from /tmp with TMPDIR=/tmp):", "", "```",
             cmd, "python -m paper_2306_08514_amd.rocprof_summary traffic <fetch dir> <write dir> ...", "```", "",
             f"Calibration: a {c['copy_bytes'] / 2**30:.0f} GiB device copy reads FETCH_SIZE "
             f"{c['fetch_counter_of_copy']:.0f} and WRITE_SIZE {c['write_counter_of_copy']:.0f} (counter units), "
             f"so one unit is {c['fetch_bytes_per_unit']:.1f} B fetched / {c['write_bytes_per_unit']:.1f} B written.",
             "", "| kernel | dispatches | fetch MB/launch | write MB/launch | total MB/launch |",
             "|---|---:|---:|---:|---:|"]
    for t, k in rec["kernels"].items():
        fb = k["fetch_bytes"]
        wb = k["write_bytes"]
        tot = k.get("bytes_per_launch")
        lines.append(f"| {t} | {k['dispatches']} | {fb / 1e6 if fb is not None else float('nan'):.3f} | "
                     f"{wb / 1e6 if wb is not None else float('nan'):.3f} | "
                     f"{tot / 1e6 if tot is not None else float('nan'):.3f} |")
    lines += ["", "Machine-readable record (read by bench.py):", "", "```json", json.dumps(rec, indent=1), "```"]
    return "\n".join(lines) + "\n"


def read_traffic_record(md_path):
    """The JSON record embedded in a traffic summary, or None."""
    try:
        text = open(md_path).read()
    except OSError:
        return None
    m = re.search(r"```json\n(.*?)\n```", text, re.S)
    return json.loads(m.group(1)) if m else None


def main(argv):
    if len(argv) >= 3 and argv[0] == "trace":
        sys.stdout.write(_md_trace(argv[1], argv[2], " ".join(argv[3:])))
    elif len(argv) >= 4 and argv[0] == "traffic":
        sys.stdout.write(_md_traffic(argv[1], argv[2], argv[3], " ".join(argv[4:])))
    else:
        sys.stderr.write(__doc__)
        return 2
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
