"""Short text summaries of rocprofv3 output (CSV format) for the kernels of
the SRP hot path, and the HBM-traffic record the benchmark reads back.

    python -m paper_2306_08514_amd.rocprof_summary trace DIR TITLE CMD... > out.md
    python -m paper_2306_08514_amd.rocprof_summary traffic FETCH_DIR WRITE_DIR TITLE CMD... > out.md

    python -m paper_2306_08514_amd.rocprof_summary counters TITLE DIR... -- CMD... > out.md
    python -m paper_2306_08514_amd.rocprof_summary clock DIR TITLE CMD... > out.md

`trace` turns a `--kernel-trace --stats` run into a table of per-kernel
calls and durations.  `counters` tabulates the per-dispatch medians of
every counter found in one or more `--pmc` runs, per kernel, with the
ratios derived from them (matrix-core and LDS busy fractions, L2 hit
rate).  `traffic` reads two `--pmc FETCH_SIZE` /
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
    # FD: FP32 128 x 128 tiles (also the LR fat stage), 16-bit / FP8 gemm_fd16;
    # the general tall GEMM: FP32 256 x 128, 16-bit / FP8 128 x 128
    (r"gemm_fd16", "gemm_fd"),
    (r"gemm_nt<float, 128, 128|gemm_ntIfLi128ELi128E|gemm_nt<[^,]+, 256, 256|gemm_ntI[^L]*Li256ELi256E", "gemm_fd"),
    (r"gemm_nt", "gemm_tall"),
    (r"tall_ws<.*, true>|tall_wsI.*Lb1E", "sspi_dense"),
    (r"tall_ws", "gemm_tall"),
    (r"sspi_gather", "sspi_gather"),
    (r"sspi_band_records", "sspi_band_records (plan)"),
    (r"sspi_band_tables", "sspi_band_tables (plan)"),
    (r"sspi_band_passes", "sspi_band_passes (plan)"),
    (r"sspi_band", "sspi_band"),
    (r"lam_gemm_f64", "lam_gemm_f64 (plan)"),
    (r"xi_to_frames|xi_rows16|rows_to_f16", "xi_to_frames"),
    (r"split_reduce", "split_reduce"),
    (r"sspi_dense_weights", "sspi_dense_weights (plan)"),
    (r"gcc_direct", "gcc_direct"),
    (r"slri_fat_global", "slri_fat_global"),
    (r"slri_fat", "slri_fat"),
    (r"phat_kernel", "phat"),
    (r"build_steering", "build_steering (plan)"),
    (r"gram_global_f64", "gram_global_f64 (plan)"),
    (r"slri_u_global_f64", "slri_u_global_f64 (plan)"),
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


def _targs(name):
    """Template arguments of a (possibly mangled) kernel name, for telling
    instances of one kernel apart: '<...>' when demangled, else the integer
    arguments 'Li<n>E' of the mangled name."""
    m = re.search(r"<([^()]*)>\(", name)
    if m:
        return m.group(1)
    ints = re.findall(r"Li(\d+)E", name)
    return ",".join(ints) if ints else name[:24]


def unique_tags(names):
    """{name: tag}, where kernels that share a tag get their template
    arguments appended."""
    by = {}
    for n in names:
        by.setdefault(tag(n), []).append(n)
    out = {}
    for t, ns in by.items():
        for n in ns:
            out[n] = t if len(ns) == 1 else f"{t} <{_targs(n)}>"
    return out


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
    names = sorted(set(fv) | set(wv))
    tags = unique_tags(names)
    for name in names:
        t = tags[name]
        if tag(name) in ("copy", "torch (bench checks)"):
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
    rows = kernel_stats(d)
    tags = unique_tags([r[1] for r in rows])
    for tg, name, calls, tot, avg, mn, mx in rows:
        if tg == "torch (bench checks)":
            continue
        lines.append(f"| {tags[name]} | {calls} | {tot / 1e6:.3f} | {avg / 1e3:.2f} | {mn / 1e3:.2f} | {mx / 1e3:.2f} | "
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


# derived ratios of the counters summary; the cycle counters are summed by
# rocprofv3 over their instances: SQ_VALU_MFMA_BUSY_CYCLES over the SIMDs,
# SQ_LDS_IDX_ACTIVE and SQ_BUSY_CU_CYCLES over the CUs, GRBM_GUI_ACTIVE over
# the XCDs (so GRBM_GUI_ACTIVE / XCDS is the kernel's length in cycles)
XCDS, CUS, SIMDS = 8, 256, 1024
DERIVED = [
    ("mfma busy", ("SQ_VALU_MFMA_BUSY_CYCLES", "GRBM_GUI_ACTIVE"), lambda m, g: m / (SIMDS * g / XCDS)),
    ("lds active", ("SQ_LDS_IDX_ACTIVE", "GRBM_GUI_ACTIVE"), lambda a, g: a / (CUS * g / XCDS)),
    ("cu busy", ("SQ_BUSY_CU_CYCLES", "GRBM_GUI_ACTIVE"), lambda b, g: b / (CUS * g / XCDS)),
    ("lds bank conflict / active", ("SQ_LDS_BANK_CONFLICT", "SQ_LDS_IDX_ACTIVE"), lambda c, a: c / a if a else 0.0),
    ("L2 hit", ("TCC_HIT_sum", "TCC_MISS_sum"), lambda h, m: h / (h + m) if h + m else 0.0),
]


def counters(dirs):
    """{tag: {"name", "dispatches", counter: median per dispatch}} over every
    counter of the *_counter_collection.csv files under dirs."""
    names = set()
    for d in dirs:
        for path in _find(d, "counter_collection.csv"):
            with open(path, newline="") as f:
                for r in csv.DictReader(f):
                    names.add(r["Counter_Name"])
    out = {}
    per = {}
    for d in dirs:
        for cname in sorted(names):
            try:
                per[(d, cname)] = counter_values(d, cname)
            except FileNotFoundError:
                continue
    tags = unique_tags({k for vals in per.values() for k in vals})
    for (d, cname), vals in per.items():
        if True:
            for kname, vs in vals.items():
                t = tags[kname]
                rec = out.setdefault(t, {"name": kname, "dispatches": len(vs)})
                rec[cname] = statistics.median(vs)
    for rec in out.values():
        for label, (a, b), fn in DERIVED:
            if a in rec and b in rec and rec[b]:
                rec[label] = fn(rec[a], rec[b])
    return out


def _md_counters(title, dirs, cmd):
    rec = counters(dirs)
    cnames = sorted({k for r in rec.values() for k in r if k.isupper() or k.startswith(("SQ_", "TCC_", "GRBM_",
                                                                                           "TCP_", "TA_", "TD_"))})
    labels = [lab for lab, _, _ in DERIVED if any(lab in r for r in rec.values())]
    lines = [f"# {title}", "", "Commands (repository root; rocprofv3 from /tmp with TMPDIR=/tmp; one run per",
             "counter group):", "", "```", cmd,
             "python -m paper_2306_08514_amd.rocprof_summary counters <title> <dirs> -- <command>", "```", "",
             f"Kernel source SHA-256: `{source_sha256()}`", "",
             "Derived ratios: matrix-core busy = SQ_VALU_MFMA_BUSY_CYCLES / (1024 SIMDs x GRBM_GUI_ACTIVE / 8 "
             "XCDs); LDS active and CU busy = SQ_LDS_IDX_ACTIVE or SQ_BUSY_CU_CYCLES / (256 CUs x "
             "GRBM_GUI_ACTIVE / 8); L2 hit = TCC_HIT / (TCC_HIT + TCC_MISS).  Medians per dispatch.", "",
             "| kernel | dispatches | " + " | ".join(labels) + " |", "|---|---:|" + "---:|" * len(labels)]
    for t, r in sorted(rec.items()):
        if t.startswith(("copy", "torch (bench checks)")) or t.endswith("(plan)"):
            continue
        lines.append(f"| {t} | {r['dispatches']} | " +
                     " | ".join(f"{100 * r[lab]:.1f} %" if lab in r else "—" for lab in labels) + " |")
    lines += ["", "Raw medians per dispatch:", "", "| kernel | " + " | ".join(cnames) + " |",
              "|---|" + "---:|" * len(cnames)]
    for t, r in sorted(rec.items()):
        if t.startswith(("copy", "torch (bench checks)")) or t.endswith("(plan)"):
            continue
        lines.append(f"| {t} | " + " | ".join(f"{r[c]:.4g}" if c in r else "—" for c in cnames) + " |")
    return "\n".join(lines) + "\n"


def clocks(d):
    """{kernel name: [(span ns, clock GHz) per dispatch]} from a `--pmc
    GRBM_GUI_ACTIVE` run: the counter, summed over the XCDs, divided by the
    XCD count and by the dispatch's span gives the clock it ran at."""
    per = {}
    for path in _find(d, "counter_collection.csv"):
        with open(path, newline="") as f:
            for r in csv.DictReader(f):
                if r["Counter_Name"] != "GRBM_GUI_ACTIVE":
                    continue
                key = (r["Kernel_Name"], r.get("Dispatch_Id") or r.get("Correlation_Id"))
                span = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
                prev = per.get(key, (0.0, span))
                per[key] = (prev[0] + float(r["Counter_Value"]), span)
    out = {}
    for (name, _), (cyc, span) in per.items():
        if span > 0:
            out.setdefault(name, []).append((span, cyc / XCDS / span))
    return out


_MANGLED_TYPES = {"DF16b": "bf16", "DF16_": "f16", "f": "f32", "d": "f64", "NS_3fp8E": "fp8"}
_DEMANGLED_TYPES = {"__bf16": "bf16", "_Float16": "f16", "float": "f32", "double": "f64", "srp::fp8": "fp8"}


def _dtype(name):
    """Operand type of a kernel template instance (first template argument),
    '' when it has none."""
    m = re.search(r"<([^,<>()]*)[,>]", name)
    if m and m.group(1).strip() in _DEMANGLED_TYPES:
        return _DEMANGLED_TYPES[m.group(1).strip()]
    m = re.search(r"\d[a-z_0-9]+I(DF16b|DF16_|NS_3fp8E|f|d)", name)
    return _MANGLED_TYPES.get(m.group(1), "") if m else ""


def _md_clock(d, title, cmd, min_us=100.0):
    rows = []
    for name, vs in clocks(d).items():
        vs = [v for v in vs if v[0] >= min_us * 1e3]
        if not vs:
            continue
        ghz = sorted(v[1] for v in vs)
        rows.append((tag(name), name, len(vs), statistics.median(v[0] for v in vs) / 1e6, statistics.median(ghz),
                     ghz[0], ghz[-1]))
    rows.sort(key=lambda r: -r[3])
    lines = [f"# {title}", "", "Command (repository root; rocprofv3 from /tmp with TMPDIR=/tmp):", "",
             "```", cmd, "python -m paper_2306_08514_amd.rocprof_summary clock <dir> ...", "```", "",
             f"Kernel source SHA-256: `{source_sha256()}`", "",
             f"Clock of a dispatch = GRBM_GUI_ACTIVE (summed over the {XCDS} XCDs) / {XCDS} / the dispatch's span; "
             f"dispatches of at least {min_us:.0f} us.", "",
             "| kernel | dispatches | median ms | median GHz | min GHz | max GHz | full name |",
             "|---|---:|---:|---:|---:|---:|---|"]
    for tg, name, n, ms, med, lo, hi in rows:
        if tg == "torch (bench checks)":
            continue
        label = f"{tg} ({_dtype(name)})" if _dtype(name) else tg
        lines.append(f"| {label} | {n} | {ms:.3f} | {med:.2f} | {lo:.2f} | {hi:.2f} | `{name[:90]}` |")
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
    elif len(argv) >= 3 and argv[0] == "clock":
        sys.stdout.write(_md_clock(argv[1], argv[2], " ".join(argv[3:])))
    elif len(argv) >= 4 and argv[0] == "counters" and "--" in argv:
        i = argv.index("--")
        sys.stdout.write(_md_counters(argv[1], argv[2:i], " ".join(argv[i + 1:])))
    else:
        sys.stderr.write(__doc__)
        return 2
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
