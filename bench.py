"""Benchmark: adaptive SDC steps of the batched workload on one MI355X.

Headline workload (the metric's configuration): 48 independent 2D
monodomain instances of sides 96..384 (3,694,813 dofs in one context), P1
triangles on [0,2]^2 cm, isotropic conductivity 1e-3 exp(0.3 g) with g a
smoothed seeded Gaussian field, Aliev-Panfilov reaction, SDC on M = 3
Radau-IIA nodes, K = 4 sweeps per step, dt = 0.2 ms, drop tolerance 1e-7,
Jacobi-PCG to rtol 1e-12 (synthetic seeded inputs).  A "step" is one SDC
time step of every instance: K sweeps, each with M restricted solves per
instance, the reaction and the active-set selection.  `--warmup` steps run
first from t = 0 (the stimulus), then exactly `--steps` steps are timed with
the device synchronised on both sides (by default 5 and 95: the timed steps
are the rest of the workload's 100-step run, t = 1..20 ms); the timed
window is repeated `--repeats` times from the same state and the median
repeat is reported.

Reported value: active dof-sweeps per second = sum over the window's steps
and sweeps of the active rows, divided by its wall time.  The roofline
entry is for the dominant kernel (the CG iteration, one launch per CG
iteration over all instances still iterating), timed with HIP events on the
library's stream in a second pass over the same window; its bytes per
launch are given three ways: the minimum the chosen matrix storage must
move, a textbook count for CSR storage (12 B per stored entry, 120 B per
row), and HBM traffic from committed rocprofv3 counters.  The
adjoint/forward ratio is the reverse pass of 100 steps (checkpoint every
10) over the forward pass of the same steps.  The CPU baseline is the FP64
oracle on one host core over the first step(s) of the same window.  Further
legs: the 2D 512^2 and 3D 128^3 single-instance workloads (a window of
their early steps with its variants, and their whole runs, T = 200 and 400
ms, with windows at fixed times and the oracle on the same steps) and the
cell-by-cell workloads.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# wall-clock speedups of adaptive over non-adaptive SDC that the paper
# reports on CPUs (Kaskade 7; 2D: Core i7-9700T, 3D: Xeon E5), for context
PAPER_SPEEDUP = {"2d_monodomain": 2.13, "2d_emi": 3.336, "3d_monodomain": 3.29, "3d_emi": 4.344}
# snapshot times (ms) of the whole runs: the first steps, and the front at
# 10, 50 and 150 ms; in 3D also the second stimulus at 120 ms (colliding fronts)
FULL_RUN_SNAPSHOTS_2D = (0.0, 10.0, 50.0, 150.0)
FULL_RUN_SNAPSHOTS_3D = (0.0, 10.0, 50.0, 120.0, 150.0)
COUNTERS = os.path.join(ROOT, "profiles", "k_cg_iter_batched48_counters.md")
COUNTERS_3D = os.path.join(ROOT, "profiles", "k_cg_iter2_3d128.md")
# the device kernels and their launch constants: counter summaries name the
# hash of these files, and their bytes are used only while it still matches
KERNEL_SRCS = [os.path.join(ROOT, "paper_2311_07206_amd", "csrc", f)
               for f in ("kernels.hip", "kernels.hpp", "device.hpp")]


def kernel_sources_sha():
    """sha256 over the kernel source files, in the order of KERNEL_SRCS."""
    import hashlib
    h = hashlib.sha256()
    for path in KERNEL_SRCS:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(path=None):
    """HBM bytes per updating CG-iteration launch from committed FETCH_SIZE /
    WRITE_SIZE runs, as a dict with "all" and, when the summary has them,
    "listed" and "all_rows" launches; None when the kernel source changed
    since the counters were taken."""
    try:
        text = open(path or COUNTERS).read()
    except OSError:
        return None
    fields = dict(line.split(":", 1) for line in text.splitlines() if line.startswith("- ") and ":" in line)
    fields = {k[2:].strip(): v.strip() for k, v in fields.items()}
    if fields.get("kernel sources sha256") != kernel_sources_sha():
        return None
    out = {"all": float(fields["measured bytes per launch"])}
    for key, name in (("listed", "measured bytes per listed launch"),
                      ("all_rows", "measured bytes per all-rows launch")):
        if name in fields:
            out[key] = float(fields[name])
    if "algorithmic bytes per launch" in fields:
        out["algorithmic"] = float(fields["algorithmic bytes per launch"])
    return out


def summarize_trace(path):
    """Markdown summary of a rocprofv3 --kernel-trace CSV: per-kernel totals and
    the CG iteration kernel's duration by grid size and by launch class.
    When the run made calibration copies (three back-to-back device copies of
    at least 50 us and within 30 % of each other's duration: the first of
    them touches its memory first), only the dispatches after the last such
    triple count (the timed window); a setup's own large copies come
    earlier."""
    import collections
    import csv
    import re
    rows = sorted(csv.DictReader(open(path)), key=lambda r: int(r["Start_Timestamp"]))   # the CSV is not in time order
    dur = [int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in rows]
    is_copy = ["copyBuffer" in r["Kernel_Name"] for r in rows]
    start = 0
    for q in range(len(rows) - 2):
        trio = dur[q:q + 3]
        if all(is_copy[q:q + 3]) and min(trio) >= 50000 and max(trio) <= 1.3 * min(trio):
            start = q + 3
    durs, grid, by_cls = collections.defaultdict(list), collections.defaultdict(list), collections.defaultdict(list)
    for r, d in list(zip(rows, dur))[start:]:
        m = re.search(r"(k_\w+)", r["Kernel_Name"])
        name = m.group(1) if m else r["Kernel_Name"].split("(")[0][:60]
        durs[name].append(d)
        if name in ("k_cg_iter", "k_cg_iter2"):   # one or two rows per thread; 256-row map entries either way
            grid[int(r["Grid_Size_X"]) // int(r["Workgroup_Size_X"])].append(d)
            by_cls[cg_launch_class(r["Kernel_Name"])].append(d)
    total = sum(sum(v) for v in durs.values())
    out = [f"dispatches counted: {len(rows) - start} of {len(rows)}"
           + (" (after the calibration copies)" if start else ""), "",
           "| kernel | calls | total ms | avg us | share |", "|---|---|---|---|---|"]
    for k, v in sorted(durs.items(), key=lambda z: -sum(z[1])):
        out.append(f"| {k} | {len(v)} | {sum(v) / 1e6:.2f} | {np.mean(v) / 1e3:.3f} | {100 * sum(v) / total:.1f}% |")
    v = np.array(durs.get("k_cg_iter", []) + durs.get("k_cg_iter2", []) or [0])
    out += ["", f"CG iteration (k_cg_iter, k_cg_iter2): {len(v)} dispatches, mean {v.mean() / 1e3:.3f} us", "",
            "| launch class | dispatches | mean us | median us | dispatches >= 5 us | their mean us |",
            "|---|---|---|---|---|---|"]
    for c in ("all_rows", "listed"):
        x = np.array(by_cls.get(c, []))
        if len(x):
            big = x[x >= 5000]
            out.append(f"| {c} | {len(x)} | {x.mean() / 1e3:.2f} | {np.median(x) / 1e3:.2f} | {len(big)} | "
                       f"{(big.mean() if len(big) else 0) / 1e3:.2f} |")
    out += ["", "| blocks (256 rows) | dispatches | median us | mean us |", "|---|---|---|---|"]
    bins = [(1, 128), (128, 256), (256, 512), (512, 1024), (1024, 1025), (1025, 1 << 30)]
    for lo, hi in bins:
        x = np.array([d for g, ds in grid.items() if lo <= g < hi for d in ds])
        if len(x):
            out.append(f"| {lo}..{hi - 1} | {len(x)} | {np.median(x) / 1e3:.2f} | {x.mean() / 1e3:.2f} |")
    return "\n".join(out)


def cg_launch_class(name):
    """'listed' or 'all_rows' for a CG-iteration kernel name, else None
    (k_cg_iter2: every row, two per thread; k_cg_iter<S, FIRST, LIST, TOT>:
    LIST 1 a listed set, 0 every row)."""
    import re
    if "k_cg_iter2" in name:
        return "all_rows"
    m = re.search(r"k_cg_iter<\s*-?\d+\s*,\s*\w+\s*,\s*(-?\d+)", name)
    if m:
        return "listed" if m.group(1) == "1" else "all_rows"
    return None


def summarize_counters(fetch_csv, write_csv, min_blocks=0):
    """Pair FETCH_SIZE and WRITE_SIZE runs dispatch by dispatch (KiB per
    dispatch).  A 256 MiB device copy (reads and writes 262144 KiB) calibrates
    each counter; the CG iteration's launches that perform an update (writes
    above 1 KiB), with at least min_blocks map entries, give the measured HBM
    bytes per launch, over all of them and by launch class (listed set or
    every row)."""
    import csv
    rows = []
    for path in (fetch_csv, write_csv):
        r = sorted(csv.DictReader(open(path)), key=lambda x: int(x["Dispatch_Id"]))
        rows.append(r)
    f, w = rows
    assert len(f) == len(w), "the two runs must dispatch the same kernels"
    cg_f, cg_w, cls, copy = [], [], [], []
    for a, b in zip(f, w):
        assert a["Kernel_Name"] == b["Kernel_Name"]
    # only the launches after the last calibration copy (the timed window)
    last = max([q for q, b in enumerate(w) if "copyBuffer" in b["Kernel_Name"]
                and abs(float(b["Counter_Value"]) - 262144.0) < 13000.0] or [-1])
    for q, (a, b) in enumerate(zip(f, w)):
        if "k_cg_iter" in a["Kernel_Name"] and q > last:
            if min_blocks and int(a["Grid_Size"]) // int(a["Workgroup_Size"]) < min_blocks:
                continue
            cg_f.append(float(a["Counter_Value"]))
            cg_w.append(float(b["Counter_Value"]))
            cls.append(cg_launch_class(a["Kernel_Name"]))
        elif "copyBuffer" in a["Kernel_Name"] and abs(float(b["Counter_Value"]) - 262144.0) < 13000.0:
            copy.append((float(a["Counter_Value"]), float(b["Counter_Value"])))
    cg_f, cg_w, cls = np.array(cg_f), np.array(cg_w), np.array(cls, dtype=object)
    work = cg_w > 1.0
    ff = 262144.0 / np.mean([c[0] for c in copy])
    fw = 262144.0 / np.mean([c[1] for c in copy])
    fetch_kib, write_kib = cg_f[work].mean(), cg_w[work].mean()
    out = {"copy_fetch_kib": [c[0] for c in copy], "copy_write_kib": [c[1] for c in copy],
           "fetch_factor": ff, "write_factor": fw, "dispatches": int(len(cg_f)), "updating": int(work.sum()),
           "fetch_kib_per_launch": fetch_kib, "write_kib_per_launch": write_kib,
           "measured_bytes_per_launch": (ff * fetch_kib + fw * write_kib) * 1024.0,
           "kernel_sources_sha256": kernel_sources_sha()}
    for c in ("listed", "all_rows"):
        sel = work & (cls == c)
        if sel.any():
            out[f"{c}_updating"] = int(sel.sum())
            out[f"{c}_bytes_per_launch"] = (ff * cg_f[sel].mean() + fw * cg_w[sel].mean()) * 1024.0
    return out


def summarize_pmc(path):
    """Mean of every counter of a rocprofv3 --pmc CSV per dispatch, for the
    CG iteration by launch class (listed set, every row) and for the 256 MiB
    calibration copies; only dispatches after the last calibration copy
    count for the CG classes.  Copies are recognised by the largest
    WRITE-side or request counts of the run (they are its biggest dispatches)."""
    import collections
    import csv
    rows = sorted(csv.DictReader(open(path)), key=lambda r: (int(r["Dispatch_Id"]), r["Counter_Name"]))
    by = collections.defaultdict(dict)
    names = {}
    for r in rows:
        d = int(r["Dispatch_Id"])
        by[d][r["Counter_Name"]] = float(r["Counter_Value"])
        names[d] = r["Kernel_Name"]
    ids = sorted(by)
    copies = [d for d in ids if "copyBuffer" in names[d]]
    big = [d for d in copies if sum(by[d].values()) >= 0.5 * max(sum(by[c].values()) for c in copies)] if copies else []
    start = max(big) if big else -1
    out = {}
    groups = {"copy_256MiB": big}
    for c in ("listed", "all_rows"):
        groups[c] = [d for d in ids if d > start and cg_launch_class(names[d]) == c]
    for g, ds in groups.items():
        if ds:
            keys = sorted(by[ds[0]])
            out[g] = {"dispatches": len(ds), **{k: float(np.mean([by[d].get(k, 0.0) for d in ds])) for k in keys}}
    return out


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=95,
                    help="timed steps of the batched workload (default: the rest of its 100-step run)")
    ap.add_argument("--warmup", type=int, default=5, help="untimed steps from t = 0 before the window")
    ap.add_argument("--repeats", type=int, default=5, help="repeats of the timed window (median reported)")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the batched workload's window and its kernel pass (profiling runs)")
    ap.add_argument("--adjoint-steps", type=int, default=100)
    ap.add_argument("--ckpt-every", type=int, default=10)
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-graph", action="store_true", help="skip the graph-captured runs of the same windows")
    ap.add_argument("--no-sequential", action="store_true",
                    help="skip the 48 instances run one after another")
    ap.add_argument("--n", type=int, default=512, help="grid side of the 2D leg (workload uses 512)")
    ap.add_argument("--steps-2d", type=int, default=20)
    ap.add_argument("--warmup-2d", type=int, default=5)
    ap.add_argument("--cpu-sample-steps", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--no-2d", action="store_true", help="skip the 512^2 single-instance leg")
    ap.add_argument("--no-3d", action="store_true", help="skip the 128^3 3D workload")
    ap.add_argument("--no-emi", action="store_true", help="skip the cell-by-cell workloads (2D and 3D)")
    ap.add_argument("--emi-steps", type=int, default=3)
    ap.add_argument("--no-emi-3d", action="store_true", help="skip the 3D cell-by-cell workload")
    ap.add_argument("--no-speedup", action="store_true",
                    help="skip the non-adaptive (theta = 0) runs over the same steps")
    ap.add_argument("--no-linearized", action="store_true",
                    help="skip the 512x512 run with the paper's linearized basic scheme")
    ap.add_argument("--no-first-sweep", action="store_true",
                    help="skip the runs with the heuristic first-sweep set")
    ap.add_argument("--no-cg-energy", action="store_true",
                    help="skip the runs with the energy-error CG stop (the paper's 1e-3)")
    ap.add_argument("--small-set-rows", type=int, default=0,
                    help="the latency curve's solver option (0: default one-launch solves of small sets, -1: off)")
    ap.add_argument("--no-full-run", action="store_true",
                    help="skip the whole runs of the 2D and 3D workloads (T = 200 and 400 ms) and their windows")
    ap.add_argument("--full-window", type=int, default=5, help="steps of each window of the whole runs")
    ap.add_argument("--full-oracle-steps", type=int, default=1,
                    help="oracle steps at the start of each window of the whole runs (0: none)")
    ap.add_argument("--full-oracle-3d", action="store_true",
                    help="also time the oracle on the 3D window of the second stimulus (about 60 s of CPU)")
    ap.add_argument("--no-latency", action="store_true",
                    help="skip the time-per-sweep curve over front-shell active sets")
    ap.add_argument("--calib", action="store_true",
                    help="device copies of 256 MiB at the start of each timed window (counter calibration and the "
                         "window's start in rocprofv3 runs)")
    ap.add_argument("--no-headline", action="store_true",
                    help="skip the batched workload (profiling runs of the 2D or 3D leg alone)")
    ap.add_argument("--no-storage-variants", action="store_true",
                    help="skip the 3D leg's runs with CSR and sliced ELL storage forced")
    ap.add_argument("--summarize-trace", metavar="KERNEL_TRACE_CSV",
                    help="print a summary of a rocprofv3 kernel trace and exit")
    ap.add_argument("--min-blocks", type=int, default=0,
                    help="with --summarize-counters: only CG launches with at least this many map entries")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="pair rocprofv3 FETCH_SIZE / WRITE_SIZE counter runs, print JSON and exit")
    ap.add_argument("--summarize-pmc", metavar="COUNTER_CSV",
                    help="per-dispatch means of every counter of a rocprofv3 --pmc run, by launch class")
    return ap.parse_args()


def cg_roofline(prof, storage, n_diag, peak=None):
    """The CG iteration's roofline over the profiled launches: bytes per
    launch three ways and the event-timed mean launch duration.

    csr_count: a textbook Jacobi-PCG iteration on CSR storage: 12 B per
      stored entry (8 value + 4 column) and, per row, 4 (row pointer) + 4
      (list entry, listed sets only) + 112 (14 vector touches);
    storage_min: what the chosen storage must move at least: the symmetric
      diagonal storage reads its nd/2 + 1 stored diagonals per row (8 B each),
      CSR 12 B per entry and a 4 B row pointer; per row 3 vectors read once
      (u, w, s scaled by the preconditioner) and the same 3 written, the
      iterate x read and written every other launch (8 B a launch) and the
      direction p read and written every other launch, with u read a second
      time there to rebuild it (12 B a launch): 68 B (dinv is formed from the
      diagonal), plus the list entry;
    achieved: storage_min bytes / mean launch duration (the reported frac):
      csr_count (a column index and the full row per entry) exceeds what
      the symmetric diagonal storage moves, so its rate can pass the HBM
      peak; it is reported beside (csr_count_GBps, frac_csr_count).
    """
    peak = peak or HBM_PEAK_GBS
    L, ms = prof["cg_launches"], prof["cg_ms"]
    rows, nnz = prof["cg_rows"], prof["cg_nnz"]
    listed_rows = rows - prof["cg_all_rows"]
    b_scope = 12.0 * nnz + 116.0 * rows + 4.0 * listed_rows
    if storage == "dia":
        b_min = (8.0 * (n_diag // 2 + 1) + 68.0) * rows + 4.0 * listed_rows
    else:
        b_min = 12.0 * nnz + 72.0 * rows + 4.0 * listed_rows
    sec = ms * 1e-3
    out = {"kernel": "k_cg_iter (all CG-iteration launches: listed sets k_cg_iter, every row k_cg_iter2)",
           "bound": "hbm", "achieved": b_min / sec / 1e9, "peak": peak, "unit": "GB/s",
           "frac": b_min / sec / 1e9 / peak, "traffic": None,
           "avg_launch_us": 1e3 * ms / L, "launches": L,
           "bytes_per_launch_storage_min": b_min / L, "bytes_per_launch_csr_count": b_scope / L,
           "csr_count_GBps": b_scope / sec / 1e9, "frac_csr_count": b_scope / sec / 1e9 / peak,
           "rows_per_launch": rows / L}
    for cls, launches, lms, lrows, lnnz, listed in (
            ("all_rows", prof["cg_all_launches"], prof["cg_all_ms"], prof["cg_all_rows"], prof["cg_all_nnz"], 0.0),
            ("listed", L - prof["cg_all_launches"], ms - prof["cg_all_ms"], listed_rows, nnz - prof["cg_all_nnz"],
             1.0)):
        if launches <= 0 or lms <= 0:
            continue
        bs = 12.0 * lnnz + (116.0 + 4.0 * listed) * lrows
        bm = ((8.0 * (n_diag // 2 + 1) + 68.0) * lrows if storage == "dia" else 12.0 * lnnz + 72.0 * lrows) \
            + 4.0 * listed * lrows
        out[cls] = {"launches": launches, "avg_launch_us": 1e3 * lms / launches, "rows_per_launch": lrows / launches,
                    "storage_min_GBps": bm / (lms * 1e-3) / 1e9, "frac": bm / (lms * 1e-3) / 1e9 / peak,
                    "csr_count_GBps": bs / (lms * 1e-3) / 1e9, "frac_csr_count": bs / (lms * 1e-3) / 1e9 / peak}
    return out


def add_traffic(roof, mt, prof):
    """Counter-measured HBM bytes per launch (committed profile of the same
    command) beside the byte models, weighted by this run's launch mix."""
    if mt is None:
        return roof
    L, La = prof["cg_launches"], prof["cg_all_launches"]
    if "listed" in mt and "all_rows" in mt:
        per = (mt["all_rows"] * La + mt["listed"] * (L - La)) / L
    else:
        per = mt["all"]
    sec = prof["cg_ms"] * 1e-3
    roof["traffic"] = per
    roof["measured_GBps"] = per * L / sec / 1e9
    roof["frac_measured"] = roof["measured_GBps"] / roof["peak"]
    for cls in ("all_rows", "listed"):
        if cls in mt and cls in roof:
            t = roof[cls]["avg_launch_us"] * 1e-6
            roof[cls]["traffic"] = mt[cls]
            roof[cls]["measured_GBps"] = mt[cls] / t / 1e9
            roof[cls]["frac_measured"] = mt[cls] / t / 1e9 / roof["peak"]
    return roof


def sweep_bytes(st, M, ident):
    """Algorithmic bytes of one sweep from its statistics.

    8 B per FP64 value, 4 B per active-list entry (absent when every row is
    active), 8 B per stored matrix value; index structure (CSR columns and
    row pointers) is storage overhead and not counted.  Per active row
    (n_a rows, z_a stored values of A in them):
      sweep start    8 z_a + idx + 8 (6M + 4)
      node RHS       8 z_a [m > 0] + idx + 8 (2m + 4)
      CG start       8 z_a + idx + 24
      CG iteration   8 z + idx + 88   per iteration (z = values of the rows
                     still iterating)
      post-solve     idx + 8 (m + 14)
      selection      2 idx + 24
    """
    na, za = st["n_active"], st["nnz_active"]
    idxb = 0 if ident else 4
    b = 8 * za + na * (idxb + 8 * (6 * M + 4))
    for m in range(M):
        rows, nnz = st["cg_row_iters"][m], st["cg_nnz_iters"][m]
        b += (8 * za if m > 0 else 0) + na * (idxb + 8 * (2 * m + 4))
        b += 8 * za + na * (24 + idxb)
        b += 8 * nnz + (88 + idxb) * rows
        b += na * (idxb + 8 * (m + 14))
    b += na * (2 * idxb + 24)
    return b


def step_bytes(N, M):
    """Per step outside the sweeps: spread (read v0, w0; write v, w, I, R at M nodes) and copy-out."""
    return N * (16 + 32 * M) + N * 32


def main():
    args = parse()
    if args.summarize_trace:
        print(summarize_trace(args.summarize_trace))
        return
    if args.summarize_counters:
        print(json.dumps(summarize_counters(*args.summarize_counters, min_blocks=args.min_blocks), indent=1))
        return
    if args.summarize_pmc:
        print(json.dumps(summarize_pmc(args.summarize_pmc), indent=1))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU (the library is single-device); --gpus must be 1"}))
        sys.exit(2)
    t_run = time.perf_counter()

    def done(leg):
        # one line per finished leg on stderr (the JSON line stays alone on stdout)
        print(f"[bench] {leg} done at {time.perf_counter() - t_run:.0f} s", file=sys.stderr, flush=True)

    out, window = ({}, None) if args.no_headline else headline(args)
    done("batched workload")
    if not args.headline_only:
        out["copy_GBps"] = copy_bandwidth()
        if "roofline" in out:
            out["roofline"]["frac_of_copy"] = out["roofline"]["achieved"] / out["copy_GBps"]
        if not args.no_2d:
            out["workload_2d"] = workload_2d(args)
            done("2D workload")
        if not args.no_3d:
            out["workload_3d"] = workload_3d(speedup=not args.no_speedup, first_sweep=not args.no_first_sweep,
                                             cg_energy=not args.no_cg_energy,
                                             variants=not args.no_storage_variants, calib=args.calib,
                                             repeats=args.repeats)
            done("3D workload window")
            if not args.no_full_run:
                from workloads import config2
                # the 3D oracle takes about 50 s to build and 11-18 s per step on
                # one core: on request it runs the window of the second stimulus
                out["workload_3d"]["full_run"] = full_run(config2(), FULL_RUN_SNAPSHOTS_3D, args.full_window,
                                                          args.repeats, args.full_oracle_steps,
                                                          cpu=args.full_oracle_3d and args.full_oracle_steps > 0,
                                                          oracle_at=(120.0,),
                                                          nonadaptive=not args.no_speedup, paper_key="3d_monodomain",
                                                          first=None if args.no_first_sweep else (3, 10))
                done("3D whole run")
        if not args.no_emi:
            out["workload_emi"] = workload_emi(args.emi_steps, speedup=not args.no_speedup, calib=args.calib)
            if not args.no_emi_3d:
                out["workload_emi_3d"] = workload_emi(args.emi_steps, speedup=not args.no_speedup, three_d=True,
                                                      calib=args.calib)
            done("cell-by-cell workloads")
    if not args.no_cpu and not args.headline_only and window is not None:
        out["cpu_baseline"] = cpu_baseline(*window, args.cpu_sample_steps, args.steps)
        done("CPU baseline")
    print(json.dumps(out), flush=True)


def headline(args):
    """The batched workload: `warmup` steps from t = 0, then the window of
    `steps` steps, timed `repeats` times from the same state (median
    reported), a kernel-timing pass over the same window, and the legs that
    belong to this workload (each instance alone, non-adaptive, adjoint)."""
    import torch

    from paper_2311_07206_amd import Solver
    from workloads import config4

    P = config4()
    dev = torch.device("cuda", 0)
    sync = torch.cuda.synchronize
    s = Solver.from_problem(P)
    v = torch.tensor(P.v_init, device=dev)
    w = torch.tensor(P.w_init, device=dev)
    for n in range(args.warmup):
        s.step(v, w, n * P.dt)
    sync()
    v_start, w_start, t_start = v.clone(), w.clone(), args.warmup * P.dt
    if args.calib:
        calibration_copies(dev)   # counter calibration, and the window's start in traces
    times, logs, v_end = [], None, None
    for r in range(max(1, args.repeats)):
        vv, ww = v_start.clone(), w_start.clone()
        el, lg = _timed_steps(s, vv, ww, t_start, P.dt, args.steps, sync)
        times.append(el)
        if logs is None:
            logs, v_end = lg, vv.cpu().numpy()
        else:   # the same window from the same state: the same sets every repeat
            assert [st["n_active"] for x in lg for st in x] == [st["n_active"] for x in logs for st in x]
    elapsed = float(np.median(times))
    dof_sweeps = sum(st["n_active"] for lg in logs for st in lg)
    nbytes = sum(sweep_bytes(st, P.M, k == 0) for lg in logs for k, st in enumerate(lg))
    nbytes += args.steps * step_bytes(P.N, P.M)
    info = s.info()
    out = {
        "metric": "active dof-sweeps/sec + HBM GB/s (% peak); adjoint/forward time ratio",
        "value": dof_sweeps / elapsed,
        "unit": "active dof-sweeps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"batched: {P.n_inst} 2D monodomain instances, sides 96..384 ({P.N} dofs), "
                        f"Aliev-Panfilov, SDC M={P.M} K={P.K} dt={P.dt} ms, theta={P.theta}, Jacobi-PCG rtol "
                        f"{P.cg_rtol}; timed steps {args.warmup}..{args.warmup + args.steps - 1} "
                        f"(t={t_start:.1f}..{t_start + args.steps * P.dt:.1f} ms), median of {len(times)} repeats",
            "instances": P.n_inst, "dofs": P.N, "nnz": s.nnz, "M": P.M, "K": P.K},
        "repeats_ms_per_step": [1e3 * t / args.steps for t in times],
        "storage": info,
        "algorithmic_GBps": nbytes / elapsed / 1e9,
        "mean_active_per_sweep": [float(np.mean([lg[k]["n_active"] for lg in logs])) for k in range(P.K)],
        "mean_cg_iters_per_node": [float(np.mean([lg[k]["cg_iters_max"][m] for lg in logs for k in range(P.K)]))
                                   for m in range(P.M)],
    }
    if not args.no_profile:
        # kernel timing in a second pass over the same window (events around each CG launch)
        s.profile(True)
        _timed_steps(s, v_start.clone(), w_start.clone(), t_start, P.dt, args.steps, sync)
        prof = s.profile_read()
        s.profile(False)
        if prof["cg_launches"]:
            roof = cg_roofline(prof, info["format"], info["n_diagonals"])
            out["roofline"] = add_traffic(roof, measured_traffic(COUNTERS), prof)
    if not args.headline_only:
        if not args.no_graph:
            out["graph"] = graph_window(P, v_start.cpu().numpy(), w_start.cpu().numpy(), t_start, args.steps,
                                        args.repeats, out["ms_per_step"], v_host=v_end)
        if not args.no_speedup:
            el0 = nonadaptive_run(P, v_start.cpu().numpy(), w_start.cpu().numpy(), t_start, args.steps)
            out["adaptive_vs_nonadaptive"] = {"nonadaptive_ms_per_step": 1e3 * el0 / args.steps,
                                              "speedup": el0 / elapsed}
        if not args.no_sequential:
            seq = sequential_instances(P, v_start.cpu().numpy(), w_start.cpu().numpy(), t_start, args.steps)
            out["sequential_ms_per_step"] = 1e3 * seq / args.steps
            out["speedup_vs_sequential"] = seq / elapsed
        if not args.no_adjoint:
            out["adjoint"] = adjoint_ratio(P, s, args.adjoint_steps, args.ckpt_every)
            out["adjoint_forward_ratio"] = out["adjoint"]["ratio"]
    s.close()
    return out, (P, v_start.cpu().numpy(), w_start.cpu().numpy(), t_start)


def calibration_copies(dev, n=3):
    """n device copies of 256 MiB: they calibrate FETCH_SIZE / WRITE_SIZE
    (known bytes) and, being the longest copies of the run, mark where the
    timed window starts in a kernel trace."""
    import torch
    src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    for _ in range(n):
        dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def graph_window(P, v0, w0, t0, nsteps, repeats, ms_host, v_host=None):
    """The same window with graph-captured sweeps (sdc_set_graph): one
    untimed pass (captures, budgets), then `repeats` timed passes from the
    same state, median reported beside the host-launched steps' time; with
    v_host (the host-launched window's final potential), whether every
    repeat ended on the same bits."""
    import torch

    from paper_2311_07206_amd import Solver
    dev = torch.device("cuda", 0)
    sync = torch.cuda.synchronize
    s = Solver.from_problem(P)
    s.set_graph(True)
    _timed_steps(s, torch.tensor(v0, device=dev), torch.tensor(w0, device=dev), t0, P.dt, nsteps, sync)
    i0 = s.info()
    times, dofs, same = [], None, v_host is not None
    for _ in range(max(1, repeats)):
        vg = torch.tensor(v0, device=dev)
        el, logs = _timed_steps(s, vg, torch.tensor(w0, device=dev), t0, P.dt, nsteps, sync)
        times.append(el)
        dofs = sum(st["n_active"] for lg in logs for st in lg)
        if v_host is not None:
            same = same and np.array_equal(vg.cpu().numpy(), v_host)
    i1 = s.info()
    s.close()
    el = float(np.median(times))
    return {"ms_per_step": 1e3 * el / nsteps, "value": dofs / el, "unit": "active dof-sweeps/s",
            "host_launched_ms_per_step": ms_host, "speedup_vs_host_launched": ms_host / (1e3 * el / nsteps),
            "graph_steps": i1["graph_steps"] - i0["graph_steps"], "redone": i1["graph_redone"] - i0["graph_redone"],
            "captures": i1["graph_captures"] - i0["graph_captures"], "repeats": len(times),
            "bitwise_equal_to_host_launched": same if v_host is not None else None}


def sequential_instances(P, v0, w0, t0, nsteps):
    """Wall time of the same window with each instance in a context of its
    own, run one after another."""
    import torch

    from paper_2311_07206_amd import Solver
    dev = torch.device("cuda", 0)
    seq = 0.0
    for i in range(P.n_inst):
        lo, hi = int(P.node_off[i]), int(P.node_off[i + 1])
        e0, e1 = int(P.elem_off[i]), int(P.elem_off[i + 1])
        si = Solver(P.coords[lo:hi], P.elems[e0:e1] - lo, P.elem_tensor[e0:e1], P.node_sigma[lo:hi],
                    P.ionic[i:i + 1], [0, hi - lo], [0, e1 - e0], P.M, P.K, P.dt, P.theta)
        vi = torch.tensor(v0[lo:hi], device=dev)
        wi = torch.tensor(w0[lo:hi], device=dev)
        si.step(vi.clone(), wi.clone(), t0)   # warm the iteration budgets
        e, _ = _timed_steps(si, vi, wi, t0, P.dt, nsteps, torch.cuda.synchronize)
        seq += e
        si.close()
    return seq


def adjoint_ratio(P, s, nsteps=100, ckpt=10):
    """Reverse mode over the batched workload's forward run of nsteps steps
    from t = 0 with checkpoints every ckpt steps: the gradient of
    0.5 ||v(T) - v_target||^2 with respect to the nodal conductivity and each
    instance's Aliev-Panfilov a, v_target from a forward run of the same
    steps with the seeded perturbed conductivity (the workload's target).
    Ratio = backward wall time (checkpoint recomputation and the first
    allocation of the recording slots included) / forward wall time; the
    loss expression's torch kernels run once untimed before the backward."""
    import torch

    from paper_2311_07206_amd import Solver
    from paper_2311_07206_amd.autograd import SDCRun
    from workloads import config4

    dev = torch.device("cuda", 0)
    sync = torch.cuda.synchronize
    T = config4(target=True)
    st = Solver.from_problem(T)
    vt = torch.tensor(T.v_init, device=dev)
    wt = torch.tensor(T.w_init, device=dev)
    for n in range(nsteps):
        st.step(vt, wt, n * T.dt)
    st.close()
    sigma = torch.tensor(P.node_sigma, device=dev, requires_grad=True)
    a = torch.tensor(P.ionic[:, 1].copy(), device=dev, requires_grad=True)
    v0 = torch.tensor(P.v_init, device=dev, requires_grad=True)
    w0 = torch.tensor(P.w_init, device=dev, requires_grad=True)
    sync()
    t = time.perf_counter()
    vT, _ = SDCRun.apply(sigma, a, v0, w0, s, nsteps, 0.0, ckpt)
    sync()
    tf = time.perf_counter() - t
    loss = 0.5 * ((vT - vt) ** 2).sum()
    # the loss's own backward kernels, once untimed: their first launch loads
    # code that is no part of the reverse pass (about 0.2 s on the 48-instance
    # workload); the library's first-call costs stay in the timing
    zv = torch.zeros_like(vT, requires_grad=True)
    (0.5 * ((zv - vt) ** 2).sum()).backward()
    sync()
    t = time.perf_counter()
    loss.backward()
    sync()
    tb = time.perf_counter() - t
    return {"workload": f"{P.n_inst} instances, {nsteps} steps from t = 0, checkpoint every {ckpt} steps; "
                        f"loss 0.5 ||v(T) - v_target||^2, v_target from the seeded perturbed-sigma forward run; "
                        f"gradients w.r.t. nodal sigma and per-instance a",
            "forward_ms": 1e3 * tf, "backward_ms": 1e3 * tb, "ratio": tb / tf, "loss": float(loss),
            "grad_sigma_norm": float(sigma.grad.norm()), "grad_a": a.grad.cpu().numpy().tolist()[:4]}


def workload_2d(args):
    """The 512^2 single-instance workload: `warmup_2d` steps from t = 0, then
    `steps_2d` timed steps; its own roofline, adaptive/non-adaptive speedup,
    the heuristic first-sweep set, the paper's CG stop, the linearized scheme
    and the time-per-sweep curve over front-shell sets."""
    import torch

    from paper_2311_07206_amd import Solver
    from workloads import config1

    P = config1(n=args.n, theta=1e-7)
    dev = torch.device("cuda", 0)
    sync = torch.cuda.synchronize
    s = Solver.from_problem(P)
    v = torch.tensor(P.v_init, device=dev)
    w = torch.tensor(P.w_init, device=dev)
    for n in range(args.warmup_2d):
        s.step(v, w, n * P.dt)
    sync()
    v_start, w_start, t_start = v.cpu().numpy().copy(), w.cpu().numpy().copy(), args.warmup_2d * P.dt
    nsteps = args.steps_2d
    if args.calib:
        calibration_copies(dev)
    # the window `repeats` times from the same state (median reported)
    times, logs, v_std = [], None, None
    for _ in range(max(1, args.repeats)):
        vv, ww = torch.tensor(v_start, device=dev), torch.tensor(w_start, device=dev)
        el, lg = _timed_steps(s, vv, ww, t_start, P.dt, nsteps, sync)
        times.append(el)
        if logs is None:
            logs, v_std = lg, vv.cpu().numpy()
    elapsed = float(np.median(times))
    out = {"workload": f"2D monodomain {args.n}x{args.n} P1 ({P.N} dofs), M={P.M} K={P.K} dt={P.dt} ms, "
                       f"theta={P.theta}; timed steps t={t_start:.1f}..{t_start + nsteps * P.dt:.1f} ms",
           "value": sum(st["n_active"] for lg in logs for st in lg) / elapsed, "unit": "active dof-sweeps/s",
           "ms_per_step": 1e3 * elapsed / nsteps, "repeats_ms_per_step": [1e3 * t / nsteps for t in times],
           "storage": s.info(),
           "mean_active_per_sweep": [float(np.mean([lg[k]["n_active"] for lg in logs])) for k in range(P.K)]}
    if not args.no_profile:
        s.profile(True)
        _timed_steps(s, torch.tensor(v_start, device=dev), torch.tensor(w_start, device=dev), t_start, P.dt,
                     nsteps, sync)
        prof = s.profile_read()
        s.profile(False)
        if prof["cg_launches"]:
            info = out["storage"]
            out["roofline"] = cg_roofline(prof, info["format"], info["n_diagonals"])
    s.close()
    if not args.no_graph:
        out["graph"] = graph_window(P, v_start, w_start, t_start, nsteps, 3, out["ms_per_step"], v_host=v_std)
    v_non = None
    if not args.no_speedup:
        el0, v_non = nonadaptive_run(P, v_start, w_start, t_start, nsteps, return_state=True)
        out["adaptive_vs_nonadaptive"] = {"nonadaptive_ms_per_step": 1e3 * el0 / nsteps, "speedup": el0 / elapsed,
                                          "paper_cpu_speedup_2d_monodomain": PAPER_SPEEDUP["2d_monodomain"]}
    if not args.no_first_sweep:
        out["first_sweep_subset"] = first_sweep_variant(P, v_start, w_start, t_start, nsteps, out["ms_per_step"],
                                                        v_std, v_non)
    if not args.no_cg_energy:
        out["cg_energy_stop"] = cg_energy_variant(P, v_start, w_start, t_start, nsteps, out["ms_per_step"], v_std,
                                                  v_non, speedup=not args.no_speedup)
    if not args.no_linearized:
        out["linearized"] = workload_linearized(P, v_start, w_start, t_start, nsteps, speedup=not args.no_speedup)
    if not args.no_latency:
        out["latency_curve"] = latency_curve(P, small_set_rows=args.small_set_rows)
    if not args.no_full_run:
        out["full_run"] = full_run(config1(n=args.n, theta=1e-7), FULL_RUN_SNAPSHOTS_2D, args.full_window,
                                   args.repeats, args.full_oracle_steps, cpu=args.full_oracle_steps > 0,
                                   nonadaptive=not args.no_speedup, paper_key="2d_monodomain",
                                   first=None if args.no_first_sweep else (4, 10))
    return out


def front_shell_masks(coords, elems, v, densities, level=0.5):
    """Synthetic active sets shaped like a front's shell: one ascending row
    list per density (fraction of the rows, at least one row).  The nodes at
    either end of a mesh edge across which v crosses `level` rank first
    (distance 0), then every other node by its Euclidean distance to the
    nearest of them, ties by index; without a crossing the node whose v is
    closest to `level` is the seed.  The lists are nested."""
    import numpy as np
    from scipy.spatial import cKDTree
    e = np.asarray(elems)
    nv = e.shape[1]
    a = np.concatenate([e[:, i] for i in range(nv) for j in range(i + 1, nv)])
    b = np.concatenate([e[:, j] for i in range(nv) for j in range(i + 1, nv)])
    cross = (v[a] - level) * (v[b] - level) < 0
    seeds = np.unique(np.concatenate([a[cross], b[cross]]))
    if seeds.size == 0:
        seeds = np.array([int(np.argmin(np.abs(v - level)))])
    dist, _ = cKDTree(coords[seeds]).query(coords)
    order = np.lexsort((np.arange(v.size), dist))
    return [np.sort(order[:max(1, int(round(d * v.size)))]).astype(np.int32) for d in densities]


def latency_curve(P, snapshots=(10.0, 50.0, 150.0), densities=(1.0, 0.5, 0.1, 0.01, 0.003, 0.001), reps=5,
                  small_set_rows=0):
    """Time per sweep against the size of its active set.  The run goes from
    the initial state (sets chosen by the drop tolerance) to each snapshot
    time; there, sweeps 1..K-1 of one step are pinned to front-shell masks of
    the given densities, and the step is repeated from the snapshot state,
    once untimed and `reps` times timed.  A sweep's time is its stream time
    by events (its launches, the next set's mapping and the host
    synchronisation); a second set of `reps` steps with kernel timing on
    gives the mean duration of the CG iteration launches on the pinned sets
    (sets solved by one workgroup in one launch, see small_set_rows, have
    none)."""
    import numpy as np
    import torch

    from paper_2311_07206_amd import Solver
    dev = torch.device("cuda", 0)
    s = Solver.from_problem(P, small_set_rows=small_set_rows)
    v = torch.tensor(P.v_init, device=dev)
    w = torch.tensor(P.w_init, device=dev)
    n_done, out = 0, []
    redone0 = s.info()["redone_steps"]
    for ts in snapshots:
        while n_done < int(round(ts / P.dt)):
            s.step(v, w, n_done * P.dt)
            n_done += 1
        t_snap = n_done * P.dt
        sel = s.step(v.clone(), w.clone(), t_snap, stats=True)
        masks = front_shell_masks(P.coords, P.elems, v.cpu().numpy(), densities)
        rows = []
        for d, idx in zip(densities, masks):
            pin = torch.tensor(idx, dtype=torch.int32, device=dev)
            for k in range(1, P.K):
                s.set_active(k, pin)
            ms, first, iters, nbytes = [], [], [], []
            for r in range(reps + 1):
                lg = s.step(v.clone(), w.clone(), t_snap, stats=True)
                if r == 0:
                    continue
                first.append(lg[0]["ms"])
                for st in lg[1:]:
                    ms.append(st["ms"])
                    iters.append(sum(st["cg_iters_max"]))
                    nbytes.append(sweep_bytes(st, P.M, False))
            s.profile(True)
            for r in range(reps):
                s.step(v.clone(), w.clone(), t_snap)
            torch.cuda.synchronize()
            pr = s.profile_read()
            s.profile(False)
            s.set_active(0, None)
            nl = pr["cg_launches"] - pr["cg_all_launches"]
            cg_ms = pr["cg_ms"] - pr["cg_all_ms"]
            row = {"density": d, "n_active": int(idx.size), "ms_per_sweep": float(np.median(ms)),
                   "cg_iterations_per_sweep": float(np.mean(iters)),
                   "sweep_us_per_cg_iteration": 1e3 * float(np.mean(ms)) / max(float(np.mean(iters)), 1.0),
                   "algorithmic_GBps": float(np.mean(nbytes)) / float(np.mean(ms)) / 1e6,
                   "first_sweep_ms": float(np.median(first))}
            if nl > 0 and cg_ms > 0:
                info = s.info()
                lr = cg_roofline(pr, info["format"], info["n_diagonals"])["listed"]
                row["cg_launch_us"] = lr["avg_launch_us"]
                row["cg_launch_GBps"] = lr["storage_min_GBps"]
            rows.append(row)
        out.append({"t_ms": t_snap, "selected_n_active": [st["n_active"] for st in sel], "masks": rows})
    redone = s.info()["redone_steps"] - redone0
    s.close()
    return {"workload": f"2D monodomain {int(round(P.N ** 0.5))}x{int(round(P.N ** 0.5))}, sweeps 1..{P.K - 1} "
                        f"pinned to front-shell masks (level v = 0.5)",
            "small_set_rows": small_set_rows, "snapshots": out, "redone_steps": redone}


def copy_bandwidth(nbytes=1 << 30, reps=10):
    """Device-to-device copy of 1 GiB (read + write counted), best of `reps`,
    timed with events: the bandwidth a plain streaming kernel reaches."""
    import torch
    dev = torch.device("cuda", 0)
    src = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = 1e30
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1) * 1e-3)
    del src, dst
    return 2 * nbytes / best / 1e9


def nonadaptive_run(P, v0, w0, t0, nsteps, warm_budget=True, return_state=False, **kw):
    """Wall time of `nsteps` steps with theta = 0 (all rows in every sweep) from
    the given state, for the adaptive/non-adaptive speedup (and the final
    potential, with return_state)."""
    import torch

    from paper_2311_07206_amd import Solver
    dev = torch.device("cuda", 0)
    s = Solver.from_problem(P, theta=0.0, **kw)
    v, w = torch.tensor(v0, device=dev), torch.tensor(w0, device=dev)
    if warm_budget:
        s.step(v.clone(), w.clone(), t0)   # iteration history for the budgets
    el, _ = _timed_steps(s, v, w, t0, P.dt, nsteps, torch.cuda.synchronize)
    s.close()
    return (el, v.cpu().numpy()) if return_state else el


def first_sweep_variant(P, v0, w0, t0, nsteps, ms_std, v_std, v_non=None, rings=4, every=10):
    """The same timed steps with the heuristic first-sweep set (first_rings
    rings of growth, all rows every first_full_every steps): throughput, the
    share of rows the first sweeps took, and how far the final potential
    lies from the standard adaptive run's (and, with the non-adaptive run's
    v_non, how far each of the two lies from that)."""
    import torch

    from paper_2311_07206_amd import Solver
    dev = torch.device("cuda", 0)
    s = Solver.from_problem(P, first_rings=rings, first_full_every=every)
    v, w = torch.tensor(v0, device=dev), torch.tensor(w0, device=dev)
    s.step(v.clone(), w.clone(), t0)   # iteration history for the budgets
    s.set_active(0, None)              # the timed run carries nothing in
    redone = s.info()["redone_steps"]
    el, logs = _timed_steps(s, v, w, t0, P.dt, nsteps, torch.cuda.synchronize)
    redone = s.info()["redone_steps"] - redone
    s.close()
    vf = v.cpu().numpy()
    out = {"first_rings": rings, "first_full_every": every, "value": sum(st["n_active"] for lg in logs for st in lg) / el,
           "unit": "active dof-sweeps/s", "ms_per_step": 1e3 * el / nsteps, "speedup_vs_standard": ms_std / (1e3 * el / nsteps),
           "first_sweep_rows_frac": float(np.mean([lg[0]["n_active"] for lg in logs])) / P.N,
           "max_abs_v_vs_standard": float(np.abs(vf - v_std).max()), "theta": P.theta, "redone_steps": redone}
    if v_non is not None:
        out["max_abs_v_vs_nonadaptive"] = float(np.abs(vf - v_non).max())
        out["standard_max_abs_v_vs_nonadaptive"] = float(np.abs(v_std - v_non).max())
    return out


def cg_energy_variant(P, v0, w0, t0, nsteps, ms_std, v_std, v_non=None, tol=1e-3, delay=4, speedup=True):
    """The same timed steps with every CG solve stopped at an estimated
    relative energy error of tol (the paper's setting, Sec. 5.1; estimated
    over delay steps) instead of the residual tolerance: throughput, CG steps
    per solve against the residual stop's, how far the final potential lies
    from the residual-stop run's (and from the non-adaptive one's), and the
    adaptive/non-adaptive speedup with the energy stop on both sides."""
    import torch

    from paper_2311_07206_amd import Solver
    dev = torch.device("cuda", 0)
    s = Solver.from_problem(P, cg_energy_tol=tol, cg_delay=delay)
    v, w = torch.tensor(v0, device=dev), torch.tensor(w0, device=dev)
    s.step(v.clone(), w.clone(), t0)   # iteration history for the budgets
    redone = s.info()["redone_steps"]
    el, logs = _timed_steps(s, v, w, t0, P.dt, nsteps, torch.cuda.synchronize)
    redone = s.info()["redone_steps"] - redone
    s.close()
    vf = v.cpu().numpy()
    solves = [it for lg in logs for st in lg if st["n_active"] > 0 for it in st["cg_iters_max"]]
    out = {"cg_energy_tol": tol, "cg_delay": delay, "value": sum(st["n_active"] for lg in logs for st in lg) / el,
           "unit": "active dof-sweeps/s", "ms_per_step": 1e3 * el / nsteps,
           "speedup_vs_residual_stop": ms_std / (1e3 * el / nsteps),
           "mean_cg_steps_per_solve": float(np.mean(solves)) if solves else 0.0,
           "max_abs_v_vs_residual_stop": float(np.abs(vf - v_std).max()), "redone_steps": redone}
    if v_non is not None:
        out["max_abs_v_vs_nonadaptive"] = float(np.abs(vf - v_non).max())
    if speedup:
        el0 = nonadaptive_run(P, v0, w0, t0, nsteps, cg_energy_tol=tol, cg_delay=delay)
        out["adaptive_vs_nonadaptive"] = {"nonadaptive_ms_per_step": 1e3 * el0 / nsteps, "speedup": el0 / el}
    return out


def full_run(P, snap_ms, window=5, repeats=5, oracle_steps=1, cpu=True, oracle_at=None, nonadaptive=False,
             paper_key=None, first=None):
    """The workload's whole run from t = 0 (every step of its schedule, all
    stimuli), timed as one pass with the device synchronised at its ends.
    Windows of `window` steps starting at the snapshot times are then timed
    `repeats` times each (median reported), each repeat from the state the
    whole run had one step earlier and that step run untimed first, so that
    the timed steps continue their predecessor as in the whole run.  With
    `cpu`, the oracle runs the first `oracle_steps` steps of each window (of
    those starting at the times `oracle_at`, default all) from the same state
    on one core, beside the GPU's median time for the same steps: both rates
    over identical steps.  With `nonadaptive`, the whole run is timed again
    with theta = 0: the speedup over the whole run, as the paper reports
    its speedups, and the distance of the two potentials at the window
    times.  With `first` = (rings, every), the whole run once more with the
    heuristic first-sweep set: its time and its distance to the
    non-adaptive run at the same times."""
    import torch

    from paper_2311_07206_amd import Solver
    dev = torch.device("cuda", 0)
    sync = torch.cuda.synchronize
    s = Solver.from_problem(P)
    v = torch.tensor(P.v_init, device=dev)
    w = torch.tensor(P.w_init, device=dev)
    starts = sorted({min(P.n_steps - window, int(round(t / P.dt))) for t in snap_ms})
    saved = {max(0, n0 - 1) for n0 in starts}
    snaps, dofs = {}, 0
    sync()
    t = time.perf_counter()
    for n in range(P.n_steps):
        if n in saved:
            snaps[n] = (v.clone(), w.clone())
        dofs += sum(st["n_active"] for st in s.step(v, w, n * P.dt, stats=True))
    sync()
    el = time.perf_counter() - t
    print(f"[bench] {P.name}: whole run of {P.n_steps} steps in {el:.1f} s", file=sys.stderr, flush=True)
    out = {"steps": P.n_steps, "t_end_ms": P.n_steps * P.dt, "seconds": el, "ms_per_step": 1e3 * el / P.n_steps,
           "value": dofs / el, "unit": "active dof-sweeps/s",
           "stimuli_ms": [float(st[0]) for st in P.stimuli], "redone_steps": s.info()["redone_steps"],
           "windows": []}
    kept = {}
    if nonadaptive:
        # the same run with theta = 0, its states kept at the same steps (the
        # final state is back at rest, so the distance is taken there)
        s0 = Solver.from_problem(P, theta=0.0)
        vn, wn = torch.tensor(P.v_init, device=dev), torch.tensor(P.w_init, device=dev)
        sync()
        t = time.perf_counter()
        for n in range(P.n_steps):
            if n in saved:
                kept[n] = vn.clone()
            s0.step(vn, wn, n * P.dt)
        sync()
        el0 = time.perf_counter() - t
        s0.close()
        dist = {}
        for n in sorted(saved):
            a, b = snaps[n][0].cpu().numpy(), kept[n].cpu().numpy()
            dist[f"{n * P.dt:g}"] = {"max_abs_v": float(np.abs(a - b).max()),
                                     "rel_l2_v": float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))}
        out["adaptive_vs_nonadaptive"] = {"nonadaptive_seconds": el0, "speedup": el0 / el,
                                          "theta": P.theta, "v_distance_at_ms": dist}
        if paper_key:
            out["adaptive_vs_nonadaptive"][f"paper_cpu_speedup_{paper_key}"] = PAPER_SPEEDUP[paper_key]
        print(f"[bench] {P.name}: non-adaptive whole run in {el0:.1f} s", file=sys.stderr, flush=True)
    if first is not None:
        rings, every = first
        s1 = Solver.from_problem(P, first_rings=rings, first_full_every=every)
        vf, wf = torch.tensor(P.v_init, device=dev), torch.tensor(P.w_init, device=dev)
        kept1 = {}
        sync()
        t = time.perf_counter()
        for n in range(P.n_steps):
            if n in saved:
                kept1[n] = vf.clone()
            s1.step(vf, wf, n * P.dt)
        sync()
        el1 = time.perf_counter() - t
        s1.close()
        fd = {"first_rings": rings, "first_full_every": every, "seconds": el1, "ms_per_step": 1e3 * el1 / P.n_steps,
              "speedup_vs_standard": el / el1}
        if kept:
            fd["speedup_vs_nonadaptive"] = out["adaptive_vs_nonadaptive"]["nonadaptive_seconds"] / el1
            fd["max_abs_v_to_nonadaptive_at_ms"] = {
                f"{n * P.dt:g}": float(np.abs(kept1[n].cpu().numpy() - kept[n].cpu().numpy()).max()) for n in sorted(saved)}
        out["first_sweep_subset"] = fd
        print(f"[bench] {P.name}: whole run with the heuristic first-sweep set in {el1:.1f} s", file=sys.stderr,
              flush=True)
    orc = None
    for n0 in starts:
        lead = 1 if n0 > 0 else 0
        times, t_first, logs, state0 = [], [], None, None
        for _ in range(max(1, repeats)):
            vv, ww = (x.clone() for x in snaps[n0 - lead])
            for k in range(lead):   # untimed: the step before the window
                s.step(vv, ww, (n0 - lead + k) * P.dt)
            if state0 is None:
                state0 = (vv.cpu().numpy(), ww.cpu().numpy())
            sync()
            t = time.perf_counter()
            lg = []
            for k in range(window):
                lg.append(s.step(vv, ww, (n0 + k) * P.dt, stats=True))
                if k + 1 == oracle_steps:
                    sync()
                    t_first.append(time.perf_counter() - t)
            sync()
            times.append(time.perf_counter() - t)
            logs = logs or lg
        el_w = float(np.median(times))
        wd = {"t0_ms": n0 * P.dt, "steps": window, "ms_per_step": 1e3 * el_w / window,
              "value": sum(st["n_active"] for x in logs for st in x) / el_w,
              "mean_active_per_sweep": [float(np.mean([x[k]["n_active"] for x in logs])) for k in range(P.K)]}
        if cpu and (oracle_at is None or any(abs(n0 * P.dt - ta) < 0.5 * P.dt for ta in oracle_at)):
            from threadpoolctl import threadpool_limits

            from oracle.sdc import build, run
            orc = orc or build(P)
            with threadpool_limits(limits=1):
                t = time.perf_counter()
                _, _, olog = run(orc, state0[0], state0[1], oracle_steps, P.K, P.stimuli, t0=n0 * P.dt)
                el_o = time.perf_counter() - t
            od = sum(info["n_active"] for step in olog for info in step)
            gd = sum(st["n_active"] for x in logs[:oracle_steps] for st in x)
            el_g = float(np.median(t_first))
            wd["oracle"] = {"steps": oracle_steps, "seconds": el_o, "value": od / el_o, "cores": 1,
                            "gpu_value_same_steps": gd / el_g, "gpu_over_oracle": (gd / el_g) / (od / el_o)}
        out["windows"].append(wd)
    s.close()
    return out


def _timed_steps(solver, v, w, t0, dt, n, sync):
    sync()
    t = time.perf_counter()
    logs = [solver.step(v, w, t0 + k * dt, stats=True) for k in range(n)]
    sync()
    return time.perf_counter() - t, logs


def workload_linearized(P, v0, w0, t0, nsteps, speedup=True):
    """The 512^2 workload with the paper's basic scheme (reaction Jacobian in
    the implicit operator, Gauss-Seidel gating), the same steps from the same
    state as the main measurement."""
    import torch

    from paper_2311_07206_amd import Solver
    dev = torch.device("cuda", 0)
    s = Solver.from_problem(P, scheme="linearized")
    v, w = torch.tensor(v0, device=dev), torch.tensor(w0, device=dev)
    s.step(v.clone(), w.clone(), t0)   # iteration history for the budgets
    el, logs = _timed_steps(s, v, w, t0, P.dt, nsteps, torch.cuda.synchronize)
    s.close()
    dofs = sum(st["n_active"] for lg in logs for st in lg)
    out = {"workload": f"2D monodomain {int(round(P.N ** 0.5))}^2, the paper's linearized basic scheme, "
                       f"M={P.M} K={P.K} dt={P.dt}, theta={P.theta}; {nsteps} steps from t={t0:.1f} ms",
           "value": dofs / el, "unit": "active dof-sweeps/s", "ms_per_step": 1e3 * el / nsteps,
           "mean_active_per_sweep": [float(np.mean([lg[k]["n_active"] for lg in logs])) for k in range(P.K)],
           "mean_cg_iters_per_node": [float(np.mean([lg[k]["cg_iters_max"][m] for lg in logs for k in range(P.K)]))
                                      for m in range(P.M)]}
    if speedup:
        el0 = nonadaptive_run(P, v0, w0, t0, nsteps, scheme="linearized")
        out["adaptive_vs_nonadaptive"] = {"nonadaptive_ms_per_step": 1e3 * el0 / nsteps, "speedup": el0 / el,
                                          "paper_cpu_speedup_2d_monodomain": PAPER_SPEEDUP["2d_monodomain"]}
    return out


def workload_3d(nsteps=10, warm=10, speedup=True, first_sweep=True, cg_energy=True, variants=True, calib=False,
                repeats=5):
    """The 128^3 3D workload (2.1M dofs, 27M stored entries): HBM-resident."""
    import torch

    from paper_2311_07206_amd import Solver
    from workloads import config2

    P = config2()
    dev = torch.device("cuda", 0)
    s = Solver.from_problem(P)
    v = torch.tensor(P.v_init, device=dev)
    w = torch.tensor(P.w_init, device=dev)
    for k in range(warm):
        s.step(v, w, k * P.dt)
    v0, w0 = v.cpu().numpy().copy(), w.cpu().numpy().copy()
    if calib:
        calibration_copies(dev)
    # the window `repeats` times from the same state (median reported)
    times, logs = [], None
    for _ in range(max(1, repeats)):
        vr, wr = torch.tensor(v0, device=dev), torch.tensor(w0, device=dev)
        t_el, lg = _timed_steps(s, vr, wr, warm * P.dt, P.dt, nsteps, torch.cuda.synchronize)
        times.append(t_el)
        if logs is None:
            logs, v, w = lg, vr, wr
    el = float(np.median(times))
    # the kernel timings from a second pass over the same steps
    s.profile(True)
    _timed_steps(s, torch.tensor(v0, device=dev), torch.tensor(w0, device=dev), warm * P.dt, P.dt, nsteps,
                 torch.cuda.synchronize)
    prof = s.profile_read()
    s.profile(False)
    dofs = sum(st["n_active"] for lg in logs for st in lg)
    nbytes = sum(sweep_bytes(st, P.M, k == 0) for lg in logs for k, st in enumerate(lg)) + nsteps * step_bytes(P.N, P.M)
    out = {"workload": f"3D monodomain 128^3 P1 tets ({P.N} dofs), M={P.M} K={P.K} dt={P.dt}, theta={P.theta}",
           "value": dofs / el, "unit": "active dof-sweeps/s", "ms_per_step": 1e3 * el / nsteps,
           "repeats_ms_per_step": [1e3 * t / nsteps for t in times],
           "algorithmic_GBps": nbytes / el / 1e9, "storage": s.info(),
           "mean_active_per_sweep": [float(np.mean([lg[k]["n_active"] for lg in logs])) for k in range(P.K)]}
    if prof["cg_launches"]:
        # the first sweep's launches on all 2.1 M rows (0.3 GB each) reach
        # beyond the Infinity Cache: its all_rows class times HBM
        info = out["storage"]
        out["roofline"] = cg_roofline(prof, info["format"], info["n_diagonals"])
        out["roofline"] = add_traffic(out["roofline"], measured_traffic(COUNTERS_3D), prof)
    s.close()
    v_std, v_non = v.cpu().numpy(), None
    if speedup:
        el0, v_non = nonadaptive_run(P, v0, w0, warm * P.dt, nsteps, return_state=True)
        out["adaptive_vs_nonadaptive"] = {"nonadaptive_ms_per_step": 1e3 * el0 / nsteps, "speedup": el0 / el,
                                          "paper_cpu_speedup_3d_monodomain": PAPER_SPEEDUP["3d_monodomain"]}
    if first_sweep:
        out["first_sweep_subset"] = first_sweep_variant(P, v0, w0, warm * P.dt, nsteps, out["ms_per_step"], v_std,
                                                        v_non, rings=3)
    if cg_energy:
        out["cg_energy_stop"] = cg_energy_variant(P, v0, w0, warm * P.dt, nsteps, out["ms_per_step"], v_std, v_non,
                                                  speedup=speedup)
    if variants:
        out["storage_variants"] = storage_variants(P, v0, w0, warm * P.dt, nsteps)
    return out


def storage_variants(P, v0, w0, t0, nsteps, formats=(("csr", 1), ("sell", 3))):
    """The same steps with the matrix storage forced (CSR, sliced ELL):
    ms per step and the setup's SpMV-shaped timing of each."""
    import torch

    from paper_2311_07206_amd import Solver
    dev = torch.device("cuda", 0)
    out = {}
    for name, fmt in formats:
        s = Solver.from_problem(P, fmt=fmt)
        v, w = torch.tensor(v0, device=dev), torch.tensor(w0, device=dev)
        s.step(v.clone(), w.clone(), t0)   # iteration history for the budgets
        el, _ = _timed_steps(s, v, w, t0, P.dt, nsteps, torch.cuda.synchronize)
        out[name] = {"ms_per_step": 1e3 * el / nsteps}
        s.close()
    return out


def workload_emi(nsteps=3, warm=1, speedup=True, three_d=False, calib=False):
    """The cell-by-cell workload, from the stimulus: CSR storage, Jacobi-PCG.
    2D: 64 x 16 myocytes (390,564 potential dofs, 81,920 membrane sites);
    3D: 8 x 3 x 2 brick myocytes (209,672 dofs, 55,392 sites, tetrahedra)."""
    import torch

    from paper_2311_07206_amd import Solver
    from workloads import config3
    from workloads.emi import config5

    P = config5() if three_d else config3()
    dev = torch.device("cuda", 0)
    s = Solver.from_problem(P, cg_maxit=200000)
    u = torch.tensor(P.v_init, device=dev)
    w = torch.tensor(P.w_init, device=dev)
    for k in range(warm):
        s.step(u, w, k * P.dt)
    u0, w0 = u.cpu().numpy().copy(), w.cpu().numpy().copy()
    if calib:
        calibration_copies(dev)
    el, logs = _timed_steps(s, u, w, warm * P.dt, P.dt, nsteps, torch.cuda.synchronize)
    print(f"[bench] {P.name}: {nsteps} timed steps in {el:.1f} s", file=sys.stderr, flush=True)
    # the kernel timings from a second pass over the same steps (events
    # around every CG launch; the synchronous solves then check their stop
    # once per event pool, so this pass is not the timed one)
    s.profile(True)
    _timed_steps(s, torch.tensor(u0, device=dev), torch.tensor(w0, device=dev), warm * P.dt, P.dt, nsteps,
                 torch.cuda.synchronize)
    prof = s.profile_read()
    s.profile(False)
    dofs = sum(st["n_active"] for lg in logs for st in lg)
    nbytes = sum(sweep_bytes(st, P.M, k == 0) for lg in logs for k, st in enumerate(lg)) + nsteps * step_bytes(P.N, P.M)
    out = {"workload": f"{'3D' if three_d else '2D'} cell-by-cell {P.N} potential dofs, "
                       f"{len(P.mem_intra)} membrane sites, M={P.M} "
                       f"K={P.K} dt={P.dt}, theta={P.theta}; steps {warm}..{warm + nsteps - 1} after the stimulus",
           "value": dofs / el, "unit": "active dof-sweeps/s", "ms_per_step": 1e3 * el / nsteps,
           "algorithmic_GBps": nbytes / el / 1e9, "storage": s.info(),
           "mean_active_per_sweep": [float(np.mean([lg[k]["n_active"] for lg in logs])) for k in range(P.K)],
           "cg_iters_sweep0": [int(np.max([lg[0]["cg_iters_max"][m] for lg in logs])) for m in range(P.M)]}
    if prof["cg_launches"]:
        info = out["storage"]
        out["roofline"] = cg_roofline(prof, info["format"], info["n_diagonals"])
    s.close()
    if speedup:
        # solves above the asynchronous budget limit run synchronously, so
        # the missing iteration history costs little here
        el0 = nonadaptive_run(P, u0, w0, warm * P.dt, nsteps, warm_budget=False, cg_maxit=200000)
        key = "3d_emi" if three_d else "2d_emi"
        out["adaptive_vs_nonadaptive"] = {"nonadaptive_ms_per_step": 1e3 * el0 / nsteps, "speedup": el0 / el,
                                          f"paper_cpu_speedup_{key}": PAPER_SPEEDUP[key]}
    return out


def cpu_baseline(P, v0, w0, t0, nsteps, window_steps):
    """The oracle on one core over the first nsteps steps of the timed window,
    from the same state (native thread pools limited to one thread)."""
    from threadpoolctl import threadpool_limits

    from oracle.sdc import build, run
    orc = build(P)
    with threadpool_limits(limits=1):
        t = time.perf_counter()
        _, _, log = run(orc, v0, w0, nsteps, P.K, P.stimuli, t0=t0)
        el = time.perf_counter() - t
    dof_sweeps = sum(info["n_active"] for step in log for info in step)
    return {"value": dof_sweeps / el, "unit": "active dof-sweeps/s", "cores": 1, "kind": "oracle",
            "sample": f"the first {nsteps} of the {window_steps} timed steps of the same workload, from the "
                      f"same state at t={t0:.1f} ms ({el:.1f} s on one core)",
            "host_cpu": cpu_model(), "host_cpu_count": os.cpu_count()}


def cpu_model():
    """The host CPU's model name as /proc/cpuinfo gives it (None elsewhere)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


if __name__ == "__main__":
    main()
