"""Write the rocprofv3 summaries under profiles/ from a profiling run's CSVs.

Usage: python paper_1109_0286_amd/profile_summary.py RUN_DIR
RUN_DIR holds trace/trace_kernel_stats.csv (kernel trace of `bench.py`),
fetch/fetch_counter_collection.csv and write/write_counter_collection.csv
(FETCH_SIZE / WRITE_SIZE runs of `bench.py --calib-copy`), trace.log and
bench.json (the bench line without the profiler).
"""

from __future__ import annotations

import csv
import json
import os
import statistics
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

TRACE_CMD = ("cd /tmp && export TMPDIR=/tmp && rocprofv3 --kernel-trace --stats -d $R/gpurun_out/p/trace -o trace "
             "--output-format csv -- python $R/bench.py --steps 5 --warmup 1 --no-cpu-baseline")
PMC_CMD = ("cd /tmp && export TMPDIR=/tmp && timeout -s KILL 120 rocprofv3 --pmc {c} --kernel-include-regex "
           "\"col_kernel<float|copyBuffer\" -d $R/gpurun_out/p/{d} -o {d} --output-format csv -- "
           "python $R/bench.py --steps 1 --warmup 0 --no-cpu-baseline --calib-copy")
CALIB = 256 << 20


def main(run: str) -> None:
    import bench
    rows = list(csv.DictReader(open(os.path.join(run, "trace", "trace_kernel_stats.csv"))))
    clean = json.loads(open(os.path.join(run, "bench.json")).read().strip().splitlines()[-1])
    col_rocprof = next(float(r["AverageNs"]) / 1e3 for r in rows if "col_kernel<float, 2048>" in r["Name"])
    with open(os.path.join(ROOT, "profiles", "fill_2048_kernel_stats.md"), "w") as f:
        f.write("# Kernel statistics: 2048x2048 fill, FP64 and FP32-operator paths (rocprofv3)\n\n")
        f.write("Command (R = repository root):\n\n```\n" + TRACE_CMD + "\n```\n\n")
        f.write(f"- `col_kernel<float,2048>` average under rocprofv3: {col_rocprof:.2f} us; "
                f"bench.py without the profiler (HIP events timestamped by each dispatch, timed region): "
                f"{clean['col_kernel_ms_in_solve']['f32'] * 1e3:.2f} us.\n")
        f.write(f"- bench.py without the profiler: mixed {clean['value']:.2f} solves/s "
                f"({clean['config']['iters_inner']} inner iterations, {clean['config']['iters_outer']} refinements), "
                f"FP64 {clean['fp64_path']['value']:.2f} solves/s ({clean['fp64_path']['iters']} iterations).\n\n")
        f.write("| kernel | calls | avg us | total ms | % |\n|---|---:|---:|---:|---:|\n")
        for r in rows[:24]:
            f.write(f"| `{r['Name'][:80]}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                    f"{float(r['TotalDurationNs']) / 1e6:.2f} | {float(r['Percentage']):.1f} |\n")
        f.write("\nModes: r2c 0 compact, 1 p = z + beta p, 2 x += alpha p / r -= alpha q, 3 full map, 4 white noise; "
                "c2r 0 compact (+dot), 1 z with r.z and r.r, 2 FP64 residual, 3 realization, 4 full map.\n")

    def load(kind):
        rr = list(csv.DictReader(open(os.path.join(run, kind, f"{kind}_counter_collection.csv"))))
        col = [float(r["Counter_Value"]) for r in rr if "col_kernel<float, 2048>" in r["Kernel_Name"]]
        cal = [float(r["Counter_Value"]) for r in rr
               if "copyBuffer" in r["Kernel_Name"] and int(r["Grid_Size"]) == 131072]
        return statistics.median(col), statistics.median(cal), len(col)

    fk, fc, n = load("fetch")
    wk, wc, _ = load("write")
    fs, ws = CALIB / (fc * 1024), CALIB / (wc * 1024)
    traffic = fk * 1024 * fs + wk * 1024 * ws
    alg = 5 * 4 * 2048 * 1024
    out = {"kernel": "col_kernel<float,2048>", "workload": "2048x2048 fill, FP32 column pass",
           "fetch_kib_per_dispatch_median": fk, "write_kib_per_dispatch_median": wk, "dispatches": n,
           "calib_copy_bytes": CALIB, "calib_fetch_kib": fc, "calib_write_kib": wc,
           "fetch_scale": fs, "write_scale": ws, "traffic_bytes": traffic, "algorithmic_bytes": alg,
           "source_hash": bench.kernel_source_hash(),
           "commands": [PMC_CMD.format(c="FETCH_SIZE", d="fetch"), PMC_CMD.format(c="WRITE_SIZE", d="write")]}
    json.dump(out, open(os.path.join(ROOT, "profiles", "col_kernel_f32_2048_traffic.json"), "w"), indent=1)
    with open(os.path.join(ROOT, "profiles", "col_kernel_f32_2048_traffic.md"), "w") as f:
        f.write("# HBM traffic of col_kernel<float,2048> (2048x2048 workload), rocprofv3 counters\n\n")
        f.write("Commands (R = repository root):\n\n```\n" + "\n".join(out["commands"]) + "\n```\n\n")
        f.write(f"- FETCH_SIZE median {fk:.1f} KiB per dispatch over {n} dispatches; WRITE_SIZE median {wk:.1f} KiB.\n")
        f.write(f"- Calibration: a plain 256 MiB device copy (`__amd_rocclr_copyBuffer`, grid 131072) reads "
                f"FETCH_SIZE {fc:.1f} KiB and WRITE_SIZE {wc:.1f} KiB: scale factors {fs:.3f} (fetch) and {ws:.3f} (write).\n")
        f.write(f"- Traffic per launch: {traffic / 1e6:.2f} MB (reads {fk * 1024 * fs / 1e6:.2f}, writes "
                f"{wk * 1024 * ws / 1e6:.2f}) against {alg / 1e6:.2f} MB algorithmic.\n")
        f.write(f"- Kernel source hash when taken: {out['source_hash']}; bench.py reports `traffic` only while it matches.\n")


if __name__ == "__main__":
    main(sys.argv[1])
