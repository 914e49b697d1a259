"""Write the rocprofv3 summaries under profiles/ from a profiling run's CSVs.

Usage: python paper_1109_0286_amd/profile_summary.py RUN_DIR N
N is 2048 (the headline workload) or 4096 (the wide cut).  RUN_DIR holds
trace/trace_kernel_stats.csv (kernel trace of `bench.py`),
fetch/fetch_counter_collection.csv and write/write_counter_collection.csv
(FETCH_SIZE / WRITE_SIZE runs of `bench.py ... --calib-copy`) and bench.json
(the bench line of the same workload without the profiler).  The kernel
whose roofline the bench line reports (its dominant kernel) is the one the
counter runs select (KERNEL below).  Writes profiles/fill_N_kernel_stats.md and
profiles/<kernel>_f32_N_traffic.{json,md}.
"""

from __future__ import annotations

import csv
import json
import os
import statistics
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

BENCH_ARGS = {
    2048: ("--steps 5 --warmup 1 --no-cpu-baseline --batch 0", "--steps 1 --warmup 0 --no-cpu-baseline --batch 0"),
    4096: ("--workload grid4096 --steps 2 --warmup 1", "--workload grid4096 --steps 1 --warmup 0"),
}
TRACE_CMD = ("cd /tmp && export TMPDIR=/tmp && rocprofv3 --kernel-trace --stats -d $OUT/p{n}/trace -o trace "
             "--output-format csv -- python $R/bench.py {a}")
PMC_CMD = ("cd /tmp && export TMPDIR=/tmp && timeout -s KILL 120 rocprofv3 --pmc {c} --kernel-include-regex "
           "\"{k}<float|copyBuffer\" -d $OUT/p{n}/{d} -o {d} --output-format csv -- "
           "python $R/bench.py {a} --calib-copy")
CALIB = 256 << 20
MODES = ("Modes: r2c 0 compact, 1 p = z + beta p, 2 x += alpha p / r -= alpha q, 3 full map, 4 white noise, "
         "5 single-reduction update; c2r 0 compact (+dot), 1 z with r.z and r.r, 2 FP64 residual, 3 realization, "
         "4 full map.  With the block preconditioner the r2c / c2r compact launches also transform the band "
         "runs' rows.")


def dominant(clean: dict) -> str:
    """Kernel name (e.g. band_solve_kernel) of the bench line's roofline."""
    return clean["roofline"]["kernel"].split("<")[0]


def bench_numbers(clean: dict, n: int) -> tuple[float, str]:
    """(live in-solve average of the dominant FP32 kernel in us, one line on the run)."""
    if n == 2048:
        live = clean["dominant_kernel_ms_in_solve"]["f32"] * 1e3
        line = (f"mixed {clean['value']:.2f} solves/s ({clean['config']['iters_inner']} inner iterations, "
                f"{clean['config']['iters_outer']} refinements), FP64 {clean['fp64_path']['value']:.2f} solves/s "
                f"({clean['fp64_path']['iters']} iterations), preconditioner {clean['config']['preconditioner']}")
    else:
        m, d = clean["paths"]["mixed"], clean["paths"]["fp64"]
        live = m["dominant_kernel_ms"] * 1e3
        line = (f"mixed {m['solves_per_s']:.2f} solves/s ({m['iters_inner']} inner iterations, "
                f"{m['iters_outer']} refinements), FP64 {d['solves_per_s']:.2f} solves/s ({d['iters_inner']} "
                f"iterations), preconditioner {clean['config']['preconditioner']}")
    return live, line


def main(run: str, n: int) -> None:
    import bench
    ta, pa = BENCH_ARGS[n]
    rows = list(csv.DictReader(open(os.path.join(run, "trace", "trace_kernel_stats.csv"))))
    clean = json.loads(open(os.path.join(run, "bench.json")).read().strip().splitlines()[-1])
    kern = dominant(clean)
    # the FP32 instance of the kernel at this size (all launches of the run)
    sel = [r for r in rows if kern + "<float" in r["Name"] and (f", {n}" in r["Name"] or kern in
                                                                 ("band_solve_kernel", "block_mv_kernel",
                                                                  "combine_kernel"))]
    calls = sum(int(r["Calls"]) for r in sel)
    col_rocprof = sum(float(r["TotalDurationNs"]) for r in sel) / max(calls, 1) / 1e3
    live, line = bench_numbers(clean, n)
    roof = clean["roofline"]
    with open(os.path.join(ROOT, "profiles", f"fill_{n}_kernel_stats.md"), "w") as f:
        f.write(f"# Kernel statistics: {n}x{n} fill, FP64 and FP32-operator paths (rocprofv3)\n\n")
        f.write("Command (R = repository root, OUT = an output directory):\n\n```\n" + TRACE_CMD.format(n=n, a=ta) +
                "\n```\n\n")
        f.write(f"- `{kern}<float>` average under rocprofv3 (every launch of the run): {col_rocprof:.2f} us; "
                f"bench.py without the profiler (HIP events timestamped by each dispatch, timed region of the "
                f"mixed path): {live:.2f} us.\n")
        f.write(f"- bench.py without the profiler: {line}.\n")
        f.write(f"- Roofline of that kernel: {roof['achieved']:.0f} GB/s algorithmic = {roof['frac']:.3f} of "
                f"{roof['peak']:.0f} GB/s; a plain device copy reaches {roof['copy_attainable_gbs']:.0f} GB/s.\n\n")
        f.write("| kernel | calls | avg us | total ms | % |\n|---|---:|---:|---:|---:|\n")
        for r in rows[:24]:
            f.write(f"| `{r['Name'][:80]}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                    f"{float(r['TotalDurationNs']) / 1e6:.2f} | {float(r['Percentage']):.1f} |\n")
        f.write("\n" + MODES + "\n")

    def load(kind):
        rr = list(csv.DictReader(open(os.path.join(run, kind, f"{kind}_counter_collection.csv"))))
        col = [float(r["Counter_Value"]) for r in rr if kern + "<float" in r["Kernel_Name"]]
        # the calibration copies are the run's last three copy dispatches
        copies = sorted((int(r["Dispatch_Id"]), float(r["Counter_Value"])) for r in rr
                        if "copyBuffer" in r["Kernel_Name"])
        cal = [v for _, v in copies[-3:]]
        return statistics.median(col), statistics.median(cal), len(col)

    fk, fc, cnt = load("fetch")
    wk, wc, _ = load("write")
    fs, ws = CALIB / (fc * 1024), CALIB / (wc * 1024)
    traffic = fk * 1024 * fs + wk * 1024 * ws
    alg = roof["bytes_per_launch"]
    out = {"kernel": f"{kern}<float> ({n}x{n})", "workload": f"{n}x{n} fill, FP32 {kern}",
           "fetch_kib_per_dispatch_median": fk, "write_kib_per_dispatch_median": wk, "dispatches": cnt,
           "calib_copy_bytes": CALIB, "calib_fetch_kib": fc, "calib_write_kib": wc,
           "fetch_scale": fs, "write_scale": ws, "traffic_bytes": traffic, "algorithmic_bytes": alg,
           "source_hash": bench.kernel_source_hash(),
           "commands": [PMC_CMD.format(c="FETCH_SIZE", d="fetch", n=n, a=pa, k=kern),
                        PMC_CMD.format(c="WRITE_SIZE", d="write", n=n, a=pa, k=kern)]}
    json.dump(out, open(os.path.join(ROOT, "profiles", f"{kern}_f32_{n}_traffic.json"), "w"), indent=1)
    with open(os.path.join(ROOT, "profiles", f"{kern}_f32_{n}_traffic.md"), "w") as f:
        f.write(f"# HBM traffic of {kern}<float> ({n}x{n} workload), rocprofv3 counters\n\n")
        f.write("Commands (R = repository root, OUT = an output directory):\n\n```\n" + "\n".join(out["commands"]) +
                "\n```\n\n")
        f.write(f"- FETCH_SIZE median {fk:.1f} KiB per dispatch over {cnt} dispatches; "
                f"WRITE_SIZE median {wk:.1f} KiB.\n")
        f.write(f"- Calibration: a plain 256 MiB device copy (`__amd_rocclr_copyBuffer`, the run's last three "
                f"dispatches) reads "
                f"FETCH_SIZE {fc:.1f} KiB and WRITE_SIZE {wc:.1f} KiB: scale factors {fs:.3f} (fetch) and "
                f"{ws:.3f} (write).\n")
        f.write(f"- Traffic per launch: {traffic / 1e6:.2f} MB (reads {fk * 1024 * fs / 1e6:.2f}, writes "
                f"{wk * 1024 * ws / 1e6:.2f}) against {alg / 1e6:.2f} MB algorithmic.\n")
        f.write(f"- Kernel source hash when taken: {out['source_hash']}; bench.py reports `traffic` only while "
                f"it matches.\n")
    print(f"wrote profiles for n = {n}")


if __name__ == "__main__":
    main(sys.argv[1], int(sys.argv[2]))
