"""Write the rocprofv3 summaries under profiles/ from a profiling run's CSVs.

Usage: python paper_1109_0286_amd/profile_summary.py RUN_DIR N
N is 2048 (the headline workload) or 4096 (the wide cut).  RUN_DIR holds
trace/trace_kernel_stats.csv (kernel trace of `bench.py`),
fetch/fetch_counter_collection.csv and write/write_counter_collection.csv
(FETCH_SIZE / WRITE_SIZE runs of `bench.py ... --calib-copy` over the FP32
kernels of a CG iteration, KERNELS below) and bench.json (the bench line of
the same workload without the profiler).  Writes profiles/fill_N_kernel_stats.md
and profiles/<kernel>_f32_N_traffic.{json,md} for each of those kernels.
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
    2048: ("--steps 5 --warmup 1 --no-cpu-baseline --batch 0 --no-extra --no-compare",
           "--steps 1 --warmup 0 --no-cpu-baseline --batch 0 --no-extra --no-compare"),
    4096: ("--workload grid4096 --steps 2 --warmup 1", "--workload grid4096 --steps 1 --warmup 0"),
}
TRACE_CMD = ("cd /tmp && export TMPDIR=/tmp && rocprofv3 --kernel-trace --stats -d $OUT/p{n}/trace -o trace "
             "--output-format csv -- python $R/bench.py {a}")
PMC_CMD = ("cd /tmp && export TMPDIR=/tmp && timeout -s KILL 120 rocprofv3 --pmc {c} --kernel-include-regex "
           "\"{k}\" -d $OUT/p{n}/{d} -o {d} --output-format csv -- "
           "python $R/bench.py {a} --calib-copy")
CALIB = 256 << 20
MODES = ("Modes: r2c 0 compact, 1 p = z + beta p, 2 x += alpha p / r -= alpha q, 3 full map, 4 white noise, "
         "5 single-reduction update; c2r 0 compact (+dot), 1 z with r.z and r.r, 2 FP64 residual, 3 realization, "
         "4 full map.  With the block preconditioner the r2c / c2r compact launches also transform the band "
         "runs' rows.")
# FP32 kernels of the mixed solve's CG iteration whose HBM bytes the counter
# runs measure: bench.py's name -> the kernel-name prefix of its dispatches
# (r2c: the p = z + beta p pass; c2r: the A p pass, the largest grid of mode 0)
KERNELS = {"bandblock": "band_block_kernel<float>", "col": "col_kernel<float, {n}",
           "r2c": "r2c_kernel<float, {n}, 1>", "c2r": "c2r_kernel<float, {n}, 0>",
           "combine": "combine_kernel<float>"}


def pmc_regex(n: int) -> str:
    return "|".join(v.format(n=n) for v in KERNELS.values()) + "|copyBuffer"


def dominant(clean: dict) -> str:
    """Kernel name (e.g. band_block_kernel) of the bench line's roofline."""
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
                                                                  "combine_kernel", "band_block_kernel"))]
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
        kr = clean.get("kernel_roofline") or {}
        if kr:
            f.write("FP32 kernels of the mixed solve's CG iteration, bench.py without the profiler (in-solve "
                    "average per launch, algorithmic bytes of bench.kernel_bytes):\n\n"
                    "| kernel | us | algorithmic MB | GB/s | frac of 8 TB/s |\n|---|---:|---:|---:|---:|\n")
            for k, v in kr.items():
                f.write(f"| {k} | {v['us_per_launch']:.2f} | {v['bytes_per_launch'] / 1e6:.2f} | "
                        f"{v['achieved_gbs']:.0f} | {v['frac']:.3f} |\n")
            f.write("\n")
        f.write("| kernel | calls | avg us | total ms | % |\n|---|---:|---:|---:|---:|\n")
        for r in rows[:24]:
            f.write(f"| `{r['Name'][:80]}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                    f"{float(r['TotalDurationNs']) / 1e6:.2f} | {float(r['Percentage']):.1f} |\n")
        f.write("\n" + MODES + "\n")

    def load(kind):
        rows_k = list(csv.DictReader(open(os.path.join(run, kind, f"{kind}_counter_collection.csv"))))
        # the calibration copies are the run's last three copy dispatches
        copies = sorted((int(r["Dispatch_Id"]), float(r["Counter_Value"])) for r in rows_k
                        if "copyBuffer" in r["Kernel_Name"])
        return rows_k, statistics.median([v for _, v in copies[-3:]])

    frows, fc = load("fetch")
    wrows, wc = load("write")
    fs, ws = CALIB / (fc * 1024), CALIB / (wc * 1024)
    info = clean.get("block_preconditioner")
    n_m = clean["config"]["n_masked"]
    regex = pmc_regex(n)
    lines = []
    for name, prefix in KERNELS.items():
        prefix = prefix.format(n=n)

        def per_dispatch(rr):
            sel = [r for r in rr if r["Kernel_Name"].replace("void fillk::", "").replace(
                "(anonymous namespace)::", "").startswith(prefix)]
            if not sel:
                return None, 0
            top = max(int(r["Grid_Size"]) for r in sel)  # the full-size launches
            vals = [float(r["Counter_Value"]) for r in sel if int(r["Grid_Size"]) == top]
            return statistics.median(vals), len(vals)

        fk, cnt = per_dispatch(frows)
        wk, _ = per_dispatch(wrows)
        if fk is None or wk is None:
            continue
        traffic = fk * 1024 * fs + wk * 1024 * ws
        alg = bench.kernel_bytes(name, 4, n, n, n_m, info)
        out = {"kernel": f"{prefix} ({n}x{n})", "workload": f"{n}x{n} fill, FP32 {bench.KERNEL_NAMES[name]}",
               "fetch_kib_per_dispatch_median": fk, "write_kib_per_dispatch_median": wk, "dispatches": cnt,
               "calib_copy_bytes": CALIB, "calib_fetch_kib": fc, "calib_write_kib": wc,
               "fetch_scale": fs, "write_scale": ws, "traffic_bytes": traffic, "algorithmic_bytes": alg,
               "source_hash": bench.kernel_source_hash(),
               "commands": [PMC_CMD.format(c="FETCH_SIZE", d="fetch", n=n, a=pa, k=regex),
                            PMC_CMD.format(c="WRITE_SIZE", d="write", n=n, a=pa, k=regex)]}
        stem = f"{bench.KERNEL_NAMES[name]}_f32_{n}_traffic"
        json.dump(out, open(os.path.join(ROOT, "profiles", stem + ".json"), "w"), indent=1)
        with open(os.path.join(ROOT, "profiles", stem + ".md"), "w") as f:
            f.write(f"# HBM traffic of {prefix}...> ({n}x{n} workload), rocprofv3 counters\n\n")
            f.write("Commands (R = repository root, OUT = an output directory):\n\n```\n" +
                    "\n".join(out["commands"]) + "\n```\n\n")
            f.write(f"- FETCH_SIZE median {fk:.1f} KiB per dispatch over {cnt} full-size dispatches; "
                    f"WRITE_SIZE median {wk:.1f} KiB.\n")
            f.write(f"- Calibration: a plain 256 MiB device copy (`__amd_rocclr_copyBuffer`, the run's last three "
                    f"dispatches) reads FETCH_SIZE {fc:.1f} KiB and WRITE_SIZE {wc:.1f} KiB: scale factors "
                    f"{fs:.3f} (fetch) and {ws:.3f} (write).\n")
            f.write(f"- Traffic per launch: {traffic / 1e6:.2f} MB (reads {fk * 1024 * fs / 1e6:.2f}, writes "
                    f"{wk * 1024 * ws / 1e6:.2f}) against {alg / 1e6:.2f} MB algorithmic "
                    f"({traffic / alg:.2f}x).\n")
            f.write(f"- Kernel source hash when taken: {out['source_hash']}; bench.py reports `traffic` only while "
                    f"it matches.\n")
        lines.append(f"| `{prefix}...>` | {alg / 1e6:.2f} | {traffic / 1e6:.2f} | {traffic / alg:.2f} |")
    with open(os.path.join(ROOT, "profiles", f"fill_{n}_kernel_stats.md"), "a") as f:
        f.write("\nHBM traffic per launch (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy's counters; the "
                f"`*_f32_{n}_traffic.md` files):\n\n| kernel | algorithmic MB | counter MB | ratio |\n"
                "|---|---:|---:|---:|\n" + "\n".join(lines) + "\n")
    print(f"wrote profiles for n = {n}")


if __name__ == "__main__":
    main(sys.argv[1], int(sys.argv[2]))
