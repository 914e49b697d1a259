"""Autotuner of the FFT kernels' shapes: elements per thread (radix-plan
variant) per precision, transform length and pass kind (row passes or column
pass), and rows per row-pass workgroup per precision and length.

Three steps, the middle one on the GPU:

  python paper_1109_0286_amd/autotune.py build
      builds one candidate library per (plan variant, row scale) pair
      (every kernel on that variant, every row pass on that row scale) under
      paper_1109_0286_amd/_tune/;
  python paper_1109_0286_amd/autotune.py measure OUT.json
      for each candidate (a child process loading it through FILL_LIBRARY)
      and each length n with two variants, times the kernels inside short
      fill solves (best of three) on an n x n grid (10% band + holes, FP32-operator and FP64
      plans, M^-1 = Px C Px): the average launch duration of the r2c, c2r and
      col kernels from HIP events around every launch;
  python paper_1109_0286_amd/autotune.py apply OUT.json
      picks per (precision, n) the fastest (variant, row scale) for the row
      passes (mean r2c + mean c2r) and the fastest variant for the column pass
      (mean col, averaged over the row scales), writes csrc/fft_tuned.hpp and
      the summary profiles/fft_autotune.md.  Rebuild with build.py afterwards.
"""

from __future__ import annotations

import json
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
TUNE = os.path.join(HERE, "_tune")
VARIANTS = (0, 1)
ROW_SCALES = (1, 2)
CANDIDATES = tuple((v, r) for v in VARIANTS for r in ROW_SCALES)
LENGTHS = (128, 256, 512, 1024, 2048, 4096)  # lengths with two plan variants
KERNELS = ("r2c", "c2r", "col")
REPS = 3
HEADER = os.path.join(HERE, "csrc", "fft_tuned.hpp")
SUMMARY = os.path.join(ROOT, "profiles", "fft_autotune.md")
VARIANT_NAMES = {0: "E=16 (radix 16 passes)", 1: "E=8 (radix <= 8 passes)"}


def cand_name(c) -> str:
    return f"v{c[0]}r{c[1]}"


def lib_path(c) -> str:
    return os.path.join(TUNE, cand_name(c), "libfill.so")


def cmd_build() -> None:
    sys.path.insert(0, HERE)
    import build as B
    for c in CANDIDATES:
        B.build(variant=c[0], rows=c[1], lib=lib_path(c))


def _child(v: str, out: str) -> None:
    """Runs with FILL_LIBRARY = candidate v: in-solve kernel timings."""
    sys.path.insert(0, ROOT)
    import numpy as np
    import torch
    import paper_1109_0286_amd as F
    import workloads as W
    res = {}
    for n in LENGTHS:
        P = W.damped_power_law(n, n, 4.0, n / 8, 1e-7)
        mask = W.band_holes_mask(n, n, W.band_rows(n, 0.10), max(4, n * n // 20000), 2.0, 12.0, 2)
        d = torch.from_numpy(W.observed_map(P, n, n, 0, mask)).cuda()
        for prec, pname in ((F.FILL_PREC_FP32_OP, "f32"), (F.FILL_PREC_FP64, "f64")):
            plan = F.Plan(n, n, mask, P, prec)
            plan.set_precond(F.FILL_PRECOND_CXX)
            plan.realize(d, 1, 1e-6)  # warm-up (and graph capture)
            for k in KERNELS:
                best = float("inf")
                for _ in range(REPS):  # best of REPS solves: small grids are noisy
                    plan.kernel_timing(getattr(F, f"FILL_K_{k.upper()}"), prec)
                    plan.realize(d, 1, 1e-6)
                    ms, cnt = plan.kernel_timing_read()
                    plan.kernel_timing(-1)
                    best = min(best, ms / max(cnt, 1))
                res[f"{pname}/{n}/{k}"] = best
            print(f"candidate {v} n {n} {pname}: " +
                  " ".join(f"{k} {res[f'{pname}/{n}/{k}'] * 1e3:.2f} us" for k in KERNELS), flush=True)
            plan.close()
    json.dump(res, open(out, "w"))


def cmd_measure(out: str) -> int:
    import tempfile
    result = {"candidates": {}}
    for c in CANDIDATES:
        lib = lib_path(c)
        if not os.path.exists(lib):
            print(f"{lib} is missing: run `autotune.py build` first", file=sys.stderr)
            return 1
        with tempfile.NamedTemporaryFile(suffix=".json", delete=False) as tf:
            part = tf.name
        env = dict(os.environ, FILL_LIBRARY=lib)
        r = subprocess.run([sys.executable, os.path.abspath(__file__), "_child", cand_name(c), part], env=env)
        if r.returncode != 0:
            return r.returncode
        result["candidates"][cand_name(c)] = json.load(open(part))
        os.unlink(part)
    try:
        import torch
        result["device"] = torch.cuda.get_device_name(0)
    except Exception:
        result["device"] = None
    json.dump(result, open(out, "w"), indent=1)
    print(f"wrote {out}")
    return 0


def choose(result: dict) -> dict:
    t = result["candidates"]
    pick = {}
    for prec in ("f32", "f64"):
        for n in LENGTHS:
            row = {c: t[cand_name(c)][f"{prec}/{n}/r2c"] + t[cand_name(c)][f"{prec}/{n}/c2r"] for c in CANDIDATES}
            col = {v: sum(t[cand_name((v, r))][f"{prec}/{n}/col"] for r in ROW_SCALES) / len(ROW_SCALES)
                   for v in VARIANTS}
            pick[(prec, n, "row")] = (min(row, key=row.get), row)
            pick[(prec, n, "col")] = (min(col, key=col.get), col)
    return pick


def cmd_apply(path: str) -> None:
    result = json.load(open(path))
    pick = choose(result)
    lines = [
        "// FFT plan variant per (precision, length, pass kind): 0 = E 16, 1 = E 8",
        "// elements per thread (fft_device.hpp); rows per row-pass workgroup relative",
        "// to the 64 KiB default.  Written by autotune.py from in-solve kernel timings",
        "// on " + str(result.get("device")) + "; lengths not listed use variant 0, scale 1.",
        "#pragma once",
        "",
        "namespace fillk {",
        "",
        "constexpr int tuned_fft_variant(bool f32, int n, int pass) {",
    ]
    lines.append("  switch (n) {")
    for n in LENGTHS:
        rv = {pr: pick[(pr, n, "row")][0][0] for pr in ("f32", "f64")}
        cv = {pr: pick[(pr, n, "col")][0] for pr in ("f32", "f64")}
        lines.append(f"    case {n}: return f32 ? (pass == 0 ? {rv['f32']} : {cv['f32']})")
        lines.append(f"                 : (pass == 0 ? {rv['f64']} : {cv['f64']});")
    lines += ["    default: return 0;", "  }", "}", "", "constexpr int tuned_row_scale(bool f32, int n) {",
              "  switch (n) {"]
    for n in LENGTHS:
        rs = {pr: pick[(pr, n, "row")][0][1] for pr in ("f32", "f64")}
        lines.append(f"    case {n}: return f32 ? {rs['f32']} : {rs['f64']};")
    lines += ["    default: return 1;", "  }", "}", "", "}  // namespace fillk", ""]
    open(HEADER, "w").write("\n".join(lines))
    md = ["# FFT plan autotuning (in-solve kernel durations, HIP events)", "",
          "Commands (R = repository root, OUT = an output directory; `build` and `apply` on the host, `measure` "
          "on the GPU):", "", "```",
          "python $R/paper_1109_0286_amd/autotune.py build",
          "python $R/paper_1109_0286_amd/autotune.py measure $OUT/tune.json",
          "python $R/paper_1109_0286_amd/autotune.py apply $OUT/tune.json", "```", "",
          f"Device: {result.get('device')}.  Variants: " +
          "; ".join(f"{v} = {VARIANT_NAMES[v]}" for v in VARIANTS) + "; row scale s = s x 64 KiB of LDS per "
          "row-pass workgroup.", "",
          "Row passes: mean r2c + mean c2r launch (us) per candidate vNrS (variant N, row scale S); column "
          "pass: mean col launch (us) per variant, averaged over the row scales.", "",
          "| precision | n | " + " | ".join(f"row {cand_name(c)}" for c in CANDIDATES) +
          " | row chosen | col v0 | col v1 | col chosen |",
          "|---|---:|" + "---:|" * len(CANDIDATES) + "---|---:|---:|---:|"]
    for prec in ("f32", "f64"):
        for n in LENGTHS:
            rc, rt = pick[(prec, n, "row")]
            cc, ct = pick[(prec, n, "col")]
            md.append(f"| {prec} | {n} | " + " | ".join(f"{rt[c] * 1e3:.2f}" for c in CANDIDATES) +
                      f" | {cand_name(rc)} | {ct[0] * 1e3:.2f} | {ct[1] * 1e3:.2f} | {cc} |")
    open(SUMMARY, "w").write("\n".join(md) + "\n")
    print(f"wrote {HEADER} and {SUMMARY}; rebuild with python paper_1109_0286_amd/build.py")


def main(argv) -> int:
    if len(argv) >= 1 and argv[0] == "build":
        cmd_build()
        return 0
    if len(argv) >= 2 and argv[0] == "measure":
        return cmd_measure(argv[1])
    if len(argv) >= 2 and argv[0] == "apply":
        cmd_apply(argv[1])
        return 0
    if len(argv) >= 3 and argv[0] == "_child":
        _child(argv[1], argv[2])
        return 0
    print(__doc__, file=sys.stderr)
    return 2


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
