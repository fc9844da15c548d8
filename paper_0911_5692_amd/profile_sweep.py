"""HBM traffic of the fused sweep from rocprofv3 counters.

Two steps, each its own process:

  run        a plain device copy of known size (the counter calibration) and
             a read-only sum over the same bytes (its cross-check), then a
             few leapfrog steps of a workload at its benchmark launch shape
             (or of the 68-lattice ensemble at its autotuned shape, or the
             adjoint of the 128^3 workload); meant to run under
               rocprofv3 --pmc FETCH_SIZE ...   and again with   --pmc WRITE_SIZE
  summarize  reads the two counter CSVs (and optionally a --kernel-trace
             --stats CSV), scales each counter by what it reads for the copy,
             and writes profiles/sweep_traffic_<workload>.json and .md.
  kernels    writes the per-kernel table of any --kernel-trace --stats run
             (every kernel a benchmark run launched) as markdown.

FETCH_SIZE and WRITE_SIZE are in KiB per dispatch.  The calibration factor of
a counter is (bytes the copy moves) / (what the counter reads for the copy).
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import re
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
COPY_MIB = 1024


def _code_only(text: str) -> str:
    """C/C++ source without comments and with whitespace runs collapsed, so
    that editing a comment does not change the hash."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def sweep_source_hash(stencil: int = 7) -> str:
    """Hash of the code (comments aside) of the sweep kernel of this stencil."""
    h = hashlib.sha256()
    main = ("lf_sweep27.hip", "lf_sweep27_tile.h") if stencil == 27 else ("lf_sweep.hip", "lf_sweep_tile.h")
    for f in (*main, "lf_sweep_common.h", "lf_internal.h", "lf_stencil.h"):
        with open(os.path.join(PKG, "csrc", f)) as fh:
            h.update(_code_only(fh.read()).encode())
    return h.hexdigest()[:16]


ENSEMBLE = "ensemble"  # the 68-lattice workload of uneven sizes (48 x 64^3 + 16 x 96^3 + 4 x 160^3)
ADJOINT = "adjoint"    # the 128^3 adjoint workload: 500 steps, checkpoints every 50, forward + backward


def _calibration_kernels() -> None:
    """A device copy of COPY_MIB MiB (reads and writes that much) and a
    read-only sum over the same bytes (reads them once, writes 4 bytes)."""
    import torch

    n = COPY_MIB * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    s = a.sum()
    torch.cuda.synchronize()
    del a, b, s


def run_ensemble(steps: int) -> None:
    import torch

    sys.path.insert(0, ROOT)
    from paper_0911_5692_amd import Ensemble
    from paper_0911_5692_amd import workloads as W

    _calibration_kernels()
    members = W.ensemble_members()
    ens = Ensemble([m.model() for m in members], dtype=torch.float32, tuned=True)
    for r, m in enumerate(members):
        ic = W.make_inputs(m, realization=r)
        ens.init_physical(r, *(torch.from_numpy(ic[k]).to("cuda") for k in ("f1", "f2", "u1", "u2")), ic["a0"])
    ens.step(steps)
    torch.cuda.synchronize()
    print(f"profile run done: ensemble {steps} steps, shape {ens.tuning}", flush=True)


def run_adjoint() -> None:
    import torch

    sys.path.insert(0, ROOT)
    from paper_0911_5692_amd import Lattice
    from paper_0911_5692_amd import workloads as W

    _calibration_kernels()
    w = W.CFG5
    ic = W.make_inputs(w)
    lat = Lattice(**w.model(), dtype=torch.float32)
    lat.init_physical(*(torch.from_numpy(ic[k]).to("cuda") for k in ("f1", "f2", "u1", "u2")), ic["a0"])
    lat.adjoint_forward(w.steps, 50)
    lat.adjoint_backward(1.0)
    torch.cuda.synchronize()
    print(f"profile run done: adjoint of {w.name}, {w.steps} steps, K = 50", flush=True)


def run(workload: str, steps: int) -> None:
    import torch

    if workload == ENSEMBLE:
        run_ensemble(steps)
        return
    if workload == ADJOINT:
        run_adjoint()
        return
    sys.path.insert(0, ROOT)
    from paper_0911_5692_amd import Lattice
    from paper_0911_5692_amd import workloads as W

    w = W.WORKLOADS[workload]
    shape = W.BENCH_SHAPES.get(w.name, {})
    _calibration_kernels()
    N = w.N
    g = torch.Generator(device="cuda")
    g.manual_seed(0)
    f = [1 + 1e-4 * torch.randn((N, N, N), dtype=torch.float64, device="cuda", generator=g),
         1e-5 * torch.randn((N, N, N), dtype=torch.float64, device="cuda", generator=g),
         -0.7 + 1e-4 * torch.randn((N, N, N), dtype=torch.float64, device="cuda", generator=g),
         1e-3 * torch.randn((N, N, N), dtype=torch.float64, device="cuda", generator=g)]
    lat = Lattice(**w.model(), dtype=torch.float32 if w.dtype == "f32" else torch.float64, **shape)
    lat.init_physical(*f, 1.0)
    del f
    lat.step(steps)
    torch.cuda.synchronize()
    print(f"profile run done: {workload} {steps} steps, shape {shape}", flush=True)


def _rows(path: str):
    with open(path) as fh:
        return list(csv.DictReader(fh))


def _find(d: str, suffix: str) -> str:
    for root, _, files in os.walk(d):
        for f in files:
            if f.endswith(suffix):
                return os.path.join(root, f)
    raise FileNotFoundError(f"{suffix} under {d}")


def _counter(path: str, name: str, kernel_pred):
    vals = [float(r["Counter_Value"]) for r in _rows(path)
            if r["Counter_Name"] == name and kernel_pred(r["Kernel_Name"])]
    return vals


def summarize(workload: str, fetch_dir: str, write_dir: str, trace_dir: str | None, out_dir: str,
              commands: list[str]) -> dict:
    sys.path.insert(0, ROOT)
    from paper_0911_5692_amd import workloads as W

    if workload == ENSEMBLE:
        sites = sum(m.sites for m in W.ensemble_members())
        alg, stencil, shape = 32 * sites, 7, "autotuned (profile run log)"
        alg_read = alg / 2
        is_sweep = lambda k: "k_sweep_ens" in k
    elif workload == ADJOINT:
        # the reverse step's field pass: per site it reads the four FP64
        # cotangents (32 B) and the stored FP32 fields of this step and of
        # the step before (16 B, the latter for the next step's sums), and
        # writes four FP64 cotangents (32 B); the first reverse step of each
        # 50-step segment (2% of launches) has no next step's fields (72 B)
        alg, stencil, shape = 80 * W.CFG5.sites, 7, "64 x 4 tiles, 16-plane chunks at 128^3"
        alg_read = 48 * W.CFG5.sites
        is_sweep = lambda k: "k_adj_fields" in k
    else:
        w = W.WORKLOADS[workload]
        esize = 4 if w.dtype == "f32" else 8
        alg, stencil, shape = 8 * esize * w.sites, w.stencil, W.BENCH_SHAPES.get(w.name, {})
        alg_read = alg / 2
        is_sweep = lambda k: "k_sweep" in k
    copy_bytes = COPY_MIB * (1 << 20)
    is_copy = lambda k: "copy" in k.lower() and "lf::" not in k
    is_sum = lambda k: "reduce_kernel" in k
    fpath, wpath = _find(fetch_dir, "counter_collection.csv"), _find(write_dir, "counter_collection.csv")
    f_copy = _counter(fpath, "FETCH_SIZE", is_copy)
    w_copy = _counter(wpath, "WRITE_SIZE", is_copy)
    f_sum = _counter(fpath, "FETCH_SIZE", is_sum)
    f_sweep = _counter(fpath, "FETCH_SIZE", is_sweep)
    w_sweep = _counter(wpath, "WRITE_SIZE", is_sweep)
    # the calibration copy is the largest copy dispatch, the read-only sum the
    # largest reduction
    fc, wc = max(f_copy) * 1024.0, max(w_copy) * 1024.0
    kf, kw = copy_bytes / fc, copy_bytes / wc
    kf_sum = copy_bytes / (max(f_sum) * 1024.0) if f_sum else None
    fetch = sum(f_sweep) / len(f_sweep) * 1024.0 * kf
    write = sum(w_sweep) / len(w_sweep) * 1024.0 * kw
    res = dict(workload=workload, sweep_source_hash=sweep_source_hash(stencil),
               launch_shape=shape, algorithmic_bytes_per_launch=alg,
               fetch_calibration_read_only=kf_sum,
               fetch_bytes_per_launch=fetch, write_bytes_per_launch=write,
               hbm_bytes_per_launch=fetch + write, fetch_calibration=kf, write_calibration=kw,
               fetch_over_algorithmic_reads=fetch / alg_read, write_over_algorithmic_writes=write / (alg - alg_read),
               launches=len(f_sweep))
    if trace_dir:
        stats = _rows(_find(trace_dir, "kernel_stats.csv"))
        res["kernel_stats"] = [dict(name=r["Name"][:90], calls=int(r["Calls"]), avg_ns=float(r["AverageNs"]),
                                    pct=float(r["Percentage"])) for r in stats[:8]]
        # sweep launches per (kernel, grid): the statistics above merge every
        # lattice size the traced run launched one kernel on
        groups: dict = {}
        for r in _rows(_find(trace_dir, "kernel_trace.csv")):
            if is_sweep(r["Kernel_Name"]):
                key = (r["Kernel_Name"].split("(")[0], int(r["Grid_Size_X"]) // int(r["Workgroup_Size_X"]))
                groups.setdefault(key, []).append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
        res["sweep_launches"] = sorted(
            (dict(name=k[0], blocks=k[1], calls=len(v), avg_ns=sum(v) / len(v)) for k, v in groups.items()),
            key=lambda g: -g["calls"] * g["avg_ns"])
    os.makedirs(out_dir, exist_ok=True)
    with open(os.path.join(out_dir, f"sweep_traffic_{workload}.json"), "w") as fh:
        json.dump(res, fh, indent=1)
    with open(os.path.join(out_dir, f"sweep_traffic_{workload}.md"), "w") as fh:
        fh.write(f"# HBM traffic of the fused sweep, workload {workload}\n\n")
        fh.write("Commands (from the repository root on the GPU host):\n\n")
        for c in commands:
            fh.write(f"    {c}\n")
        fh.write(f"\nCalibration: a device copy of {COPY_MIB} MiB reads FETCH_SIZE = {fc / 1024:.1f} KiB "
                 f"and WRITE_SIZE = {wc / 1024:.1f} KiB, so the counters are scaled by "
                 f"{kf:.4f} (fetch) and {kw:.4f} (write).")
        if kf_sum:
            fh.write(f"  Cross-check: a read-only sum over the same {COPY_MIB} MiB reads FETCH_SIZE = "
                     f"{max(f_sum):.1f} KiB, a fetch factor of {kf_sum:.4f}.")
        fh.write("\n\n")
        fh.write("| quantity | per sweep launch |\n|---|---|\n")
        fh.write(f"| algorithmic bytes ({'80' if workload == ADJOINT else '32'} B/site) | {alg / 1e9:.4f} GB |\n")
        fh.write(f"| HBM fetch (scaled) | {fetch / 1e9:.4f} GB = {res['fetch_over_algorithmic_reads']:.3f} x algorithmic reads |\n")
        fh.write(f"| HBM write (scaled) | {write / 1e9:.4f} GB = {res['write_over_algorithmic_writes']:.3f} x algorithmic writes |\n")
        fh.write(f"| total HBM traffic | {(fetch + write) / 1e9:.4f} GB |\n")
        fh.write(f"| sweep launches averaged | {len(f_sweep)} |\n")
        fh.write(f"| sweep source hash | {res['sweep_source_hash']} |\n")
        fh.write(f"| launch shape | {res['launch_shape']} |\n")
        if trace_dir:
            fh.write("\nKernel trace (rocprofv3 --kernel-trace --stats):\n\n| kernel | calls | avg ns | % |\n|---|---|---|---|\n")
            for k in res["kernel_stats"]:
                fh.write(f"| {k['name']} | {k['calls']} | {k['avg_ns']:.0f} | {k['pct']:.1f} |\n")
            fh.write("\nSweep launches of the same trace by grid (kernel trace, end - start):\n\n"
                     "| kernel | blocks | calls | avg ns |\n|---|---|---|---|\n")
            for g in res["sweep_launches"]:
                fh.write(f"| {g['name']} | {g['blocks']} | {g['calls']} | {g['avg_ns']:.0f} |\n")
    return res


def kernel_table(trace_dir: str, out_path: str, commands: list[str], title: str) -> None:
    """Markdown table of every kernel of a rocprofv3 --kernel-trace --stats run
    (calls, average and total duration), with the commands that made it."""
    stats = _rows(_find(trace_dir, "kernel_stats.csv"))
    with open(out_path, "w") as fh:
        fh.write(f"# {title}\n\nCommands (from the repository root on the GPU host):\n\n")
        for c in commands:
            fh.write(f"    {c}\n")
        fh.write("\n| kernel | calls | avg us | total ms | % |\n|---|---|---|---|---|\n")
        for r in stats:
            name = r["Name"].replace("(anonymous namespace)::", "").split("(")[0][:100]
            fh.write(f"| {name} | {int(r['Calls'])} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['TotalDurationNs']) / 1e6:.2f} | {float(r['Percentage']):.2f} |\n")


def main() -> int:
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    r = sub.add_parser("run")
    r.add_argument("--workload", default="m2phi2_512c_f32", help="a workload name, 'ensemble' or 'adjoint'")
    r.add_argument("--steps", type=int, default=4)
    s = sub.add_parser("summarize")
    s.add_argument("--workload", default="m2phi2_512c_f32")
    s.add_argument("--fetch-dir", required=True)
    s.add_argument("--write-dir", required=True)
    s.add_argument("--trace-dir")
    s.add_argument("--out-dir", default=os.path.join(ROOT, "profiles"))
    s.add_argument("--command", action="append", default=[])
    k = sub.add_parser("kernels")
    k.add_argument("--trace-dir", required=True)
    k.add_argument("--out", required=True)
    k.add_argument("--title", default="Kernel trace")
    k.add_argument("--command", action="append", default=[])
    a = ap.parse_args()
    if a.cmd == "run":
        run(a.workload, a.steps)
    elif a.cmd == "kernels":
        kernel_table(a.trace_dir, a.out, a.command, a.title)
    else:
        res = summarize(a.workload, a.fetch_dir, a.write_dir, a.trace_dir, a.out_dir, a.command)
        print(json.dumps(res))
    return 0


if __name__ == "__main__":
    sys.exit(main())
