#!/usr/bin/env python3
"""Throughput of the FRW two-field lattice leapfrog on one MI355X.

Workload (default): the chaotic-inflation model of Sainio, arXiv:0911.5692,
Sec. III — V = m^2 phi^2/2 + g^2 phi^2 chi^2/2 in program units (m = 1,
G = g^2 phi0^2/m^2 = 2.5e5, r = 3/2, s = 0) on a 512^3 periodic lattice, FP32
lattice arrays, vacuum-spectrum initial fluctuations from a fixed seed.

A step is one leapfrog step of the whole path: the FP64 scale-factor update,
the fused kick-drift sweep of both fields and the volume averages for the
next a''.  Inputs are resident in HBM before the timed region starts.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "Gsite-updates/s per leapfrog step, 512³ 2-field FP32; % of HBM roofline"


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def measured_traffic(workload: str, stencil: int, shape: dict):
    """HBM bytes per sweep launch from the committed rocprofv3 counter summary,
    or None when it is missing or was taken on a different sweep source or
    launch shape."""
    from paper_0911_5692_amd.profile_sweep import sweep_source_hash
    path = os.path.join(ROOT, "profiles", f"sweep_traffic_{workload}.json")
    try:
        with open(path) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    if d.get("sweep_source_hash") != sweep_source_hash(stencil) or d.get("launch_shape") != shape:
        return None
    return d.get("hbm_bytes_per_launch")


def cpu_model() -> str:
    """The host CPU's model name (/proc/cpuinfo), or "unknown"."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.lower().startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, ic) -> dict:
    import oracle as O
    cores = int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count() or 1)
    m = O.Model(**w.model())
    st = O.start_physical(m, ic["f1"], ic["f2"], ic["u1"], ic["u2"], ic["a0"])
    t0 = time.perf_counter()
    O.evolve(st, 1)
    per = time.perf_counter() - t0
    n = max(1, min(48, int(12.0 / max(per, 1e-3))))  # about 12 s of wall time
    log(f"cpu baseline: 1 step {per:.2f} s, timing {n} more")
    t0 = time.perf_counter()
    O.evolve(st, n)
    el = time.perf_counter() - t0
    out = {"value": w.sites * n / el / 1e9, "unit": "Gsite-updates/s", "cores": cores,
           "kind": "oracle", "cpu_model": cpu_model(),
           "precision": f"FP64 oracle (the GPU path computes in {w.dtype.upper()})",
           "sample": f"{n} leapfrog steps of the {w.N}^3 workload, FP64 C oracle, OpenMP {cores} threads"}
    # one more step on a single thread (the oracle's OpenMP loops, one thread)
    try:
        gomp = ctypes.CDLL("libgomp.so.1")
        gomp.omp_set_num_threads(1)
        t0 = time.perf_counter()
        O.evolve(st, 1)
        el1 = time.perf_counter() - t0
        gomp.omp_set_num_threads(cores)
        out["single_thread"] = {"value": w.sites / el1 / 1e9, "sample": "1 leapfrog step, 1 thread"}
    except OSError:
        out["single_thread"] = None
    # 20 steps of the 256^3 workload (lambda phi^4, its own inputs), all threads
    try:
        from paper_0911_5692_amd import workloads as W
        w2 = W.CFG2
        ic2 = W.make_inputs(w2)
        m2 = O.Model(**w2.model())
        st2 = O.start_physical(m2, ic2["f1"], ic2["f2"], ic2["u1"], ic2["u2"], ic2["a0"])
        t0 = time.perf_counter()
        O.evolve(st2, 20)
        el2 = time.perf_counter() - t0
        out["at_256"] = {"value": w2.sites * 20 / el2 / 1e9, "sample": f"20 leapfrog steps of the {w2.N}^3 "
                         f"workload ({w2.name}), OpenMP {cores} threads"}
    except MemoryError:
        out["at_256"] = None
    return out


def time_extras(w, dtype) -> tuple[dict, dict]:
    """Wall times at the workload's size of the on-device vacuum
    initialisation (noise, FFTs, filter, Friedmann initialisation) and of one
    power spectrum (f1): first call (FFT plan setup included) and a second."""
    import torch

    from paper_0911_5692_amd import Lattice
    from paper_0911_5692_amd import workloads as W

    spec = W.vacuum_spec(w, seed=w.cfg)
    lat = Lattice(**w.model(), dtype=dtype, device="cuda:0")

    def timed(fn):
        out = {}
        for key in ("first_ms", "warm_ms"):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            out[key] = round((time.perf_counter() - t0) * 1e3, 2)
        return out

    init = timed(lambda: lat.init_vacuum(spec, 1.0))
    spectrum = timed(lambda: lat.spectrum("f1"))
    lat.close()
    return init, spectrum


def copy_reference(N: int, reps: int = 20) -> dict:
    """Rate of lf_stream_copy over the sweep's bytes at N^3 (four FP32 arrays
    read, four written, no arithmetic): what the device streams for this
    read/write mix, timed with HIP events on the current stream."""
    import torch

    from paper_0911_5692_amd import stream_copy

    src = [torch.zeros(N ** 3, dtype=torch.float32, device="cuda:0") for _ in range(4)]
    dst = [torch.empty_like(src[0]) for _ in range(4)]
    for _ in range(3):
        stream_copy(src, dst)
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        stream_copy(src, dst)
    e.record()
    e.synchronize()
    ms = s.elapsed_time(e) / reps
    del src, dst
    return {"kernel": "lf_stream_copy (one float per lane, blocks in address order, non-temporal stores)",
            "bytes": 32 * N ** 3,
            "ms": round(ms, 5), "GBps": round(32 * N ** 3 / (ms * 1e-3) / 1e9, 1)}


def time_slab_share(lat, w, gpus: int = 8, reps: int = 20) -> dict:
    """One GPU's share of the lattice split into `gpus` z-slabs: the sweep
    (lf_slab_sweep) on planes [0, N/gpus) with its halo planes in separate
    buffers, automatic z-chunk, timed with HIP events on the lattice's stream.
    The coefficients are the lattice's last step's; halo exchange and the
    cross-slab sum are not part of it."""
    import torch

    N = w.N
    nz = N // gpus
    state, _ = lat.get_state()
    slab = [s[:nz].clone() for s in state]
    lo = [s[[N - 2, N - 1]].clone() for s in state[:2]] + [s[[N - 1]].clone() for s in state[2:]]
    hi = [s[[nz]].clone() for s in state[:2]]
    del state
    out, _ = lat.slab_sweep(slab, lo, hi)
    for _ in range(3):
        lat.slab_sweep(slab, lo, hi, out=out)
    st = lat.stream
    s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s0.record(st)
    for _ in range(reps):
        lat.slab_sweep(slab, lo, hi, out=out)
    s1.record(st)
    s1.synchronize()
    ms = s0.elapsed_time(s1) / reps
    sites = N * N * nz
    esize = 4 if w.dtype == "f32" else 8
    alg = 8 * esize * sites
    halo = 8 * esize * N * N  # d: 2 planes below, 1 above; e: 1 below (both fields)
    return {"gpus": gpus, "planes": nz, "N": N, "rows": lat.slab_rows(nz), "ms": round(ms, 5),
            "gsite_updates_per_s": round(sites / (ms * 1e-3) / 1e9, 2),
            "algorithmic_GBps": round(alg / (ms * 1e-3) / 1e9, 1), "halo_bytes": halo,
            "frac_of_peak": round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}


def time_additions() -> dict:
    """Measured numbers of the rows and additions beyond the step itself:
    the 256^3 lambda phi^4 workload (its 1000 steps; its eight arrays, 512 MB,
    are only twice the 256 MB MALL, so its rate is not a pure HBM figure),
    rho/p per site at 512^3 (algorithmic 16 B read + 8 B written per site,
    FP32 outputs), the ensemble of uneven lattices (500 steps), and the
    adjoint of the 128^3 workload (500 steps, checkpoints every 50)."""
    import torch

    from paper_0911_5692_amd import Ensemble, Lattice
    from paper_0911_5692_amd import workloads as W

    out = {}
    w2 = W.CFG2
    ic = W.make_inputs(w2)
    lat = Lattice(**w2.model(), dtype=torch.float32, device="cuda:0")
    lat.init_physical(*(torch.from_numpy(ic[k]).to("cuda:0") for k in ("f1", "f2", "u1", "u2")), ic["a0"])
    lat.step(20)
    torch.cuda.synchronize()
    lat.step(w2.steps)
    ms = lat.last_step_ms() / w2.steps
    out["lphi4_256"] = {"N": w2.N, "steps": w2.steps, "ms_per_step": round(ms, 5),
                        "Gsite_updates_per_s": round(w2.sites / ms / 1e6, 2),
                        "hbm_frac_algorithmic": round(32 * w2.sites / ms / 1e6 / HBM_PEAK_GBS, 4)}
    lat.close()
    del ic

    w = W.CFG3
    lat = Lattice(**w.model(), dtype=torch.float32, device="cuda:0", **W.BENCH_SHAPES[w.name])
    lat.init_vacuum(W.vacuum_spec(w, seed=w.cfg), 1.0)
    lat.step(20)
    lat.rho_p(dtype=torch.float32)
    torch.cuda.synchronize()
    reps = 5
    t0 = time.perf_counter()
    for _ in range(reps):
        lat.rho_p(dtype=torch.float32)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    alg = 24 * w.sites
    out["rho_p"] = {"N": w.N, "ms": round(ms, 3), "algorithmic_bytes": alg, "GBps": round(alg / ms / 1e6, 1),
                    "hbm_frac": round(alg / ms / 1e6 / HBM_PEAK_GBS, 4)}
    lat.close()

    members = W.ensemble_members()
    # launch shape from the ensemble autotuner's cache (a tuning run, outside
    # the timed steps, when the cache has no line for this device)
    ens = Ensemble([m.model() for m in members], dtype=torch.float32, device="cuda:0", tuned=True)
    for r, m in enumerate(members):
        ic = W.make_inputs(m, realization=r)
        ens.init_physical(r, *(torch.from_numpy(ic[k]).to("cuda:0") for k in ("f1", "f2", "u1", "u2")),
                          ic["a0"])
    ens.step(10)
    torch.cuda.synchronize()
    ens.step(W.ENSEMBLE_STEPS)
    ms = ens.last_step_ms() / W.ENSEMBLE_STEPS
    sites = sum(m.sites for m in members)
    tuning = {k: ens.tuning[k] for k in ("tile_x", "tile_y", "ztarget", "ms")}
    tuning["zchunks_by_N"] = {m.N: z for m, z in zip(members, ens.tuning["zchunks"])}
    out["ensemble"] = {"realizations": len(members), "sites": sites, "ms_per_step": round(ms, 4),
                       "Gsite_updates_per_s": round(sites / ms / 1e6, 2),
                       "hbm_frac_algorithmic": round(32 * sites / ms / 1e6 / HBM_PEAK_GBS, 4),
                       "launch_shape": tuning}
    ens.close()

    w5 = W.CFG5
    ic = W.make_inputs(w5)
    lat = Lattice(**w5.model(), dtype=torch.float32, device="cuda:0")
    dev_ic = [torch.from_numpy(ic[k]).to("cuda:0") for k in ("f1", "f2", "u1", "u2")]
    passes = []
    for _ in range(2):  # the second pass is reported; the first includes one-time set-up
        lat.init_physical(*dev_ic, ic["a0"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lat.adjoint_forward(w5.steps, 50)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        lat.adjoint_backward(1.0)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        passes.append((round((t1 - t0) * 1e3, 1), round((t2 - t1) * 1e3, 1)))
    out["adjoint"] = {"N": w5.N, "steps": w5.steps, "K": 50, "forward_ms": passes[1][0],
                      "backward_ms": passes[1][1], "first_forward_ms": passes[0][0],
                      "first_backward_ms": passes[0][1]}
    lat.close()
    return out


PAPER_MS_PER_STEP = 22.0  # Sec. III: 256^3, 2 fields, GTX 260, FP32, 27-point, energy kernel every 512 steps


def time_paper_config(blocks: int = 4) -> dict:
    """The configuration the paper times (Sec. III): 256^3, two fields,
    V = m^2 phi^2/2 + g^2 phi^2 chi^2/2, dt = 2^-10/m, FP32, 27-point
    Laplacian, with the energy-density and pressure kernel once every 512
    steps.  Vacuum initial state generated on the device.  Wall time per step
    over `blocks` x 512 steps (the rho/p call at each block end included)."""
    import torch

    from paper_0911_5692_amd import Lattice
    from paper_0911_5692_amd import workloads as W

    w = W.PAPER_256_S27
    lat = Lattice(**w.model(), dtype=torch.float32, device="cuda:0", **W.BENCH_SHAPES[w.name])
    lat.init_vacuum(W.vacuum_spec(w, seed=w.cfg), 1.0)
    lat.step(512)
    lat.rho_p(arrays=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(blocks):
        lat.step(512)
        lat.rho_p(arrays=False)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / (512 * blocks)
    lat.close()
    return {"workload": w.name, "stencil": 27, "N": w.N, "steps": 512 * blocks, "ms_per_step": round(ms, 5),
            "paper_ms_per_step": PAPER_MS_PER_STEP, "paper_hardware": "GTX 260 (context only)",
            "speedup": round(PAPER_MS_PER_STEP / ms, 1)}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="m2phi2_512c_f32")
    ap.add_argument("--kernel-steps", type=int, default=50,
                    help="eager steps timed per kernel with HIP events (roofline)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-init-timing", action="store_true",
                    help="skip timing the on-device vacuum initialisation and spectrum")
    ap.add_argument("--no-paper-config", action="store_true",
                    help="skip timing the paper's own 256^3 27-point configuration")
    ap.add_argument("--no-additions", action="store_true",
                    help="skip timing rho/p, the ensemble and the adjoint")
    ap.add_argument("--no-slab", action="store_true",
                    help="skip timing the sweep on one GPU's z-slab share")
    ap.add_argument("--autotune", action="store_true",
                    help="re-run the launch-shape autotuner instead of the committed shape")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: runs on one GPU only.  Of the multi-GPU z-slab path only the sweep on one GPU's "
              "slab share is built (timed as slab_share); halo exchange and the cross-slab sums are not. "
              "Run with --gpus 1.", file=sys.stderr)
        return 2

    import torch

    from paper_0911_5692_amd import Lattice
    from paper_0911_5692_amd import workloads as W

    w = W.WORKLOADS[args.workload]
    dtype = torch.float32 if w.dtype == "f32" else torch.float64
    esize = 4 if w.dtype == "f32" else 8
    log(f"workload {w.name}: N={w.N} dtype={w.dtype}; generating seeded inputs")
    t0 = time.perf_counter()
    ic = W.make_inputs(w)
    host_inputs_s = time.perf_counter() - t0
    log(f"inputs ready in {host_inputs_s:.1f} s")

    shape = dict(W.BENCH_SHAPES.get(w.name, {}))
    if args.autotune:
        from paper_0911_5692_amd import autotune
        t = autotune(**w.model(), dtype=dtype, cache_path=None)
        shape = {k: t[k] for k in ("tile_x", "tile_y", "zchunk")}
        log(f"autotuned shape {shape} ({t['ms']:.4f} ms/step)")
    lat = Lattice(**w.model(), dtype=dtype, device="cuda:0", **shape)
    dev = [torch.from_numpy(ic[k]).to("cuda:0") for k in ("f1", "f2", "u1", "u2")]
    ad0 = lat.init_physical(*dev, ic["a0"])
    del dev
    torch.cuda.synchronize()
    # Eager steps before the warmup: after the device has idled (input
    # generation, upload), its first milliseconds of work run about 10%
    # slower while the clocks come up; these bring them up, so that a short
    # timed run sees the rate of a long one.  The per-kernel timing for the
    # roofline is taken again after the timed region.
    log(f"initialised, a'(0) = {ad0:.6f}; bringing the clocks up with {args.kernel_steps} eager steps")
    lat.time_kernels(args.kernel_steps)
    log(f"warmup {args.warmup} steps")
    lat.step(args.warmup)
    torch.cuda.synchronize()

    log(f"timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat.step(args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = lat.last_step_ms()
    ms_per_step = ev_ms / args.steps
    value = w.sites / (ms_per_step * 1e-3) / 1e9
    log(f"{ms_per_step:.4f} ms/step (events), wall {wall * 1e3 / args.steps:.4f} ms/step, "
        f"{value:.2f} Gsite-updates/s")
    en = lat.energies()
    log(f"energies after {en['step']} steps: a={en['a']:.6f} R={en['R']:.3e}")

    kms = lat.time_kernels(args.kernel_steps)
    sweep_ms = kms[1]
    alg_bytes = 8 * esize * w.sites  # read f, v; write v, f_new; two fields
    achieved = alg_bytes / (sweep_ms * 1e-3) / 1e9
    traffic = measured_traffic(w.name, w.stencil, shape)
    log(f"kernel ms: a-update {kms[0]:.4f}, sweep {sweep_ms:.4f}, reduce {kms[2]:.4f}; "
        f"sweep {achieved:.0f} GB/s")
    slab = None
    if not args.no_slab:
        slab = time_slab_share(lat, w)
        slab["frac_of_full_lattice_rate"] = round(slab["gsite_updates_per_s"] / (w.sites / (sweep_ms * 1e-3) / 1e9),
                                                  4)
        log(f"one GPU's z-slab share: {slab}")
    lat.close()
    torch.cuda.synchronize()
    copy = None
    if w.dtype == "f32":
        copy = copy_reference(w.N)
        copy["sweep_frac_of_copy"] = round(achieved / copy["GBps"], 4)
        log(f"stream copy of the same bytes: {copy}")

    init = spectrum = None
    if not args.no_init_timing:
        init, spectrum = time_extras(w, dtype)
        init["host_generator_s"] = round(host_inputs_s, 2)
        log(f"device vacuum initialisation: {init}; spectrum: {spectrum}")

    paper = None
    if not args.no_paper_config:
        paper = time_paper_config()
        log(f"paper's configuration: {paper}")

    additions = None
    if not args.no_additions:
        additions = time_additions()
        log(f"additions: {additions}")

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the oracle on the host (bounded sample)")
        cpu = cpu_baseline(w, ic)
        log(f"cpu baseline {cpu['value']:.4f} Gsite-updates/s on {cpu['cores']} threads")

    line = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "Gsite-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 6),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": w.dtype,
        "data": "synthetic",
        "config": {"workload": f"{w.name}: m^2 phi^2 + g^2 phi^2 chi^2 (G=2.5e5), {w.N}^3 periodic, "
                               f"L={w.L}, dt={w.dt}, {w.stencil}-point Laplacian, vacuum fluctuations, "
                               f"seed [3,0,i,k]",
                   "N": w.N, "sites": w.sites, "lattice_dtype": w.dtype, "stencil": w.stencil,
                   "launch_shape": shape,
                   "step_hbm_frac_algorithmic": round(value * 1e9 * 8 * esize / 1e9 / HBM_PEAK_GBS, 4)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "kernel": "k_sweep_lds27 (fused kick-drift, 27-point)" if w.stencil == 27
                     else "k_sweep_lds (fused kick-drift, 7-point)",
                     "kernel_ms": round(sweep_ms, 5), "bytes_per_launch": alg_bytes,
                     "copy_reference": copy},
        "cpu_baseline": cpu,
        "slab_share": slab,
        "init": init,
        "spectrum": spectrum,
        "paper_config": paper,
        "additions": additions,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
