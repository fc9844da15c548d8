"""Python handle of one lattice context of liblf (C ABI in include/lf.h).

PyTorch provides the device memory (workspace and field tensors) and the
stream; every step of the evolution runs in liblf's HIP kernels.
"""
from __future__ import annotations

import ctypes
import os
import shutil

import torch

from ._lib import LF_F32, LF_F64, Params, Report, Scalars, Vacuum, check, lib

_DT = {torch.float32: LF_F32, torch.float64: LF_F64}


def _dev_ptr(t: torch.Tensor, dtype: torch.dtype, shape) -> ctypes.c_void_p:
    if not t.is_cuda:
        raise ValueError("tensor must be on the GPU")
    if t.dtype != dtype:
        raise ValueError(f"tensor dtype {t.dtype}, expected {dtype}")
    if tuple(t.shape) != tuple(shape) or not t.is_contiguous():
        raise ValueError(f"tensor must be contiguous with shape {tuple(shape)}")
    if t.data_ptr() % 256:
        raise ValueError("tensor storage must be 256-byte aligned")
    return ctypes.c_void_p(t.data_ptr())


DEFAULT_TUNE_CACHE = os.environ.get(
    "LF_AUTOTUNE_CACHE", os.path.join(os.path.dirname(os.path.abspath(__file__)), "autotune_cache.jsonl"))
# Choices the autotuners made on an MI355X (gfx950) for the benchmark's
# workloads; a new default cache starts as a copy of them.
SEED_TUNE_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_seed_gfx950.jsonl")


def _cache(path: str | None) -> str | None:
    """The cache file to use: the default one is created from the seed."""
    if path and path == DEFAULT_TUNE_CACHE and not os.path.exists(path) and os.path.exists(SEED_TUNE_CACHE):
        shutil.copyfile(SEED_TUNE_CACHE, path)
    return path


def autotune(N: int, L: float, dt: float, beta: int, c1: float, G: float, r: float, s: float,
             kappa2: float, dtype: torch.dtype = torch.float32, device="cuda",
             cache_path: str | None = DEFAULT_TUNE_CACHE, stencil: int = 7) -> dict:
    """Fastest sweep launch shape for this lattice size, dtype, beta and
    stencil on the current device (liblf's lf_autotune; cached per
    architecture in a JSONL file).  Returns dict(tile_x, tile_y, zchunk, ms)
    (ms = -1 on a cache hit)."""
    p = Params(int(N), _DT[dtype], float(L), float(dt), int(beta), 0, float(c1), float(G), float(r),
               float(s), float(kappa2), 0, 0, 0, int(stencil))
    size = ctypes.c_size_t()
    check(lib().lf_autotune_workspace_bytes(ctypes.byref(p), ctypes.byref(size)))
    ws = torch.empty(size.value, dtype=torch.uint8, device=device)
    stream = torch.cuda.current_stream(torch.device(device))
    best, ms = Params(), ctypes.c_double()
    cache_path = _cache(cache_path)
    check(lib().lf_autotune(ctypes.byref(p), ctypes.c_void_p(stream.cuda_stream), ctypes.c_void_p(ws.data_ptr()),
                            size.value, cache_path.encode() if cache_path else None, ctypes.byref(best),
                            ctypes.byref(ms)))
    return dict(tile_x=best.tile_x, tile_y=best.tile_y, zchunk=best.zchunk, ms=ms.value)


def _vacuum(spec: dict) -> Vacuum:
    """lf_vacuum from dict(f0=(f1, f2), u0=(u1, u2), m2=(m1^2, m2^2), eps2, seed,
    cutoff=0)."""
    v = Vacuum()
    for i in range(2):
        v.f0[i], v.u0[i], v.m2[i] = float(spec["f0"][i]), float(spec["u0"][i]), float(spec["m2"][i])
    v.eps2 = float(spec["eps2"])
    v.cutoff = float(spec.get("cutoff", 0.0))
    v.seed = int(spec["seed"])
    return v


def vacuum_fields(N: int, L: float, spec: dict, device="cuda", stream: torch.cuda.Stream | None = None):
    """Vacuum initial state generated on the device (liblf's lf_vacuum_fields):
    (f1, f2, u1, u2) as FP64 tensors of shape (N, N, N).  spec: see _vacuum."""
    device = torch.device(device)
    p = Params(int(N), LF_F64, float(L), 1.0, 2, 0, 1.0, 0.0, 1.5, 0.0, 0.0, 0, 0, 0, 0)
    size = ctypes.c_size_t()
    check(lib().lf_vacuum_workspace_bytes(ctypes.byref(p), ctypes.byref(size)))
    ws = torch.empty(size.value, dtype=torch.uint8, device=device)
    out = [torch.empty((N, N, N), dtype=torch.float64, device=device) for _ in range(4)]
    st = stream if stream is not None else torch.cuda.current_stream(device)
    v = _vacuum(spec)
    check(lib().lf_vacuum_fields(ctypes.byref(p), ctypes.byref(v), ctypes.c_void_p(st.cuda_stream),
                                 ctypes.c_void_p(ws.data_ptr()), size.value,
                                 *(ctypes.c_void_p(t.data_ptr()) for t in out)))
    return tuple(out)


def stream_copy(src, dst, stream: torch.cuda.Stream | None = None) -> None:
    """dst[j] = src[j] for four contiguous float32 tensors of one size
    (lf_stream_copy, the bandwidth reference of the benchmark); asynchronous
    on `stream` (default: the current stream)."""
    if len(src) != 4 or len(dst) != 4:
        raise ValueError("four source and four destination tensors")
    n = src[0].numel()
    for t in (*src, *dst):
        if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous() or t.numel() != n:
            raise ValueError("contiguous float32 device tensors of one size")
    st = stream or torch.cuda.current_stream(src[0].device)
    check(lib().lf_stream_copy(*(ctypes.c_void_p(t.data_ptr()) for t in (*src, *dst)), int(n),
                               ctypes.c_void_p(st.cuda_stream)))


def _aligned(t: torch.Tensor) -> torch.Tensor:
    return t if (t.is_contiguous() and t.data_ptr() % 256 == 0) else t.contiguous().clone()


class Lattice:
    """One N^3 two-field lattice (Sainio, arXiv:0911.5692, Sec. II).

    Parameters are program units: box side L, time step dt, potential
    V_pr = c1 a^p1 f1^beta/beta + G a^p2 f1^2 f2^2 / 2, rescaling exponents
    r, s (s - 2r + 3 = 0) and kappa2 = 8 pi G_N / A^2.  dtype is the element
    type of the lattice arrays (float32 or float64).  stencil selects the
    Laplacian: 7 (6 neighbours) or 27 (the paper's own, Sec. II.C).
    """

    def __init__(self, N: int, L: float, dt: float, beta: int, c1: float, G: float, r: float,
                 s: float, kappa2: float, dtype: torch.dtype = torch.float32,
                 device: str | torch.device = "cuda", tile_y: int = 0, zchunk: int = 0,
                 tile_x: int = 0, stream: torch.cuda.Stream | None = None, stencil: int = 7,
                 tuned: bool | str = False):
        """tuned: take the launch shape from the autotuner (its cache, or a
        tuning run on a miss) when no tile_y / zchunk / tile_x is given; a
        string is the cache path (default: LF_AUTOTUNE_CACHE or the package's
        autotune_cache.jsonl)."""
        if dtype not in _DT:
            raise ValueError("dtype must be torch.float32 or torch.float64")
        if tuned and not (tile_y or zchunk or tile_x):
            t = autotune(N, L, dt, beta, c1, G, r, s, kappa2, dtype=dtype, device=device,
                         cache_path=tuned if isinstance(tuned, str) else DEFAULT_TUNE_CACHE, stencil=stencil)
            tile_x, tile_y, zchunk = t["tile_x"], t["tile_y"], t["zchunk"]
        self.launch_shape = dict(tile_x=int(tile_x), tile_y=int(tile_y), zchunk=int(zchunk))
        self.N, self.dtype = int(N), dtype
        self.device = torch.device(device)
        self.params = Params(int(N), _DT[dtype], float(L), float(dt), int(beta), 0, float(c1),
                             float(G), float(r), float(s), float(kappa2), int(tile_y), int(zchunk),
                             int(tile_x), int(stencil))
        size = ctypes.c_size_t()
        check(lib().lf_workspace_bytes(ctypes.byref(self.params), ctypes.byref(size)))
        self.ws_bytes = size.value
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        ctx = ctypes.c_void_p()
        check(lib().lf_create(ctypes.byref(self.params), ctypes.c_void_p(self.stream.cuda_stream),
                              ctypes.c_void_p(self.ws.data_ptr()), self.ws_bytes, ctypes.byref(ctx)))
        self._ctx = ctx
        self._keep = ()

    # ------------------------------------------------------------ lifecycle
    def close(self) -> None:
        if getattr(self, "_ctx", None):
            lib().lf_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def shape(self):
        return (self.N, self.N, self.N)

    # ------------------------------------------------------------ init
    def init_vacuum(self, spec: dict, a0: float = 1.0) -> float:
        """Generate a vacuum state on the device (lf_init_vacuum; spec as for
        vacuum_fields) and initialise from it with the Friedmann a'_0, which
        is returned."""
        size = ctypes.c_size_t()
        check(lib().lf_init_vacuum_workspace_bytes(ctypes.byref(self.params), ctypes.byref(size)))
        ws = torch.empty(size.value, dtype=torch.uint8, device=self.device)
        ad0 = ctypes.c_double()
        v = _vacuum(spec)
        check(lib().lf_init_vacuum(self._ctx, ctypes.byref(v), float(a0), ctypes.c_void_p(ws.data_ptr()),
                                   size.value, ctypes.byref(ad0)))
        return ad0.value

    def spectrum(self, which: str = "f1", nbins: int | None = None):
        """Shell-averaged power spectrum of a synchronised field (lf_spectrum):
        which in f1, f2, v1, v2.  Returns (power, count) as float64 numpy
        arrays of nbins (default: every shell)."""
        import numpy as np

        idx = ("f1", "f2", "v1", "v2").index(which)
        nmax = lib().lf_spectrum_bins(self.N)
        nb = nmax if nbins is None else int(nbins)
        size = ctypes.c_size_t()
        check(lib().lf_spectrum_workspace_bytes(ctypes.byref(self.params), ctypes.byref(size)))
        ws = torch.empty(size.value, dtype=torch.uint8, device=self.device)
        power = np.zeros(nb)
        count = np.zeros(nb)
        dp = ctypes.POINTER(ctypes.c_double)
        check(lib().lf_spectrum(self._ctx, idx, nb, power.ctypes.data_as(dp), count.ctypes.data_as(dp),
                                ctypes.c_void_p(ws.data_ptr()), size.value))
        return power, count

    def init(self, f1, f2, v1, v2, a0: float, ad0: float) -> None:
        """Synchronised program-unit state at tau = 0 (float32 or float64 tensors)."""
        ts = [_aligned(t) for t in (f1, f2, v1, v2)]
        dt = ts[0].dtype
        ptrs = [_dev_ptr(t, dt, self.shape) for t in ts]
        check(lib().lf_init(self._ctx, *ptrs, _DT[dt], float(a0), float(ad0)))
        self._keep = ts  # inputs must outlive the enqueued kernels
        self.stream.synchronize()
        self._keep = ()

    def init_physical(self, f1, f2, u1, u2, a0: float = 1.0) -> float:
        """Fields and rescaled physical velocities; returns a'(0) from Friedmann."""
        ts = [_aligned(t) for t in (f1, f2, u1, u2)]
        dt = ts[0].dtype
        ptrs = [_dev_ptr(t, dt, self.shape) for t in ts]
        ad0 = ctypes.c_double()
        check(lib().lf_init_physical(self._ctx, *ptrs, _DT[dt], float(a0), ctypes.byref(ad0)))
        return ad0.value

    # ------------------------------------------------------------ evolution
    def step(self, n: int = 1) -> None:
        check(lib().lf_step(self._ctx, int(n)))

    def last_step_ms(self) -> float:
        ms = ctypes.c_double()
        check(lib().lf_last_step_ms(self._ctx, ctypes.byref(ms)))
        return ms.value

    def time_kernels(self, n: int):
        """Average ms per kernel over n eager steps: (a-update, sweep, reduce)."""
        ms = (ctypes.c_double * 3)()
        check(lib().lf_time_kernels(self._ctx, int(n), ms, 3))
        return tuple(ms)

    def set_coupling(self, G: float) -> None:
        check(lib().lf_set_coupling(self._ctx, float(G)))

    # ------------------------------------------------------------ outputs
    def energies(self, check_finite: bool = True) -> dict:
        rep = Report()
        rc = lib().lf_energies(self._ctx, ctypes.byref(rep))
        if check_finite or rc not in (0, 3):
            check(rc)
        return dict(step=rep.step, a=rep.a, ad=rep.ad, hubble=rep.hubble, K1=rep.K[0],
                    K2=rep.K[1], G1=rep.Gr[0], G2=rep.Gr[1], P=rep.P, rho=rep.rho, R=rep.R,
                    status=rep.status)

    def rho_p(self, arrays: bool = True, dtype: torch.dtype = torch.float64):
        """Energy density and pressure at the synchronised time: (rho, p) tensors
        (or None) and dict(rho, p, w) of volume averages, w = <p>/<rho>."""
        out = [torch.empty(self.shape, dtype=dtype, device=self.device) for _ in range(2)] if arrays else [None, None]
        ptrs = [(_dev_ptr(t, dtype, self.shape) if t is not None else None) for t in out]
        avg = (ctypes.c_double * 3)()
        check(lib().lf_rho_p(self._ctx, ptrs[0], ptrs[1], _DT[dtype], avg))
        return out[0], out[1], dict(rho=avg[0], p=avg[1], w=avg[2])

    def history(self, steps: int, every: int, w: bool = True) -> dict:
        """Evolve `steps` steps and record, at the start and after every
        `every` steps, the synchronised step, a, a'/a, rho, the Friedmann
        residual R and (w=True) the equation of state w = <p>/<rho>: the
        series the paper plots in Sec. III.  Returns numpy arrays."""
        import numpy as np

        if every < 1:
            raise ValueError("every must be >= 1")
        rec = {k: [] for k in ("step", "a", "hubble", "rho", "R", "w")}

        def take():
            e = self.energies()
            for k in ("step", "a", "hubble", "rho", "R"):
                rec[k].append(e[k])
            rec["w"].append(self.rho_p(arrays=False)[2]["w"] if w else float("nan"))

        take()
        done = 0
        while done < steps:
            n = min(every, steps - done)
            self.step(n)
            done += n
            take()
        return {k: np.asarray(v) for k, v in rec.items()}

    def fields(self, synchronized: bool = False, dtype: torch.dtype = torch.float64):
        """(f1, f2, v1, v2) as new tensors: f(k+1/2) and v(k), or f(k), v(k)."""
        out = [torch.empty(self.shape, dtype=dtype, device=self.device) for _ in range(4)]
        ptrs = [_dev_ptr(t, dtype, self.shape) for t in out]
        check(lib().lf_get_fields(self._ctx, *ptrs, _DT[dtype], 1 if synchronized else 0))
        self.stream.synchronize()
        return tuple(out)

    # ------------------------------------------------------------ checkpoint
    def get_state(self):
        """Bitwise checkpoint: (deviation tensors d1, d2, e1, e2, Scalars)."""
        out = [torch.empty(self.shape, dtype=self.dtype, device=self.device) for _ in range(4)]
        ptrs = [_dev_ptr(t, self.dtype, self.shape) for t in out]
        sc = Scalars()
        check(lib().lf_get_state(self._ctx, *ptrs, ctypes.byref(sc)))
        return tuple(out), sc

    def set_state(self, arrays, scalars: Scalars) -> None:
        ptrs = [_dev_ptr(t, self.dtype, self.shape) for t in arrays]
        check(lib().lf_set_state(self._ctx, *ptrs, ctypes.byref(scalars)))


    # ------------------------------------------------------------ z-slab share
    def slab_rows(self, nz: int, zchunk: int = 0) -> int:
        """Partial-sum rows lf_slab_sweep writes for a slab of nz planes."""
        rows = ctypes.c_int64()
        check(lib().lf_slab_rows(self._ctx, int(nz), int(zchunk), ctypes.byref(rows)))
        return rows.value

    def slab_sweep(self, slab, lo, hi, out=None, zchunk: int = 0):
        """One step's sweep on a z-slab of this lattice with halo planes
        (lf_slab_sweep): slab = (d1, d2, e1, e2), each (nz, N, N) in the
        stored deviation form; lo = (d1, d2 of planes -2, -1; e1, e2 of plane
        -1); hi = (d1, d2 of plane nz).  Uses the coefficients of the last
        step.  Returns (out arrays, partial rows (rows, 4) float64);
        asynchronous on the lattice's stream."""
        N, dt, dev = self.N, self.dtype, self.ws.device
        nz = int(slab[0].shape[0])
        want = [(nz, N, N)] * 4
        lo_shapes = [(2, N, N), (2, N, N), (1, N, N), (1, N, N)]
        for t, shp in zip((*slab, *lo, *hi), want + lo_shapes + [(1, N, N)] * 2):
            if tuple(t.shape) != shp or t.dtype != dt or not t.is_contiguous() or t.device != dev:
                raise ValueError(f"slab arrays: contiguous {dt} tensors of shape {shp} on {dev}")
        if out is None:
            out = tuple(torch.empty((nz, N, N), dtype=dt, device=dev) for _ in range(4))
        rows = self.slab_rows(nz, zchunk)
        part = torch.empty((rows, 4), dtype=torch.float64, device=dev)
        arr = lambda ts: (ctypes.c_void_p * len(ts))(*(t.data_ptr() for t in ts))
        check(lib().lf_slab_sweep(self._ctx, nz, int(zchunk), arr(slab), arr(lo), arr(hi), arr(out),
                                  ctypes.c_void_p(part.data_ptr()), rows))
        self._keep = (slab, lo, hi, out, part)
        return out, part

    def slab_sweep_sums(self, slab, lo, hi, out, sums, zchunk: int = 0):
        """The sweep of slab_sweep without a partial-row buffer
        (lf_slab_sweep_sums): the rows go to the library's static device
        array and their totals into `sums` (float64 tensor of 4 on the
        device).  `out` and `sums` are the caller's; nothing is allocated.
        Asynchronous on the lattice's stream."""
        N, dt, dev = self.N, self.dtype, self.ws.device
        nz = int(slab[0].shape[0])
        want = [(nz, N, N)] * 4
        lo_shapes = [(2, N, N), (2, N, N), (1, N, N), (1, N, N)]
        for t, shp in zip((*slab, *lo, *hi, *out), want + lo_shapes + [(1, N, N)] * 2 + want):
            if tuple(t.shape) != shp or t.dtype != dt or not t.is_contiguous() or t.device != dev:
                raise ValueError(f"slab arrays: contiguous {dt} tensors of shape {shp} on {dev}")
        if tuple(sums.shape) != (4,) or sums.dtype != torch.float64 or sums.device != dev:
            raise ValueError(f"sums: float64 tensor of shape (4,) on {dev}")
        arr = lambda ts: (ctypes.c_void_p * len(ts))(*(t.data_ptr() for t in ts))
        check(lib().lf_slab_sweep_sums(self._ctx, nz, int(zchunk), arr(slab), arr(lo), arr(hi), arr(out),
                                       ctypes.c_void_p(sums.data_ptr())))
        self._keep = (slab, lo, hi, out, sums)
        return out, sums

    # ------------------------------------------------------------ adjoint
    def adjoint_forward(self, n: int, K: int, weights=(0.0, 1.0, 0.0, 1.0)) -> float:
        """Run n steps with checkpoints every K steps; returns the loss
        w0 K1 + w1 K2 + w2 G1 + w3 G2 at the end (synchronised energies)."""
        size = ctypes.c_size_t()
        check(lib().lf_adj_workspace_bytes(ctypes.byref(self.params), int(n), int(K), ctypes.byref(size)))
        self.adj_ws = torch.empty(size.value, dtype=torch.uint8, device=self.device)
        w = (ctypes.c_double * 4)(*[float(x) for x in weights])
        loss = ctypes.c_double()
        check(lib().lf_adj_forward(self._ctx, int(n), int(K), w, ctypes.c_void_p(self.adj_ws.data_ptr()),
                                   size.value, ctypes.byref(loss)))
        return loss.value

    def adjoint_backward(self, dL: float = 1.0) -> dict:
        """Gradient of dL * loss: dict(G, a0, ad0 floats; f1, f2, v1, v2 FP64 tensors
        with respect to the synchronised initial state)."""
        g = [torch.empty(self.shape, dtype=torch.float64, device=self.device) for _ in range(4)]
        ptrs = [_dev_ptr(t, torch.float64, self.shape) for t in g]
        dG, da0, dad0 = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        check(lib().lf_adj_backward(self._ctx, float(dL), ctypes.byref(dG), *ptrs, ctypes.byref(da0),
                                    ctypes.byref(dad0)))
        self.adj_ws = None
        return dict(G=dG.value, a0=da0.value, ad0=dad0.value, f1=g[0], f2=g[1], v1=g[2], v2=g[3])


class LeapfrogLoss(torch.autograd.Function):
    """Loss of the synchronised energies after n leapfrog steps as a
    differentiable function of G (a 0-d tensor) and the initial fields.

    forward(G, f1, f2, v1, v2, spec) -> loss (0-d FP64 tensor), where spec is
    a dict with the Lattice arguments (N, L, dt, beta, c1, r, s, kappa2,
    dtype) and n, K, a0, ad0, weights.  The gradient runs liblf's adjoint
    kernels (reverse steps with checkpoints every K steps)."""

    @staticmethod
    def forward(ctx, G, f1, f2, v1, v2, spec):
        kw = {k: spec[k] for k in ("N", "L", "dt", "beta", "c1", "r", "s", "kappa2")}
        kw["stencil"] = spec.get("stencil", 7)
        lat = Lattice(**kw, G=float(G), dtype=spec.get("dtype", torch.float32), device=f1.device)
        lat.init(f1.detach(), f2.detach(), v1.detach(), v2.detach(), spec["a0"], spec["ad0"])
        loss = lat.adjoint_forward(spec["n"], spec["K"], spec.get("weights", (0.0, 1.0, 0.0, 1.0)))
        ctx.lat = lat
        ctx.dtypes = (f1.dtype, f2.dtype, v1.dtype, v2.dtype)
        ctx.G_device = G.device if isinstance(G, torch.Tensor) else torch.device("cpu")
        return torch.tensor(loss, dtype=torch.float64, device=f1.device)

    @staticmethod
    def backward(ctx, grad):
        g = ctx.lat.adjoint_backward(float(grad))
        ctx.lat.close()
        out = [g[k].to(dt) for k, dt in zip(("f1", "f2", "v1", "v2"), ctx.dtypes)]
        return (torch.tensor(g["G"], dtype=torch.float64, device=ctx.G_device), *out, None)


def _report_dict(rep: Report) -> dict:
    return dict(step=rep.step, a=rep.a, ad=rep.ad, hubble=rep.hubble, K1=rep.K[0], K2=rep.K[1],
                G1=rep.Gr[0], G2=rep.Gr[1], P=rep.P, rho=rep.rho, R=rep.R, status=rep.status)


def _ens_params(members, dtype, tile_x=0, tile_y=0, zchunks=None):
    arr = (Params * len(members))()
    for i, m in enumerate(members):
        zc = int(zchunks[i]) if zchunks is not None else 0
        arr[i] = Params(int(m["N"]), _DT[dtype], float(m["L"]), float(m["dt"]), int(m["beta"]), 0,
                        float(m["c1"]), float(m["G"]), float(m["r"]), float(m["s"]),
                        float(m["kappa2"]), int(tile_y), zc, int(tile_x), int(m.get("stencil", 7)))
    return arr


def ens_autotune(members, dtype: torch.dtype = torch.float32, device="cuda",
                 cache_path: str | None = DEFAULT_TUNE_CACHE) -> dict:
    """Fastest ensemble launch shape for these realizations on the current
    device (liblf's lf_ens_autotune; cached per architecture and multiset of
    lattice sizes).  Returns dict(tile_x, tile_y, ztarget, zchunks, ms), with
    zchunks the per-realization z-chunks of the target (ms = -1 on a cache
    hit)."""
    arr = _ens_params(members, dtype)
    R = len(members)
    size = ctypes.c_size_t()
    check(lib().lf_ens_autotune_workspace_bytes(R, arr, ctypes.byref(size)))
    ws = torch.empty(size.value, dtype=torch.uint8, device=device)
    stream = torch.cuda.current_stream(torch.device(device))
    tx, ty, zt, ms = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
    cache_path = _cache(cache_path)
    check(lib().lf_ens_autotune(R, arr, ctypes.c_void_p(stream.cuda_stream), ctypes.c_void_p(ws.data_ptr()),
                                size.value, cache_path.encode() if cache_path else None, ctypes.byref(tx),
                                ctypes.byref(ty), ctypes.byref(zt), ctypes.byref(ms)))
    del ws
    zchunks = [lib().lf_ens_zchunk(int(m["N"]), zt.value) for m in members]
    return dict(tile_x=tx.value, tile_y=ty.value, ztarget=zt.value, zchunks=zchunks, ms=ms.value)


class Ensemble:
    """R independent lattices stepped together by liblf's batched kernels.

    members: list of dicts with the Lattice keyword arguments N, L, dt, beta,
    c1, G, r, s, kappa2 and optionally stencil (dtype, beta and stencil
    common to all).  tuned: take the tile and z-chunks from the ensemble
    autotuner (its cache, or a tuning run on a miss; a string is the cache
    path) unless a tile or z-chunks are given."""

    def __init__(self, members, dtype: torch.dtype = torch.float32, device="cuda", tile_x: int = 0,
                 tile_y: int = 0, zchunks=None, stream: torch.cuda.Stream | None = None,
                 tuned: bool | str = False):
        self.R = len(members)
        self.dtype = dtype
        self.device = torch.device(device)
        self.tuning = None
        if tuned and not (tile_x or tile_y or zchunks is not None):
            self.tuning = ens_autotune(members, dtype, device,
                                       cache_path=tuned if isinstance(tuned, str) else DEFAULT_TUNE_CACHE)
            tile_x, tile_y, zchunks = self.tuning["tile_x"], self.tuning["tile_y"], self.tuning["zchunks"]
        arr = _ens_params(members, dtype, tile_x, tile_y, zchunks)
        self.params = arr
        self.Ns = [int(m["N"]) for m in members]
        size = ctypes.c_size_t()
        check(lib().lf_ens_workspace_bytes(self.R, arr, ctypes.byref(size)))
        self.ws = torch.empty(size.value, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        check(lib().lf_ens_create(self.R, arr, ctypes.c_void_p(self.stream.cuda_stream),
                                  ctypes.c_void_p(self.ws.data_ptr()), size.value, ctypes.byref(h)))
        self._h = h

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib().lf_ens_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init_physical(self, r: int, f1, f2, u1, u2, a0: float = 1.0) -> float:
        N = self.Ns[r]
        ts = [_aligned(t) for t in (f1, f2, u1, u2)]
        dt = ts[0].dtype
        ptrs = [_dev_ptr(t, dt, (N, N, N)) for t in ts]
        ad0 = ctypes.c_double()
        check(lib().lf_ens_init_physical(self._h, int(r), *ptrs, _DT[dt], float(a0), ctypes.byref(ad0)))
        return ad0.value

    def step(self, n: int = 1) -> None:
        check(lib().lf_ens_step(self._h, int(n)))

    def last_step_ms(self) -> float:
        ms = ctypes.c_double()
        check(lib().lf_ens_last_step_ms(self._h, ctypes.byref(ms)))
        return ms.value

    def energies(self):
        reps = (Report * self.R)()
        check(lib().lf_ens_energies(self._h, reps))
        return [_report_dict(reps[i]) for i in range(self.R)]

    def fields(self, r: int, synchronized: bool = False, dtype: torch.dtype = torch.float64):
        N = self.Ns[r]
        out = [torch.empty((N, N, N), dtype=dtype, device=self.device) for _ in range(4)]
        ptrs = [_dev_ptr(t, dtype, (N, N, N)) for t in out]
        check(lib().lf_ens_get_fields(self._h, int(r), *ptrs, _DT[dtype], 1 if synchronized else 0))
        self.stream.synchronize()
        return tuple(out)
