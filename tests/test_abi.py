"""liblf.so loads on a host without a GPU, exports every entry point that
include/lf.h declares, and rejects invalid arguments before touching HIP."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def LB():
    from paper_0911_5692_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_0911_5692_amd import build
        build.build()
    return _lib


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "lf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|const char \*)\s*(lf_\w+)\s*\(", src, flags=re.M)))


def test_exports_every_declared_symbol(LB):
    names = declared_symbols()
    assert len(names) >= 14, names
    cdll = ctypes.CDLL(LB.LIB_PATH)
    missing = [n for n in names if not hasattr(cdll, n)]
    assert not missing, missing
    # every declared entry point has a Python signature (the binding covers the ABI)
    assert not [n for n in names if n not in LB.SIGNATURES], [n for n in names if n not in LB.SIGNATURES]


def _params(LB, **kw):
    d = dict(N=32, dtype=0, L=20.0, dt=0.03125, beta=4, flags=0, c1=1.0, G=100.0, r=1.0, s=-1.0,
             kappa2=1.0, tile_y=0, zchunk=0)
    d.update(kw)
    return LB.Params(**d)


def test_abi_version_and_workspace(LB):
    lib = LB.lib()
    assert lib.lf_abi_version() == 2
    size = ctypes.c_size_t()
    assert lib.lf_workspace_bytes(ctypes.byref(_params(LB)), ctypes.byref(size)) == 0
    assert size.value >= 8 * 32 ** 3 * 4
    s64 = ctypes.c_size_t()
    assert lib.lf_workspace_bytes(ctypes.byref(_params(LB, dtype=1)), ctypes.byref(s64)) == 0
    assert s64.value > size.value
    # the size limits: N = 4 and N = 2048 (8 FP32 arrays of 2048^3: 275 GB) are
    # accepted, N = 2049 is not
    for n in (4, 2048):
        assert lib.lf_workspace_bytes(ctypes.byref(_params(LB, N=n)), ctypes.byref(size)) == 0
        assert size.value >= 8 * n ** 3 * 4
    assert lib.lf_workspace_bytes(ctypes.byref(_params(LB, N=2049)), ctypes.byref(size)) == LB.LF_EINVAL


@pytest.mark.parametrize("kw,frag", [
    (dict(N=3), "N=3"), (dict(N=4096), "N=4096"), (dict(dtype=2), "dtype"),
    (dict(L=0.0), "L must"), (dict(dt=-1.0), "dt must"), (dict(beta=1), "beta"),
    (dict(beta=7), "beta"), (dict(flags=1), "flags"), (dict(r=1.0, s=0.0), "s - 2r + 3"),
    (dict(kappa2=-1.0), "kappa2"), (dict(G=float("nan")), "non-finite"), (dict(tile_y=-1), "tile_y"),
])
def test_invalid_params_rejected(LB, kw, frag):
    lib = LB.lib()
    size = ctypes.c_size_t()
    rc = lib.lf_workspace_bytes(ctypes.byref(_params(LB, **kw)), ctypes.byref(size))
    assert rc == LB.LF_EINVAL
    assert frag in lib.lf_last_error().decode()


def test_create_argument_checks_before_any_device_call(LB):
    lib = LB.lib()
    p = _params(LB)
    ctx = ctypes.c_void_p()
    assert lib.lf_create(ctypes.byref(p), None, None, 1 << 30, ctypes.byref(ctx)) == LB.LF_EINVAL
    assert lib.lf_create(ctypes.byref(p), None, ctypes.c_void_p(0x1000 + 8), 1 << 30,
                         ctypes.byref(ctx)) == LB.LF_EINVAL
    assert "aligned" in lib.lf_last_error().decode()
    assert lib.lf_create(ctypes.byref(p), None, ctypes.c_void_p(0x100000), 16,
                         ctypes.byref(ctx)) == LB.LF_ENOMEM
    assert lib.lf_step(None, 1) == LB.LF_EINVAL
    assert lib.lf_destroy(None) == LB.LF_OK


def test_autotune_workspace_covers_every_candidate(LB):
    lib = LB.lib()
    p = _params(LB, N=48)
    a, b = ctypes.c_size_t(), ctypes.c_size_t()
    assert lib.lf_autotune_workspace_bytes(ctypes.byref(p), ctypes.byref(a)) == 0
    assert lib.lf_workspace_bytes(ctypes.byref(p), ctypes.byref(b)) == 0
    assert a.value >= b.value
    size = ctypes.c_size_t()
    assert lib.lf_adj_workspace_bytes(ctypes.byref(p), 100, 7, ctypes.byref(size)) == 0
    assert size.value > 7 * 4 * 48 ** 3 * 4
    assert lib.lf_adj_workspace_bytes(ctypes.byref(p), 0, 7, ctypes.byref(size)) == LB.LF_EINVAL


def test_ensemble_workspace_and_validation(LB):
    lib = LB.lib()
    arr = (LB.Params * 3)(_params(LB, N=16), _params(LB, N=24), _params(LB, N=40))
    size = ctypes.c_size_t()
    assert lib.lf_ens_workspace_bytes(3, arr, ctypes.byref(size)) == 0
    assert size.value > 8 * (16 ** 3 + 24 ** 3 + 40 ** 3) * 4
    bad = (LB.Params * 2)(_params(LB, N=16), _params(LB, N=16, dtype=1))
    assert lib.lf_ens_workspace_bytes(2, bad, ctypes.byref(size)) == LB.LF_EINVAL
    assert lib.lf_ens_workspace_bytes(0, arr, ctypes.byref(size)) == LB.LF_EINVAL


def _vac(LB, **kw):
    v = LB.Vacuum()
    v.f0[0], v.u0[0], v.m2[0], v.m2[1] = 1.0, -0.7, 1.0, 100.0
    v.eps2, v.cutoff, v.seed = 1e-10, 0.0, 7
    for k, val in kw.items():
        if k == "m2":
            v.m2[1] = val
        else:
            setattr(v, k, val)
    return v


@pytest.mark.parametrize("kw,frag", [(dict(eps2=-1.0), "eps2"), (dict(cutoff=-2.0), "cutoff"),
                                     (dict(m2=-1e6), "imaginary"), (dict(eps2=float("inf")), "eps2")])
def test_vacuum_spec_rejected_before_any_device_call(LB, kw, frag):
    lib = LB.lib()
    p = _params(LB, N=16, dtype=1)
    buf = ctypes.c_void_p(0x100000)
    rc = lib.lf_vacuum_fields(ctypes.byref(p), ctypes.byref(_vac(LB, **kw)), None, buf, 1 << 30, buf, buf, buf, buf)
    assert rc == LB.LF_EINVAL
    assert frag in lib.lf_last_error().decode()
    rc = lib.lf_vacuum_fields(ctypes.byref(p), ctypes.byref(_vac(LB)), None, None, 1 << 30, buf, buf, buf, buf)
    assert rc == LB.LF_EINVAL and "workspace" in lib.lf_last_error().decode()
    ad0 = ctypes.c_double()
    assert lib.lf_init_vacuum(None, ctypes.byref(_vac(LB)), 1.0, buf, 1 << 30, ctypes.byref(ad0)) == LB.LF_EINVAL


def test_spectrum_arguments_checked_before_any_device_call(LB):
    lib = LB.lib()
    assert lib.lf_spectrum_bins(0) == 0 and lib.lf_spectrum_bins(512) == 444
    # ensemble z-chunk of a target item length: fewest equal chunks of at most target planes
    assert [lib.lf_ens_zchunk(n, t) for n, t in ((160, 64), (96, 48), (64, 0), (64, 1 << 20), (160, 80), (7, 3))] \
        == [54, 48, 0, 64, 80, 3]
    buf = (ctypes.c_double * 8)()
    assert lib.lf_spectrum(None, 0, 4, buf, buf, ctypes.c_void_p(0x100000), 1 << 20) == LB.LF_EINVAL
    assert "ctx" in lib.lf_last_error().decode()


def test_stream_copy_arguments_checked_before_any_device_call(LB):
    lib = LB.lib()
    p = ctypes.c_void_p(0x100000)  # aligned, never dereferenced: the checks come first
    assert lib.lf_stream_copy(p, p, p, p, p, p, p, p, 6, None) == LB.LF_EINVAL
    assert "multiple of 4" in lib.lf_last_error().decode()
    assert lib.lf_stream_copy(p, p, p, p, p, p, p, None, 8, None) == LB.LF_EINVAL
    assert "b3" in lib.lf_last_error().decode()
    assert lib.lf_stream_copy(p, ctypes.c_void_p(0x100004), p, p, p, p, p, p, 8, None) == LB.LF_EINVAL
    assert "a1" in lib.lf_last_error().decode()


def test_slab_sweep_arguments_checked_before_any_device_call(LB):
    lib = LB.lib()
    rows = ctypes.c_int64()
    assert lib.lf_slab_rows(None, 8, 0, ctypes.byref(rows)) == LB.LF_EINVAL
    assert "ctx" in lib.lf_last_error().decode()
    p = (ctypes.c_void_p * 4)(0x100000, 0x100000, 0x100000, 0x100000)
    assert lib.lf_slab_sweep(None, 8, 0, p, p, p, p, ctypes.c_void_p(0x100000), 1 << 20) == LB.LF_EINVAL
    assert "ctx" in lib.lf_last_error().decode()
