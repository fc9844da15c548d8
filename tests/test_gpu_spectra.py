"""Power spectra on the device (hipFFT + deterministic shell binning) against
the oracle's spectrum of the same fields, up to the 512^3 benchmark size."""
import numpy as np
import pytest
import torch

from oracle import spectra as OS
from _parity import gpu_run, log
from paper_0911_5692_amd import workloads as W

pytestmark = pytest.mark.gpu

WHICH = ("f1", "f2", "v1", "v2")


def _deviations(lat, dt):
    """Synchronised deviations from the background, FP64, as the device forms
    them: d - (dt/2) e for the fields, e for the velocities."""
    (d1, d2, e1, e2), _ = lat.get_state()
    d1, d2, e1, e2 = (x.double() for x in (d1, d2, e1, e2))
    return [d1 - 0.5 * dt * e1, d2 - 0.5 * dt * e2, e1, e2]


def _compare(lat, w, tag):
    """Shells >= 1 against the oracle's spectrum of the same deviation field
    (within 1e-10 relative, or 1e-14 of the largest such shell); shell 0
    against the full field's mean."""
    L = w.L
    full = lat.fields(synchronized=True, dtype=torch.float64)
    for which, g, dev in zip(WHICH, full, _deviations(lat, w.dt)):
        p, c = lat.spectrum(which)
        rp, rc = OS.shell_spectrum(dev.cpu().numpy(), L)
        assert np.array_equal(c, rc), which
        err = np.abs(p[1:] - rp[1:])
        bound = 1e-10 * rp[1:] + 1e-14 * np.max(rp[1:])
        rel = float(np.max(err / np.maximum(rp[1:], 1e-300)))
        p0 = L ** 3 / w.N ** 6 * float(g.sum()) ** 2
        log(f"[spec] {tag} {which}: shells>=1 max rel err {rel:.2e}; shell 0 {p[0]!r} vs {p0!r}")
        assert np.all(err <= bound), (which, float(np.max(err - bound)))
        assert abs(p[0] - p0) <= 1e-12 * p0 + 1e-14 * np.max(rp[1:]), which


@pytest.mark.parametrize("N", [33, 64])
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_spectrum_matches_oracle(N, dtype):
    w = W.CFG3.resized(N)
    ic = W.make_inputs(w)
    lat, _ = gpu_run(w, ic, 100, dtype=dtype)
    _compare(lat, w, f"N={N} {dtype}")


def test_spectrum_27_point_lattice_and_partial_bins():
    from dataclasses import replace
    w = replace(W.CFG2, stencil=27).resized(40)
    ic = W.make_inputs(w)
    lat, _ = gpu_run(w, ic, 50)
    _compare(lat, w, "s27 N=40")
    p, c = lat.spectrum("f2", nbins=10)
    pf, cf = lat.spectrum("f2")
    assert np.array_equal(p, pf[:10]) and np.array_equal(c, cf[:10])


def test_full_size_512_parseval_determinism_and_oracle():
    """The benchmark lattice: two calls bitwise equal, Parseval on the
    deviation, and every shell against the oracle's spectrum."""
    w = W.CFG3
    ic = W.make_inputs(w)
    lat, _ = gpu_run(w, ic, 20, **W.BENCH_SHAPES[w.name])
    p1, c1 = lat.spectrum("f2")
    p2, c2 = lat.spectrum("f2")
    assert np.array_equal(p1, p2) and np.array_equal(c1, c2)
    dev = _deviations(lat, w.dt)[1]
    g = lat.fields(synchronized=True, dtype=torch.float64)[1]
    p0 = w.L ** 3 / w.N ** 6 * float(g.sum()) ** 2
    lhs = float(np.sum(p1[1:] * c1[1:])) + p0
    rhs = float((dev * dev).sum() - dev.sum() ** 2 / w.N ** 3) * w.L ** 3 / w.N ** 3 + p0
    log(f"[spec512] Parseval {lhs!r} vs {rhs!r}")
    assert abs(lhs - rhs) <= 1e-11 * rhs
    rp, rc = OS.shell_spectrum(dev.cpu().numpy(), w.L)
    assert np.array_equal(c1, rc)
    assert np.all(np.abs(p1[1:] - rp[1:]) <= 1e-10 * rp[1:] + 1e-14 * np.max(rp[1:]))
