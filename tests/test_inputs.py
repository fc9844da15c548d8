"""The seeded input generators: reproducibility and the spectra they promise."""
import numpy as np

from oracle.spectra import shell_spectrum
from paper_0911_5692_amd import inputs, workloads


def _shells(f, L):
    pw, cnt = shell_spectrum(f, L)
    return np.arange(len(pw)), pw, cnt


def test_seeded_and_reproducible():
    a = inputs.white_noise(8, 1e-3, inputs.rng_for(1, 0, 0, 0))
    b = inputs.white_noise(8, 1e-3, inputs.rng_for(1, 0, 0, 0))
    c = inputs.white_noise(8, 1e-3, inputs.rng_for(1, 0, 1, 0))
    assert np.array_equal(a, b) and not np.array_equal(a, c)


def test_grf_spectrum_cutoff_and_mean():
    N, L, m2 = 48, 6.0, 3.0
    k_of = lambda n: 2 * np.pi * n / L
    vals = []
    for rep in range(3):
        f = inputs.gaussian_random_field(N, L, m2, inputs.rng_for(99, rep, 0, 0), amplitude2=2.0)
        n, pw, cnt = _shells(f, L)
        vals.append(pw)
        assert abs(f.mean()) < 1e-12 * f.std() * N ** 3
        # nothing above the cutoff N/4 (shells above 12.5 rounded up are empty of power)
        assert np.all(pw[n >= 14][cnt[n >= 14] > 0] < 1e-25)
    pw = np.mean(vals, axis=0)
    P = 2.0 / (2 * np.sqrt(k_of(n) ** 2 + m2))
    # shells well inside the cutoff: within sampling error (cnt modes * 3 draws)
    sel = (n >= 2) & (n <= 11)
    rel = np.abs(pw[sel] / P[sel] - 1)
    tol = 4.0 / np.sqrt(3 * cnt[sel] / 2)
    assert np.all(rel < tol), (rel, tol)


def test_grf_exact_std_and_velocity_kind():
    f = inputs.gaussian_random_field(32, 5.0, 100.0, inputs.rng_for(2, 0, 1, 0), std=1e-3)
    assert abs(f.std() - 1e-3) < 1e-15
    v = inputs.gaussian_random_field(32, 5.0, 100.0, inputs.rng_for(2, 0, 1, 1), amplitude2=1.0,
                                     kind="velocity")
    n, pw, cnt = _shells(v, 5.0)
    k = 2 * np.pi * n / 5.0
    sel = (n >= 2) & (n <= 7)
    assert np.all(np.abs(pw[sel] / (np.sqrt(k[sel] ** 2 + 100.0) / 2) - 1) < 4 / np.sqrt(cnt[sel] / 2))


def test_workload_inputs_shapes():
    w = workloads.CFG1
    ic = workloads.make_inputs(w)
    assert ic["f1"].shape == (32, 32, 32) and ic["a0"] == 1.0
    assert abs(ic["f1"].mean() - 1.0) < 1e-4 and abs(ic["f2"].std() - 1e-3) < 1e-4
    w3 = workloads.CFG3.resized(32)
    ic3 = workloads.make_inputs(w3)
    assert abs(ic3["u1"].mean() - workloads.U0_INFLATON) < 1e-8
    t = workloads.tile_inputs(ic3, 2)
    assert t["f1"].shape == (64, 64, 64) and np.array_equal(t["f1"][32:, :32, 32:], ic3["f1"])
