"""Pins of the oracle's shell power spectrum: Parseval, the exact power of a
plane wave, the brute-force mode count per shell, and the expectation of
white noise and of a field drawn with a known spectrum."""
import itertools

import numpy as np
import pytest

from oracle import spectra as S
from oracle import vacuum as V


@pytest.mark.parametrize("N", [8, 9])
def test_mode_counts_brute_force(N):
    _, cnt = S.shell_spectrum(np.zeros((N, N, N)), 1.0)
    brute = np.zeros(S.shell_count_max(N))
    half = [n if n <= N // 2 else n - N for n in range(N)]  # any representative works: |n| is even in n
    for a, b, c in itertools.product(half, repeat=3):
        brute[int(np.rint(np.sqrt(a * a + b * b + c * c)))] += 1
    assert np.array_equal(cnt, brute)
    assert cnt.sum() == N ** 3


@pytest.mark.parametrize("N", [12, 13])
def test_parseval(N):
    rng = np.random.default_rng(N)
    f = 1.3 + rng.standard_normal((N, N, N))
    L = 2.7
    p, c = S.shell_spectrum(f, L)
    assert abs(np.sum(p * c) - L ** 3 / N ** 3 * np.sum(f * f)) <= 1e-12 * np.sum(p * c)


def test_plane_wave_power():
    """f = A cos(2 pi n.x/N) puts |F|^2 = (A N^3/2)^2 on the two modes +-n:
    power[rint |n|] = 2 (L^3/N^6)(A N^3/2)^2 / count, zero elsewhere but
    rounding."""
    N, L, A = 16, 3.0, 0.7
    n = np.array([3, 1, 2])
    z, y, x = np.meshgrid(*(np.arange(N),) * 3, indexing="ij")
    f = A * np.cos(2 * np.pi * (n[0] * x + n[1] * y + n[2] * z) / N)
    p, c = S.shell_spectrum(f, L)
    s = int(np.rint(np.linalg.norm(n)))
    expect = 2 * L ** 3 / N ** 6 * (A * N ** 3 / 2) ** 2 / c[s]
    assert abs(p[s] - expect) <= 1e-12 * expect
    others = np.delete(p, s)
    assert np.max(others) <= 1e-20 * expect


def test_white_noise_and_known_spectrum_expectation():
    """White noise of variance sigma^2: E power = sigma^2 L^3/N^3 in every
    shell; a field drawn with P(k) (the vacuum generator): E power[s] = P on
    the shell's modes."""
    N, L = 64, 5.0
    rng = np.random.default_rng(3)
    sig = 0.2
    p, c = S.shell_spectrum(sig * rng.standard_normal((N, N, N)), L)
    for s in (3, 10, 25, 40, 50):
        assert abs(p[s] / (sig ** 2 * L ** 3 / N ** 3) - 1) < 5 / np.sqrt(c[s] / 2), s
    m2, eps2 = 4.0, 1e-6
    f = V.fluctuation(N, L, m2, eps2, "field", seed=4, j=0)
    p, c = S.shell_spectrum(f, L)
    for s in (4, 8, 12, 15):
        k = 2 * np.pi * s / L
        Ps = eps2 / (2 * np.sqrt(k * k + m2))
        # the shell holds |n| in [s - 1/2, s + 1/2): allow the P(k) spread across it
        spread = abs(np.log(np.sqrt((2 * np.pi * (s + 0.5) / L) ** 2 + m2) / np.sqrt((2 * np.pi * (s - 0.5) / L) ** 2 + m2)))
        assert abs(np.log(p[s] / Ps)) < 5 / np.sqrt(c[s] / 2) + spread, s
    # the generator's cutoff |n| <= N/4 leaves the shells above it empty of power
    assert np.max(p[N // 4 + 1:]) <= 1e-20 * np.max(p)
