"""Pins of the oracle's vacuum initial state (Sec. II.B: homogeneous values as
input, random fluctuations generated through an FFT).

The counter-based generator is checked against the published known-answer
vectors of Philox4x32-10 (Random123 distribution of Salmon et al., SC'11); the
normal deviates against their moments; the filtered fields against the
per-mode power, the exact cutoff and the closed-form variance sum_k P(k)/L^3.
"""
import numpy as np
import pytest

from oracle import vacuum as V

# (counter, key) -> output, Random123 known-answer vectors for philox4x32_10
KAT = [
    ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
]


@pytest.mark.parametrize("ctr,key,out", KAT)
def test_philox_known_answers(ctr, key, out):
    got = V.philox4x32_10(*ctr, *key)
    assert tuple(int(g) for g in got) == out


def test_philox_vectorised_equals_scalar():
    c0 = np.array([1, 2, 3, 0xFFFFFFFF], dtype=np.uint32)
    vec = V.philox4x32_10(c0, 5, 6, 7, 11, 13)
    for n in range(4):
        one = V.philox4x32_10(int(c0[n]), 5, 6, 7, 11, 13)
        assert all(int(vec[w][n]) == int(one[w]) for w in range(4))


def test_uniform53_range_and_exactness():
    """Every 53-bit value maps exactly to (m + 1) / 2^53: the smallest is
    2^-53 (log finite), the largest exactly 1, neighbours differ by 2^-53."""
    assert V.uniform53(0, 0) == 2.0 ** -53
    assert V.uniform53(0xFFFFFFFF, 0xFFFFFFFF) == 1.0
    a = V.uniform53(0x12345678, 0x9ABCDEF0)
    b = V.uniform53(0x12345678, 0x9ABCDEF0 + (1 << 11))
    assert b - a == 2.0 ** -53


def test_white_noise_moments_and_independence():
    N = 48
    a = V.white_noise(N, 1234, 0)
    b = V.white_noise(N, 1234, 1)
    n = N ** 3
    for g in (a, b):
        assert abs(g.mean()) < 5 / np.sqrt(n)
        assert abs(g.var() - 1.0) < 5 * np.sqrt(2.0 / n)
        assert abs(np.mean(g ** 4) - 3.0) < 5 * np.sqrt(96.0 / n)
    assert abs(np.mean(a * b)) < 5 / np.sqrt(n)
    # sampled sites agree with the full array; another seed differs
    idx = np.array([0, 1, 777, n - 1])
    assert np.array_equal(V.white_noise(N, 1234, 0, sites=idx), a.ravel()[idx])
    assert not np.array_equal(V.white_noise(N, 1235, 0, sites=idx), a.ravel()[idx])


@pytest.mark.parametrize("kind", ["field", "velocity"])
def test_fluctuation_spectrum(kind):
    """Per-shell mean of |FFT f|^2 L^3/N^6 equals P(k) within its sampling
    error; modes above the cutoff and k = 0 are zero; the variance is
    sum_k P(k)/L^3."""
    N, L, m2, eps2 = 48, 7.5, 2.0, 3e-6
    f = V.fluctuation(N, L, m2, eps2, kind, seed=99, j=2)
    F = np.fft.rfftn(f)
    nn = V.mode_norm(N)
    power = np.abs(F) ** 2 * L ** 3 / N ** 6
    P = V.spectrum(N, L, m2, eps2, kind)
    assert np.max(np.abs(F[nn > N / 4])) < 1e-12 * np.max(np.abs(F))
    assert abs(F[0, 0, 0]) < 1e-12 * np.max(np.abs(F))
    shells = np.rint(nn).astype(int)
    for s in range(1, N // 4 + 1):
        sel = (shells == s) & (nn <= N / 4) & (nn > 0)
        # count each stored mode once; the conjugate half adds no information
        ratio = np.mean(power[sel] / P[sel])
        assert abs(ratio - 1.0) < 5.0 / np.sqrt(sel.sum()) + 1e-12, (s, ratio)
    wgt = np.ones_like(nn)
    wgt[..., 1:] = 2.0
    if N % 2 == 0:
        wgt[..., -1] = 1.0
    var_expected = np.sum(wgt * P) / L ** 3
    # a realisation's variance scatters by ~ sqrt(2 / modes)
    assert abs(np.mean(f * f) / var_expected - 1.0) < 0.1


def test_vacuum_state_assembly():
    N, L = 16, 4.0
    st = V.vacuum_state(N, L, (1.0, 0.0), (-0.7, 0.0), (1.0, 50.0), 1e-8, seed=5)
    assert abs(st["f1"].mean() - 1.0) < 1e-14 and abs(st["u1"].mean() + 0.7) < 1e-14
    assert abs(st["f2"].mean()) < 1e-14
    # array j of the generator feeds f1, f2, u1, u2 in that order
    ref = V.fluctuation(N, L, 50.0, 1e-8, "velocity", 5, 3)
    assert np.array_equal(st["u2"], ref)
