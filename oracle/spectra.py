"""Oracle of the field power spectra (TEST INFRASTRUCTURE ONLY: only tests/,
the smoke entry and the benchmark's CPU baseline use it).

The paper lists power spectra through the FFT as the natural next step of
the program (Sec. IV).  The spectrum computed here is the shell average of
the discrete Fourier power of a lattice field f (N^3, x fastest):
  F_n = sum_x f(x) exp(-2 pi i n.x / N),  n the FFT-signed integer vector,
  shell s = rint(|n|),
  count[s] = number of lattice modes n with rint(|n|) = s,
  power[s] = (L^3 / N^6) * (sum over those modes of |F_n|^2) / count[s],
so that sum_s count[s] power[s] = (L^3 / N^3) sum_x f(x)^2 (Parseval), and a
Gaussian field with power spectrum P(k), normalised as <f^2> = sum_k P(k)/L^3,
has E power[s] = P(k) on the modes of shell s.
numpy's FFT is a library step; the half spectrum of rfftn counts the modes
0 < n_x < N/2 twice (their conjugates), the others once.
"""
from __future__ import annotations

import numpy as np


def shell_count_max(N: int) -> int:
    """Number of shells holding every lattice mode: rint(sqrt(3) (N div 2)) + 1."""
    h = N // 2
    return int(np.rint(np.sqrt(3.0 * h * h))) + 1


def shell_spectrum(f: np.ndarray, L: float, nbins: int | None = None):
    """(power, count) per shell s < nbins (default: all shells), FP64."""
    N = f.shape[0]
    nbins = shell_count_max(N) if nbins is None else nbins
    F = np.fft.rfftn(np.asarray(f, dtype=np.float64))
    n0 = np.fft.fftfreq(N) * N
    n2 = np.fft.rfftfreq(N) * N
    nn = np.sqrt(n0[:, None, None] ** 2 + n0[None, :, None] ** 2 + n2[None, None, :] ** 2)
    wgt = np.full(nn.shape, 2.0)
    wgt[..., 0] = 1.0
    if N % 2 == 0:
        wgt[..., -1] = 1.0
    shell = np.rint(nn).astype(np.int64).ravel()
    keep = shell < nbins
    p = (np.abs(F) ** 2).ravel() * wgt.ravel()
    cnt = np.bincount(shell[keep], weights=wgt.ravel()[keep], minlength=nbins)
    tot = np.bincount(shell[keep], weights=p[keep], minlength=nbins)
    power = np.zeros(nbins)
    nz = cnt > 0
    power[nz] = tot[nz] / cnt[nz] * L ** 3 / N ** 6
    return power, cnt
