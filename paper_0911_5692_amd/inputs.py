"""Seeded synthetic initial data (FP64, host).

This module draws random fields and nothing else: it holds no step of the
evolution.  Both the GPU library and the oracle consume the arrays it returns.
The spectra are the usual lattice initial conditions that the paper takes
from DEFROST (Sec. II.B): homogeneous values given as input plus random
fluctuations generated through an FFT.

Conventions: arrays have shape (N, N, N), x last; wavevector k = 2 pi n / L
with n the FFT-signed integer vector; a random field with power spectrum P(k)
is white noise w filtered as  f = irfftn( rfftn(w) * sqrt(N^3 P(k) / L^3) ),
so that <f^2> = sum_k P(k) / L^3, the lattice form of int d^3k/(2pi)^3 P(k).
The k = 0 mode and every |n| above the cutoff are zero.
"""
from __future__ import annotations

import os

import numpy as np
import scipy.fft as sfft

_WORKERS = min(16, os.cpu_count() or 1)


def rng_for(*key: int) -> np.random.Generator:
    """Generator seeded by SeedSequence(key), e.g. (workload, realization, field, kind)."""
    return np.random.default_rng(np.random.SeedSequence(list(key)))


def white_noise(N: int, sigma: float, rng: np.random.Generator) -> np.ndarray:
    """IID normal N(0, sigma^2) per site, float64 (N, N, N)."""
    return sigma * rng.standard_normal((N, N, N))


def _mode_norm(N: int) -> np.ndarray:
    n0 = np.fft.fftfreq(N) * N
    n2 = np.fft.rfftfreq(N) * N
    return np.sqrt(n0[:, None, None] ** 2 + n0[None, :, None] ** 2 + n2[None, None, :] ** 2)


def gaussian_random_field(N: int, L: float, m_eff2: float, rng: np.random.Generator, *,
                          amplitude2: float = 1.0, cutoff: float | None = None,
                          kind: str = "field", std: float | None = None) -> np.ndarray:
    """Gaussian random field with P(k) = amplitude2 / (2 omega_k) (kind="field")
    or amplitude2 * omega_k / 2 (kind="velocity"), omega_k = sqrt(k^2 + m_eff2),
    zero for |n| > cutoff (default N/4).  If std is given the sample is
    rescaled to that exact standard deviation."""
    if cutoff is None:
        cutoff = N / 4
    w = rng.standard_normal((N, N, N))
    W = sfft.rfftn(w, workers=_WORKERS)
    del w
    nn = _mode_norm(N)
    k = 2.0 * np.pi * nn / L
    omega = np.sqrt(k * k + m_eff2)
    if kind == "field":
        P = amplitude2 / (2.0 * omega)
    elif kind == "velocity":
        P = amplitude2 * omega / 2.0
    else:
        raise ValueError(kind)
    P[(nn == 0) | (nn > cutoff)] = 0.0
    W *= np.sqrt(N ** 3 * P / L ** 3)
    del P, omega, k, nn
    f = sfft.irfftn(W, s=(N, N, N), workers=_WORKERS)
    if std is not None:
        f *= std / f.std()
    return f
