"""Temporally correlated 1/f noise by the method of Timmer and Koenig
(1995), as the paper prescribes for P_pn (section 2.6).  FP64.

Readings where the paper is silent:
  * the PSD S(f) = A f^-alpha is one-sided, in W^2/Hz;
  * the series is generated at N = the next power of two >= T samples and
    the first T samples are kept; the DC and Nyquist bins are zero;
  * bin j (frequency f_j = j f_s / N) gets X_j = c_j (z_re + i z_im) with
    z from the pink-noise Philox stream and c_j^2 = S(f_j) N f_s / 4, so
    that the expected periodogram (2 / (N f_s)) |X_j|^2 equals S(f_j);
  * x = the inverse real DFT of X including its 1/N factor;
  * A_k, when not given per channel, is NEP^2_ref,k * f_knee^alpha_k, i.e.
    the 1/f PSD equals the white photon-noise PSD of the reference spectrum
    at the knee frequency.

Oracle -- test infrastructure only.
"""
from __future__ import annotations

import numpy as np

from . import philox as _philox


def fft_length(t_total: int) -> int:
    n = 2
    while n < t_total:
        n *= 2
    return n


def amplitude(nep2_ref, alpha, knee_hz, A=None):
    """Per-channel 1/f levels A_k of S = A_k f^-alpha_k (section 2.6).  The
    paper leaves A a free level per channel: explicit levels A are used as
    given; without them the knee reading above applies."""
    if A is not None:
        return np.asarray(A, dtype=np.float64)
    return np.asarray(nep2_ref) * knee_hz ** np.asarray(alpha)


def spectrum(seed, p, k, A, alpha, t_total, f_s):
    """The N/2+1 complex bins X_j of series (pixel p, channel k)."""
    N = fft_length(t_total)
    M = N // 2
    X = np.zeros(M + 1, dtype=np.complex128)
    j = np.arange(1, M, dtype=np.int64)
    if j.size:
        zr, zi = _philox.pink_normals(seed, j, k, p)
        f = j * (f_s / N)
        c = np.sqrt(A * f ** (-alpha) * N * f_s / 4.0)
        X[1:M] = c * (zr + 1j * zi)
    return X


def series(seed, p, k, A, alpha, t_total, f_s):
    """P_pn for (pixel p, channel k): first t_total samples of irfft."""
    N = fft_length(t_total)
    X = spectrum(seed, p, k, A, alpha, t_total, f_s)
    return np.fft.irfft(X, N)[:t_total]
