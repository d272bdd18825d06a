"""Channel responses eta_filt(f, nu) (section 2.3, Eqs. lorentzians and
filterbank).  FP64.  Oracle -- test infrastructure only."""
from __future__ import annotations

import numpy as np

from .physics import H_PLANCK


def lorentzian(nu_hz, f_hz, R):
    """Unit-peak Lorentzian 1 / (1 + 4 R^2 (nu/f - 1)^2).

    The printed denominator lacks the leading 1 and would be singular at
    nu = f; with it the curve has peak 1 and FWHM f/R."""
    return 1.0 / (1.0 + 4.0 * R ** 2 * (nu_hz / f_hz - 1.0) ** 2)


def response_matrix(filters, nu_hz, delta_J):
    """eta[F][K] for the channel set.

    lorentz     eta_k = eta_peak_k * L_k(nu)                (Eq. lorentzians)
    filterbank  eta_k = (eta_peak_k - sum_{upstream m} eta_m) * L_k(nu)
                with upstream = strictly higher centre frequency, and for
                equal f the lower channel index upstream      (Eq. filterbank)
    matrix      the user's curves.
    Photons with h*nu < 2*Delta are not detected: those rows are zero
    (section 2.3, the gap cutoff)."""
    nu = np.asarray(nu_hz, dtype=np.float64)
    if filters.mode == "matrix":
        eta = np.array(filters.matrix, dtype=np.float64, copy=True)
    else:
        f = np.asarray(filters.f_hz, dtype=np.float64)
        R = np.asarray(filters.R, dtype=np.float64)
        pk = np.asarray(filters.eta_peak, dtype=np.float64)
        K = f.size
        eta = np.zeros((nu.size, K), dtype=np.float64)
        if filters.mode == "lorentz":
            for k in range(K):
                eta[:, k] = pk[k] * lorentzian(nu, f[k], R[k])
        elif filters.mode == "filterbank":
            # descending f, ties broken by ascending index
            order = sorted(range(K), key=lambda k: (-f[k], k))
            absorbed = np.zeros(nu.size, dtype=np.float64)
            for k in order:
                eta[:, k] = (pk[k] - absorbed) * lorentzian(nu, f[k], R[k])
                absorbed += eta[:, k]
        else:
            raise ValueError(f"unknown filter mode {filters.mode!r}")
    eta[H_PLANCK * nu < 2.0 * delta_J, :] = 0.0
    return eta
