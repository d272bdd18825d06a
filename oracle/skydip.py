"""Brightness-temperature (Kelvin) output by a simulated skydip (section
2.7).  FP64.  Oracle -- test infrastructure only.

The paper sets up a linear map between the detected power and the
line-of-sight brightness temperature T_b by varying the PWV (which varies
T_b) while recording the power.  Readings where it is silent:
  * the sweep holds the elevation fixed (the observation's), steps the
    zenith PWV uniformly over [pwv_lo, pwv_hi] in n steps, has no source,
    and records the noise-free channel power (the expectation of P_tot);
  * T_b of channel k is the channel-weighted brightness temperature of the
    atmosphere along the line of sight,
        T_b,k = sum_j w_j eta_jk (1 - eta_atm,j) T_atm / sum_j w_j eta_jk;
  * the map is the ordinary least-squares line P_k = a_k + b_k T_b,k, and
    the Kelvin output is T = (P - a_k) / b_k;
  * a channel without response (sum_j w_j eta_jk = 0) or whose T_b does
    not vary over the sweep has no brightness scale: a_k = b_k = NaN.
"""
from __future__ import annotations

import numpy as np

from . import filters as _filters
from . import tod as _tod


def sweep(sc, el_rad, pwv_lo, pwv_hi, n):
    """(PWV grid, P_KID [n][K], T_b [n][K]) of the skydip."""
    spec = sc.spectral
    eta = _filters.response_matrix(spec.filters, spec.nu_hz, sc.kid.delta_J)
    pwv = np.linspace(pwv_lo, pwv_hi, n)
    eta_z, _ = _tod.lut_transmission(spec, pwv)
    eta_atm = eta_z ** (1.0 / np.sin(el_rad))
    P = _tod.cascade(sc, eta_atm, None)
    p_kid, _ = _tod.contract(sc, P, eta)
    wq = spec.w_hz[:, None] * eta
    den = wq.sum(axis=0)
    with np.errstate(invalid="ignore", divide="ignore"):
        t_b = ((1.0 - eta_atm) * spec.t_atm_K) @ wq / den
    t_b[:, den == 0.0] = np.nan
    return pwv, p_kid, t_b


def fit(p_kid, t_b):
    """Per-channel least-squares line P = a + b T_b: slope = centred
    cross moment over centred second moment of T_b, intercept through the
    means."""
    n, K = p_kid.shape
    a = np.full(K, np.nan)
    b = np.full(K, np.nan)
    for k in range(K):
        x, y = t_b[:, k], p_kid[:, k]
        if not np.all(np.isfinite(x)):
            continue
        mx, my = x.mean(), y.mean()
        sxx = np.sum((x - mx) ** 2)
        if sxx == 0.0:
            continue
        b[k] = np.sum((x - mx) * (y - my)) / sxx
        a[k] = my - b[k] * mx
    return a, b


def skydip(sc, el_rad, pwv_lo, pwv_hi, n):
    _, p_kid, t_b = sweep(sc, el_rad, pwv_lo, pwv_hi, n)
    return fit(p_kid, t_b)


def to_kelvin(tod, a, b):
    """tod [P][K][T] in W -> K."""
    return (tod - a[None, :, None]) / b[None, :, None]
