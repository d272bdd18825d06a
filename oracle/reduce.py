"""Common-mode atmosphere subtraction and inverse-variance gridding of
brightness-temperature TODs (section 4.3, Eqs. common_mode and Sj).  FP64.
Oracle -- test infrastructure only.

Readings where the paper is silent:
  * the observation's mean zenith PWV is the mean of the zenith PWV output
    over every spaxel and sample;
  * the zenith transmission at channel k is the channel-weighted mean of the
    table's transmission at that PWV,
        eta_z,k = sum_j w_j eta_jk eta_z,j / sum_j w_j eta_jk,
    and eta_atm,i(t, k) = eta_z,k ** (1 / sin theta_i(t)) with the elevation
    of the airmass, theta_i(t) = theta(t) + theta0 + dtheta_i (Eq. airmass);
  * a spaxel is off source when its offset radius sqrt(dphi^2 + dtheta^2)
    exceeds r_out strictly; no off-source spaxel is an error;
  * gridding bins every sample of spaxel i at (phi(t) + dphi_i,
    theta(t) + dtheta_i) to the nearest node of an n x n grid spanning
    +-half on both axes (samples farther than half a node spacing outside
    the outer nodes are dropped); each spaxel gives, per channel and cell,
    the mean and its variance s^2 / m (unbiased s^2 over the cell's m
    samples, m >= 2 and s^2 > 0, else no contribution); the cells of all
    spaxels are combined with weights m / s^2; a cell without contribution
    is NaN with weight 0.
"""
from __future__ import annotations

import numpy as np

from . import filters as _filters
from . import tod as _tod


def pwv_mean(pwv):
    """Mean zenith PWV of an observation from its [P][T] PWV output."""
    return float(np.mean(np.asarray(pwv, dtype=np.float64)))


def channel_zenith_transmission(sc, pwv_mm):
    """eta_z,k at a zenith PWV [K] (NaN for a channel without response)."""
    spec = sc.spectral
    eta = _filters.response_matrix(spec.filters, spec.nu_hz, sc.kid.delta_J)
    eta_z, _ = _tod.lut_transmission(spec, np.array([pwv_mm], dtype=np.float64))
    wq = spec.w_hz[:, None] * eta
    den = wq.sum(axis=0)
    with np.errstate(invalid="ignore", divide="ignore"):
        return (eta_z[0] @ wq) / den


def spaxel_transmission(sc, eta_zk, n):
    """eta_atm,i(t, k) [P][K][T] at absolute samples n."""
    _, theta = _tod.scan_offsets(sc, n)
    el = theta[None, :] + sc.scan.theta0 + np.asarray(sc.dtheta)[:, None]
    csc = 1.0 / np.sin(el)
    return np.asarray(eta_zk)[None, :, None] ** csc[:, None, :]


def off_source(sc, r_out):
    """S_j of Eq. Sj."""
    return np.hypot(np.asarray(sc.dphi), np.asarray(sc.dtheta)) > r_out


def common_mode(sc, t_b, pwv_mm, r_out, t0=0, channels=None):
    """T*_a,i(t, k) of Eq. common_mode for a [P][K][T] Kelvin TOD holding
    samples t0 .. t0 + T - 1 (or only the listed channels)."""
    t_b = np.asarray(t_b, dtype=np.float64)
    T = t_b.shape[2]
    eta_zk = channel_zenith_transmission(sc, pwv_mm)
    if channels is not None:
        eta_zk = eta_zk[list(channels)]
    eta = spaxel_transmission(sc, eta_zk, t0 + np.arange(T))
    S = off_source(sc, r_out)
    n_out = int(S.sum())
    if n_out == 0:
        raise ValueError("no spaxel lies outside r_out")
    common = (t_b[S] / (1.0 - eta[S])).sum(axis=0) / n_out
    return t_b / eta - (1.0 - eta) / eta * common[None]


def grid_cells(sc, half, n, T, t0=0):
    """Cell index [P][T] of each sample (-1 outside the grid)."""
    phi, theta = _tod.scan_offsets(sc, t0 + np.arange(T))
    d = 2.0 * half / (n - 1)
    cells = np.full((sc.n_pix, T), -1, dtype=np.int64)
    for p in range(sc.n_pix):
        ix = np.floor((phi + sc.dphi[p] + half) / d + 0.5)
        iy = np.floor((theta + sc.dtheta[p] + half) / d + 0.5)
        ok = (ix >= 0) & (ix < n) & (iy >= 0) & (iy < n)
        cells[p, ok] = (iy[ok] * n + ix[ok]).astype(np.int64)
    return cells


def spaxel_maps(sc, tod, half, n, t0=0):
    """Per spaxel, channel and cell: (count [P][n*n], mean [P][K][n*n],
    unbiased variance [P][K][n*n]); NaN where count < 2."""
    tod = np.asarray(tod, dtype=np.float64)
    P, K, T = tod.shape
    cells = grid_cells(sc, half, n, T, t0)
    C = n * n
    count = np.zeros((P, C))
    mean = np.full((P, K, C), np.nan)
    var = np.full((P, K, C), np.nan)
    for p in range(P):
        ok = cells[p] >= 0
        c = cells[p, ok]
        m = np.bincount(c, minlength=C).astype(np.float64)
        count[p] = m
        has = m >= 2
        for k in range(K):
            v = tod[p, k, ok]
            s1 = np.bincount(c, weights=v, minlength=C)
            mu = np.divide(s1, m, out=np.zeros(C), where=m > 0)
            s2 = np.bincount(c, weights=(v - mu[c]) ** 2, minlength=C)
            mean[p, k, has] = mu[has]
            var[p, k, has] = s2[has] / (m[has] - 1.0)
    return count, mean, var


def combine(count, mean, var):
    """Inverse-variance combination over spaxels: (map [K][C], weight
    [K][C]) with weight_i = m_i / s_i^2."""
    P, K, C = mean.shape
    w = np.zeros((P, K, C))
    use = np.isfinite(var) & (var > 0)
    w[use] = (count[:, None, :] * np.ones((1, K, 1)))[use] / var[use]
    wsum = w.sum(axis=0)
    num = np.where(use, w * np.nan_to_num(mean), 0.0).sum(axis=0)
    with np.errstate(invalid="ignore", divide="ignore"):
        m = np.where(wsum > 0, num / wsum, np.nan)
    return m, wsum


def reduce_maps(sc, t_b, pwv_mm, r_out, half, n, t0=0):
    """Common-mode subtraction, then gridding: (T*, map, weight)."""
    ts = common_mode(sc, t_b, pwv_mm, r_out, t0)
    count, mean, var = spaxel_maps(sc, ts, half, n, t0)
    m, w = combine(count, mean, var)
    return ts, m, w
