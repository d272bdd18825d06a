"""Input preparation (section 2.2): aperture illumination, far-field
pattern, source-beam convolution (Eq. convolve_src) and the footprint
smoothing of the PWV screen.  FP64.  Oracle -- test infrastructure only.

Readings where the printed equations are garbled or silent:
  * Eq. aper_dist: circularly symmetric Gaussian amplitude illumination
    with edge taper t_edge dB (negative) at the rim r = R_tel,
        A(r) = 10 ** (t_edge (r / R_tel)^2 / 20)  for r < R_tel, else 0;
  * F = |FT{A}|^2 normalised to its peak: the continuous two-dimensional
    Fourier transform of A over aperture coordinates in wavelengths, which
    for a circularly symmetric field is the Hankel transform
        F(rho) = [ int_0^R A(r) J0(2 pi rho r / lambda) r dr
                   / int_0^R A(r) r dr ]^2,
    rho the angular distance (small angles); the paper samples this with
    an FFT;
  * Eq. convolve_src on the cube's own (phi, theta) grid: the integral is
    the rectangle-rule sum over every grid node, with the flat-sky angular
    distance sqrt(dphi^2 + dtheta^2) between nodes, and A_p = pi R_tel^2;
  * screen footprint: each screen cell becomes the A-weighted mean of the
    cells whose centres lie within R_tel of it (weights A(r), normalised
    to sum 1), indices clamped at the screen edges.
"""
from __future__ import annotations

import numpy as np
from scipy import integrate, special

C_LIGHT = 299792458.0


def aperture_field(r_m, R_tel, t_edge_db):
    r = np.asarray(r_m, dtype=np.float64)
    return np.where(r < R_tel, 10.0 ** (t_edge_db * (r / R_tel) ** 2 / 20.0),
                    0.0)


def _hankel(rho, lam, R_tel, t_edge_db):
    k = 2.0 * np.pi * rho / lam
    f = lambda r: (10.0 ** (t_edge_db * (r / R_tel) ** 2 / 20.0)
                   * special.j0(k * r) * r)
    # split at the zeros of J0 so that each piece is smooth and one-signed
    n_osc = int(k * R_tel / np.pi) + 1
    edges = np.linspace(0.0, R_tel, n_osc + 1)
    tol = 1e-15 * R_tel * R_tel
    return sum(integrate.quad(f, a, b, epsabs=tol, epsrel=1e-12, limit=200)[0]
               for a, b in zip(edges[:-1], edges[1:]))


def far_field(rho_rad, nu_hz, R_tel, t_edge_db):
    """Peak-normalised far-field power pattern at angular distances rho
    (any shape) for one frequency."""
    lam = C_LIGHT / nu_hz
    rho = np.asarray(rho_rad, dtype=np.float64)
    h0 = _hankel(0.0, lam, R_tel, t_edge_db)
    out = np.empty(rho.shape)
    flat = out.reshape(-1)
    for i, r in enumerate(rho.reshape(-1)):
        flat[i] = (_hankel(float(r), lam, R_tel, t_edge_db) / h0) ** 2
    return out


def convolve_source(I, nu_hz, az0, daz, el0, del_, R_tel, t_edge_db):
    """P_nu,src [n_el][n_az][F] from the specific intensity I [n_el][n_az]
    [F] (W m^-2 Hz^-1 sr^-1) on the grid az = az0 + i daz, el = el0 + j del
    (Eq. convolve_src)."""
    I = np.asarray(I, dtype=np.float64)
    n_el, n_az, F = I.shape
    a_p = np.pi * R_tel ** 2
    el = el0 + del_ * np.arange(n_el)
    ia = np.arange(n_az)
    ie = np.arange(n_el)
    da = (ia[:, None] - ia[None, :]) * daz          # [i][i']
    de = (ie[:, None] - ie[None, :]) * del_         # [j][j']
    rho = np.sqrt(da[None, :, None, :] ** 2 + de[:, None, :, None] ** 2)
    out = np.empty_like(I)
    src = I * np.cos(el)[:, None, None]              # I(phi', theta') cos theta'
    rho_u, inv = np.unique(rho, return_inverse=True)
    for f in range(F):
        Fb = far_field(rho_u, nu_hz[f], R_tel, t_edge_db)[inv].reshape(rho.shape)
        out[:, :, f] = a_p * daz * del_ * np.einsum("jikl,kl->ji", Fb,
                                                    src[:, :, f])
    return out


def source_power_at(I_f, nu_f, daz, el0, del_, R_tel, t_edge_db, i, j):
    """One node (i, j) of Eq. convolve_src at one frequency, from the
    intensity plane I_f [n_el][n_az] of that frequency."""
    I_f = np.asarray(I_f, dtype=np.float64)
    n_el, n_az = I_f.shape
    ia = np.arange(n_az)
    ie = np.arange(n_el)
    rho = np.sqrt(((i - ia)[None, :] * daz) ** 2 + ((j - ie)[:, None] * del_) ** 2)
    rho_u, inv = np.unique(rho, return_inverse=True)
    Fb = far_field(rho_u, nu_f, R_tel, t_edge_db)[inv].reshape(rho.shape)
    src = I_f * np.cos(el0 + del_ * ie)[:, None]
    return np.pi * R_tel ** 2 * daz * del_ * float(np.sum(Fb * src))


def footprint_weights(dx_m, dy_m, R_tel, t_edge_db):
    """Normalised weights [2 ry + 1][2 rx + 1] of the screen footprint."""
    rx = int(np.floor(R_tel / dx_m))
    ry = int(np.floor(R_tel / dy_m))
    x = dx_m * np.arange(-rx, rx + 1)
    y = dy_m * np.arange(-ry, ry + 1)
    r = np.sqrt(x[None, :] ** 2 + y[:, None] ** 2)
    w = aperture_field(r, R_tel, t_edge_db)
    return w / w.sum()


def convolve_screen(scr, dx_m, dy_m, R_tel, t_edge_db):
    """Footprint-smoothed screen [ny][nx] (edge-clamped)."""
    scr = np.asarray(scr, dtype=np.float64)
    ny, nx = scr.shape
    w = footprint_weights(dx_m, dy_m, R_tel, t_edge_db)
    ry, rx = (w.shape[0] - 1) // 2, (w.shape[1] - 1) // 2
    out = np.zeros_like(scr)
    xs = np.arange(nx)
    ys = np.arange(ny)
    for a in range(-ry, ry + 1):
        yy = np.clip(ys + a, 0, ny - 1)
        for b in range(-rx, rx + 1):
            if w[a + ry, b + rx] == 0.0:
                continue
            xx = np.clip(xs + b, 0, nx - 1)
            out += w[a + ry, b + rx] * scr[yy][:, xx]
    return out
