"""Seeded synthetic inputs for the TOD simulator.

This module only draws and lays out inputs: frequency grids with their
quadrature weights, PWV screens, zenith-transmission tables standing in for
the ATM tables, filter parameters, cascade stage parameters, pre-convolved
source cubes and specific-intensity cubes, spaxel offsets, user-defined scan
trajectories and request streams.  It holds none of the simulator's arithmetic (no cascade, no filter
response, no contraction, no noise model); both the FP64 oracle and the GPU
path consume exactly the arrays produced here.

Everything is deterministic in its seed (numpy PCG64).
"""
from __future__ import annotations

import os

import numpy as np

ARCSEC = np.pi / (180.0 * 3600.0)
DEG = np.pi / 180.0
C_LIGHT = 299792458.0
JY = 1.0e-26  # W m^-2 Hz^-1


# --------------------------------------------------------------------------
# frequency grid
# --------------------------------------------------------------------------
def nu_grid(F: int, lo_hz: float = 200e9, hi_hz: float = 460e9):
    """F uniform bins over [lo, hi]; centres and midpoint-rule weights (Hz)."""
    dnu = (hi_hz - lo_hz) / F
    nu = lo_hz + (np.arange(F, dtype=np.float64) + 0.5) * dnu
    w = np.full(F, dnu, dtype=np.float64)
    return nu, w


# --------------------------------------------------------------------------
# synthetic zenith transmission table (stand-in for the ATM table)
# --------------------------------------------------------------------------
def absorption_lines(seed: int = 7, n_lines: int = 5, lo_hz: float = 200e9,
                     hi_hz: float = 460e9):
    rng = np.random.default_rng(seed)
    return dict(
        nu_hz=rng.uniform(lo_hz, hi_hz, n_lines),
        gamma_hz=rng.uniform(1e9, 8e9, n_lines),
        a_per_mm=10.0 ** rng.uniform(-1.5, 0.3, n_lines),
        base_per_mm=0.01,
    )


def zenith_transmission_table(nu_hz, lines, pwv0_mm=0.0, dpwv_mm=0.01,
                              n_pwv=301):
    """eta_z[i, j] = exp(-tau(nu_j) * PWV_i), tau a sum of Lorentzian lines.

    Returns (eta_z[n_pwv, F] float64, pwv0_mm, dpwv_mm)."""
    nu = np.asarray(nu_hz, dtype=np.float64)
    tau = np.full_like(nu, lines["base_per_mm"])
    for nl, g, a in zip(lines["nu_hz"], lines["gamma_hz"], lines["a_per_mm"]):
        tau += a / (1.0 + ((nu - nl) / g) ** 2)
    pwv = pwv0_mm + dpwv_mm * np.arange(n_pwv, dtype=np.float64)
    eta = np.exp(-np.outer(pwv, tau))
    return eta, pwv0_mm, dpwv_mm


# --------------------------------------------------------------------------
# PWV screen: 2-D power-law Fourier field
# --------------------------------------------------------------------------
def pwv_screen(ny: int, nx: int, seed: int, mean_mm: float = 1.0,
               rms_mm: float = 0.02, slope: float = -11.0 / 3.0,
               cell_m: float = 0.2) -> np.ndarray:
    """FP64 [ny][nx] screen (x, the wind axis, contiguous) whose power
    spectrum falls as |k|^slope; k = 0 removed; rescaled to the given rms
    and shifted to the given mean."""
    import scipy.fft as sfft

    rng = np.random.default_rng(seed)
    ky = np.fft.fftfreq(ny, d=cell_m)
    kx = np.fft.rfftfreq(nx, d=cell_m)
    nkx = kx.size
    spec = np.empty((ny, nkx), dtype=np.complex128)
    # row blocks bound the peak memory for the 2 GiB screens
    blk = max(1, (1 << 24) // nkx)
    for r0 in range(0, ny, blk):
        r1 = min(ny, r0 + blk)
        k2 = ky[r0:r1, None] ** 2 + kx[None, :] ** 2
        with np.errstate(divide="ignore"):
            amp = np.where(k2 > 0.0, k2 ** (slope / 4.0), 0.0)
        re = rng.standard_normal((r1 - r0, nkx))
        im = rng.standard_normal((r1 - r0, nkx))
        spec[r0:r1] = amp * (re + 1j * im)
    del k2, amp, re, im
    field = sfft.irfft2(spec, s=(ny, nx), workers=os.cpu_count() or 1,
                        overwrite_x=True)
    del spec
    field -= field.mean()
    field *= rms_mm / field.std()
    field += mean_mm
    return np.ascontiguousarray(field, dtype=np.float64)


def uniform_screen(ny: int, nx: int, value_mm: float) -> np.ndarray:
    return np.full((ny, nx), value_mm, dtype=np.float64)


# --------------------------------------------------------------------------
# spaxel layouts
# --------------------------------------------------------------------------
def square_spaxels(n_side: int, pitch_rad: float):
    """p = n_side*row + col; elevation (row) is the outer axis."""
    c = (n_side - 1) / 2.0
    rows, cols = np.meshgrid(np.arange(n_side), np.arange(n_side),
                             indexing="ij")
    dphi = ((cols - c) * pitch_rad).ravel().astype(np.float64)
    dtheta = ((rows - c) * pitch_rad).ravel().astype(np.float64)
    return dphi, dtheta


def hex_spaxels(r_hex: int, pitch_rad: float):
    """Packed hexagon with 3R(R+1)+1 spaxels: centre first, then rings
    counter-clockwise starting on the +azimuth corner."""
    pts = [(0.0, 0.0)]
    ang = np.arange(7) * (np.pi / 3.0)
    corners = np.stack([np.cos(ang), np.sin(ang)], axis=1)
    for r in range(1, r_hex + 1):
        for s in range(6):
            a, b = corners[s], corners[s + 1]
            for i in range(r):
                v = r * a + i * (b - a)
                pts.append((v[0], v[1]))
    pts = np.asarray(pts, dtype=np.float64) * pitch_rad
    return pts[:, 0].copy(), pts[:, 1].copy()


# --------------------------------------------------------------------------
# user-defined scan: raster trajectory
# --------------------------------------------------------------------------
def raster_trajectory(t_total: int, f_s: float, half_az_rad: float,
                      speed_rad_s: float, el_step_rad: float,
                      half_el_rad: float) -> np.ndarray:
    """(phi, theta)[t_total][2] FP64 for an azimuth triangle wave of
    amplitude half_az at constant speed, stepping elevation by el_step at
    each turn-around, back and forth over +-half_el."""
    t = np.arange(t_total, dtype=np.float64) / f_s
    leg_s = 2.0 * half_az_rad / speed_rad_s
    ph = t / leg_s
    leg = np.floor(ph)
    u = ph - leg
    even = (leg % 2) == 0
    az = np.where(even, -half_az_rad + 2.0 * half_az_rad * u,
                  half_az_rad - 2.0 * half_az_rad * u)
    n_steps = int(round(2.0 * half_el_rad / el_step_rad))
    m = leg % (2 * n_steps)
    m = np.where(m > n_steps, 2 * n_steps - m, m)
    el = -half_el_rad + el_step_rad * m
    return np.ascontiguousarray(np.stack([az, el], axis=1))


# --------------------------------------------------------------------------
# pre-convolved source cubes (beam convolution done analytically here)
# --------------------------------------------------------------------------
def beam_fwhm_rad(nu_hz, dish_m: float = 10.0, k: float = 1.2):
    return k * C_LIGHT / (np.asarray(nu_hz) * dish_m)


def source_cube(nu_hz, n_grid: int, half_extent_rad: float, phi0: float,
                theta0: float, components, a_p_m2: float):
    """P_nu,src cube float32 [n_el][n_az][F] (W/Hz) on a square grid
    centred on (phi0, theta0).

    components: list of dicts with keys
      flux_jy   -- callable nu_hz -> total flux density (Jy) or array (F,)
      fwhm_rad  -- source FWHM (0 for a point source)
      off_rad   -- (d_az, d_el) offset from the grid centre
      peak_w_hz -- optional: fixes the peak P (W/Hz) instead of the flux
    A Gaussian source convolved with the Gaussian beam is again Gaussian;
    its amplitude keeps the total flux."""
    nu = np.asarray(nu_hz, dtype=np.float64)
    off = np.linspace(-half_extent_rad, half_extent_rad, n_grid)
    d_az = off[None, :, None]
    d_el = off[:, None, None]
    sb = beam_fwhm_rad(nu) / np.sqrt(8.0 * np.log(2.0))
    cube = np.zeros((n_grid, n_grid, nu.size), dtype=np.float64)
    for comp in components:
        ss = comp.get("fwhm_rad", 0.0) / np.sqrt(8.0 * np.log(2.0))
        s2 = ss ** 2 + sb ** 2
        oa, oe = comp.get("off_rad", (0.0, 0.0))
        r2 = (d_az - oa) ** 2 + (d_el - oe) ** 2
        shape = np.exp(-r2 / (2.0 * s2[None, None, :]))
        if "peak_w_hz" in comp:
            amp = np.full_like(nu, comp["peak_w_hz"])
        else:
            flux = comp["flux_jy"]
            flux = flux(nu) if callable(flux) else np.asarray(flux)
            amp = a_p_m2 * flux * JY * (sb ** 2 / s2)
        cube += amp[None, None, :] * shape
    d = 2.0 * half_extent_rad / (n_grid - 1)
    grid = dict(n_az=n_grid, n_el=n_grid, az0=phi0 - half_extent_rad,
                daz=d, el0=theta0 - half_extent_rad, del_=d)
    return np.ascontiguousarray(cube.astype(np.float32)), grid


def intensity_cube(nu_hz, n_grid: int, half_extent_rad: float, seed: int,
                   n_blobs: int = 4, peak=1e-18):
    """Specific-intensity cube float32 [n_grid][n_grid][F] (W m^-2 Hz^-1
    sr^-1): seeded Gaussian blobs (widths 5-40 arcsec) with power-law
    spectra, plus a faint flat floor."""
    rng = np.random.default_rng(seed)
    nu = np.asarray(nu_hz, dtype=np.float64)
    off = np.linspace(-half_extent_rad, half_extent_rad, n_grid)
    cube = np.full((n_grid, n_grid, nu.size), 1e-3 * peak)
    for _ in range(n_blobs):
        ca, ce = rng.uniform(-0.6, 0.6, 2) * half_extent_rad
        s = rng.uniform(5, 40) * ARCSEC
        shape = np.exp(-((off[None, :] - ca) ** 2 + (off[:, None] - ce) ** 2)
                       / (2 * s * s))
        spec = rng.uniform(0.2, 1.0) * peak * (nu / 300e9) ** rng.uniform(-1, 3)
        cube += shape[:, :, None] * spec[None, None, :]
    return np.ascontiguousarray(cube.astype(np.float32))


# --------------------------------------------------------------------------
# request stream for the serving workload
# --------------------------------------------------------------------------
def request_stream(n: int = 256, rate_hz: float = 20.0, seed: int = 5,
                   pix_choices=(1, 7, 19, 49), k_choices=(64, 347, 720),
                   f_choices=tuple(range(1000, 4001, 250)),
                   dur_s=(10.0, 600.0), n_screens: int = 4):
    rng = np.random.default_rng(seed)
    arrivals = np.cumsum(rng.exponential(1.0 / rate_hz, n))
    reqs = []
    for i in range(n):
        reqs.append(dict(
            rid=i,
            arrival_s=float(arrivals[i]),
            n_pix=int(rng.choice(pix_choices)),
            K=int(rng.choice(k_choices)),
            F=int(rng.choice(f_choices)),
            duration_s=float(rng.uniform(*dur_s)),
            screen=int(rng.integers(0, n_screens)),
            seed=int(rng.integers(0, 2**63 - 1)),
        ))
    return reqs
