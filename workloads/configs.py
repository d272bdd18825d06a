"""The five synthetic workloads and small variants of them.

c1  plain method, tiny: 1 px stare, 64 Lorentzians (R=500), F=1000, 10 s.
c2  single-pixel spectrometer: 1 px raster, 347-channel filterbank, F=3000,
    600 s, 512x65536 screen, 6-stage cascade.
c3  IFU: 7x7 px daisy, as c2 otherwise, 1 h, 1024x262144 screen.
c4  c3 plus a faint extended source, split-precision contraction.
c5  serving stream of 256 requests (see workloads.gen.request_stream).

Shapes, sizes and value ranges follow the DESHIMA 2.0 / ASTE setting of the
paper (Table 1, section 3.1) where the paper gives them; the atmosphere
table, screens and sources are seeded synthetic stand-ins.
"""
from __future__ import annotations

import numpy as np

from . import gen
from .gen import ARCSEC, DEG
from .scenario import (KID, Filters, Scan, Scenario, Screen, Source,
                       Spectral, Stage, Telescope)

F_SAMPLE = 160.0
THETA0 = 60.0 * DEG
A_P = np.pi * 5.0 ** 2


def lorentz_bank(K: int, lo_hz=220e9, hi_hz=440e9, R=500.0, eta_peak=1.0,
                 mode="lorentz"):
    k = np.arange(K, dtype=np.float64)
    f = lo_hz * (hi_hz / lo_hz) ** (k / max(K - 1, 1))
    return Filters(mode=mode, f_hz=f, R=np.full(K, R),
                   eta_peak=np.full(K, eta_peak))


def cascade_c1():
    return [Stage("reflect", eta=0.95, t_K=280.0),
            Stage("reflect", eta=0.8, t_K=40.0),
            Stage("reflect", eta=0.6, t_K=4.0)]


def cascade_c2():
    """Table-1-shaped: spillover, Ohmic-Al, secondary spillover to the sky,
    AR-coated window, leaky lens."""
    return [Stage("reflect", eta=0.99, t_K=273.0),
            Stage("ohmic", eps_ref=0.0025, nu_ref_hz=840e9, t_K=273.0),
            Stage("atm_coupled", eta=0.85),
            Stage("refractive", d_m=4e-3, n_index=3.41, tan_delta=1e-4,
                  t_K=290.0, t_refl_K=290.0, ar_coated=True),
            Stage("reflect", eta=0.7, t_K=4.0)]


def cascade_table2():
    """Table-2-shaped cascade with non-coated lenses (3 passes each)."""
    return [Stage("reflect", eta=0.99, t_K=273.0),
            Stage("ohmic", t_K=273.0),
            Stage("ohmic", t_K=273.0),
            Stage("atm_coupled", eta=0.85),
            Stage("refractive", d_m=10e-3, n_index=3.4, tan_delta=1e-5,
                  t_K=290.0, t_refl_K=290.0),
            Stage("refractive", d_m=4e-3, n_index=3.4, tan_delta=1e-5,
                  t_K=290.0, t_refl_K=290.0),
            Stage("reflect", eta=0.65, t_K=4.0),
            Stage("refractive", d_m=25.56e-3, n_index=3.4, tan_delta=1e-5,
                  t_K=4.0, t_refl_K=4.0),
            Stage("refractive", d_m=16e-3, n_index=3.4, tan_delta=1e-5,
                  t_K=4.0, t_refl_K=4.0),
            Stage("reflect", eta=0.7, t_K=4.0)]


def spectral(F, filters, stages, lut_seed=7, ref_pwv=1.0, ref_el=THETA0,
             lo_hz=200e9, hi_hz=460e9):
    nu, w = gen.nu_grid(F, lo_hz, hi_hz)
    lines = gen.absorption_lines(lut_seed, lo_hz=lo_hz, hi_hz=hi_hz)
    eta_z, pwv0, dpwv = gen.zenith_transmission_table(nu, lines)
    return Spectral(nu_hz=nu, w_hz=w, eta_z=eta_z, pwv0_mm=pwv0,
                    dpwv_mm=dpwv, t_atm_K=273.0, stages=stages,
                    filters=filters, ref_pwv_mm=ref_pwv, ref_el_rad=ref_el)


def screen(ny, nx, seed, mean=1.0, rms=0.02, uniform=False):
    arr = (gen.uniform_screen(ny, nx, mean) if uniform
           else gen.pwv_screen(ny, nx, seed, mean, rms))
    return Screen(pwv_mm=arr, dx_m=0.2, dy_m=0.2, ix0=32.0,
                  iy0=(ny - 1) / 2.0, h_column_m=1537.0, wind_mps=10.0)


def point_source(nu, n_grid=55, half=70 * ARCSEC, flux_jy=1e-3):
    cube, g = gen.source_cube(nu, n_grid, half, 0.0, THETA0,
                              [dict(flux_jy=np.full(nu.size, flux_jy),
                                    fwhm_rad=0.0)], A_P)
    return Source(cube=cube, az0=g["az0"], daz=g["daz"], el0=g["el0"],
                  del_=g["del_"])


def line_source(nu, n_grid=55, half=70 * ARCSEC, faint=False):
    def flux(n):
        return 0.1 + 1.0 * np.exp(-4 * np.log(2) * (n - 350e9) ** 2
                                  / (0.5e9) ** 2)
    comps = [dict(flux_jy=flux, fwhm_rad=10 * ARCSEC)]
    if faint:
        # flat peak 1e-4 of a nominal loading of 0.1 * k_B * 273 K
        comps.append(dict(peak_w_hz=1e-4 * 0.1 * 1.380649e-23 * 273.0,
                          fwhm_rad=60 * ARCSEC))
    cube, g = gen.source_cube(nu, n_grid, half, 0.0, THETA0, comps, A_P)
    return Source(cube=cube, az0=g["az0"], daz=g["daz"], el0=g["el0"],
                  del_=g["del_"])


def c1(noise=True, uniform_screen=False, t_total=1600):
    sp = spectral(1000, lorentz_bank(64), cascade_c1())
    dphi, dth = np.zeros(1), np.zeros(1)
    return Scenario(
        name="c1", f_sample_hz=F_SAMPLE, spectral=sp,
        screen=screen(64, 4096, 1001, uniform=uniform_screen),
        scan=Scan("stare", phi0=0.0, theta0=THETA0), dphi=dphi, dtheta=dth,
        t_total=t_total, source=point_source(sp.nu_hz), seed=1,
        photon_noise=noise,
        pink_alpha=np.ones(64) if noise else None, pink_knee_hz=1.0)


def c2(t_total=96000, screen_shape=(512, 65536), noise=True, F=3000, K=347):
    sp = spectral(F, lorentz_bank(K, eta_peak=0.16, mode="filterbank"),
                  cascade_c2())
    traj = gen.raster_trajectory(t_total, F_SAMPLE, 60 * ARCSEC,
                                 0.5 * DEG, 10 * ARCSEC, 60 * ARCSEC)
    return Scenario(
        name="c2", f_sample_hz=F_SAMPLE, spectral=sp,
        screen=screen(*screen_shape, 1002),
        scan=Scan("traj", phi0=0.0, theta0=THETA0, traj=traj),
        dphi=np.zeros(1), dtheta=np.zeros(1), t_total=t_total,
        source=line_source(sp.nu_hz), seed=2, photon_noise=noise,
        pink_alpha=np.ones(K) if noise else None, pink_knee_hz=1.0)


def daisy_scan():
    om = 2 * np.pi * 1.54
    return Scan("daisy", phi0=0.0, theta0=THETA0, r_petal=90 * ARCSEC,
                omega=om, Omega=om / 50.0)


def c3(t_total=576000, screen_shape=(1024, 262144), n_side=7, noise=True,
       F=3000, K=347, faint=False, name="c3", seed=3, reuse_screen=None):
    """reuse_screen: a Screen made by an earlier call with the same
    screen_shape (c3 and c4 share theirs), to skip regenerating it."""
    sp = spectral(F, lorentz_bank(K, eta_peak=0.16, mode="filterbank"),
                  cascade_c2())
    dphi, dth = gen.square_spaxels(n_side, 12 * ARCSEC)
    if reuse_screen is not None:
        assert reuse_screen.pwv_mm.shape == tuple(screen_shape)
    return Scenario(
        name=name, f_sample_hz=F_SAMPLE, spectral=sp,
        screen=(reuse_screen if reuse_screen is not None
                else screen(*screen_shape, 1003)),
        scan=daisy_scan(), dphi=dphi, dtheta=dth, t_total=t_total,
        source=line_source(sp.nu_hz, n_grid=121, half=150 * ARCSEC,
                           faint=faint),
        seed=seed, photon_noise=noise,
        pink_alpha=np.ones(K) if noise else None, pink_knee_hz=1.0)


def c4(**kw):
    kw.setdefault("faint", True)
    return c3(name="c4", seed=4, **kw)


# --------------------------------------------------------------------------
# c5: serving stream
# --------------------------------------------------------------------------
def c5_spectral(K, F):
    """Spectral setup of a serving request: K-channel filterbank (R=500,
    eta_peak 0.16) over 220-440 GHz, F bins, Table-1-shaped cascade."""
    return spectral(F, lorentz_bank(K, eta_peak=0.16, mode="filterbank"),
                    cascade_c2())


def c5_screens(n=4, shape=(512, 65536)):
    return [screen(*shape, 50 + i) for i in range(n)]


def c5_pixels(n_pix):
    if n_pix == 49:
        return gen.square_spaxels(7, 12 * ARCSEC)
    r = {1: 0, 7: 1, 19: 2}[n_pix]
    return gen.hex_spaxels(r, 12 * ARCSEC)


def c5_requests(n=256, rate_hz=20.0, seed=5, **kw):
    """Request parameters (arrival, pixels, channels, bins, duration,
    screen, seed); samples = round(duration * 160 Hz)."""
    reqs = gen.request_stream(n, rate_hz, seed, **kw)
    for r in reqs:
        r["t_total"] = int(round(r["duration_s"] * F_SAMPLE))
    return reqs


def c5_scenario(req, screens, spectral_cache=None, source_cache=None):
    """Scenario of one serving request (daisy scan, c2-style line source on
    a 55x55 grid over +-70 arcsec).  Caches let requests share setups."""
    K, F = req["K"], req["F"]
    sp = spectral_cache.get((K, F)) if spectral_cache is not None else None
    if sp is None:
        sp = c5_spectral(K, F)
        if spectral_cache is not None:
            spectral_cache[(K, F)] = sp
    src = source_cache.get(F) if source_cache is not None else None
    if src is None:
        src = line_source(sp.nu_hz)
        if source_cache is not None:
            source_cache[F] = src
    dphi, dth = c5_pixels(req["n_pix"])
    return Scenario(
        name=f"c5-r{req['rid']}", f_sample_hz=F_SAMPLE, spectral=sp,
        screen=screens[req["screen"]], scan=daisy_scan(), dphi=dphi,
        dtheta=dth, t_total=req["t_total"], source=src, seed=req["seed"],
        photon_noise=True, pink_alpha=np.ones(K), pink_knee_hz=1.0)
