"""FP64 forward model: pointing, screen and source sampling, cascade,
filterbank contraction, photon noise and the TOD (paper sections 2.2-2.7).

Follows the paper's order stage by stage; no cascade collapse, no
reference-row trick, no blocking.  Where the paper is silent the readings
are stated in each docstring.  Oracle -- test infrastructure only.
"""
from __future__ import annotations

import numpy as np

from . import filters as _filters
from . import philox as _philox
from . import physics as _ph


# --------------------------------------------------------------------------
# interpolation helpers (sections 2.4 and 2.2)
# --------------------------------------------------------------------------
def _clamped_cell(g, n):
    """Clamp the fractional index to [0, n-1]; cell = min(floor(g), n-2);
    weight = g - cell.  Returns (cell, weight, was_clamped)."""
    gc = np.clip(g, 0.0, n - 1.0)
    cell = np.minimum(np.floor(gc), n - 2).astype(np.int64)
    return cell, gc - cell, gc != g


def bilinear_clamped(grid, gx, gy):
    """Bilinear interpolation on grid[y][x] at fractional indices (gx, gy);
    out-of-range positions take the edge value.  Returns (value, clamped)."""
    ny, nx = grid.shape
    cx, wx, ox = _clamped_cell(gx, nx)
    cy, wy, oy = _clamped_cell(gy, ny)
    v = ((1.0 - wx) * (1.0 - wy) * grid[cy, cx]
         + wx * (1.0 - wy) * grid[cy, cx + 1]
         + (1.0 - wx) * wy * grid[cy + 1, cx]
         + wx * wy * grid[cy + 1, cx + 1])
    return v, ox | oy


def lut_transmission(spec, pwv_mm):
    """eta_atm,z(nu) at each PWV from the 2-D lookup table (section 2.4).

    The paper does not say how the table is interpolated.  Reading: linear
    in optical depth tau = -ln(eta_z) between the two bracketing PWV rows,
    which is exact wherever the zenith opacity is linear in PWV; PWV outside
    the table axis is clamped to it.  Table entries must lie in (0, 1].
    Returns ([rows][F], clamped[rows])."""
    n = spec.eta_z.shape[0]
    g = (np.asarray(pwv_mm, np.float64) - spec.pwv0_mm) / spec.dpwv_mm
    i, w, clamped = _clamped_cell(g, n)
    tau = -np.log(spec.eta_z)
    tz = (1.0 - w)[:, None] * tau[i, :] + w[:, None] * tau[i + 1, :]
    return np.exp(-tz), clamped


def source_power(src, az, el):
    """P_nu,src at spaxel pointings by bilinear interpolation on the cube;
    zero where the pointing falls outside the cube grid (section 2.4).  The
    grid is the closed interval [0, n-1] in fractional index on both axes.
    Returns [rows][F]."""
    rows = np.asarray(az).size
    if src is None:
        return None
    cube = src.cube.astype(np.float64)
    ga = (np.asarray(az, np.float64) - src.az0) / src.daz
    ge = (np.asarray(el, np.float64) - src.el0) / src.del_
    inside = (ga >= 0) & (ga <= src.n_az - 1) & (ge >= 0) & (ge <= src.n_el - 1)
    ca, wa, _ = _clamped_cell(ga, src.n_az)
    ce, we, _ = _clamped_cell(ge, src.n_el)
    wa = wa[:, None]
    we = we[:, None]
    out = ((1.0 - wa) * (1.0 - we) * cube[ce, ca]
           + wa * (1.0 - we) * cube[ce, ca + 1]
           + (1.0 - wa) * we * cube[ce + 1, ca]
           + wa * we * cube[ce + 1, ca + 1])
    out[~inside] = 0.0
    assert out.shape[0] == rows
    return out


# --------------------------------------------------------------------------
# scanning (section 2.4)
# --------------------------------------------------------------------------
def scan_offsets(sc, n):
    """(phi(t), theta(t)) of the scan pattern at absolute samples n, with
    t = n / f_sample.  stare: (0, 0); daisy: Eq. daisy; traj: the user's
    trajectory array."""
    n = np.asarray(n, dtype=np.int64)
    t = n.astype(np.float64) / sc.f_sample_hz
    s = sc.scan
    if s.kind == "stare":
        return np.zeros_like(t), np.zeros_like(t)
    if s.kind == "daisy":
        phi = s.r_petal * np.cos(s.Omega * t) * np.sin(s.omega * t)
        theta = s.r_petal * np.sin(s.Omega * t) * np.sin(s.omega * t)
        return phi, theta
    if s.kind == "traj":
        return s.traj[n, 0].astype(np.float64), s.traj[n, 1].astype(np.float64)
    raise ValueError(s.kind)


def row_geometry(sc, p, n):
    """Per-row quantities for pixel p at absolute samples n.

    Screen coordinates follow Eq. xy_atm literally (scan plus spaxel
    offset, without the scan offset (phi0, theta0)); the airmass uses the
    full elevation theta + theta0 + dtheta_p (Eq. airmass); the source is
    sampled at the full spaxel pointing (section 2.4)."""
    t = np.asarray(n, np.float64) / sc.f_sample_hz
    phi, theta = scan_offsets(sc, n)
    scr = sc.screen
    x = scr.h_column_m * np.tan(phi + sc.dphi[p]) + scr.wind_mps * t
    y = scr.h_column_m * np.tan(theta + sc.dtheta[p])
    gx = x / scr.dx_m + scr.ix0
    gy = y / scr.dy_m + scr.iy0
    pwv, scr_clamped = bilinear_clamped(scr.pwv_mm, gx, gy)
    el = theta + sc.scan.theta0 + sc.dtheta[p]
    az = phi + sc.scan.phi0 + sc.dphi[p]
    return dict(t=t, pwv=pwv, csc=1.0 / np.sin(el), az=az, el=el,
                screen_clamped=scr_clamped)


# --------------------------------------------------------------------------
# radiative-transfer cascade (section 2.5)
# --------------------------------------------------------------------------
def cascade(sc, eta_atm, p_src):
    """Spectral power after the last stage.

    P_0 = eta_t eta_surf eta_pol P_src + P_JN(T_CMB); stage 0 is the
    atmosphere, P_1 = eta_atm P_0 + (1 - eta_atm) P_JN(T_atm) (Eq. radtrans
    with eta_0 = eta_atm); every later pass applies Eq. radtrans with its
    own eta and parasitic power, which for a sky-coupled stage is
    (1 - eta_atm) P_JN(T_atm) + eta_atm P_JN(T_CMB).
    eta_atm: [rows][F]; p_src: [rows][F] or None.  Returns [rows][F]."""
    spec = sc.spectral
    nu = spec.nu_hz
    b_cmb = _ph.johnson_nyquist(nu, sc.t_cmb_K)
    b_atm = _ph.johnson_nyquist(nu, spec.t_atm_K)
    eps = _ph.aperture_efficiency(nu, sc.telescope)
    P = np.broadcast_to(b_cmb, eta_atm.shape).copy()
    if p_src is not None:
        P += eps * p_src
    P = eta_atm * P + (1.0 - eta_atm) * b_atm
    for stage in spec.stages:
        for kind, eta, t_K in _ph.stage_passes(stage, nu):
            if kind == "fixed":
                parasitic = _ph.johnson_nyquist(nu, t_K)
            else:
                parasitic = (1.0 - eta_atm) * b_atm + eta_atm * b_cmb
            P = eta * P + (1.0 - eta) * parasitic
    return P


# --------------------------------------------------------------------------
# filterbank contraction and photon noise (sections 2.5-2.6)
# --------------------------------------------------------------------------
def contract(sc, P, eta_filt=None):
    """P_KID = int eta_filt P dnu and
    NEP^2 = 2 int eta_filt P (h nu + eta_filt P + 2 Delta / eta_pb) dnu,
    both by the midpoint rule with the per-bin weights w (Hz).  The NEP
    integrand is split by distributivity into a P term and a P^2 term.
    P: [rows][F].  Returns (P_KID [rows][K], NEP2 [rows][K])."""
    spec = sc.spectral
    if eta_filt is None:
        eta_filt = _filters.response_matrix(spec.filters, spec.nu_hz,
                                            sc.kid.delta_J)
    w = spec.w_hz
    hv = _ph.H_PLANCK * spec.nu_hz
    gap = 2.0 * sc.kid.delta_J / sc.kid.eta_pb
    p_kid = (P * w) @ eta_filt
    nep2 = 2.0 * ((P * (w * (hv + gap))) @ eta_filt
                  + (P * P * w) @ (eta_filt * eta_filt))
    return p_kid, nep2


def sigma_of(sc, nep2):
    """sigma = NEP sqrt(f_sample / 2) (section 2.6)."""
    return np.sqrt(nep2) * np.sqrt(0.5 * sc.f_sample_hz)


def reference_nep2(sc, eta_filt=None):
    """NEP^2 per channel of the noise-free, source-free spectrum at the
    reference operating point (zenith PWV ref_pwv_mm, elevation ref_el_rad).
    Sets the 1/f amplitude: the pink PSD equals this white level at the
    knee frequency."""
    spec = sc.spectral
    eta_z, _ = lut_transmission(spec, np.array([spec.ref_pwv_mm]))
    eta_atm = eta_z ** (1.0 / np.sin(spec.ref_el_rad))
    P = cascade(sc, eta_atm, None)
    return contract(sc, P, eta_filt)[1][0]


# --------------------------------------------------------------------------
# full forward model on a window of rows
# --------------------------------------------------------------------------
def simulate(sc, t_begin=0, t_end=None, pixels=None, chunk=2048,
             photon_noise=None):
    """Noise-free power, sigma, white noise and TOD (without pink noise)
    for pixels x samples [t_begin, t_end).

    Returns dict of arrays shaped [n_pixels][K][T_window]:
      p_kid, sigma, tod (= p_kid + sigma z when photon noise is on),
    plus pwv [n_pixels][T_window] (zenith PWV at the row) and
    clamps (screen positions clamped to the screen edge)."""
    if t_end is None:
        t_end = sc.t_total
    if pixels is None:
        pixels = range(sc.n_pix)
    pixels = list(pixels)
    if photon_noise is None:
        photon_noise = sc.photon_noise
    spec = sc.spectral
    eta_filt = _filters.response_matrix(spec.filters, spec.nu_hz,
                                        sc.kid.delta_J)
    K = eta_filt.shape[1]
    Tw = t_end - t_begin
    out = {k: np.zeros((len(pixels), K, Tw)) for k in ("p_kid", "sigma",
                                                       "tod")}
    out["pwv"] = np.zeros((len(pixels), Tw))
    clamps = 0
    for ip, p in enumerate(pixels):
        for a in range(t_begin, t_end, chunk):
            b = min(t_end, a + chunk)
            n = np.arange(a, b, dtype=np.int64)
            g = row_geometry(sc, p, n)
            clamps += int(g["screen_clamped"].sum())
            eta_z, _ = lut_transmission(spec, g["pwv"])
            eta_atm = eta_z ** g["csc"][:, None]
            psrc = source_power(sc.source, g["az"], g["el"])
            P = cascade(sc, eta_atm, psrc)
            p_kid, nep2 = contract(sc, P, eta_filt)
            sig = sigma_of(sc, nep2)
            tod = p_kid.copy()
            if photon_noise:
                kk = np.arange(K, dtype=np.int64)
                z = _philox.white_normal(sc.seed, n[:, None], kk[None, :], p)
                tod += sig * z
            s = slice(a - t_begin, b - t_begin)
            out["p_kid"][ip, :, s] = p_kid.T
            out["sigma"][ip, :, s] = sig.T
            out["tod"][ip, :, s] = tod.T
            out["pwv"][ip, s] = g["pwv"]
    out["clamps"] = clamps
    return out
