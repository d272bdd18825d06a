"""Physical constants, blackbody power and efficiencies (FP64).

Paper sections: 2.3 (telescope and instrument), 2.5 (radiative-transfer
cascade).  Oracle -- test infrastructure only.
"""
from __future__ import annotations

import numpy as np

H_PLANCK = 6.62607015e-34   # J s (exact SI)
K_BOLTZ = 1.380649e-23      # J/K (exact SI)
C_LIGHT = 299792458.0       # m/s (exact SI)


def johnson_nyquist(nu_hz, t_K):
    """Single-mode Johnson-Nyquist spectral power h*nu / (exp(h*nu/kT) - 1)
    in W/Hz (section 2.5, the CMB and stage-temperature terms).  The paper
    does not print the formula; this is the single-polarisation,
    zero-point-free form.  T = 0 gives 0."""
    nu = np.asarray(nu_hz, dtype=np.float64)
    if t_K <= 0.0:
        return np.zeros_like(nu)
    x = H_PLANCK * nu / (K_BOLTZ * t_K)
    with np.errstate(over="ignore"):
        return H_PLANCK * nu / np.expm1(x)


def ruze(nu_hz, rho_surf_m):
    """Ruze surface efficiency exp(-(4 pi rho / lambda)^2) (section 2.3;
    the printed parenthesisation squares outside the exponential, read here
    as the standard Ruze form)."""
    lam = C_LIGHT / np.asarray(nu_hz, dtype=np.float64)
    return np.exp(-(4.0 * np.pi * rho_surf_m / lam) ** 2)


def aperture_efficiency(nu_hz, tel):
    """eta_t * eta_surf * eta_pol, the factor on the source at stage 0
    (section 2.5, effective source seen by the 0th stage)."""
    return tel.eta_taper * ruze(nu_hz, tel.rho_surf_m) * tel.eta_pol


def ohmic_eta(nu_hz, eps_ref, nu_ref_hz):
    """Ohmic-loss stage efficiency 1 - eps_ref * sqrt(nu / nu_ref)
    (section 2.5, Ohmic reflector losses)."""
    return 1.0 - eps_ref * np.sqrt(np.asarray(nu_hz, np.float64) / nu_ref_hz)


def refractive_eta(nu_hz, d_m, n_index, tan_delta):
    """Dielectric absorption pass exp(-2 pi d n tan(delta) / lambda)
    (section 2.5, Eq. eta_refr)."""
    lam = C_LIGHT / np.asarray(nu_hz, dtype=np.float64)
    return np.exp(-2.0 * np.pi * d_m * n_index * tan_delta / lam)


def surface_eta(n_index):
    """Surface pass 1 - ((1 - n) / (1 + n))^2 at normal incidence
    (section 2.5, Eq. eta_refl)."""
    return 1.0 - ((1.0 - n_index) / (1.0 + n_index)) ** 2


def stage_passes(stage, nu_hz):
    """Expand one optics stage into the passes of Eq. radtrans it stands for.

    Returns a list of (kind, eta[F], t_K) with kind 'fixed' (couples to
    the stage temperature) or 'atm' (couples to the sky: parasitic power
    (1-eta_atm) P_JN(T_atm) + eta_atm P_JN(T_CMB)).
    A refractive stage is reflect - absorb - reflect; with an AR coating
    only the absorbing pass remains (section 2.5)."""
    nu = np.asarray(nu_hz, dtype=np.float64)
    F = nu.size

    def vec(e):
        return np.broadcast_to(np.asarray(e, dtype=np.float64), (F,)).copy()

    k = stage.kind
    if k == "reflect":
        return [("fixed", vec(stage.eta), stage.t_K)]
    if k == "atm_coupled":
        return [("atm", vec(stage.eta), None)]
    if k == "ohmic":
        return [("fixed", ohmic_eta(nu, stage.eps_ref, stage.nu_ref_hz),
                 stage.t_K)]
    if k == "refractive":
        absorb = ("fixed", refractive_eta(nu, stage.d_m, stage.n_index,
                                          stage.tan_delta), stage.t_K)
        if stage.ar_coated:
            return [absorb]
        surf = ("fixed", vec(surface_eta(stage.n_index)), stage.t_refl_K)
        return [surf, absorb, surf]
    raise ValueError(f"unknown stage kind {k!r}")
