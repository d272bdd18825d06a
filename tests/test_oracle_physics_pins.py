"""Pins of the oracle's efficiency and noise-level formulas against physics
that is derived here independently of the formulas' printed text.

Each test computes the quantity from its physical definition (a Monte-Carlo
of surface phase errors, the boundary conditions of a dielectric interface,
a plane wave in a lossy medium, the periodogram of the generated noise) and
compares it with the oracle function.  A plausible misreading of the printed
formula (a square outside the exponential, a dropped square, the wavelength
in the medium, sqrt(f_s) for sqrt(f_s / 2)) fails at least one of them.
"""
import numpy as np
import pytest

from oracle import physics as ph
from oracle import pink as opk
from oracle import tod as ot
from workloads import Stage, configs
from workloads.scenario import Telescope

EPS0 = 8.8541878128e-12   # F/m


# --------------------------------------------------------------------------
# Ruze surface efficiency (section 2.3, Ruze equation)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("nu_hz", [150e9, 350e9, 600e9])
def test_ruze_is_the_gain_loss_of_gaussian_surface_errors(nu_hz):
    """A reflector whose surface deviates normally by e ~ N(0, rho^2)
    lengthens the reflected path by 2e, a phase error 2 e (2 pi / lambda).
    The on-axis field is the aperture mean of exp(i phase); the gain falls
    by |<exp(i phase)>|^2.  Estimated here by Monte-Carlo over 4 million
    independent surface patches."""
    rho = 42e-6
    lam = ph.C_LIGHT / nu_hz
    rng = np.random.default_rng(20260423)
    n = 4_000_000
    e = rng.normal(0.0, rho, n)
    phase = 2.0 * e * (2.0 * np.pi / lam)
    field = np.mean(np.exp(1j * phase))
    gain = abs(field) ** 2
    # sd of |mean|^2 ~ 2 |mean| sd(cos)/sqrt(n) with sd(cos) <= 1/sqrt(2)
    tol = 5 * 2 * np.sqrt(gain) * np.sqrt(0.5 / n)
    got = ph.ruze(np.array([nu_hz]), rho)[0]
    assert abs(got - gain) < tol, (got, gain, tol)
    # the literal exp(-x)^2 reading and a 2 pi rho / lambda phase both fail
    x = 4 * np.pi * rho / lam
    assert abs(np.exp(-x) ** 2 - gain) > 10 * tol
    assert abs(np.exp(-(x / 2) ** 2) - gain) > 10 * tol


def test_ruze_by_gauss_hermite_quadrature():
    """The same expectation <cos(phase)> evaluated by Gauss-Hermite
    quadrature of the Gaussian surface distribution (<sin> = 0 by
    symmetry): deterministic, to 1e-12."""
    t, w = np.polynomial.hermite_e.hermegauss(80)   # weight exp(-t^2 / 2)
    w = w / np.sqrt(2 * np.pi)
    rho = 42e-6
    nu = np.array([100e9, 220e9, 350e9, 440e9, 900e9])
    lam = ph.C_LIGHT / nu
    c = np.array([np.sum(w * np.cos(2 * (rho * t) * 2 * np.pi / l))
                  for l in lam])
    np.testing.assert_allclose(ph.ruze(nu, rho), c ** 2, rtol=1e-12)


def test_aperture_efficiency_is_taper_times_surface_times_polarisation():
    """The factor on the source at stage 0 (section 2.5) for the ASTE-like
    telescope of section 3.1: eta_t = 0.85, rho = 42 um, one polarisation.
    The surface term is the quadrature gain loss above, not ph.ruze."""
    t, w = np.polynomial.hermite_e.hermegauss(80)
    w = w / np.sqrt(2 * np.pi)
    tel = Telescope()
    nu = np.array([250e9, 350e9])
    lam = ph.C_LIGHT / nu
    surf = np.array([np.sum(w * np.cos(4 * np.pi * tel.rho_surf_m * t / l))
                     for l in lam]) ** 2
    np.testing.assert_allclose(ph.aperture_efficiency(nu, tel),
                               0.85 * surf * 0.5, rtol=1e-12)


# --------------------------------------------------------------------------
# dielectric surface pass (section 2.5, Eq. eta_refl)
# --------------------------------------------------------------------------
def _fresnel_normal_incidence(n):
    """Power transmittance from vacuum into index n at normal incidence,
    from the boundary conditions: tangential E continuous (1 + r = t),
    tangential H continuous (1 - r = n t, H proportional to n E).  The
    transmitted power flux is n |t|^2 per unit incident flux."""
    A = np.array([[1.0, -1.0], [-1.0, -n]], dtype=np.float64)
    b = np.array([-1.0, -1.0])
    r, t = np.linalg.solve(A, b)
    assert abs(r) ** 2 + n * abs(t) ** 2 == pytest.approx(1.0, rel=1e-14)
    return n * t * t


@pytest.mark.parametrize("n", [1.0, 1.5, 2.0, 3.41, 9.0])
def test_surface_pass_is_fresnel_transmittance(n):
    got = ph.surface_eta(n)
    assert got == pytest.approx(_fresnel_normal_incidence(n), rel=1e-14)
    # a dropped square (1 - |r|) is not the transmittance
    if n != 1.0:
        assert abs((1 - abs((1 - n) / (1 + n))) - got) > 1e-3


def test_refractive_stage_surface_passes_use_fresnel():
    nu = np.array([300e9])
    st = Stage("refractive", d_m=4e-3, n_index=3.41, tan_delta=1e-4,
               t_K=290.0, t_refl_K=77.0)
    passes = ph.stage_passes(st, nu)
    T = _fresnel_normal_incidence(3.41)
    assert passes[0][1][0] == pytest.approx(T, rel=1e-14)
    assert passes[2][1][0] == pytest.approx(T, rel=1e-14)


# --------------------------------------------------------------------------
# dielectric absorption pass (section 2.5, Eq. eta_refr)
# --------------------------------------------------------------------------
def _lossy_slab_power(nu_hz, d_m, n, tan_delta):
    """Power remaining after a plane wave crosses thickness d of a medium
    with relative permittivity eps = n^2 (1 - i tan_delta) (the loss
    tangent is eps'' / eps'): the field goes as exp(-i k0 n_c z) with the
    complex index n_c = sqrt(eps) taken in the lower half plane."""
    eps = n * n * (1.0 - 1j * tan_delta)
    n_c = np.sqrt(eps + 0j)
    if n_c.imag > 0:
        n_c = -n_c
    k0 = 2.0 * np.pi * nu_hz / ph.C_LIGHT
    return np.abs(np.exp(-1j * k0 * n_c * d_m)) ** 2


@pytest.mark.parametrize("nu_hz,d_m,n,tan_delta", [
    (300e9, 4e-3, 3.41, 1e-4),     # the Table 1 window
    (300e9, 0.10, 3.41, 1e-3),     # thick and lossy: exponent about 2.1
    (150e9, 0.05, 1.52, 3e-4),
    (440e9, 0.02, 2.0, 2e-3),
])
def test_absorption_pass_is_lossy_plane_wave_decay(nu_hz, d_m, n, tan_delta):
    got = ph.refractive_eta(np.array([nu_hz]), d_m, n, tan_delta)[0]
    ref = _lossy_slab_power(nu_hz, d_m, n, tan_delta)
    # the exact complex root differs from n (1 - i tan_delta / 2) only at
    # order tan_delta^2 in the exponent
    assert np.log(got) == pytest.approx(np.log(ref), rel=2e-6)
    lam = ph.C_LIGHT / nu_hz
    ex = 2 * np.pi * d_m * n * tan_delta / lam
    if ex > 0.5:
        # lambda in the medium (lambda / n) or a missing n both fail
        assert abs(np.log(ref) + ex * n) > 0.3 * ex
        assert abs(np.log(ref) + ex / n) > 0.3 * ex


# --------------------------------------------------------------------------
# Ohmic loss (section 2.5): the sqrt(nu) law of a good conductor
# --------------------------------------------------------------------------
def test_ohmic_loss_follows_the_hagen_rubens_law():
    """For a good conductor the normal-incidence absorptivity is
    1 - R = 2 sqrt(2 eps0 omega / sigma) (Hagen-Rubens), proportional to
    sqrt(nu).  Fixing eps_ref from it at nu_ref, the oracle's loss at any
    other frequency must equal Hagen-Rubens there."""
    sigma_al = 3.77e7   # S/m
    nu = np.array([100e9, 220e9, 350e9, 840e9, 2e12])

    def hr(f):
        return 2.0 * np.sqrt(2.0 * EPS0 * 2.0 * np.pi * f / sigma_al)

    nu_ref = 840e9
    eps_ref = hr(nu_ref)
    np.testing.assert_allclose(1.0 - ph.ohmic_eta(nu, eps_ref, nu_ref),
                               hr(nu), rtol=1e-13)
    # the paper's 0.25 % at 840 GHz is the Hagen-Rubens loss of a metal of
    # aluminium's order of conductivity (here within 30 %)
    assert 0.7 < 0.0025 / eps_ref < 1.3


# --------------------------------------------------------------------------
# photon-noise sigma (section 2.6): sigma = NEP sqrt(f_s / 2)
# --------------------------------------------------------------------------
def test_white_noise_psd_equals_nep_squared():
    """NEP^2 is a one-sided power spectral density (W^2 / Hz).  The white
    noise tod - p_kid of a uniform stare, sampled at f_s, must therefore
    have the mean one-sided periodogram (2 / (T f_s)) |X_j|^2 = NEP^2 over
    its interior bins, for every channel.  NEP^2 comes from the contraction
    of the row's spectrum (pinned by the Lorentzian integrals), so this
    fixes the conversion sigma_of and the noise draw together."""
    sc = configs.c1(uniform_screen=True, t_total=65536)
    sc.source = None
    T, fs = sc.t_total, sc.f_sample_hz
    out = ot.simulate(sc, pixels=[0])
    x = out["tod"][0] - out["p_kid"][0]            # [K][T]
    g = ot.row_geometry(sc, 0, np.array([0], dtype=np.int64))
    eta_z, _ = ot.lut_transmission(sc.spectral, g["pwv"])
    P = ot.cascade(sc, eta_z ** g["csc"][:, None],
                   ot.source_power(sc.source, g["az"], g["el"])
                   if sc.source is not None else None)
    _, nep2 = ot.contract(sc, P)
    nep2 = nep2[0]                                  # [K]
    X = np.fft.rfft(x, axis=-1)[:, 1:T // 2]
    psd = 2.0 / (T * fs) * np.abs(X) ** 2
    ratio = psd.mean(axis=-1) / nep2
    # each bin is exponential (sd = mean): the mean over T/2 - 1 bins has
    # relative sd 1/sqrt(T/2)
    band = 5.0 / np.sqrt(T / 2)
    # (sqrt(f_s) in place of sqrt(f_s / 2) would give a ratio of 2)
    assert np.all(np.abs(ratio - 1.0) < band), ratio


# --------------------------------------------------------------------------
# 1/f level at the knee (section 2.6 with the knee reading of the level)
# --------------------------------------------------------------------------
def test_pink_psd_meets_the_white_psd_at_the_knee():
    """The knee is the frequency where the 1/f PSD equals the white
    photon-noise PSD of the reference spectrum.  Both sides are measured
    by periodogram here: the white noise of a uniform stare at the
    reference operating point (PWV 1 mm, elevation 60 deg, no source) and
    1/f series drawn with the knee-derived levels, averaged over 32 series
    and the bins within 10 % of a 2 Hz knee, with the f^alpha slope taken
    out.  This fixes amplitude and reference_nep2 together (a level of
    NEP^2 without the knee factor would be off by 2)."""
    sc = configs.c1(uniform_screen=True, t_total=65536)
    sc.source = None
    sc.pink_knee_hz = 2.0
    T, fs = sc.t_total, sc.f_sample_hz
    assert sc.spectral.ref_pwv_mm == 1.0
    assert sc.spectral.ref_el_rad == sc.scan.theta0
    out = ot.simulate(sc, pixels=[0])
    assert np.all(out["pwv"] == 1.0)
    ks = np.array([3, 30, 60])
    x = out["tod"][0, ks] - out["p_kid"][0, ks]
    white = (2.0 / (T * fs) * np.abs(np.fft.rfft(x, axis=-1)[:, 1:T // 2])
             ** 2).mean(axis=-1)
    A = opk.amplitude(ot.reference_nep2(sc), sc.pink_alpha, sc.pink_knee_hz)
    f = np.arange(T // 2 + 1) * fs / T
    near = np.abs(f / sc.pink_knee_hz - 1.0) < 0.1
    for i, k in enumerate(ks):
        al = sc.pink_alpha[k]
        per = []
        for p in range(32):
            xs = opk.series(sc.seed, p, k, A[k], al, T, fs)
            X = np.fft.rfft(xs)
            per.append(2.0 / (T * fs) * np.abs(X[near]) ** 2
                       * (f[near] / sc.pink_knee_hz) ** al)
        level = np.mean(per)
        n = np.size(per)
        band = 5.0 / np.sqrt(n) + 5.0 / np.sqrt(T / 2)
        assert abs(level / white[i] - 1.0) < band, (k, level / white[i])
