"""Pins of the FP64 oracle against what the paper and mathematics fix.

Each test ties an oracle function to something other than itself: closed
forms, invariants, limits, brute force on tiny inputs, an independent
Philox implementation, statistics of the noise, and constants printed in
the paper (tests/golden/paper_constants.json).
"""
import copy
import json
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
from oracle import filters as of
from oracle import philox as op
from oracle import physics as ph
from oracle import pink as opk
from oracle import tod as ot
from workloads import Filters, Scan, Scenario, Screen, Source, Spectral, Stage
from workloads import configs, gen

HERE = os.path.dirname(os.path.abspath(__file__))


def tiny_scenario(F=8, K=3, P=2, T=5, stages=None, filt="filterbank",
                  uniform=None, scan="daisy", source=True, seed=11):
    """A hand-sized scenario: F bins over 300-340 GHz, K channels."""
    nu, w = gen.nu_grid(F, 300e9, 340e9)
    lines = gen.absorption_lines(3, lo_hz=300e9, hi_hz=340e9)
    eta_z, p0, dp = gen.zenith_transmission_table(nu, lines, 0.0, 0.05, 61)
    if filt == "matrix":
        rng = np.random.default_rng(seed)
        fil = Filters("matrix", matrix=rng.uniform(0, 0.5, (F, K)))
    else:
        fil = configs.lorentz_bank(K, 305e9, 335e9, R=40.0, eta_peak=0.5,
                                   mode=filt)
    if stages is None:
        stages = configs.cascade_c2()
    sp = Spectral(nu_hz=nu, w_hz=w, eta_z=eta_z, pwv0_mm=p0, dpwv_mm=dp,
                  t_atm_K=270.0, stages=stages, filters=fil)
    scr = (gen.uniform_screen(16, 64, uniform) if uniform is not None
           else gen.pwv_screen(16, 64, seed, 1.0, 0.1))
    screen = Screen(pwv_mm=scr, dx_m=0.5, dy_m=0.5, ix0=4.0, iy0=7.5)
    if scan == "daisy":
        sc_ = Scan("daisy", theta0=np.pi / 3, r_petal=40 * gen.ARCSEC,
                   omega=2 * np.pi * 1.54, Omega=2 * np.pi * 1.54 / 50)
    else:
        sc_ = Scan("stare", theta0=np.pi / 3)
    dphi, dth = gen.hex_spaxels(1, 12 * gen.ARCSEC)
    src = None
    if source:
        cube, g = gen.source_cube(nu, 9, 60 * gen.ARCSEC, 0.0, np.pi / 3,
                                  [dict(flux_jy=np.full(F, 5.0),
                                        fwhm_rad=10 * gen.ARCSEC)],
                                  np.pi * 25)
        src = Source(cube=cube, az0=g["az0"], daz=g["daz"], el0=g["el0"],
                     del_=g["del_"])
    return Scenario(name="tiny", f_sample_hz=160.0, spectral=sp,
                    screen=screen, scan=sc_, dphi=dphi[:P], dtheta=dth[:P],
                    t_total=T, source=src, seed=seed)


# --------------------------------------------------------------------------
# paper constants (golden)
# --------------------------------------------------------------------------
def test_paper_constants_cutoff_and_rates():
    g = json.load(open(os.path.join(HERE, "golden", "paper_constants.json")))
    sc = tiny_scenario()
    assert sc.kid.delta_J == pytest.approx(g["delta_al_ev"]["value"]
                                           * 1.602176634e-19, rel=1e-15)
    cut = 2 * sc.kid.delta_J / ph.H_PLANCK
    assert abs(cut / g["cutoff_hz_about"]["value"] - 1) < g[
        "cutoff_hz_about"]["rel_tol"]
    assert sc.kid.eta_pb == g["eta_pb"]["value"]
    assert sc.t_cmb_K == g["t_cmb_K"]["value"]
    assert sc.telescope.eta_pol == g["eta_pol"]["value"]
    fs = eval(g["deshima_f_sample_hz"]["expr"])
    assert round(fs) == g["deshima_f_sample_hz"]["about"]
    # Ohmic-Al at the reference frequency loses exactly eps_ref
    e = ph.ohmic_eta(np.array([840e9]), 0.0025, 840e9)
    assert e[0] == pytest.approx(1 - g["ohmic_eps_ref"]["value"], abs=1e-16)


def test_gap_cutoff_zeroes_rows_below_2delta():
    nu = np.linspace(80e9, 100e9, 41)
    fil = Filters("lorentz", f_hz=np.array([95e9]), R=np.array([5.0]),
                  eta_peak=np.array([1.0]))
    delta = 188e-6 * 1.602176634e-19
    eta = of.response_matrix(fil, nu, delta)
    below = ph.H_PLANCK * nu < 2 * delta
    assert below.any() and (~below).any()
    assert np.all(eta[below] == 0)
    assert np.all(eta[~below] > 0)


# --------------------------------------------------------------------------
# P9: Johnson-Nyquist limits
# --------------------------------------------------------------------------
def test_planck_limits():
    nu = np.array([1e9, 10e9, 100e9, 350e9])
    T = 1e4
    x = ph.H_PLANCK * nu / (ph.K_BOLTZ * T)
    B = ph.johnson_nyquist(nu, T)
    kT = ph.K_BOLTZ * T
    # Rayleigh-Jeans: B = kT x/(e^x-1) = kT (1 - x/2 + x^2/12 - ...)
    assert np.all(np.abs(B / kT - (1 - x / 2)) <= x ** 2 / 12 * 1.01)
    # Wien: B -> h nu e^{-x} for x >> 1
    nu_w = np.array([2e12])
    Tw = 5.0
    xw = ph.H_PLANCK * nu_w / (ph.K_BOLTZ * Tw)
    assert ph.johnson_nyquist(nu_w, Tw)[0] == pytest.approx(
        ph.H_PLANCK * nu_w[0] * np.exp(-xw[0]), rel=1e-12)
    assert np.all(ph.johnson_nyquist(nu, 0.0) == 0)
    # T -> 0: B = h nu e^{-x} / (1 - e^{-x}) vanishes
    xs = ph.H_PLANCK * nu / (ph.K_BOLTZ * 1e-3)
    bs = ph.johnson_nyquist(nu, 1e-3)
    np.testing.assert_allclose(bs, ph.H_PLANCK * nu * np.exp(-xs)
                               / (-np.expm1(-xs)), rtol=1e-12)
    assert bs[-1] == 0.0


# --------------------------------------------------------------------------
# P10: bilinear exact on ramps and at nodes
# --------------------------------------------------------------------------
def test_bilinear_ramp_and_nodes():
    ny, nx = 7, 11
    yy, xx = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    grid = 0.25 + 2.0 * xx - 3.5 * yy
    rng = np.random.default_rng(0)
    gx = rng.uniform(0, nx - 1, 200)
    gy = rng.uniform(0, ny - 1, 200)
    v, cl = ot.bilinear_clamped(grid, gx, gy)
    assert not cl.any()
    np.testing.assert_allclose(v, 0.25 + 2.0 * gx - 3.5 * gy, rtol=0,
                               atol=1e-12)
    g2 = rng.standard_normal((ny, nx))
    iy, ix = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    v2, _ = ot.bilinear_clamped(g2, ix.ravel().astype(float),
                                iy.ravel().astype(float))
    assert np.array_equal(v2, g2.ravel())
    # out of range takes the edge value and is flagged
    v3, cl3 = ot.bilinear_clamped(grid, np.array([-3.0, nx + 2.0]),
                                  np.array([2.0, 2.0]))
    assert cl3.all()
    np.testing.assert_allclose(v3, [grid[2, 0], grid[2, nx - 1]])


def test_source_zero_outside_grid_and_exact_at_nodes():
    """Closed grid [0, n-1] on both axes; nodes return the cube exactly;
    outside is zero.  Grid spacing is a binary fraction so that positions
    at the edge round-trip exactly."""
    rng = np.random.default_rng(3)
    cube = rng.uniform(1, 2, (9, 9, 4)).astype(np.float32)
    s = Source(cube=cube, az0=-1.0, daz=0.25, el0=0.5, del_=0.125)
    ia = np.array([0, 3, 8, 8, -0.01, 8.01, 4, 2.5])
    ie = np.array([0, 5, 8, 0, 4, 4, -0.2, 8.0])
    P = ot.source_power(s, s.az0 + s.daz * ia, s.el0 + s.del_ * ie)
    np.testing.assert_array_equal(P[0], cube[0, 0])
    np.testing.assert_array_equal(P[1], cube[5, 3])
    np.testing.assert_array_equal(P[2], cube[8, 8])
    np.testing.assert_array_equal(P[3], cube[0, 8])
    assert np.all(P[4:7] == 0)
    np.testing.assert_allclose(P[7], 0.5 * (cube[8, 2].astype(float)
                                            + cube[8, 3]), rtol=1e-15)


def test_lut_follows_exponential_law_between_nodes():
    """The synthetic table is eta_z = exp(-tau(nu) PWV); interpolation in
    optical depth reproduces it at any PWV, and eta_z^csc equals
    exp(-tau PWV csc)."""
    sc = tiny_scenario()
    sp = sc.spectral
    lines = gen.absorption_lines(3, lo_hz=300e9, hi_hz=340e9)
    tau = lines["base_per_mm"] + sum(
        a / (1 + ((sp.nu_hz - n) / g) ** 2)
        for n, g, a in zip(lines["nu_hz"], lines["gamma_hz"],
                           lines["a_per_mm"]))
    pwv = np.array([0.0, 0.35, 0.987654, 1.5, 2.999])
    eta, cl = ot.lut_transmission(sp, pwv)
    assert not cl.any()
    csc = 1 / np.sin(np.pi / 3)
    np.testing.assert_allclose(eta ** csc, np.exp(-np.outer(pwv, tau) * csc),
                               rtol=1e-13)
    # beyond the axis: clamped to the first / last row
    eta2, cl2 = ot.lut_transmission(sp, np.array([99.0, -1.0]))
    assert cl2.all()
    np.testing.assert_allclose(eta2[0], sp.eta_z[-1], rtol=1e-15)
    np.testing.assert_array_equal(eta2[1], sp.eta_z[0])
    # halfway between rows: geometric mean of the two rows
    mid, _ = ot.lut_transmission(sp, np.array([sp.pwv0_mm + 2.5 * sp.dpwv_mm]))
    np.testing.assert_allclose(mid[0], np.sqrt(sp.eta_z[2] * sp.eta_z[3]),
                               rtol=1e-14)


# --------------------------------------------------------------------------
# P1, P2 and equilibrium: cascade
# --------------------------------------------------------------------------
def identity_stages():
    return [Stage("reflect", eta=1.0, t_K=300.0),
            Stage("atm_coupled", eta=1.0),
            Stage("ohmic", eps_ref=0.0, t_K=300.0),
            Stage("refractive", d_m=1e-3, n_index=1.0, tan_delta=0.0,
                  t_K=300.0, t_refl_K=77.0),
            Stage("refractive", d_m=1e-3, n_index=3.4, tan_delta=0.0,
                  t_K=300.0, ar_coated=True)]


def test_p1_unit_efficiencies_reproduce_input():
    sc = tiny_scenario(stages=identity_stages(), uniform=0.0, scan="stare")
    rows = 6
    eta_z, _ = ot.lut_transmission(sc.spectral, np.zeros(rows))
    assert np.all(eta_z == 1.0)
    rng = np.random.default_rng(1)
    psrc = rng.uniform(0, 1e-24, (rows, sc.F))
    P = ot.cascade(sc, eta_z ** 2.0, psrc)
    nu = sc.spectral.nu_hz
    P0 = (ph.aperture_efficiency(nu, sc.telescope) * psrc
          + ph.johnson_nyquist(nu, sc.t_cmb_K))
    np.testing.assert_array_equal(P, P0)


def test_p2_single_stage_closed_form():
    """Atmosphere only: P_1 = e^{-tau PWV csc} P_0 + (1 - e^{...}) B(T_atm)."""
    sc = tiny_scenario(stages=[], scan="stare", source=False)
    sp = sc.spectral
    lines = gen.absorption_lines(3, lo_hz=300e9, hi_hz=340e9)
    tau = lines["base_per_mm"] + sum(
        a / (1 + ((sp.nu_hz - n) / g) ** 2)
        for n, g, a in zip(lines["nu_hz"], lines["gamma_hz"],
                           lines["a_per_mm"]))
    pwv = np.array([sp.dpwv_mm * 20.37])
    csc = 1 / np.sin(np.pi / 3)
    eta_z, _ = ot.lut_transmission(sp, pwv)
    P = ot.cascade(sc, eta_z ** csc, None)[0]
    e = np.exp(-tau * pwv[0] * csc)
    b_cmb = ph.johnson_nyquist(sp.nu_hz, sc.t_cmb_K)
    b_atm = ph.johnson_nyquist(sp.nu_hz, sp.t_atm_K)
    np.testing.assert_allclose(P, e * b_cmb + (1 - e) * b_atm, rtol=1e-13)


def test_thermal_equilibrium_any_cascade():
    """All temperatures equal, no source: a passive cascade in equilibrium
    with its input emits P_JN(T) whatever the efficiencies (Kirchhoff)."""
    T = 150.0
    stages = configs.cascade_table2()
    for st in stages:
        st.t_K = T
        st.t_refl_K = T
    sc = tiny_scenario(stages=stages, source=False)
    sc.t_cmb_K = T
    sc.spectral.t_atm_K = T
    rng = np.random.default_rng(2)
    eta_atm = rng.uniform(0.05, 1.0, (5, sc.F))
    P = ot.cascade(sc, eta_atm, None)
    B = ph.johnson_nyquist(sc.spectral.nu_hz, T)
    np.testing.assert_allclose(P, np.broadcast_to(B, P.shape), rtol=1e-13)


def test_refractive_stage_passes():
    """Non-coated: surface, absorption, surface; AR-coated: absorption only;
    a lossless index-1 slab is transparent."""
    nu = np.array([300e9])
    st = Stage("refractive", d_m=4e-3, n_index=3.41, tan_delta=1e-4,
               t_K=290.0, t_refl_K=77.0)
    passes = ph.stage_passes(st, nu)
    assert [p[2] for p in passes] == [77.0, 290.0, 77.0]
    r = ((1 - 3.41) / (1 + 3.41)) ** 2
    assert passes[0][1][0] == pytest.approx(1 - r, rel=1e-15)
    lam = ph.C_LIGHT / 300e9
    assert passes[1][1][0] == pytest.approx(
        np.exp(-2 * np.pi * 4e-3 * 3.41 * 1e-4 / lam), rel=1e-15)
    st.ar_coated = True
    assert len(ph.stage_passes(st, nu)) == 1
    st2 = Stage("refractive", d_m=4e-3, n_index=1.0, tan_delta=0.0)
    assert all(p[1][0] == 1.0 for p in ph.stage_passes(st2, nu))


# --------------------------------------------------------------------------
# P3, P4: filters and their integrals
# --------------------------------------------------------------------------
def test_p3_filterbank_product_form_and_sum_rule():
    nu = np.linspace(200e9, 460e9, 3001)
    K = 40
    f = 220e9 * 2 ** (np.arange(K) / (K - 1))
    # shuffle channel order to exercise the upstream ordering
    perm = np.random.default_rng(4).permutation(K)
    fil = Filters("filterbank", f_hz=f[perm], R=np.full(K, 300.0),
                  eta_peak=np.full(K, 0.16))
    eta = of.response_matrix(fil, nu, 0.0)
    L = np.stack([1 / (1 + 4 * 300.0 ** 2 * (nu / fk - 1) ** 2)
                  for fk in f[perm]], axis=1)
    # product form: eta_k = eta_p L_k prod_{f_m > f_k} (1 - L_m)
    prod = np.ones_like(eta)
    for k in range(K):
        for m in range(K):
            if f[perm][m] > f[perm][k]:
                prod[:, k] *= 1 - L[:, m]
    np.testing.assert_allclose(eta, 0.16 * L * prod, rtol=1e-12, atol=1e-18)
    resid = 0.16 * np.prod(1 - L, axis=1)
    np.testing.assert_allclose(eta.sum(axis=1) + resid, 0.16, rtol=1e-12)
    top = int(np.argmax(f[perm]))
    np.testing.assert_allclose(eta[:, top], 0.16 * L[:, top], rtol=1e-15)


def test_filterbank_equal_frequencies_lower_index_upstream():
    nu = np.linspace(300e9, 320e9, 201)
    fil = Filters("filterbank", f_hz=np.array([310e9, 310e9]),
                  R=np.array([100.0, 100.0]), eta_peak=np.array([1.0, 1.0]))
    eta = of.response_matrix(fil, nu, 0.0)
    L = of.lorentzian(nu, 310e9, 100.0)
    np.testing.assert_allclose(eta[:, 0], L, rtol=1e-15)
    np.testing.assert_allclose(eta[:, 1], (1 - L) * L, rtol=1e-14)


def test_p4_lorentzian_integrals_pin_contraction():
    """For a flat spectrum P0 the contraction reduces to closed-form
    integrals of the Lorentzian (fine grid, >= 20 bins per FWHM)."""
    f, R, pk = 330e9, 500.0, 0.7
    lo, hi = 300e9, 360e9
    F = 40000
    nu, w = gen.nu_grid(F, lo, hi)
    assert (f / R) / (w[0]) >= 20
    sc = tiny_scenario()
    sc.spectral = Spectral(nu_hz=nu, w_hz=w, eta_z=np.ones((2, F)),
                           pwv0_mm=0, dpwv_mm=1, t_atm_K=0, stages=[],
                           filters=Filters("lorentz", f_hz=np.array([f]),
                                           R=np.array([R]),
                                           eta_peak=np.array([pk])))
    P0 = 3.7e-21
    P = np.full((1, F), P0)
    p_kid, nep2 = ot.contract(sc, P)
    ua, ub = 2 * R * (lo / f - 1), 2 * R * (hi / f - 1)
    I0 = f / (2 * R) * (np.arctan(ub) - np.arctan(ua))
    I1 = f ** 2 / (2 * R) * ((np.arctan(ub) - np.arctan(ua))
                             + (np.log1p(ub ** 2) - np.log1p(ua ** 2)) / (4 * R))
    I2 = f / (2 * R) * ((ub / (2 * (1 + ub ** 2)) - ua / (2 * (1 + ua ** 2)))
                        + (np.arctan(ub) - np.arctan(ua)) / 2)
    gap = 2 * sc.kid.delta_J / sc.kid.eta_pb
    assert p_kid[0, 0] == pytest.approx(P0 * pk * I0, rel=2e-6)
    expect = 2 * (P0 * pk * (ph.H_PLANCK * I1 + gap * I0) + P0 ** 2 * pk ** 2 * I2)
    assert nep2[0, 0] == pytest.approx(expect, rel=2e-6)


# --------------------------------------------------------------------------
# P11: brute force on tiny shapes
# --------------------------------------------------------------------------
@pytest.mark.parametrize("filt", ["filterbank", "lorentz", "matrix"])
def test_p11_brute_force_tiny(filt):
    sc = tiny_scenario(filt=filt, stages=configs.cascade_table2())
    out = ot.simulate(sc)
    sp = sc.spectral
    F, K, P, T = sc.F, sc.K, sc.n_pix, sc.t_total
    h, kB, c = ph.H_PLANCK, ph.K_BOLTZ, ph.C_LIGHT

    def B(nu, T_):
        return 0.0 if T_ <= 0 else h * nu / np.expm1(h * nu / (kB * T_))

    def lor(nu, f, R):
        return 1 / (1 + 4 * R * R * (nu / f - 1) ** 2)

    # filter matrix by scalar loops
    eta = np.zeros((F, K))
    for j in range(F):
        if filt == "matrix":
            for k in range(K):
                eta[j, k] = sp.filters.matrix[j, k]
        elif filt == "lorentz":
            for k in range(K):
                eta[j, k] = sp.filters.eta_peak[k] * lor(
                    sp.nu_hz[j], sp.filters.f_hz[k], sp.filters.R[k])
        else:
            # channels are ordered by ascending f: fill from the top
            for k in reversed(range(K)):
                up = sum(eta[j, m] for m in range(k + 1, K))
                eta[j, k] = (sp.filters.eta_peak[k] - up) * lor(
                    sp.nu_hz[j], sp.filters.f_hz[k], sp.filters.R[k])
    tel = sc.telescope
    for p in range(P):
        for n in range(T):
            t = n / sc.f_sample_hz
            s = sc.scan
            phi = s.r_petal * np.cos(s.Omega * t) * np.sin(s.omega * t)
            the = s.r_petal * np.sin(s.Omega * t) * np.sin(s.omega * t)
            x = sc.screen.h_column_m * np.tan(phi + sc.dphi[p]) + \
                sc.screen.wind_mps * t
            y = sc.screen.h_column_m * np.tan(the + sc.dtheta[p])
            gx = x / sc.screen.dx_m + sc.screen.ix0
            gy = y / sc.screen.dy_m + sc.screen.iy0
            cx, cy = int(np.floor(gx)), int(np.floor(gy))
            wx, wy = gx - cx, gy - cy
            S = sc.screen.pwv_mm
            pwv = ((1 - wx) * (1 - wy) * S[cy, cx] + wx * (1 - wy) * S[cy, cx + 1]
                   + (1 - wx) * wy * S[cy + 1, cx] + wx * wy * S[cy + 1, cx + 1])
            gl = (pwv - sp.pwv0_mm) / sp.dpwv_mm
            il = int(np.floor(gl))
            wl = gl - il
            el = the + s.theta0 + sc.dtheta[p]
            az = phi + s.phi0 + sc.dphi[p]
            src = sc.source
            ga = (az - src.az0) / src.daz
            ge = (el - src.el0) / src.del_
            ia, ie = int(np.floor(ga)), int(np.floor(ge))
            wa, we = ga - ia, ge - ie
            for j in range(F):
                nu = sp.nu_hz[j]
                ez = np.exp((1 - wl) * np.log(sp.eta_z[il, j])
                            + wl * np.log(sp.eta_z[il + 1, j]))
                ea = ez ** (1 / np.sin(el))
                C = src.cube.astype(np.float64)
                ps = ((1 - wa) * (1 - we) * C[ie, ia, j] + wa * (1 - we) * C[ie, ia + 1, j]
                      + (1 - wa) * we * C[ie + 1, ia, j] + wa * we * C[ie + 1, ia + 1, j])
                eps = tel.eta_taper * np.exp(-(4 * np.pi * tel.rho_surf_m * nu / c) ** 2) * tel.eta_pol
                Pj = eps * ps + B(nu, sc.t_cmb_K)
                Pj = ea * Pj + (1 - ea) * B(nu, sp.t_atm_K)
                for st in sp.stages:
                    for kind, e, tk in ph.stage_passes(st, np.array([nu])):
                        par = (B(nu, tk) if kind == "fixed" else
                               (1 - ea) * B(nu, sp.t_atm_K) + ea * B(nu, sc.t_cmb_K))
                        Pj = e[0] * Pj + (1 - e[0]) * par
                eta_col = eta[j]
                if j == 0:
                    pk = np.zeros(K)
                    n2 = np.zeros(K)
                pk += sp.w_hz[j] * eta_col * Pj
                n2 += 2 * sp.w_hz[j] * eta_col * Pj * (
                    h * nu + eta_col * Pj + 2 * sc.kid.delta_J / sc.kid.eta_pb)
            np.testing.assert_allclose(out["p_kid"][p, :, n], pk, rtol=1e-12)
            sig = np.sqrt(n2) * np.sqrt(sc.f_sample_hz / 2)
            np.testing.assert_allclose(out["sigma"][p, :, n], sig, rtol=1e-12)
            for k in range(K):
                z = op.white_normal(sc.seed, n, k, p)
                assert out["tod"][p, k, n] == pytest.approx(pk[k] + sig[k] * z,
                                                            rel=1e-12)


# --------------------------------------------------------------------------
# scan geometry
# --------------------------------------------------------------------------
def test_daisy_bounds_and_origin():
    sc = tiny_scenario()
    n = np.arange(0, 20000)
    phi, the = ot.scan_offsets(sc, n)
    assert phi[0] == 0 and the[0] == 0
    assert np.all(np.hypot(phi, the) <= sc.scan.r_petal * (1 + 1e-15))
    # radius |sin(omega t)| r
    t = n / sc.f_sample_hz
    np.testing.assert_allclose(np.hypot(phi, the),
                               sc.scan.r_petal * np.abs(np.sin(sc.scan.omega * t)),
                               rtol=1e-12, atol=1e-20)


def test_wind_advances_screen_coordinate():
    sc = tiny_scenario(scan="stare")
    g0 = ot.row_geometry(sc, 0, np.array([0]))
    # stare on a ramp screen: PWV changes by slope * u_w / f_s / dx per sample
    ny, nx = sc.screen.pwv_mm.shape
    sc.screen.pwv_mm = np.tile(1.0 + 0.01 * np.arange(nx), (ny, 1))
    n = np.arange(0, 5)
    g = ot.row_geometry(sc, 0, n)
    step = 0.01 * sc.screen.wind_mps / sc.f_sample_hz / sc.screen.dx_m
    np.testing.assert_allclose(np.diff(g["pwv"]), step, rtol=1e-9)
    assert g0["csc"][0] == pytest.approx(1 / np.sin(np.pi / 3 + sc.dtheta[0]))


def test_zenith_airmass_is_identity():
    sc = tiny_scenario(scan="stare", source=False, stages=[])
    sc.scan.theta0 = np.pi / 2
    sc.dtheta[:] = 0
    g = ot.row_geometry(sc, 0, np.array([0]))
    assert g["csc"][0] == 1.0


# --------------------------------------------------------------------------
# P8: Philox against rocRAND's engine; P6 and P7: noise statistics
# --------------------------------------------------------------------------
@pytest.fixture(scope="module")
def rocrand_probe():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    d = tempfile.mkdtemp()
    exe = os.path.join(d, "probe")
    r = subprocess.run([hipcc, "-x", "hip", "--offload-arch=gfx950", "-O1",
                        os.path.join(HERE, "rocrand_philox_probe.cpp"),
                        "-o", exe], capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("could not build the rocRAND probe: " + r.stderr[-400:])
    return exe


@pytest.mark.parametrize("seed,n,k,p,s", [
    (0x123456789ABCDEF, 0, 0, 0, 0), (1, 5, 3, 2, 0), (2**63 + 12345, 77, 346, 48, 1),
    (42, 2**31 + 7, 700, 3, 1), (0, 0, 0, 0, 0)])
def test_p8_philox_matches_rocrand(rocrand_probe, seed, n, k, p, s):
    """Counter (n, k, p, s) under key seed: rocRAND's subsequence fills
    counter words 2-3 and its offset (in 32-bit outputs) words 0-1."""
    sub = p | (s << 32)
    off = 4 * (n + (k << 32))
    r = subprocess.run([rocrand_probe, str(seed), str(sub), str(off), "8"],
                       capture_output=True, text=True, check=True)
    ref = np.array([int(v) for v in r.stdout.split()], dtype=np.uint32)
    o = op.philox4x32_10(np.array([n, n + 1]), k, p, s, op.key_of(seed))
    mine = np.stack(o, axis=1).ravel()
    np.testing.assert_array_equal(mine, ref)


def test_uniforms_exact_and_open_interval():
    o = np.array([0, 0xFFFFFFFF, 0x1FF, 0x200, 0x80000000], dtype=np.uint32)
    u = op.to_uniform(o)
    assert u[0] == 2.0 ** -24 and u[1] == 1 - 2.0 ** -24
    assert u[2] == u[0] and u[3] == 3 * 2.0 ** -24
    assert u[4] == 0.5 + 2.0 ** -24
    assert np.all(u.astype(np.float32).astype(np.float64) == u)


def test_p6_photon_noise_variance_and_mean():
    sc = configs.c1(uniform_screen=True, t_total=96000)
    sc.source = None
    out = ot.simulate(sc, pixels=[0])
    z = (out["tod"] - out["p_kid"]) / out["sigma"]
    T = z.shape[-1]
    # sigma is constant in time for a uniform stare
    assert np.all(np.ptp(out["sigma"], axis=-1) <= 1e-12 * out["sigma"][..., 0])
    var = z.var(axis=-1)
    band = 5 * np.sqrt(2 / T)
    assert np.all(np.abs(var - 1) < band)
    assert np.all(np.abs(z.mean(axis=-1)) < 5 / np.sqrt(T))
    # channels are independent
    c = np.corrcoef(z[0, :8])
    assert np.all(np.abs(c[~np.eye(8, dtype=bool)]) < 5 / np.sqrt(T))


def test_p7_pink_expected_variance_and_psd():
    """Averaged over series, var(x) -> sum_j S(f_j) df and the periodogram
    follows A f^-alpha; Parseval holds for each realisation."""
    T, fs, alpha, A = 4096, 160.0, 1.0, 2.5e-34
    N = opk.fft_length(T)
    assert N == T
    n_ser = 400
    xs = np.stack([opk.series(9, p, 0, A, alpha, T, fs) for p in range(n_ser)])
    j = np.arange(1, N // 2)
    f = j * fs / N
    S = A * f ** -alpha
    expect_var = np.sum(S) * fs / N
    v = xs.var(axis=1) + xs.mean(axis=1) ** 2  # mean is exactly zero
    assert abs(xs.mean()) < 1e-12 * np.sqrt(expect_var)
    assert v.mean() == pytest.approx(expect_var, rel=5 * v.std() / np.sqrt(n_ser) / expect_var)
    X = np.fft.rfft(xs, axis=1)
    per = 2.0 / (N * fs) * np.abs(X[:, 1:N // 2]) ** 2
    ratio = per.mean(axis=0) / S
    assert abs(ratio.mean() - 1) < 0.02
    slope = np.polyfit(np.log(f), np.log(per.mean(axis=0)), 1)[0]
    assert slope == pytest.approx(-alpha, abs=0.03)
    Xs = opk.spectrum(9, 0, 0, A, alpha, T, fs)
    x0 = xs[0]
    assert np.sum(x0 ** 2) == pytest.approx(
        (2 * np.sum(np.abs(Xs[1:-1]) ** 2)) / N, rel=1e-12)


def test_pink_short_series_edge_cases():
    assert opk.fft_length(1) == 2 and opk.fft_length(2) == 2
    assert opk.fft_length(3) == 4 and opk.fft_length(1600) == 2048
    x = opk.series(1, 0, 0, 1e-34, 1.0, 1, 160.0)
    assert x.shape == (1,) and x[0] == 0.0


# --------------------------------------------------------------------------
# P5: uniform screen gives a constant TOD
# --------------------------------------------------------------------------
def test_p5_uniform_screen_constant_tod():
    sc = configs.c1(noise=False, uniform_screen=True, t_total=400)
    out = ot.simulate(sc)
    pk = out["p_kid"]
    assert np.max(np.ptp(pk, axis=-1) / pk.mean(axis=-1)) < 1e-14
    assert np.array_equal(out["tod"], pk)


def test_sky_coupled_stage_limits():
    """A sky-coupled stage sees the CMB through a transparent sky and the
    atmosphere's own emission through an opaque one."""
    sc = tiny_scenario(stages=[Stage("atm_coupled", eta=0.5)], source=False)
    nu = sc.spectral.nu_hz
    b_cmb = ph.johnson_nyquist(nu, sc.t_cmb_K)
    b_atm = ph.johnson_nyquist(nu, sc.spectral.t_atm_K)
    P = ot.cascade(sc, np.ones((1, sc.F)), None)[0]
    np.testing.assert_allclose(P, b_cmb, rtol=1e-15)
    P = ot.cascade(sc, np.zeros((1, sc.F)), None)[0]
    np.testing.assert_allclose(P, b_atm, rtol=1e-15)
    sc.spectral.stages = [Stage("atm_coupled", eta=0.25)]
    P = ot.cascade(sc, np.full((1, sc.F), 0.5), None)[0]
    P1 = 0.5 * b_cmb + 0.5 * b_atm
    np.testing.assert_allclose(P, 0.25 * P1 + 0.75 * P1, rtol=1e-15)


def test_daisy_petal_direction_rotates_at_Omega():
    sc = tiny_scenario()
    n = np.arange(1, 3000)
    phi, the = ot.scan_offsets(sc, n)
    t = n / sc.f_sample_hz
    s = np.sin(sc.scan.omega * t)
    ok = np.abs(s) > 0.1
    ang = np.arctan2(the * np.sign(s), phi * np.sign(s))
    d = np.angle(np.exp(1j * (ang - sc.scan.Omega * t)))
    assert np.max(np.abs(d[ok])) < 1e-9


def test_screen_coordinates_exclude_scan_offset():
    """Eq. xy_atm uses phi(t)+dphi and theta(t)+dtheta only: a stare at
    theta0 = 60 deg reads the screen at y = h tan(dtheta), not at the
    boresight elevation."""
    sc = tiny_scenario(scan="stare", source=False)
    ny, nx = sc.screen.pwv_mm.shape
    yy, xx = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    sc.screen.pwv_mm = 1.0 + 0.01 * xx + 0.02 * yy
    g = ot.row_geometry(sc, 1, np.array([0, 3]))
    assert not g["screen_clamped"].any()
    t = np.array([0, 3]) / sc.f_sample_hz
    gx = (sc.screen.h_column_m * np.tan(sc.dphi[1]) + sc.screen.wind_mps * t) \
        / sc.screen.dx_m + sc.screen.ix0
    gy = sc.screen.h_column_m * np.tan(sc.dtheta[1]) / sc.screen.dy_m \
        + sc.screen.iy0
    np.testing.assert_allclose(g["pwv"], 1.0 + 0.01 * gx + 0.02 * gy,
                               rtol=1e-12)


def test_source_sampled_at_full_pointing():
    """Stare at the cube centre: pixel 0 sees the centre spectrum; a pixel
    offset by one grid step sees the neighbouring node."""
    sc = tiny_scenario(scan="stare")
    s = sc.source
    sc.dphi = np.array([0.0, s.daz])
    sc.dtheta = np.array([0.0, 0.0])
    for p, col in ((0, 4), (1, 5)):
        g = ot.row_geometry(sc, p, np.array([0]))
        P = ot.source_power(s, g["az"], g["el"])
        np.testing.assert_allclose(P[0], s.cube[4, col], rtol=1e-9)


# --------------------------------------------------------------------------
# Kelvin output by skydip (section 2.7)
# --------------------------------------------------------------------------
def test_skydip_brightness_limits():
    """A transparent sky has T_b = 0; an opaque one T_b = T_atm."""
    from oracle import skydip as osd
    sc = tiny_scenario(F=16, K=3)
    sp = sc.spectral
    sp.eta_z = np.vstack([np.ones(sc.F), np.full(sc.F, 1e-300)])
    sp.pwv0_mm, sp.dpwv_mm = 0.0, 1.0
    _, _, t_b = osd.sweep(sc, np.pi / 2, 0.0, 1.0, 2)
    np.testing.assert_allclose(t_b[0], 0.0, atol=1e-12)
    np.testing.assert_allclose(t_b[1], sp.t_atm_K, rtol=1e-12)


def test_skydip_exact_for_single_bin_channels():
    """Channels that see one frequency bin each make power exactly linear in
    T_b: the fit reproduces every sweep point, with slope D_j / T_atm per
    unit weight (D = power difference between opaque and clear sky)."""
    from oracle import skydip as osd
    F, K = 12, 4
    sc = tiny_scenario(F=F, K=K, filt="matrix", stages=configs.cascade_c2())
    m = np.zeros((F, K))
    for k, j in enumerate((1, 4, 7, 10)):
        m[j, k] = 0.3 + 0.1 * k
    sc.spectral.filters.matrix = m
    el = np.pi / 3
    pwv, p_kid, t_b = osd.sweep(sc, el, 0.2, 2.5, 9)
    a, b = osd.fit(p_kid, t_b)
    np.testing.assert_allclose(a + b * t_b, p_kid, rtol=1e-12)
    clear = ot.cascade(sc, np.ones((1, F)), None)[0]
    opaque = ot.cascade(sc, np.zeros((1, F)), None)[0]
    for k, j in enumerate((1, 4, 7, 10)):
        wq = sc.spectral.w_hz[j] * m[j, k]
        assert a[k] == pytest.approx(wq * clear[j], rel=1e-12)
        assert b[k] == pytest.approx(wq * (opaque[j] - clear[j])
                                     / sc.spectral.t_atm_K, rel=1e-12)


def test_to_kelvin_inverts_the_line():
    from oracle import skydip as osd
    a = np.array([1.0, 2.0])
    b = np.array([0.5, 4.0])
    T = np.random.default_rng(0).uniform(0, 300, (3, 2, 7))
    P = a[None, :, None] + b[None, :, None] * T
    np.testing.assert_allclose(osd.to_kelvin(P, a, b), T, rtol=1e-14)


def test_skydip_fit_matches_polyfit_and_flags_degenerate_channels():
    """The closed-form fit agrees with numpy's least-squares polynomial fit;
    a constant or undefined T_b column gives NaN."""
    from oracle import skydip as osd
    rng = np.random.default_rng(11)
    t = rng.uniform(5, 60, (40, 4))
    p = 3e-12 + 2e-14 * t + rng.normal(0, 1e-16, t.shape)
    t[:, 2] = 7.0
    t[:, 3] = np.nan
    a, b = osd.fit(p, t)
    for k in range(2):
        bk, ak = np.polyfit(t[:, k], p[:, k], 1)
        assert a[k] == pytest.approx(ak, rel=1e-10)
        assert b[k] == pytest.approx(bk, rel=1e-10)
    assert np.isnan(a[2:]).all() and np.isnan(b[2:]).all()


def test_skydip_dead_channel_has_no_scale():
    from oracle import skydip as osd
    F, K = 12, 2
    sc = tiny_scenario(F=F, K=K, filt="matrix")
    m = np.zeros((F, K))
    m[3, 0] = 0.5
    sc.spectral.filters.matrix = m
    a, b = osd.skydip(sc, np.pi / 3, 0.3, 2.0, 5)
    assert np.isfinite(a[0]) and np.isfinite(b[0]) and b[0] > 0
    assert np.isnan(a[1]) and np.isnan(b[1])


# --------------------------------------------------------------------------
# common-mode subtraction and gridding (section 4.3)
# --------------------------------------------------------------------------
def _reduce_scenario(T=400, P=7):
    sc = tiny_scenario(F=30, K=4, P=P, T=T, filt="lorentz")
    return sc


def test_channel_transmission_single_bin_and_airmass():
    """Single-bin channels see exactly that bin's table transmission; the
    transmission at elevation 30 degrees is the zenith one squared, and at
    the zenith it is the zenith one."""
    from oracle import reduce as orr
    F, K = 10, 3
    sc = tiny_scenario(F=F, K=K, P=1, T=4, filt="matrix", scan="stare")
    m = np.zeros((F, K))
    bins = (2, 5, 8)
    for k, j in enumerate(bins):
        m[j, k] = 0.4
    sc.spectral.filters.matrix = m
    sp = sc.spectral
    row = 37
    pwv = sp.pwv0_mm + row * sp.dpwv_mm
    ez = orr.channel_zenith_transmission(sc, pwv)
    np.testing.assert_allclose(ez, sp.eta_z[row, list(bins)], rtol=1e-13)
    sc.dtheta = np.zeros(1)
    sc.scan.theta0 = np.pi / 2
    np.testing.assert_allclose(orr.spaxel_transmission(sc, ez, np.arange(4))[0],
                               np.repeat(ez[:, None], 4, axis=1), rtol=1e-14)
    sc.scan.theta0 = np.pi / 6
    np.testing.assert_allclose(orr.spaxel_transmission(sc, ez, np.arange(4))[0],
                               np.repeat(ez[:, None] ** 2, 4, axis=1), rtol=1e-13)


def test_common_mode_removes_a_common_atmosphere():
    """T_b = T_sky(t, k) (1 - eta_i) + s_i with s = 0 off source gives
    T* = s_i / eta_i on source and 0 off source, whatever T_sky is."""
    from oracle import reduce as orr
    sc = _reduce_scenario()
    P, K, T = sc.n_pix, sc.K, sc.t_total
    r_out = 10 * gen.ARCSEC            # hexagon: centre on, ring off
    S = orr.off_source(sc, r_out)
    assert S.sum() == P - 1 and not S[0]
    pwv = 0.9
    eta = orr.spaxel_transmission(sc, orr.channel_zenith_transmission(sc, pwv),
                                  np.arange(T))
    rng = np.random.default_rng(5)
    t_sky = rng.uniform(250, 280, (K, T))
    s = np.zeros((P, K, T))
    s[0] = rng.normal(0, 1e-3, (K, T))
    t_b = t_sky[None] * (1 - eta) + s
    ts = orr.common_mode(sc, t_b, pwv, r_out)
    np.testing.assert_allclose(ts[0], s[0] / eta[0], rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(ts[1:], 0.0, atol=1e-11)
    with pytest.raises(ValueError):
        orr.common_mode(sc, t_b, pwv, 1.0)


def test_gridding_matches_brute_force_loops():
    """Per-spaxel cell statistics against explicit per-sample loops."""
    from oracle import reduce as orr
    sc = _reduce_scenario(T=300, P=3)
    rng = np.random.default_rng(9)
    tod = rng.normal(1.0, 0.2, (3, sc.K, 300))
    half, n = 50 * gen.ARCSEC, 5
    count, mean, var = orr.spaxel_maps(sc, tod, half, n)
    d = 2 * half / (n - 1)
    for p in range(3):
        acc = {}
        for t in range(300):
            phi = sc.scan.r_petal * np.cos(sc.scan.Omega * t / 160.0) * np.sin(sc.scan.omega * t / 160.0)
            th = sc.scan.r_petal * np.sin(sc.scan.Omega * t / 160.0) * np.sin(sc.scan.omega * t / 160.0)
            ix = int(np.floor((phi + sc.dphi[p] + half) / d + 0.5))
            iy = int(np.floor((th + sc.dtheta[p] + half) / d + 0.5))
            if 0 <= ix < n and 0 <= iy < n:
                acc.setdefault(iy * n + ix, []).append(t)
        for c in range(n * n):
            ts = acc.get(c, [])
            assert count[p, c] == len(ts)
            for k in range(sc.K):
                if len(ts) >= 2:
                    v = tod[p, k, ts]
                    assert mean[p, k, c] == pytest.approx(np.mean(v), rel=1e-12)
                    assert var[p, k, c] == pytest.approx(np.var(v, ddof=1), rel=1e-10)
                else:
                    assert np.isnan(mean[p, k, c]) and np.isnan(var[p, k, c])
    assert count.sum() > 0.8 * 3 * 300


def test_inverse_variance_combination_closed_form():
    """Two spaxels with identical cells: means m1, m2 with variances
    s1^2 = 1, s2^2 = 4 over equal counts m combine to (4 m1 + m2) / 5 with
    weight 5 m / 4; a cell only one spaxel reaches takes its mean."""
    from oracle import reduce as orr
    C = 3
    count = np.array([[4.0, 4.0, 4.0], [4.0, 4.0, 1.0]])
    mean = np.array([[[1.0, 2.0, 3.0]], [[3.0, -1.0, 9.0]]])
    var = np.array([[[1.0, 1.0, 1.0]], [[4.0, 4.0, np.nan]]])
    m, w = orr.combine(count, mean, var)
    assert m.shape == (1, C)
    np.testing.assert_allclose(m[0, :2], [(4 * 1 + 3) / 5, (4 * 2 - 1) / 5])
    np.testing.assert_allclose(w[0, :2], [5.0, 5.0])
    assert m[0, 2] == 3.0 and w[0, 2] == 4.0


# --------------------------------------------------------------------------
# input preparation (section 2.2)
# --------------------------------------------------------------------------
def test_far_field_uniform_aperture_is_airy():
    """No taper: the far field of a uniformly lit disc is the Airy pattern
    [2 J1(x) / x]^2, x = 2 pi rho R / lambda."""
    from scipy import special
    from oracle import inputs as oin
    nu, R = 300e9, 5.0
    lam = 299792458.0 / nu
    rho = np.array([0.0, 1e-6, 5 * gen.ARCSEC, 11 * gen.ARCSEC, 30 * gen.ARCSEC])
    got = oin.far_field(rho, nu, R, 0.0)
    x = 2 * np.pi * rho[1:] * R / lam
    np.testing.assert_allclose(got[1:], (2 * special.j1(x) / x) ** 2,
                               rtol=1e-9, atol=1e-14)
    assert got[0] == pytest.approx(1.0, abs=1e-14)


def test_far_field_taper_widens_the_beam():
    from oracle import inputs as oin
    rho = 15 * gen.ARCSEC
    f0 = oin.far_field(rho, 350e9, 5.0, 0.0)
    f10 = oin.far_field(rho, 350e9, 5.0, -10.0)
    assert 0 < f0 < f10 < 1


def test_source_convolution_of_a_single_node():
    """A source in one grid node spreads as A_p I cos(theta') dphi dtheta
    F(distance)."""
    from oracle import inputs as oin
    n, F = 5, 2
    nu = np.array([250e9, 400e9])
    d = 10 * gen.ARCSEC
    el0 = 0.8
    I = np.zeros((n, n, F))
    I[1, 3, :] = [2e-18, 5e-18]
    P = oin.convolve_source(I, nu, -2 * d, d, el0, d, 5.0, -10.0)
    for f in range(F):
        for j in range(n):
            for i in range(n):
                rho = np.hypot((i - 3) * d, (j - 1) * d)
                exp = (np.pi * 25.0 * d * d * I[1, 3, f] * np.cos(el0 + d)
                       * oin.far_field(rho, nu[f], 5.0, -10.0))
                assert P[j, i, f] == pytest.approx(exp, rel=1e-12)


def test_screen_footprint_constant_delta_and_edges():
    """Constant screens are unchanged; a unit cell in the interior spreads
    into the normalised weights; edges clamp (brute-force loops)."""
    from oracle import inputs as oin
    dx = dy = 0.5
    R, te = 1.6, -12.0
    w = oin.footprint_weights(dx, dy, R, te)
    assert w.shape == (7, 7) and w.sum() == pytest.approx(1.0, rel=1e-15)
    assert w[0, 0] == 0.0 and w[3, 3] == w.max()
    np.testing.assert_allclose(oin.convolve_screen(np.full((9, 12), 0.7), dx,
                                                   dy, R, te), 0.7, rtol=1e-14)
    s = np.zeros((11, 13))
    s[5, 6] = 1.0
    out = oin.convolve_screen(s, dx, dy, R, te)
    np.testing.assert_allclose(out[2:9, 3:10], w[::-1, ::-1], rtol=1e-14)
    rng = np.random.default_rng(4)
    s = rng.uniform(0.5, 1.5, (6, 8))
    out = oin.convolve_screen(s, dx, dy, R, te)
    for y in range(6):
        for x in range(8):
            acc = 0.0
            for a in range(-3, 4):
                for b in range(-3, 4):
                    acc += w[a + 3, b + 3] * s[min(max(y + a, 0), 5),
                                               min(max(x + b, 0), 7)]
            assert out[y, x] == pytest.approx(acc, rel=1e-13)
