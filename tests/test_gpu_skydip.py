"""Brightness-temperature output (simulated skydip, section 2.7): the GPU
skydip against the oracle's, and KELVIN jobs against the oracle's TOD put
on the oracle's scale.

Tolerances: the sweep and the fit are FP64 on both sides, so p_kid, t_b, a
and b agree within 1e-9 relative.  A KELVIN TOD is T = (P - a) / b; an
error e |P| in watts is e |P| / |b| kelvin, so the bar of the watts TOD
(1e-6 relative) reads |T_gpu - T_oracle| |b| <= 1e-6 |P_oracle|, and the
1/f part keeps its bar of 1e-5 of its rms.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2604_23305_amd as g
from oracle import pink as opk
from oracle import skydip as osd
from paper_2604_23305_amd.binding import GtodError
from tests.gpu_util import new_ctx
from tests.test_oracle_pins import tiny_scenario
from workloads import configs

pytestmark = pytest.mark.gpu

TOL_FIT = 1e-9
TOL_TOD = 1e-6
TOL_PINK = 1e-5


@pytest.fixture(scope="module")
def ctx():
    c = new_ctx()
    yield c
    g.free(c)


def _check_sweep(ctx, sc, el, lo, hi, n):
    run = g.ScenarioRun(ctx, sc)
    a, b, pk, tb = g.skydip(ctx, run.spec_id, sc.K, el, lo, hi, n,
                            return_sweep=True)
    _, pk_o, tb_o = osd.sweep(sc, el, lo, hi, n)
    a_o, b_o = osd.fit(pk_o, tb_o)
    live = np.isfinite(b_o)
    for name, got, ref in (("p_kid", pk, pk_o), ("t_b", tb[:, live], tb_o[:, live]),
                           ("a", a[live], a_o[live]), ("b", b[live], b_o[live])):
        err = np.where(ref == 0, np.abs(got),
                       np.abs(got - ref) / np.where(ref == 0, 1.0, np.abs(ref)))
        print(f"  {name}: max rel err {err.max():.2e}", flush=True)
        assert err.max() <= TOL_FIT, name
    assert np.array_equal(np.isnan(a), ~live) and np.array_equal(np.isnan(b), ~live)
    return run, a, b


def test_skydip_tiny_matches_oracle(ctx):
    sc = tiny_scenario(F=40, K=5, P=1, T=8)
    _check_sweep(ctx, sc, np.pi / 3, 0.2, 2.4, 37)


def test_skydip_filterbank_full_spectral_size(ctx):
    """347-channel filterbank over 3000 bins with the six-pass cascade,
    at the 60 degree observing elevation."""
    sc = configs.c2(t_total=256, screen_shape=(64, 4096))
    _check_sweep(ctx, sc, configs.THETA0, 0.3, 3.0, 64)


def test_skydip_clamps_and_dead_channels(ctx):
    """Sweep reaching past the table axis (clamped on both sides) and a
    channel without response (no scale)."""
    sc = tiny_scenario(F=24, K=3, P=1, T=8, filt="matrix")
    sc.spectral.filters.matrix[:, 2] = 0.0
    top = sc.spectral.pwv0_mm + (sc.spectral.eta_z.shape[0] - 1) * sc.spectral.dpwv_mm
    _check_sweep(ctx, sc, 0.7, -0.5, top + 0.5, 20)


def test_skydip_argument_errors(ctx):
    sc = tiny_scenario(F=16, K=3, P=1, T=8)
    run = g.ScenarioRun(ctx, sc)
    out = run.alloc()
    with pytest.raises(GtodError, match="EINVAL"):
        g.simulate_tod(ctx, [run.signal_job(out, kelvin=True)])
    for el, lo, hi, n in ((0.0, 0.1, 1.0, 8), (np.pi, 0.1, 1.0, 8),
                          (1.0, 1.0, 1.0, 8), (1.0, 0.1, 1.0, 1),
                          (1.0, 0.1, 1.0, g._abi.SKYDIP_MAX_N + 1),
                          (1.0, np.nan, 1.0, 8)):
        with pytest.raises(GtodError, match="EINVAL"):
            g.skydip(ctx, run.spec_id, sc.K, el, lo, hi, n)
    with pytest.raises(GtodError, match="ENOTFOUND"):
        g.skydip(ctx, 987654, sc.K, 1.0, 0.1, 1.0, 8)
    strict = new_ctx(strict_range=True, workspace_bytes=64 << 20)
    try:
        r2 = g.ScenarioRun(strict, sc)
        with pytest.raises(GtodError, match="ERANGE"):
            g.skydip(strict, r2.spec_id, sc.K, 1.0, -1.0, 1.0, 8)
        g.skydip(strict, r2.spec_id, sc.K, 1.0, 0.1, 1.0, 8)
    finally:
        g.free(strict)


def _kelvin_bar(got_K, exp_W, a, b):
    exp_K = (exp_W - a[None, :, None]) / b[None, :, None]
    err = np.abs(got_K - exp_K) * np.abs(b)[None, :, None] / np.abs(exp_W)
    print(f"  kelvin tod: max err (W-relative) {err.max():.2e}", flush=True)
    return err.max()


@pytest.mark.parametrize("precision", [g.PREC_FP32, g.PREC_SPLIT_BF16])
def test_kelvin_signal_matches_oracle(ctx, precision):
    """Signal and photon noise, several contraction tiles and a ragged
    tail, in kelvin."""
    sc = configs.c2(t_total=700, screen_shape=(64, 4096), F=600, K=70)
    run = g.ScenarioRun(ctx, sc)
    a_o, b_o = osd.skydip(sc, sc.scan.theta0, 0.3, 3.0, 48)
    a, b = g.skydip(ctx, run.spec_id, sc.K, sc.scan.theta0, 0.3, 3.0, 48)
    np.testing.assert_allclose(a, a_o, rtol=TOL_FIT)
    np.testing.assert_allclose(b, b_o, rtol=TOL_FIT)
    out = run.alloc(with_p_kid=True)
    g.simulate_tod(ctx, [run.signal_job(out, precision=precision,
                                        kelvin=True)])
    torch.cuda.synchronize()
    ref = oracle.tod.simulate(sc)
    assert _kelvin_bar(out.tod.cpu().numpy(), ref["tod"], a_o, b_o) <= TOL_TOD
    # the noise-free power stays in watts
    err = np.abs(out.p_kid.cpu().numpy() - ref["p_kid"]) / np.abs(ref["p_kid"])
    assert err.max() <= TOL_TOD


def test_kelvin_pink_and_accumulate(ctx):
    """1/f noise job in kelvin, then signal accumulated on top: the sum is
    the oracle's (tod + pink - a) / b."""
    sc = tiny_scenario(F=48, K=4, P=2, T=3000)
    sc.photon_noise = True
    sc.pink_alpha = np.array([1.0, 0.5, 2.0, 1.5])
    sc.pink_knee_hz = 1.0
    run = g.ScenarioRun(ctx, sc)
    a_o, b_o = osd.skydip(sc, sc.scan.theta0, 0.2, 2.5, 33)
    g.skydip(ctx, run.spec_id, sc.K, sc.scan.theta0, 0.2, 2.5, 33)
    tod = torch.zeros((sc.n_pix, sc.K, sc.t_total), device="cuda")
    g.simulate_tod(ctx, [run.pink_job(tod, accumulate=False, kelvin=True)])
    torch.cuda.synchronize()
    pink_K = tod.cpu().numpy()
    nep2 = oracle.tod.reference_nep2(sc)
    A = opk.amplitude(nep2, sc.pink_alpha, sc.pink_knee_hz)
    pink_W = np.stack([np.stack([opk.series(sc.seed, p, k, A[k],
                                            sc.pink_alpha[k], sc.t_total,
                                            sc.f_sample_hz)
                                 for k in range(sc.K)])
                       for p in range(sc.n_pix)])
    for p in range(sc.n_pix):
        for k in range(sc.K):
            ref = pink_W[p, k] / b_o[k]
            err = np.abs(pink_K[p, k] - ref).max() / ref.std()
            assert err <= TOL_PINK, (p, k, err)
    out = g.Outputs(tod=tod, t0=0, length=sc.t_total)
    g.simulate_tod(ctx, [run.signal_job(out, accumulate=True, kelvin=True)])
    torch.cuda.synchronize()
    ref = oracle.tod.simulate(sc)
    exp_W = ref["tod"] + pink_W
    got = tod.cpu().numpy()
    exp_K = (exp_W - a_o[None, :, None]) / b_o[None, :, None]
    pink_rms = (pink_W / b_o[None, :, None]).std(axis=2, keepdims=True)
    err = np.abs(got - exp_K) / (TOL_TOD * np.abs(exp_W) / np.abs(b_o)[None, :, None]
                                 + TOL_PINK * pink_rms)
    print(f"  kelvin tod + pink: max err / bar {err.max():.2e}", flush=True)
    assert err.max() <= 1.0


def test_kelvin_dead_channel_is_nan(ctx):
    sc = tiny_scenario(F=24, K=3, P=1, T=200, filt="matrix")
    sc.spectral.filters.matrix[:, 1] = 0.0
    run = g.ScenarioRun(ctx, sc)
    g.skydip(ctx, run.spec_id, sc.K, 1.0, 0.2, 2.0, 16)
    out = run.alloc()
    g.simulate_tod(ctx, [run.signal_job(out, kelvin=True)])
    torch.cuda.synchronize()
    t = out.tod.cpu().numpy()
    assert np.isnan(t[:, 1]).all()
    assert np.isfinite(t[:, [0, 2]]).all()
