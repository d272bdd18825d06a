"""Common-mode subtraction and gridding (gtod_reduce) against the oracle.

Inputs never come from the HIP path: the Kelvin TOD fed to both sides is
the oracle's simulation put on the oracle's skydip scale (rounded to FP32),
or, at full size, a synthetic common atmosphere built from the oracle's
transmissions.

Tolerances: T* is computed in FP64 and stored in FP32, so |T*_gpu -
T*_oracle| <= 2^-23 |T*_oracle| + 1e-10 s, with s = (|T_b| + (1 - eta) |M|)
/ eta the size of the two terms that cancel; maps (FP64 throughout) within
1e-9 of the same scale, weights within 1e-8 relative.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2604_23305_amd as g
from oracle import reduce as orr
from oracle import skydip as osd
from paper_2604_23305_amd.binding import GtodError
from tests.gpu_util import new_ctx
from workloads import configs, gen

pytestmark = pytest.mark.gpu

ARC = gen.ARCSEC


@pytest.fixture(scope="module")
def ctx():
    c = new_ctx()
    yield c
    g.free(c)


def hex_scenario(T=3000, F=400, K=24, r_px=60 * ARC):
    """7-spaxel hexagon with a wide pitch so that the ring is off source,
    daisy scan, c2-style spectral setup and line source."""
    sc = configs.c2(t_total=T, screen_shape=(64, 4096), F=F, K=K)
    sc.scan = configs.daisy_scan()
    sc.dphi, sc.dtheta = gen.hex_spaxels(1, r_px)
    return sc


def kelvin_input(sc):
    """The oracle's TOD and PWV, on the oracle's skydip scale, in FP32."""
    ref = oracle.tod.simulate(sc)
    a, b = osd.skydip(sc, sc.scan.theta0, 0.25, 2.75, 64)
    t_b = osd.to_kelvin(ref["tod"], a, b).astype(np.float32)
    return t_b, ref["pwv"].astype(np.float32)


def check_tstar(sc, got, t_b, pwv_mean, r_out, channels=None, t0=0):
    ref = orr.common_mode(sc, t_b, pwv_mean, r_out, t0=t0, channels=channels)
    eta_zk = orr.channel_zenith_transmission(sc, pwv_mean)
    if channels is not None:
        eta_zk = eta_zk[list(channels)]
    eta = orr.spaxel_transmission(sc, eta_zk, t0 + np.arange(t_b.shape[2]))
    S = orr.off_source(sc, r_out)
    M = (t_b[S].astype(np.float64) / (1 - eta[S])).sum(axis=0) / S.sum()
    scale = (np.abs(t_b) + (1 - eta) * np.abs(M)[None]) / eta
    err = np.abs(got - ref) / (2.0 ** -23 * np.abs(ref) + 1e-10 * scale)
    print(f"  T*: max err / bar {err.max():.2e}", flush=True)
    assert err.max() <= 1.0
    return ref, scale


def test_reduce_small_matches_oracle(ctx):
    sc = hex_scenario()
    t_b, pwv = kelvin_input(sc)
    run = g.ScenarioRun(ctx, sc)
    d_tb = torch.from_numpy(t_b).cuda()
    d_pwv = torch.from_numpy(pwv).cuda()
    ts = torch.zeros_like(d_tb)
    n = 15
    mp = torch.zeros((sc.K, n, n), dtype=torch.float64, device="cuda")
    wt = torch.zeros_like(mp)
    r_out, half = 30 * ARC, 150 * ARC
    g.reduce(ctx, run.reduce_desc(d_tb, r_out, t_star=ts, maps=(mp, wt),
                                  map_n=n, map_half_rad=half, pwv=d_pwv))
    torch.cuda.synchronize()
    pwv_mean = orr.pwv_mean(pwv)
    ref, scale = check_tstar(sc, ts.cpu().numpy(), t_b, pwv_mean, r_out)
    count, mean, var = orr.spaxel_maps(sc, ref, half, n)
    m_o, w_o = orr.combine(count, mean, var)
    m_g = mp.cpu().numpy().reshape(sc.K, -1)
    w_g = wt.cpu().numpy().reshape(sc.K, -1)
    assert np.array_equal(np.isnan(m_g), np.isnan(m_o))
    assert np.array_equal(w_g > 0, w_o > 0)
    assert (w_o > 0).sum() > sc.K * 20
    live = w_o > 0
    tol = 1e-9 * scale.max()
    err_m = np.abs(m_g[live] - m_o[live]).max()
    err_w = (np.abs(w_g[live] - w_o[live]) / w_o[live]).max()
    print(f"  map: max abs err {err_m:.2e} (bar {tol:.2e}); weight max rel "
          f"err {err_w:.2e}", flush=True)
    assert err_m <= tol and err_w <= 1e-8


def test_reduce_host_pwv_and_channel_groups(ctx):
    """Mean PWV given by the caller; a workspace that holds only a few
    channels per group; T* not stored; stare scan; a window of samples."""
    sc = hex_scenario(T=1500, F=200, K=9)
    t_b, _ = kelvin_input(sc)
    small = new_ctx(workspace_bytes=96 << 10)   # three channels per group
    try:
        run = g.ScenarioRun(small, sc)
        t0, T = 300, 1100
        d_tb = torch.from_numpy(np.ascontiguousarray(t_b[:, :, t0:t0 + T])).cuda()
        n = 9
        mp = torch.zeros((sc.K, n, n), dtype=torch.float64, device="cuda")
        wt = torch.zeros_like(mp)
        r_out, half = 30 * ARC, 120 * ARC
        d = run.reduce_desc(d_tb, r_out, maps=(mp, wt), map_n=n,
                            map_half_rad=half, pwv_mean_mm=1.1, t0=t0)
        g.reduce(small, d)
        torch.cuda.synchronize()
        ref = orr.common_mode(sc, t_b[:, :, t0:t0 + T], 1.1, r_out, t0=t0)
        count, mean, var = orr.spaxel_maps(sc, ref, half, n, t0=t0)
        m_o, w_o = orr.combine(count, mean, var)
        m_g = mp.cpu().numpy().reshape(sc.K, -1)
        w_g = wt.cpu().numpy().reshape(sc.K, -1)
        live = w_o > 0
        assert np.array_equal(w_g > 0, live)
        assert np.abs(m_g[live] - m_o[live]).max() <= 1e-9 * np.abs(t_b).max() * 4
        assert (np.abs(w_g[live] - w_o[live]) / w_o[live]).max() <= 1e-8
    finally:
        g.free(small)


def test_reduce_argument_errors(ctx):
    sc = hex_scenario(T=200, F=100, K=4)
    run = g.ScenarioRun(ctx, sc)
    tb = torch.zeros((sc.n_pix, sc.K, 200), device="cuda")
    ts = torch.zeros_like(tb)
    mp = torch.zeros((sc.K, 5, 5), dtype=torch.float64, device="cuda")
    for kw in (dict(r_out=1.0, t_star=ts),                     # no off spaxel
               dict(r_out=30 * ARC),                           # no output
               dict(r_out=30 * ARC, maps=(mp, mp), map_n=1, map_half_rad=1e-3),
               dict(r_out=30 * ARC, maps=(mp, mp), map_n=49, map_half_rad=1e-3),
               dict(r_out=30 * ARC, maps=(mp, mp), map_n=5, map_half_rad=0.0)):
        r_out = kw.pop("r_out")
        d = run.reduce_desc(tb, r_out, pwv_mean_mm=1.0, **kw)
        with pytest.raises(GtodError, match="EINVAL"):
            g.reduce(ctx, d)
    d = run.reduce_desc(tb, 30 * ARC, t_star=ts)
    with pytest.raises(GtodError, match="EINVAL"):   # no PWV given
        g.reduce(ctx, d)
    d = run.reduce_desc(tb, 30 * ARC, t_star=ts, pwv_mean_mm=1.0)
    d.spec_id = 424242
    with pytest.raises(GtodError, match="ENOTFOUND"):
        g.reduce(ctx, d)
