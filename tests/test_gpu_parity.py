"""GPU (HIP) path against the FP64 oracle, through the C-ABI.

Tolerances (stated for the FP32 path): noise-free P_KID and the TOD within
1e-6 relative of the oracle, element by element; photon-noise sigma within
1e-5 relative; the 1/f series within 1e-5 of its rms; Philox words
bit-exact.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2604_23305_amd as g
from oracle import philox as op
from oracle import pink as opk
from tests.gpu_util import new_ctx, rel_err, report, run_signal
from tests.test_oracle_pins import tiny_scenario
from workloads import configs
from workloads import gen

pytestmark = pytest.mark.gpu

TOL_PKID = 1e-6
TOL_SIGMA = 1e-5
TOL_PINK = 1e-5


@pytest.fixture(scope="module")
def ctx():
    c = new_ctx()
    yield c
    g.free(c)


def test_philox_words_bit_exact(ctx):
    rng = np.random.default_rng(0)
    n = 4096
    ctr = rng.integers(0, 2**32, size=(n, 4), dtype=np.uint64).astype(np.uint32)
    ctr[:16] = 0
    ctr[16:32, 0] = np.arange(16)
    for seed in (0, 1, 0x123456789ABCDEF, 2**64 - 1):
        d_ctr = torch.from_numpy(ctr.view(np.int32)).cuda()
        d_out = torch.zeros((n, 4), dtype=torch.int32, device="cuda")
        g.philox(ctx, d_ctr, d_out, n, seed)
        torch.cuda.synchronize()
        got = d_out.cpu().numpy().view(np.uint32)
        ref = np.stack(op.philox4x32_10(ctr[:, 0], ctr[:, 1], ctr[:, 2],
                                        ctr[:, 3], op.key_of(seed)), axis=1)
        np.testing.assert_array_equal(got, ref)


def _compare(sc, out, ref, tol_pk=TOL_PKID, t_slice=slice(None)):
    pk = out.p_kid.cpu().numpy()[..., t_slice]
    e_pk = rel_err(pk, ref["p_kid"])
    report("p_kid", e_pk)
    e_sg = rel_err(out.sigma.cpu().numpy()[..., t_slice], ref["sigma"])
    report("sigma", e_sg)
    e_tod = rel_err(out.tod.cpu().numpy()[..., t_slice], ref["tod"])
    report("tod", e_tod)
    assert e_pk.max() <= tol_pk
    assert e_sg.max() <= TOL_SIGMA
    assert e_tod.max() <= tol_pk


@pytest.mark.parametrize("noise", [False, True])
def test_c1_full_parity(ctx, noise):
    sc = configs.c1(noise=noise)
    ref = oracle.tod.simulate(sc)
    _, out = run_signal(ctx, sc, with_pwv=True)
    _compare(sc, out, ref)
    np.testing.assert_allclose(out.pwv.cpu().numpy(), ref["pwv"], rtol=1e-7)


@pytest.mark.parametrize("prec", [g.PREC_FP32, g.PREC_SPLIT_BF16])
@pytest.mark.parametrize("filt", ["filterbank", "lorentz", "matrix"])
@pytest.mark.parametrize("shape", [(8, 3, 2, 5), (29, 70, 2, 200),
                                   (37, 33, 3, 131), (100, 130, 2, 300)])
def test_tiny_and_ragged_shapes(ctx, filt, shape, prec):
    """Shapes that leave ragged F, K and T tiles; every cascade kind; both
    contraction kernels (a K tail of one or two 32-channel tiles, or of a
    partly live channel group)."""
    F, K, P, T = shape
    sc = tiny_scenario(F=F, K=K, P=P, T=T, filt=filt,
                       stages=configs.cascade_table2())
    ref = oracle.tod.simulate(sc)
    _, out = run_signal(ctx, sc, precision=prec)
    _compare(sc, out, ref)


def test_large_source_grid_coarse_buckets(ctx):
    """A 300 x 300 source grid has more cells than the panel's row sort
    keeps buckets (65536), so rows are bucketed by 2 x 2 cells; 7 pixels
    sweep the grid on a daisy."""
    from workloads.scenario import Source
    sc = tiny_scenario(F=24, K=5, P=7, T=3000)
    cube, gr = gen.source_cube(sc.spectral.nu_hz, 300, 60 * gen.ARCSEC, 0.0,
                               np.pi / 3,
                               [dict(flux_jy=np.full(24, 5.0),
                                     fwhm_rad=10 * gen.ARCSEC),
                                dict(flux_jy=np.full(24, 2.0),
                                     fwhm_rad=4 * gen.ARCSEC,
                                     off_rad=(20 * gen.ARCSEC, -15 * gen.ARCSEC))],
                               np.pi * 25)
    sc.source = Source(cube=cube, az0=gr["az0"], daz=gr["daz"], el0=gr["el0"],
                       del_=gr["del_"])
    ref = oracle.tod.simulate(sc)
    _, out = run_signal(ctx, sc)
    _compare(sc, out, ref)


def test_sorted_panel_with_zero_cube_matches_no_cube(ctx):
    """With an all-zero source cube the rows take the bucketed panel (row
    records in scalar registers, neighbour reuse of table rows) and add a
    zero source term; without a cube they take the unsorted panel.  Both
    compute the same powers, so P_KID and sigma agree element by element
    to FP32 rounding (the two kernels may contract their products
    differently); a row or bin mix-up in either, even one confined to weak
    channels or rows, would show at the level of the PWV variation."""
    from workloads.scenario import Source
    sc0 = tiny_scenario(F=24, K=5, P=7, T=3000)
    sc1 = tiny_scenario(F=24, K=5, P=7, T=3000)
    cube, gr = gen.source_cube(sc1.spectral.nu_hz, 300, 60 * gen.ARCSEC, 0.0,
                               np.pi / 3,
                               [dict(flux_jy=np.full(24, 5.0),
                                     fwhm_rad=10 * gen.ARCSEC)],
                               np.pi * 25)
    sc1.source = Source(cube=np.zeros_like(cube), az0=gr["az0"], daz=gr["daz"],
                        el0=gr["el0"], del_=gr["del_"])
    sc0.source = None
    _, out0 = run_signal(ctx, sc0, photon_noise=False)
    _, out1 = run_signal(ctx, sc1, photon_noise=False)
    for name in ("p_kid", "sigma"):
        a = getattr(out0, name).cpu().numpy().astype(np.float64)
        b = getattr(out1, name).cpu().numpy()
        err = rel_err(b, a)
        report(name, err)
        assert err.max() <= 1e-6, (name, err.max())


@pytest.mark.parametrize("prec", [g.PREC_FP32, g.PREC_SPLIT_BF16])
def test_table_axis_clamp_matches_oracle(prec):
    """Screen PWV that leaves the table's PWV axis at both ends (section 2.4
    lookup table; PWV outside the axis is clamped to it, reading R6), in
    the default (non-strict) mode: every output element against the oracle,
    and the table-clamp counter equal to the number of rows whose PWV lies
    outside the axis (an integer, compared exactly).  The axis is narrow,
    0.9-1.1 mm, and the screen spans 0.77-1.26 mm, so that the spectra stay
    within the range the reference-row contraction keeps to 1e-6 (a sky
    far from the reference, such as a 0-3 mm sweep through opaque lines,
    loses accuracy as c0 / P_KID grows)."""
    import dataclasses
    from workloads.scenario import Screen
    sc = tiny_scenario(F=40, K=7, P=3, T=2000)
    lines = gen.absorption_lines(3, lo_hz=300e9, hi_hz=340e9)
    ez, p0, dp = gen.zenith_transmission_table(sc.spectral.nu_hz, lines,
                                               0.9, 0.01, 21)
    sc.spectral = dataclasses.replace(sc.spectral, eta_z=ez, pwv0_mm=p0,
                                      dpwv_mm=dp)
    sc.screen = Screen(pwv_mm=gen.pwv_screen(16, 512, 33, 1.0, 0.15),
                       dx_m=0.5, dy_m=0.5, ix0=4.0, iy0=7.5)
    ref = oracle.tod.simulate(sc)
    sp = sc.spectral
    top = sp.pwv0_mm + (sp.eta_z.shape[0] - 1) * sp.dpwv_mm
    low = int((ref["pwv"] < sp.pwv0_mm).sum())
    high = int((ref["pwv"] > top).sum())
    print(f"  rows below the axis {low}, above {high}", flush=True)
    assert low > 1000 and high > 1000
    c = new_ctx()
    try:
        _, out = run_signal(c, sc, precision=prec, with_pwv=True)
        _compare(sc, out, ref)
        np.testing.assert_allclose(out.pwv.cpu().numpy(), ref["pwv"],
                                   rtol=1e-7, atol=1e-9)
        assert g.counters(c)[:3] == (int(ref["clamps"]), low + high, 0)
    finally:
        g.free(c)


def test_trajectory_elevation_outside_range_is_counted():
    """A user trajectory whose elevation leaves (0, pi) has no airmass
    (Eq. airmass, 1/sin(el)): the rows that do are counted per (pixel,
    sample) in the third range counter, and every other row still matches
    the oracle element by element."""
    from workloads.scenario import Scan
    sc = tiny_scenario(F=16, K=3, P=2, T=400, scan="stare")
    traj = np.zeros((400, 2))
    traj[:, 0] = np.linspace(-20, 20, 400) * gen.ARCSEC
    traj[:, 1] = np.linspace(-10, 10, 400) * gen.ARCSEC
    traj[100:150, 1] = -np.pi / 2          # el = pi/3 - pi/2 < 0
    traj[300:320, 1] = 2.2                 # el = pi/3 + 2.2 > pi
    sc.scan = Scan("traj", theta0=np.pi / 3, traj=traj)
    keep = np.r_[0:100, 150:300, 320:400]
    ref = oracle.tod.simulate(sc, photon_noise=False)
    c = new_ctx()
    try:
        _, out = run_signal(c, sc, photon_noise=False)
        assert g.counters(c)[2] == sc.n_pix * (50 + 20)
        e = rel_err(out.p_kid.cpu().numpy()[..., keep], ref["p_kid"][..., keep])
        report("p_kid (rows with an airmass)", e)
        assert e.max() <= TOL_PKID
    finally:
        g.free(c)


def _far_elements(sc):
    """Oracle count of (row, bin) elements with |P - P_ref| > P / 8, and
    how close the nearest one lies to the threshold (relative)."""
    spec = sc.spectral
    eta_z, _ = oracle.tod.lut_transmission(spec, np.array([spec.ref_pwv_mm]))
    pref = oracle.tod.cascade(sc, eta_z ** (1.0 / np.sin(spec.ref_el_rad)),
                              None)[0]
    n = np.arange(sc.t_total, dtype=np.int64)
    count, margin = 0, np.inf
    for p in range(sc.n_pix):
        geo = oracle.tod.row_geometry(sc, p, n)
        ez, _ = oracle.tod.lut_transmission(spec, geo["pwv"])
        P = oracle.tod.cascade(sc, ez ** geo["csc"][:, None],
                               oracle.tod.source_power(sc.source, geo["az"],
                                                       geo["el"]))
        r = np.abs(P - pref) / P
        count += int((r > 0.125).sum())
        margin = min(margin, float(np.min(np.abs(r / 0.125 - 1.0))))
    return count, margin


def test_far_from_reference_is_counted():
    """Range counter 3 counts (row, bin) elements with |P - P_ref| > P / 8,
    beyond which the stated 1e-6 of the reference-row contraction is no
    longer guaranteed: zero for the c1 workload, and exactly the oracle's
    count for a source a million times brighter than the tiny scenario's
    (no element lies within 1e-4 of the threshold)."""
    from workloads.scenario import Source
    c = new_ctx()
    try:
        sc = configs.c1(noise=False)
        run_signal(c, sc)
        assert g.counters(c)[3] == 0
        sc = tiny_scenario(F=24, K=3, P=2, T=600)
        s = sc.source
        sc.source = Source(cube=s.cube * 1e6, az0=s.az0, daz=s.daz,
                           el0=s.el0, del_=s.del_)
        want, margin = _far_elements(sc)
        print(f"  oracle: {want} elements far from the reference "
              f"(nearest {margin:.1e} from the threshold)", flush=True)
        assert want > 0 and margin > 1e-4
        run_signal(c, sc, precision=g.PREC_SPLIT_BF16)
        assert g.counters(c)[3] == want
    finally:
        g.free(c)


def test_window_of_rows_only(ctx):
    """t_begin/t_end select rows; the rest of tod stays untouched."""
    sc = configs.c1()
    ref = oracle.tod.simulate(sc, 300, 777)
    run, out = run_signal(ctx, sc, 300, 777)
    pk = out.p_kid.cpu().numpy()
    assert np.all(pk[..., :300] == 0) and np.all(pk[..., 777:] == 0)
    _compare(sc, out, ref, t_slice=slice(300, 777))


def test_accumulate_adds_into_tod(ctx):
    sc = configs.c1(noise=False)
    run = g.ScenarioRun(ctx, sc)
    out = run.alloc(with_p_kid=True)
    out.tod.fill_(1.0e-12)
    g.simulate_tod(ctx, [run.signal_job(out, accumulate=True)])
    torch.cuda.synchronize()
    np.testing.assert_allclose(out.tod.cpu().numpy(),
                               out.p_kid.cpu().numpy().astype(np.float64) + 1e-12,
                               rtol=1e-6)


@pytest.mark.parametrize("prec", [g.PREC_FP32, g.PREC_SPLIT_BF16])
def test_accumulate_is_one_fp32_add(ctx, prec):
    """Adding into an existing TOD gives, element by element, exactly the
    FP32 sum of the old value and the TOD the same job writes on its own
    (noise on; 70 channels leave a partly live channel group and 32-channel
    tile, whose dead rows must neither be loaded nor stored)."""
    sc = tiny_scenario(F=40, K=70, P=3, T=700, stages=configs.cascade_table2())
    run, ref = run_signal(ctx, sc, precision=prec)
    out = run.alloc()
    gen_ = torch.Generator(device="cpu").manual_seed(5)
    prev = torch.randn(out.tod.shape, generator=gen_).float().cuda()
    out.tod.copy_(prev)
    g.simulate_tod(ctx, [run.signal_job(out, precision=prec, accumulate=True)])
    torch.cuda.synchronize()
    want = (prev + ref.tod).cpu().numpy()
    got = out.tod.cpu().numpy()
    assert np.array_equal(got, want), float(np.abs(got - want).max())


def test_uniform_screen_gives_constant_tod(ctx):
    sc = configs.c1(noise=False, uniform_screen=True)
    _, out = run_signal(ctx, sc)
    pk = out.p_kid.cpu().numpy().astype(np.float64)
    spread = np.ptp(pk, axis=-1) / pk.mean(axis=-1)
    assert spread.max() <= 2e-7


def test_chunking_is_invisible(ctx):
    """A small workspace forces many chunks: outputs are bit-identical."""
    sc = configs.c1()
    _, out_a = run_signal(ctx, sc)
    small = new_ctx(workspace_bytes=8 << 20)
    try:
        _, out_b = run_signal(small, sc)
        assert torch.equal(out_a.tod, out_b.tod)
        assert torch.equal(out_a.sigma, out_b.sigma)
    finally:
        g.free(small)


def test_pink_series_match_oracle(ctx):
    sc = configs.c1()
    run = g.ScenarioRun(ctx, sc)
    tod = torch.zeros((sc.n_pix, sc.K, sc.t_total), device="cuda")
    g.simulate_tod(ctx, [run.pink_job(tod, accumulate=False)])
    torch.cuda.synchronize()
    got = tod.cpu().numpy()
    nep2 = oracle.tod.reference_nep2(sc)
    A = opk.amplitude(nep2, sc.pink_alpha, sc.pink_knee_hz)
    for k in (0, 1, 17, 63):
        ref = opk.series(sc.seed, 0, k, A[k], sc.pink_alpha[k], sc.t_total,
                         sc.f_sample_hz)
        err = np.abs(got[0, k] - ref).max() / ref.std()
        print(f"  pink k={k}: max err / rms {err:.3e}", flush=True)
        assert err <= TOL_PINK


@pytest.mark.parametrize("T", [4097, 9000])
def test_pink_explicit_levels_per_channel(ctx, T):
    """Independent per-channel levels A_k and slopes alpha_k (section 2.6:
    A is a free level per channel), unrelated to the knee; a zero level
    gives a zero series."""
    sc = tiny_scenario(F=16, K=4, P=2, T=T)
    sc.pink_alpha = np.array([1.0, 0.5, 2.0, 1.3])
    sc.pink_A = np.array([3.0e-34, 1.0e-33, 4.0e-35, 0.0])
    sc.pink_knee_hz = 0.0   # unused when the levels are explicit
    run = g.ScenarioRun(ctx, sc)
    tod = torch.full((sc.n_pix, sc.K, T), 7.0, device="cuda")
    g.simulate_tod(ctx, [run.pink_job(tod, accumulate=False)])
    torch.cuda.synchronize()
    got = tod.cpu().numpy()
    A = opk.amplitude(None, sc.pink_alpha, None, A=sc.pink_A)
    for p in range(2):
        for k in range(3):
            ref = opk.series(sc.seed, p, k, A[k], sc.pink_alpha[k], T, 160.0)
            err = np.abs(got[p, k] - ref).max() / ref.std()
            print(f"  pink A p{p} k{k}: max err / rms {err:.3e}", flush=True)
            assert err <= TOL_PINK
        assert np.all(got[p, 3] == 0.0)


def test_pink_explicit_levels_validated(ctx):
    sc = tiny_scenario(F=16, K=3, P=1, T=64)
    sc.pink_alpha = np.ones(3)
    sc.pink_A = np.array([1e-34, -1e-34, 1e-34])
    run = g.ScenarioRun(ctx, sc)
    tod = torch.zeros((sc.n_pix, sc.K, 64), device="cuda")
    with pytest.raises(g.GtodError):
        g.simulate_tod(ctx, [run.pink_job(tod, accumulate=False)])


@pytest.mark.parametrize("T", [1, 2, 3, 100, 4097, 9000])
def test_pink_lengths(ctx, T):
    """Lengths around powers of two, down to a single sample; includes the
    two-pass transform (T > 8192)."""
    sc = tiny_scenario(F=16, K=3, P=2, T=T)
    sc.pink_alpha = np.array([1.0, 0.5, 2.0])
    run = g.ScenarioRun(ctx, sc)
    tod = torch.zeros((sc.n_pix, sc.K, T), device="cuda")
    g.simulate_tod(ctx, [run.pink_job(tod, accumulate=False)])
    torch.cuda.synchronize()
    got = tod.cpu().numpy()
    nep2 = oracle.tod.reference_nep2(sc)
    A = opk.amplitude(nep2, sc.pink_alpha, 1.0)
    for p in range(2):
        for k in range(3):
            ref = opk.series(sc.seed, p, k, A[k], sc.pink_alpha[k], T, 160.0)
            if T <= 2:
                assert np.all(got[p, k] == 0) and np.all(ref == 0)
                continue
            err = np.abs(got[p, k] - ref).max() / ref.std()
            assert err <= TOL_PINK, (p, k, err)


@pytest.mark.parametrize("T,offset", [(4096, 0), (4095, 0), (9000, 0),
                                      (9001, 0), (9000, 1)])
def test_pink_accumulate_adds_into_tod(ctx, T, offset):
    """ACCUMULATE adds the 1/f series into what the TOD holds, with one
    FP32 rounding per sample: bit-identical to the written series added on
    the host.  Even lengths take the paired 8-byte accesses, odd lengths and
    an output starting one float past an 8-byte boundary the 4-byte ones;
    4096 and 4095 are one-pass transforms, 9000 and 9001 two-pass."""
    sc = tiny_scenario(F=16, K=3, P=2, T=T)
    sc.pink_alpha = np.array([1.0, 0.5, 2.0])
    run = g.ScenarioRun(ctx, sc)
    n = sc.n_pix * sc.K * T
    written = torch.zeros((sc.n_pix, sc.K, T), device="cuda")
    g.simulate_tod(ctx, [run.pink_job(written, accumulate=False)])
    base = torch.randn(n, generator=torch.Generator().manual_seed(T + offset))
    buf = torch.zeros(offset + n, device="cuda")
    tod = buf[offset:].view(sc.n_pix, sc.K, T)
    tod.copy_(base.view(sc.n_pix, sc.K, T).to("cuda"))
    g.simulate_tod(ctx, [run.pink_job(tod, accumulate=True)])
    torch.cuda.synchronize()
    expect = base.view(sc.n_pix, sc.K, T) + written.cpu()
    assert torch.equal(tod.cpu(), expect)


def test_pink_batches_are_invisible(ctx):
    """A workspace too small for all series at once: the 111 series of
    40000 samples (two-pass transforms, 16 columns) go in 5 batches of 27
    (the last one of 3).  The TOD, added into random values, is
    bit-identical to the one-batch run of a large workspace; three series,
    one per pixel and in different batches, match the oracle."""
    T = 40000
    sc = tiny_scenario(F=16, K=37, P=3, T=T)
    sc.pink_alpha = np.linspace(0.5, 2.0, sc.K)
    nep2 = oracle.tod.reference_nep2(sc)
    A = opk.amplitude(nep2, sc.pink_alpha, sc.pink_knee_hz)
    refs = {(p, k): opk.series(sc.seed, p, k, A[k], sc.pink_alpha[k], T,
                               sc.f_sample_hz)
            for p, k in ((0, 5), (1, 20), (2, 36))}
    # values at the series' own level, so that subtracting them again
    # costs only rounding
    level = float(np.mean([r.std() for r in refs.values()]))
    base = level * torch.randn((sc.n_pix, sc.K, T),
                               generator=torch.Generator().manual_seed(9))
    outs = []
    for ws in (28 << 20, 1 << 30):
        c = new_ctx(workspace_bytes=ws)
        try:
            run = g.ScenarioRun(c, sc)
            tod = base.to("cuda")
            g.simulate_tod(c, [run.pink_job(tod, accumulate=True)])
            torch.cuda.synchronize()
            outs.append(tod.cpu())
        finally:
            g.free(c)
    assert torch.equal(outs[0], outs[1])
    got = outs[0].double().numpy() - base.double().numpy()
    for (p, k), ref in refs.items():
        err = np.abs(got[p, k] - ref).max() / ref.std()
        print(f"  pink p={p} k={k}: max err / rms {err:.3e}", flush=True)
        assert err <= TOL_PINK


@pytest.mark.parametrize("T,K", [(2**21 + 5, 2), (2**25 - 3, 1)])
def test_pink_long_series(ctx, T, K):
    """Long series: four-step splits with 512 and with 4096 columns (the
    longest series accepted), i.e. pass 2 with 4 columns per workgroup and
    with a single one."""
    sc = tiny_scenario(F=16, K=K, P=1, T=T)
    sc.pink_alpha = np.array([1.0, 2.0])[:K]
    run = g.ScenarioRun(ctx, sc)
    tod = torch.zeros((1, K, T), device="cuda")
    g.simulate_tod(ctx, [run.pink_job(tod, accumulate=False)])
    torch.cuda.synchronize()
    got = tod.cpu().numpy()
    del tod
    nep2 = oracle.tod.reference_nep2(sc)
    A = opk.amplitude(nep2, sc.pink_alpha, 1.0)
    for k in range(K):
        ref = opk.series(sc.seed, 0, k, A[k], sc.pink_alpha[k], T, 160.0)
        err = np.abs(got[0, k] - ref).max() / ref.std()
        print(f"  T={T} k={k}: max err / rms {err:.3e}", flush=True)
        assert err <= TOL_PINK, (k, err)


def test_nep2_reference_matches_oracle(ctx):
    sc = configs.c2(t_total=256, screen_shape=(64, 4096))
    run = g.ScenarioRun(ctx, sc)
    got = g.spec_nep2_ref(ctx, run.spec_id, sc.K)
    ref = oracle.tod.reference_nep2(sc)
    assert np.max(np.abs(got / ref - 1)) <= 1e-6


@pytest.mark.parametrize("prec", [g.PREC_FP32, g.PREC_SPLIT_BF16])
def test_c2_full_run_windows(ctx, prec):
    """Single-pixel spectrometer at full size (raster, 96k samples): the
    whole run on the GPU, three 2048-sample windows against the oracle."""
    sc = configs.c2()
    run, out = run_signal(ctx, sc, precision=prec)
    T = sc.t_total
    for a in (0, T // 2 - 1024, T - 2048):
        ref = oracle.tod.simulate(sc, a, a + 2048)
        print(f" window {a}", flush=True)
        _compare(sc, out, ref, t_slice=slice(a, a + 2048))


def test_split_matches_fp32_closely(ctx):
    sc = configs.c1(noise=False)
    _, o32 = run_signal(ctx, sc, precision=g.PREC_FP32)
    _, obf = run_signal(ctx, sc, precision=g.PREC_SPLIT_BF16)
    d = rel_err(obf.p_kid.cpu().numpy(), o32.p_kid.cpu().numpy().astype(np.float64))
    report("split vs fp32", d)
    assert d.max() <= 1e-6


def test_error_paths(ctx):
    sc = configs.c1()
    run = g.ScenarioRun(ctx, sc)
    out = run.alloc()
    job = run.signal_job(out)
    bad = run.signal_job(out)
    bad.spec_id = 999
    with pytest.raises(g.GtodError, match="ENOTFOUND"):
        g.simulate_tod(ctx, [job, bad])
    bad = run.signal_job(out, 0, sc.t_total)
    bad.t_end = sc.t_total + 1
    with pytest.raises(g.GtodError, match="EINVAL"):
        g.simulate_tod(ctx, [bad])
    bad = run.signal_job(out)
    bad.n_az = 1
    with pytest.raises(g.GtodError, match="EINVAL"):
        g.simulate_tod(ctx, [bad])
    with pytest.raises(g.GtodError, match="ENOTFOUND"):
        g.free(ctx, g.OBJ_SCREEN, 12345)
    tiny = new_ctx(hbm_budget_bytes=64 << 20, workspace_bytes=1 << 30)
    try:
        r2 = g.ScenarioRun(tiny, sc)
        o2 = r2.alloc()
        with pytest.raises(g.GtodError, match="EBUDGET"):
            g.simulate_tod(tiny, [r2.signal_job(o2)])
    finally:
        g.free(tiny)


@pytest.mark.parametrize("F,K,why", [(1 << 20, 1 << 10, "response plane"),
                                     ((1 << 22) + 1, 1, "panel rows")])
def test_response_plane_of_4_gib_is_rejected(ctx, F, K, why):
    """F x K whose padded response plane reaches 4 GiB, or F whose 256
    padded panel rows do (the contractions' 32-bit operand offsets), is
    refused before anything is allocated."""
    nu = np.linspace(200e9, 460e9, F)
    w = np.full(F, nu[1] - nu[0])
    eta_z = np.full((2, F), 0.9)
    f = np.linspace(210e9, 450e9, K)
    with pytest.raises(g.GtodError, match="EINVAL.*" + why):
        g.load_filters(ctx, nu, w, eta_z, 0.0, 1.0, 270.0, [], "lorentz",
                       f_hz=f, R=np.full(K, 500.0), eta_peak=np.full(K, 0.5))


def test_strict_range_rejects_leaving_screen():
    sc = configs.c1()
    c = new_ctx(strict_range=True)
    try:
        run = g.ScenarioRun(c, sc)
        out = run.alloc()
        sc.dtheta[0] = 0.05   # 77 m off a 12.8 m-wide screen
        run.dtheta[0] = 0.05
        with pytest.raises(g.GtodError, match="ERANGE"):
            g.simulate_tod(c, [run.signal_job(out)])
    finally:
        g.free(c)


def test_empty_calls_and_windows_change_nothing(ctx):
    sc = configs.c1(t_total=400)
    run = g.ScenarioRun(ctx, sc)
    out = run.alloc()
    out.tod.fill_(3.0)
    g.simulate_tod(ctx, [])
    g.simulate_tod(ctx, [run.signal_job(out, 200, 200)])
    torch.cuda.synchronize()
    assert torch.all(out.tod == 3.0)


def test_pink_length_limit_is_an_error(ctx):
    sc = tiny_scenario(F=16, K=3, P=1, T=8)
    sc.pink_alpha = np.ones(3)
    run = g.ScenarioRun(ctx, sc)
    tod = torch.zeros(4, device="cuda")
    job = run.pink_job(tod, accumulate=False)
    job.t_total = (1 << 25) + 1
    with pytest.raises(g.GtodError, match="EINVAL"):
        g.simulate_tod(ctx, [job])


def test_pixel_subset_with_pix0_matches_full_job(ctx):
    """A job over pixels [2, 5) with pix0 = 2 gives, bit for bit, rows 2..4
    of one job over all seven pixels (signal, photon and 1/f noise)."""
    sc = tiny_scenario(F=40, K=5, P=7, T=1500)
    sc.pink_alpha = np.array([1.0, 0.7, 1.3, 2.0, 0.5])
    run = g.ScenarioRun(ctx, sc)
    full = run.alloc()
    g.simulate_tod(ctx, [run.pink_job(full.tod, accumulate=False),
                         run.signal_job(full, accumulate=True)])
    part = torch.zeros((3, sc.K, sc.t_total), device="cuda")
    sig = run.signal_job(full, accumulate=True)
    sig.n_pix, sig.pix0 = 3, 2
    sig.dphi_rad = run.dphi[2:].ctypes.data
    sig.dtheta_rad = run.dtheta[2:].ctypes.data
    sig.tod = part.data_ptr()
    pk = run.pink_job(part, accumulate=False)
    pk.n_pix, pk.pix0 = 3, 2
    g.simulate_tod(ctx, [pk, sig])
    torch.cuda.synchronize()
    assert torch.equal(part, full.tod[2:5])
