"""Out-of-core runs (gtod_simulate_to_disk): the files hold, bit for bit,
what one in-memory run over all pixels gives, whatever the pixel grouping,
and that run agrees with the oracle."""
import numpy as np
import pytest
import torch

import oracle
import paper_2604_23305_amd as g
from oracle import pink as opk
from paper_2604_23305_amd.binding import GtodError
from tests.gpu_util import new_ctx
from workloads import configs, gen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = new_ctx(workspace_bytes=64 << 20)
    yield c
    g.free(c)


def scenario(T=12000, K=20, F=300):
    sc = configs.c2(t_total=T, screen_shape=(64, 4096), F=F, K=K)
    sc.scan = configs.daisy_scan()
    sc.dphi, sc.dtheta = gen.hex_spaxels(1, 12 * gen.ARCSEC)
    return sc


def in_memory(ctx, run, pink=True):
    out = run.alloc(with_pwv=True)
    jobs = ([run.pink_job(out.tod, accumulate=False)] if pink else []) + \
        [run.signal_job(out, accumulate=pink)]
    g.simulate_tod(ctx, jobs)
    torch.cuda.synchronize()
    return out


def test_groups_of_three_bitwise_and_oracle(ctx, tmp_path):
    sc = scenario()
    run = g.ScenarioRun(ctx, sc)
    ref = in_memory(ctx, run)
    K, T = sc.K, sc.t_total
    per_pix = K * T * 4 + T * 4
    wall, nbytes, groups, G = g.simulate_to_disk(
        ctx, run.signal_job(ref), run.pink_job(ref.tod), tmp_path,
        device_bytes=2 * 3 * per_pix, host_bytes=2 << 20)
    print(f"  {groups} groups of {G} px, {nbytes / 1e6:.1f} MB in {wall:.2f} s",
          flush=True)
    assert (groups, G) == (3, 3)
    tod = np.load(tmp_path / "tod.npy", mmap_mode="r")
    assert tod.shape == (sc.n_pix, K, T) and tod.dtype == np.float32
    assert np.array_equal(tod, ref.tod.cpu().numpy())
    assert np.array_equal(np.load(tmp_path / "pwv.npy"), ref.pwv.cpu().numpy())
    assert np.array_equal(np.load(tmp_path / "time.npy"),
                          np.arange(T) / sc.f_sample_hz)
    assert nbytes == sc.n_pix * (K * T * 4 + T * 4)
    # pixel 5 (second group) over a window, signal + 1/f, against the oracle
    p, a, b = 5, 4000, 6000
    o = oracle.tod.simulate(sc, a, b, pixels=[p])
    A = opk.amplitude(oracle.tod.reference_nep2(sc), sc.pink_alpha,
                      sc.pink_knee_hz)
    pink = np.stack([opk.series(sc.seed, p, k, A[k], sc.pink_alpha[k], T,
                                sc.f_sample_hz)[a:b] for k in range(K)])
    expect = o["tod"][0] + pink
    err = np.abs(tod[p, :, a:b] - expect) / np.abs(expect)
    print(f"  pixel {p} vs oracle: max rel err {err.max():.2e}", flush=True)
    assert err.max() <= 1e-6


def test_signal_only_automatic_groups(ctx, tmp_path):
    sc = scenario(T=5000, K=12, F=200)
    sc.pink_alpha = None
    run = g.ScenarioRun(ctx, sc)
    ref = in_memory(ctx, run, pink=False)
    per_pix = sc.K * sc.t_total * 4
    wall, nbytes, groups, G = g.simulate_to_disk(
        ctx, run.signal_job(ref), None, tmp_path, device_bytes=5 * per_pix,
        host_bytes=2 << 20, pwv=False)
    assert (groups, G) == (4, 2)
    assert not (tmp_path / "pwv.npy").exists()
    assert np.array_equal(np.load(tmp_path / "tod.npy"), ref.tod.cpu().numpy())


def test_sink_errors(ctx, tmp_path):
    sc = scenario(T=1000, K=8, F=100)
    run = g.ScenarioRun(ctx, sc)
    out = run.alloc()
    sig, pk = run.signal_job(out), run.pink_job(out.tod)
    with pytest.raises(GtodError, match="EINVAL"):
        g.simulate_to_disk(ctx, sig, pk, tmp_path, device_bytes=1000)
    with pytest.raises(GtodError, match="EINVAL"):
        g.simulate_to_disk(ctx, sig, pk, tmp_path, device_bytes=1 << 24,
                           host_bytes=1 << 20)
    bad = run.pink_job(out.tod)
    bad.seed += 1
    with pytest.raises(GtodError, match="EINVAL"):
        g.simulate_to_disk(ctx, sig, bad, tmp_path, device_bytes=1 << 24)
    half = run.signal_job(out, 0, 500)
    with pytest.raises(GtodError, match="EINVAL"):
        g.simulate_to_disk(ctx, half, pk, tmp_path, device_bytes=1 << 24)
    blocker = tmp_path / "file"
    blocker.write_text("x")
    with pytest.raises(GtodError, match="EIO"):
        g.simulate_to_disk(ctx, sig, pk, blocker / "sub", device_bytes=1 << 24)
