"""gtod_simulate_tod_noalloc against gtod_simulate_tod, through the C-ABI.

The no-alloc call runs the same kernels in the library's static per-GPU
scratch, so it chunks rows and 1/f series differently from a stream
workspace; no result depends on the chunking, so every output must be
bit-identical to the allocating call's (stronger than the 1e-6 bar).  Two
calls in a row, the second smaller than the first, then a job too large
for the scratch, which must be refused before anything is enqueued.
"""
import numpy as np
import pytest
import torch

import paper_2604_23305_amd as g
from workloads import configs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = g.sim_init(device=0, workspace_bytes=1 << 30)
    yield c
    g.free(c)


def _simulate(fn, ctx, run, precision):
    out = run.alloc(with_p_kid=True, with_sigma=True, with_pwv=True)
    jobs = [run.signal_job(out, precision=precision)]
    if run.sc.pink_alpha is not None:
        jobs.append(run.pink_job(out.tod, accumulate=True))
    fn(ctx, jobs)
    torch.cuda.synchronize()
    return out


def _same(a, b):
    for name in ("tod", "p_kid", "sigma", "pwv"):
        x, y = getattr(a, name), getattr(b, name)
        print(f"  {name}: shape {tuple(x.shape)}, "
              f"max |diff| {float((x - y).abs().max()):.3e}", flush=True)
        assert torch.equal(x, y), name


def test_noalloc_matches_simulate_tod_two_calls(ctx):
    # call 1: 9-pixel daisy over a source cube (bucketed panel), 40000
    # samples x 347 channels x 3000 bins, FP32, photon + 1/f noise; the
    # scratch takes 2304-sample chunks and ~990-series 1/f batches where
    # the 1 GiB workspace takes 7296 and ~1020
    big = configs.c3(t_total=40000, screen_shape=(256, 16384), n_side=3)
    run = g.ScenarioRun(ctx, big)
    print("call 1: 9 px x 347 ch x 40000 samples, FP32", flush=True)
    ref = _simulate(g.simulate_tod, ctx, run, g.PREC_FP32)
    got = _simulate(g.simulate_tod_noalloc, ctx, run, g.PREC_FP32)
    _same(got, ref)
    assert float(got.tod.abs().max()) > 0
    del ref, got
    # call 2, smaller: 1-pixel stare, 64 channels x 1000 bins x 1600
    # samples, split BF16 (single-pass 1/f transforms)
    small = configs.c1()
    run = g.ScenarioRun(ctx, small)
    print("call 2: 1 px x 64 ch x 1600 samples, split BF16", flush=True)
    ref = _simulate(g.simulate_tod, ctx, run, g.PREC_SPLIT_BF16)
    got = _simulate(g.simulate_tod_noalloc, ctx, run, g.PREC_SPLIT_BF16)
    _same(got, ref)


def test_noalloc_refuses_a_job_beyond_its_scratch(ctx):
    # 600000 bins: 128 panel rows need 307 MB, more than the 248 MiB the
    # scratch leaves after its staging slots (a 1 GiB workspace holds them)
    F = 600000
    nu = np.linspace(200e9, 460e9, F)
    w = np.full(F, nu[1] - nu[0])
    eta_z = np.full((2, F), 0.9)
    spec = g.load_filters(ctx, nu, w, eta_z, 0.0, 3.0, 273.0, [], "lorentz",
                          np.array([330e9]), np.array([500.0]),
                          np.array([1.0]))
    sc = configs.c1(noise=False, t_total=256)
    run = g.ScenarioRun(ctx, sc, spec_id=spec)
    run.cube = None
    out = run.alloc()
    print("too-large job: F = 600000", flush=True)
    with pytest.raises(g.GtodError, match="no-alloc scratch"):
        g.simulate_tod_noalloc(ctx, [run.signal_job(out)])
    torch.cuda.synchronize()
    assert float(out.tod.abs().max()) == 0.0
    g.free(ctx, g.OBJ_SPEC, spec)
