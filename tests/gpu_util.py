"""Helpers for the GPU tests: run a scenario through the C-ABI and compare
with the oracle."""
import numpy as np
import torch

import paper_2604_23305_amd as g


def new_ctx(**kw):
    kw.setdefault("workspace_bytes", 1 << 30)
    return g.sim_init(**kw)


def run_signal(ctx, sc, t_begin=0, t_end=None, precision=-1,
               photon_noise=None, run=None, with_pwv=False):
    """SIGNAL job over [t_begin, t_end) writing tod, p_kid, sigma."""
    run = run or g.ScenarioRun(ctx, sc)
    out = run.alloc(with_p_kid=True, with_sigma=True, with_pwv=with_pwv)
    job = run.signal_job(out, t_begin, t_end, precision=precision,
                         photon_noise=photon_noise)
    g.simulate_tod(ctx, [job])
    torch.cuda.synchronize()
    return run, out


def rel_err(gpu, ref):
    gpu = np.asarray(gpu, dtype=np.float64)
    return np.abs(gpu - ref) / np.abs(ref)


def report(name, err):
    print(f"  {name}: max {err.max():.3e} p99.99 "
          f"{np.quantile(err, 0.9999):.3e} median {np.median(err):.3e}",
          flush=True)
