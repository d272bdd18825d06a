"""The serving workload at full size: all 256 requests of the seeded stream
(1-49 pixels, 64-720 channels, 1000-4000 bins, 10-600 s) through the
engine on the split-BF16 path, with sampled requests checked against the
oracle: the sixteen smallest in full (every pixel, channel and sample),
sixteen others on their last pixel over the last 128 samples of four
channels.  Same bar as the other serving tests: TOD (signal, photon and 1/f
noise) within 1e-6 relative."""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
import torch

import oracle
import paper_2604_23305_amd as g
from oracle import pink as opk
from paper_2604_23305_amd.serve import Engine, Request
from workloads import configs

pytestmark = pytest.mark.gpu

N_FULL, N_WIN, WIN, N_CH = 16, 16, 128, 4


def oracle_tod(sc, p, ks, a, b):
    ref = oracle.tod.simulate(sc, a, b, pixels=[p])["tod"][0][ks]
    A = opk.amplitude(oracle.tod.reference_nep2(sc), sc.pink_alpha,
                      sc.pink_knee_hz)
    pink = np.stack([opk.series(sc.seed, p, k, A[k], sc.pink_alpha[k],
                                sc.t_total, sc.f_sample_hz)[a:b] for k in ks])
    return ref + pink


def test_c5_stream_sampled_against_oracle():
    reqs = configs.c5_requests()
    screens = configs.c5_screens()
    ctx = g.sim_init(device=0, precision=g.PREC_SPLIT_BF16,
                     workspace_bytes=4 << 30)
    try:
        scr_ids = [g.load_screen(ctx, s.pwv_mm, s.dx_m, s.dy_m, s.ix0, s.iy0,
                                 s.h_column_m, s.wind_mps) for s in screens]
        sp_cache, src_cache, spec_ids, cubes, scen = {}, {}, {}, {}, {}
        requests = []
        for r in reqs:
            sc = configs.c5_scenario(r, screens, sp_cache, src_cache)
            key = (r["K"], r["F"])
            run = g.ScenarioRun(ctx, sc, screen_id=scr_ids[r["screen"]],
                                spec_id=spec_ids.get(key),
                                cube=cubes.get(r["F"]))
            spec_ids[key] = run.spec_id
            cubes[r["F"]] = run.cube
            requests.append(Request.from_run(run, r["rid"], r["arrival_s"]))
            scen[r["rid"]] = sc
        by_size = sorted(requests, key=lambda q: q.det_samples)
        full = {q.rid for q in by_size[:N_FULL]}
        rest = by_size[N_FULL:]
        win = {q.rid for q in rest[:: max(1, len(rest) // N_WIN)][:N_WIN]}
        got = {}

        def keep(r):
            if r.rid in full:
                got[r.rid] = r.tod.cpu().numpy()
            elif r.rid in win:
                ks = np.linspace(0, r.K - 1, N_CH).round().astype(int)
                got[r.rid] = r.tod[r.n_pix - 1, ks, -WIN:].cpu().numpy()
        stats = Engine(ctx, n_streams=4, hbm_budget_bytes=150 << 30,
                       on_done=keep).run(requests, realtime=False)
        assert len(stats.records) == len(requests)
        print(f"  {len(requests)} requests, {stats.summary()['det_samples']:.3e} "
              "detector-samples", flush=True)
        # oracle per (request, pixel), in threads (NumPy releases the GIL)
        jobs = []
        for rid in sorted(full):
            sc = scen[rid]
            jobs += [(rid, p, list(range(sc.K)), 0, sc.t_total)
                     for p in range(sc.n_pix)]
        for rid in sorted(win):
            sc = scen[rid]
            ks = list(np.linspace(0, sc.K - 1, N_CH).round().astype(int))
            jobs.append((rid, sc.n_pix - 1, ks, sc.t_total - WIN, sc.t_total))
        with ThreadPoolExecutor(min(16, os.cpu_count() or 1)) as ex:
            outs = list(ex.map(lambda j: oracle_tod(scen[j[0]], *j[1:]), jobs))
        expects = {}
        for j, o in zip(jobs, outs):
            expects.setdefault(j[0], []).append(o)
        worst = 0.0
        for rid in sorted(full | win):
            sc = scen[rid]
            expect = (np.stack(expects[rid]) if rid in full
                      else expects[rid][0])
            err = np.abs(got[rid] - expect) / np.abs(expect)
            worst = max(worst, float(err.max()))
            assert err.max() <= 1e-6, (rid, sc.n_pix, sc.K, sc.F, sc.t_total,
                                       float(err.max()))
        print(f"  {len(full)} full + {len(win)} windowed requests: max rel err "
              f"{worst:.2e}", flush=True)
    finally:
        g.free(ctx)
