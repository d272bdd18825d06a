"""Serving engine: continuous batching over several streams, HBM-budget
admission, results independent of batch composition, and engine outputs
(signal + photon noise + 1/f noise) against the oracle."""
import numpy as np
import pytest
import torch

import oracle
import paper_2604_23305_amd as g
from oracle import pink as opk
from paper_2604_23305_amd.serve import Engine, Request
from tests.gpu_util import new_ctx
from workloads import Scenario, configs

pytestmark = pytest.mark.gpu


def small_requests():
    """Eight small requests with mixed pixels, channels, bins, lengths."""
    screens = [configs.screen(64, 4096, 60 + i) for i in range(2)]
    rng = np.random.default_rng(3)
    reqs, specs, srcs = [], {}, {}
    for i in range(8):
        r = dict(rid=i, arrival_s=0.0, n_pix=int(rng.choice([1, 7])),
                 K=int(rng.choice([40, 70])), F=int(rng.choice([500, 750])),
                 t_total=int(rng.integers(300, 2500)),
                 screen=int(rng.integers(0, 2)),
                 seed=int(rng.integers(0, 2**40)))
        reqs.append(configs.c5_scenario(r, screens, specs, srcs))
    return reqs


@pytest.fixture(scope="module")
def setup():
    ctx = new_ctx(precision=g.PREC_SPLIT_BF16, workspace_bytes=256 << 20)
    scens = small_requests()
    runs, ids = [], {}
    for sc in scens:
        key = (id(sc.screen), id(sc.spectral))
        run = g.ScenarioRun(ctx, sc,
                            screen_id=ids.get(("scr", id(sc.screen))),
                            spec_id=ids.get(("spec", id(sc.spectral))))
        ids[("scr", id(sc.screen))] = run.screen_id
        ids[("spec", id(sc.spectral))] = run.spec_id
        runs.append(run)
    yield ctx, scens, runs
    g.free(ctx)


def _reqs(runs):
    return [Request.from_run(r, i, 0.0) for i, r in enumerate(runs)]


def _serve(ctx, reqs, **kw):
    outs = {}
    eng = Engine(ctx, keep_outputs=True,
                 on_done=lambda r: outs.__setitem__(r.rid, r.tod), **kw)
    stats = eng.run(reqs, realtime=False)
    return outs, stats


def test_alone_equals_in_mix_bitwise(setup):
    ctx, scens, runs = setup
    alone = {}
    for i, run in enumerate(runs):
        o, _ = _serve(ctx, [Request.from_run(run, i, 0.0)], n_streams=1,
                      chunk_rows=1 << 20)
        alone[i] = o[i]
    mixed, stats = _serve(ctx, _reqs(runs), n_streams=4, chunk_rows=2048)
    assert len(stats.records) == len(runs)
    for i in range(len(runs)):
        assert torch.equal(alone[i], mixed[i]), i


def test_budget_admission_queues_and_completes(setup):
    ctx, scens, runs = setup
    reqs = _reqs(runs)
    biggest = max(r.out_bytes for r in reqs)
    budget = biggest + 1
    seen = []
    eng = Engine(ctx, n_streams=2, hbm_budget_bytes=budget, chunk_rows=4096,
                 keep_outputs=True)
    orig = eng._admit

    def admit(now):
        orig(now)
        seen.append(eng.used)
    eng._admit = admit
    stats = eng.run(reqs, realtime=False)
    assert len(stats.records) == len(reqs)
    assert max(seen) <= budget
    too_big = max(_reqs(runs), key=lambda r: r.out_bytes)
    with pytest.raises(ValueError):
        Engine(ctx, hbm_budget_bytes=biggest - 1).run([too_big],
                                                      realtime=False)


def test_engine_outputs_match_oracle(setup):
    ctx, scens, runs = setup
    outs, _ = _serve(ctx, _reqs(runs[:3]), n_streams=2, chunk_rows=1024)
    for i in range(3):
        sc = scens[i]
        ref = oracle.tod.simulate(sc)
        nep2 = oracle.tod.reference_nep2(sc)
        A = opk.amplitude(nep2, sc.pink_alpha, sc.pink_knee_hz)
        pink = np.stack([np.stack([opk.series(sc.seed, p, k, A[k],
                                              sc.pink_alpha[k], sc.t_total,
                                              sc.f_sample_hz)
                                   for k in range(sc.K)])
                         for p in range(sc.n_pix)])
        expect = ref["tod"] + pink
        got = outs[i].cpu().numpy().astype(np.float64)
        err = np.abs(got - expect) / np.abs(expect)
        print(f"  request {i}: {sc.n_pix} px {sc.K} ch {sc.F} bins "
              f"{sc.t_total} samples: max rel err {err.max():.2e}", flush=True)
        assert err.max() <= 1e-6


def test_realtime_arrivals_and_latency(setup):
    ctx, scens, runs = setup
    reqs = [Request.from_run(r, i, 0.02 * i) for i, r in enumerate(runs)]
    eng = Engine(ctx, n_streams=4, chunk_rows=4096)
    stats = eng.run(reqs, realtime=True)
    s = stats.summary()
    assert s["requests"] == len(reqs)
    for rec in stats.records:
        assert rec["done_s"] >= rec["arrival_s"]
        assert rec["admit_s"] >= rec["arrival_s"] - 1e-3
    assert s["p99_ms"] >= s["p50_ms"] > 0


def test_engine_close_releases_its_stream_workspaces(setup):
    """An engine that made its own streams returns their workspaces to the
    context's budget on close(); streams passed in are left alone, and
    releasing a stream without a workspace is ENOTFOUND."""
    ctx, scens, runs = setup
    used0, _ = g.memory(ctx)
    eng = Engine(ctx, n_streams=3)
    eng.run(_reqs(runs[:3]), realtime=False)
    torch.cuda.synchronize()
    used1, _ = g.memory(ctx)
    assert used1 > used0
    eng.close()
    assert g.memory(ctx)[0] == used0
    s = torch.cuda.Stream()
    eng2 = Engine(ctx, streams=[s])
    eng2.run(_reqs(runs[:1]), realtime=False)
    eng2.close()
    assert g.memory(ctx)[0] > used0
    g.release_stream(ctx, s)
    assert g.memory(ctx)[0] == used0
    with pytest.raises(g.GtodError, match="ENOTFOUND"):
        g.release_stream(ctx, s)


def test_engine_jsonl_log(setup, tmp_path):
    """With log_path the engine appends one JSON record per completed
    request, the same records stats.records holds."""
    import json
    ctx, scens, runs = setup
    log = tmp_path / "requests.jsonl"
    eng = Engine(ctx, n_streams=2, log_path=str(log))
    stats = eng.run(_reqs(runs[:4]), realtime=False)
    eng.close()
    lines = [json.loads(x) for x in log.read_text().splitlines()]
    assert len(lines) == 4
    assert sorted(r["rid"] for r in lines) == [0, 1, 2, 3]
    assert lines == stats.records
