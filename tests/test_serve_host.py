"""Host-side logic of the serving engine (no GPU): request construction
from a scenario binding, chunk sizing and the summary statistics."""
import types

import numpy as np

from paper_2604_23305_amd import _abi
from paper_2604_23305_amd.serve import EngineStats, Request
from workloads import configs


def fake_run(sc):
    return types.SimpleNamespace(
        sc=sc, spec_id=3, screen_id=5, dphi=np.asarray(sc.dphi, float),
        dtheta=np.asarray(sc.dtheta, float), cube=None,
        alpha=np.asarray(sc.pink_alpha, float))


def test_request_from_run_carries_the_scenario():
    screens = [configs.screen(64, 4096, 1, uniform=True)]
    r = dict(rid=7, arrival_s=1.5, n_pix=7, K=64, F=1000, t_total=3000,
             screen=0, seed=123)
    sc = configs.c5_scenario(r, screens)
    q = Request.from_run(fake_run(sc), 7, 1.5)
    assert (q.rid, q.arrival_s, q.spec_id, q.screen_id) == (7, 1.5, 3, 5)
    assert (q.K, q.n_pix, q.t_total, q.seed) == (64, 7, 3000, 123)
    assert q.scan_kind == _abi.SCAN_DAISY
    assert q.scan_params == (sc.scan.r_petal, sc.scan.omega, sc.scan.Omega)
    assert q.det_samples == 7 * 64 * 3000 and q.out_bytes == 4 * q.det_samples
    assert q.cube_grid[:3] == (55, 55, 1000)


def test_chunk_length_multiple_of_tile():
    from paper_2604_23305_amd.serve import Engine
    eng = Engine.__new__(Engine)
    eng.chunk_rows = 1 << 18
    q = types.SimpleNamespace(n_pix=49, t_total=96000)
    n = Engine.chunk_len(eng, q)
    assert n % 128 == 0 and n * 49 <= 1 << 18
    q = types.SimpleNamespace(n_pix=1, t_total=1000)
    assert Engine.chunk_len(eng, q) == 1000


def test_stats_summary():
    st = EngineStats(records=[
        dict(latency_ms=10.0, det_samples=100, arrival_s=0.0, done_s=1.0),
        dict(latency_ms=30.0, det_samples=300, arrival_s=0.5, done_s=2.0)])
    s = st.summary()
    assert s["requests"] == 2 and s["det_samples"] == 400
    assert s["det_samples_per_s"] == 200.0
    assert s["p50_ms"] == 20.0
