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


class _FakeEvent:
    def __init__(self, **kw):
        self.stream = None

    def record(self, stream):
        self.stream = stream

    def query(self):
        return False


def _host_engine(monkeypatch, n_streams=3):
    """Engine with the device calls replaced by recorders."""
    from paper_2604_23305_amd import serve
    calls = []
    monkeypatch.setattr(serve, "simulate_tod",
                        lambda ctx, jobs, stream: calls.append((stream, jobs)))
    eng = serve.Engine.__new__(serve.Engine)
    eng.torch = types.SimpleNamespace(
        cuda=types.SimpleNamespace(Event=_FakeEvent))
    eng.ctx = None
    eng.streams = [f"s{i}" for i in range(n_streams)]
    eng.chunk_rows = 1 << 12
    eng.max_inflight = 2
    eng.inflight = {i: __import__("collections").deque()
                    for i in range(n_streams)}
    eng.active = []
    eng._rr = 0
    return eng, calls


def _req(rid, n_pix, K, t_total, next_t=0, stream=-1):
    q = Request(rid=rid, arrival_s=0.0, spec_id=0, screen_id=0, K=K,
                n_pix=n_pix, dphi=np.zeros(n_pix), dtheta=np.zeros(n_pix),
                t_total=t_total, seed=rid, tod=types.SimpleNamespace(
                    data_ptr=lambda: 0))
    q.next_t, q.stream_idx = next_t, stream
    q._need_pink = False
    return q


def test_new_request_goes_to_least_loaded_stream(monkeypatch):
    eng, _ = _host_engine(monkeypatch)
    eng.active = [_req(0, 49, 720, 96000, stream=0),
                  _req(1, 1, 64, 1600, stream=1),
                  _req(2, 7, 347, 9600, stream=2)]
    assert eng._pick_stream() == 1
    # ties go round robin from the stream after the last pick
    eng.active = []
    assert [eng._pick_stream() for _ in range(4)] == [2, 0, 1, 2]


def test_finishing_chunks_go_first_in_their_own_call(monkeypatch):
    eng, calls = _host_engine(monkeypatch)
    big = _req(0, 7, 347, 100000, stream=1)       # several chunks left
    small = _req(1, 1, 64, 1000, stream=1)        # one chunk: finishes now
    mid = _req(2, 1, 64, 50000, stream=1)         # several chunks left
    other = _req(3, 1, 64, 500, stream=0)         # another stream
    eng.active = [big, small, mid, other]
    assert eng._issue(1, now=0.0)
    assert len(calls) == 2 and all(s == "s1" for s, _ in calls)
    (_, fin), (_, rest) = calls
    assert [(j.t_begin, j.t_end, j.t_total) for j in fin] == [(0, 1000, 1000)]
    # the rest ordered by the work their requests have left, least first
    assert [j.t_total for j in rest] == [50000, 100000]
    assert small.done_event is not None and small.done_event is not \
        eng.inflight[1][-1]
    assert big.done_event is None and mid.done_event is None
    assert other.next_t == 0 and len(eng.inflight[1]) == 1


def test_engine_runs_on_given_streams():
    from paper_2604_23305_amd.serve import Engine
    eng = Engine(None, n_streams=4, streams=["a", "b"])
    assert eng.streams == ["a", "b"] and sorted(eng.inflight) == [0, 1]
