"""Continuous-batching request engine on top of the gtod C-ABI.

Requests (each one whole simulation: pixels x channels x samples) arrive
over time.  The engine
  * admits a request when its arrival time has passed and its output fits in
    the HBM budget (first come, first served; later arrivals wait behind an
    earlier one that does not fit yet);
  * pins each admitted request to one of several HIP streams, the one with
    the least outstanding work (detector samples not yet issued), so that
    work of different requests runs concurrently on the device and a small
    request does not queue behind a large one when another stream is idle;
  * issues, per stream, one gtod_simulate_tod call holding the next sample
    chunk of every active request on that stream, keeping a bounded number
    of calls in flight per stream.  The jobs of a call run one after the
    other, so they are ordered by the work their requests have left, least
    first, and the chunks that complete a request go in a call of their own
    ahead of the rest, so that its completion event does not wait for them;
  * records completion with device events, frees the request's memory and
    admits waiting requests as memory frees up.
Every request first gets its 1/f job (written into its TOD), then its
signal chunks, which accumulate.  Chunks are fixed in request-local sample
indices and every noise value is keyed by (seed, pixel, channel, sample), so
a request's TOD does not depend on what it was batched with.

Screens, spectral setups and source cubes are resident and shared; the
caller loads them (load_screen / load_filters) and passes their ids.
"""
from __future__ import annotations

import collections
import json
import time
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional

import numpy as np

from . import _abi
from .binding import simulate_tod


@dataclass
class Request:
    """One simulation.  Pixel offsets are host arrays; the source cube is a
    device tensor [n_el][n_az][F] (or None)."""
    rid: int
    arrival_s: float
    spec_id: int
    screen_id: int
    K: int
    n_pix: int
    dphi: np.ndarray
    dtheta: np.ndarray
    t_total: int
    seed: int
    scan_kind: int = _abi.SCAN_DAISY
    scan_params: tuple = (0.0, 0.0, 0.0)
    phi0: float = 0.0
    theta0: float = np.pi / 3
    cube: object = None
    cube_grid: tuple = (0, 0, 0, 0.0, 0.0, 0.0, 0.0)  # n_az, n_el, ld, az0, daz, el0, del
    pink_alpha: Optional[np.ndarray] = None
    pink_knee_hz: float = 1.0
    pink_A: Optional[np.ndarray] = None   # [K] levels; None = knee-derived
    photon_noise: bool = True
    precision: int = -1
    # filled by the engine
    tod: object = None
    stream_idx: int = -1
    next_t: int = 0
    t_admit: float = float("nan")
    t_first: float = float("nan")
    t_done: float = float("nan")
    done_event: object = None

    @property
    def det_samples(self) -> int:
        return self.n_pix * self.K * self.t_total

    @property
    def remaining(self) -> int:
        """Detector samples not yet issued."""
        return self.n_pix * self.K * (self.t_total - self.next_t)

    @property
    def out_bytes(self) -> int:
        return self.det_samples * 4

    @staticmethod
    def from_run(run, rid, arrival_s, precision=-1) -> "Request":
        """Request for a binding.ScenarioRun (resident screen, spectral
        setup and source cube)."""
        sc = run.sc
        cube_grid = (0, 0, 0, 0.0, 0.0, 0.0, 0.0)
        if sc.source is not None:
            s = sc.source
            cube_grid = (s.n_az, s.n_el, s.cube.shape[2], s.az0, s.daz,
                         s.el0, s.del_)
        kind = {"stare": _abi.SCAN_STARE, "daisy": _abi.SCAN_DAISY}[
            sc.scan.kind]
        return Request(rid=rid, arrival_s=arrival_s, spec_id=run.spec_id,
                       screen_id=run.screen_id, K=sc.K, n_pix=sc.n_pix,
                       dphi=run.dphi, dtheta=run.dtheta, t_total=sc.t_total,
                       seed=sc.seed, scan_kind=kind,
                       scan_params=(sc.scan.r_petal, sc.scan.omega,
                                    sc.scan.Omega),
                       phi0=sc.scan.phi0, theta0=sc.scan.theta0,
                       cube=run.cube, cube_grid=cube_grid,
                       pink_alpha=run.alpha, pink_knee_hz=sc.pink_knee_hz,
                       pink_A=getattr(run, "pink_A", None),
                       photon_noise=sc.photon_noise, precision=precision)


@dataclass
class EngineStats:
    records: List[dict] = field(default_factory=list)

    def summary(self):
        lat = np.array([r["latency_ms"] for r in self.records])
        det = sum(r["det_samples"] for r in self.records)
        first = min(r["arrival_s"] for r in self.records)
        last = max(r["done_s"] for r in self.records)
        return {"requests": len(self.records),
                "p50_ms": float(np.percentile(lat, 50)),
                "p99_ms": float(np.percentile(lat, 99)),
                "mean_ms": float(lat.mean()),
                "det_samples": int(det),
                "makespan_s": last - first,
                "det_samples_per_s": det / (last - first)}


class Engine:
    def __init__(self, ctx, n_streams=4, hbm_budget_bytes=64 << 30,
                 chunk_rows=1 << 18, max_inflight=2, keep_outputs=False,
                 on_done: Optional[Callable[[Request], None]] = None,
                 streams=None, log_path: Optional[str] = None):
        """streams: torch.cuda.Stream objects to run on (n_streams is then
        ignored).  The library keeps a workspace per stream until the
        stream is released, so engines that follow one another on a context
        should share their streams; streams the engine makes itself are
        released by close().  log_path: append one JSON line per completed
        request (its record in stats.records) to this file."""
        import torch
        self.torch = torch
        self.ctx = ctx
        self._own_streams = streams is None
        self.streams = list(streams) if streams is not None else [
            torch.cuda.Stream() for _ in range(n_streams)]
        n_streams = len(self.streams)
        self.budget = hbm_budget_bytes
        self.used = 0
        self.chunk_rows = chunk_rows
        self.max_inflight = max_inflight
        self.keep_outputs = keep_outputs
        self.on_done = on_done
        self.inflight: Dict[int, collections.deque] = {
            i: collections.deque() for i in range(n_streams)}
        self.active: List[Request] = []
        self.pending: collections.deque = collections.deque()
        self.done: List[Request] = []
        self.stats = EngineStats()
        self.log_path = log_path
        self._rr = 0
        self._t0_event = None
        self._t0_wall = None

    def close(self):
        """Release the workspaces of the streams this engine created (after
        their queued work); streams passed in stay with the caller."""
        if self._own_streams:
            from . import binding
            for s in self.streams:
                try:
                    binding.release_stream(self.ctx, s)
                except binding.GtodError as e:
                    if e.status != _abi.ENOTFOUND:
                        raise
            self.streams = []
            self._own_streams = False

    # ------------------------------------------------------------------
    def chunk_len(self, r: Request) -> int:
        n = max(128, (self.chunk_rows // r.n_pix) // 128 * 128)
        return min(n, r.t_total)

    def _signal_job(self, r: Request, a: int, b: int) -> _abi.Job:
        j = _abi.Job(kind=_abi.JOB_SIGNAL, screen_id=r.screen_id,
                     spec_id=r.spec_id, n_pix=r.n_pix,
                     dphi_rad=r.dphi.ctypes.data,
                     dtheta_rad=r.dtheta.ctypes.data,
                     scan_kind=r.scan_kind, precision=r.precision,
                     phi0_rad=r.phi0, theta0_rad=r.theta0,
                     t_begin=a, t_end=b, t_total=r.t_total, seed=r.seed,
                     flags=_abi.JOB_ACCUMULATE
                     | (_abi.JOB_PHOTON_NOISE if r.photon_noise else 0),
                     tod=r.tod.data_ptr())
        for i, v in enumerate(r.scan_params):
            j.scan_params[i] = v
        if r.cube is not None:
            n_az, n_el, ld, az0, daz, el0, del_ = r.cube_grid
            j.cube = r.cube.data_ptr()
            j.n_az, j.n_el, j.cube_ld = n_az, n_el, ld
            j.az0_rad, j.daz_rad, j.el0_rad, j.del_rad = az0, daz, el0, del_
        return j

    def _pink_job(self, r: Request) -> _abi.Job:
        return _abi.Job(kind=_abi.JOB_PINK, spec_id=r.spec_id, n_pix=r.n_pix,
                        t_total=r.t_total, seed=r.seed, flags=0,
                        pink_alpha=r.pink_alpha.ctypes.data,
                        pink_knee_hz=r.pink_knee_hz,
                        pink_A=(r.pink_A.ctypes.data
                                if r.pink_A is not None else None),
                        tod=r.tod.data_ptr())

    def _now(self) -> float:
        return time.perf_counter() - self._t0_wall

    def _pick_stream(self) -> int:
        """Stream with the least outstanding work; ties go round robin."""
        n = len(self.streams)
        load = [0] * n
        for r in self.active:
            load[r.stream_idx] += r.remaining
        order = [(self._rr + i) % n for i in range(n)]
        si = min(order, key=lambda i: load[i])
        self._rr = (si + 1) % n
        return si

    # ------------------------------------------------------------------
    def _admit(self, now: float):
        torch = self.torch
        while self.pending and self.pending[0].arrival_s <= now:
            r = self.pending[0]
            if r.out_bytes > self.budget:
                raise ValueError(f"request {r.rid} needs {r.out_bytes} B, "
                                 f"more than the whole budget")
            if self.used + r.out_bytes > self.budget:
                break
            self.pending.popleft()
            self.used += r.out_bytes
            r.stream_idx = self._pick_stream()
            # allocate (and zero) on the request's own stream so that its
            # kernels are ordered after the fill
            alloc = torch.empty if r.pink_alpha is not None else torch.zeros
            shape = (r.n_pix, r.K, r.t_total)
            with torch.cuda.stream(self.streams[r.stream_idx]):
                try:
                    r.tod = alloc(shape, dtype=torch.float32, device="cuda")
                except torch.cuda.OutOfMemoryError:
                    # blocks cached for other streams: release and retry
                    torch.cuda.synchronize()
                    torch.cuda.empty_cache()
                    r.tod = alloc(shape, dtype=torch.float32, device="cuda")
            r.t_admit = now
            r.next_t = 0
            self.active.append(r)
            r._need_pink = r.pink_alpha is not None

    def _issue(self, si: int, now: float) -> bool:
        torch = self.torch
        q = self.inflight[si]
        while q and q[0].query():
            q.popleft()
        if len(q) >= self.max_inflight:
            return False
        # requests whose last chunk goes out now get a call (and completion
        # event) of their own, ahead of the others on this stream
        fin_jobs, rest_jobs, finishing = [], [], []
        mine = [r for r in self.active
                if r.stream_idx == si and r.next_t < r.t_total]
        for r in sorted(mine, key=lambda r: (r.remaining, r.rid)):
            a = r.next_t
            b = min(r.t_total, a + self.chunk_len(r))
            jobs = fin_jobs if b >= r.t_total else rest_jobs
            if getattr(r, "_need_pink", False):
                jobs.append(self._pink_job(r))
                r._need_pink = False
            jobs.append(self._signal_job(r, a, b))
            r.next_t = b
            if np.isnan(r.t_first):
                r.t_first = now
            if b >= r.t_total:
                finishing.append(r)
        if not fin_jobs and not rest_jobs:
            return False
        stream = self.streams[si]
        ev = None
        for jobs in (fin_jobs, rest_jobs):
            if not jobs:
                continue
            simulate_tod(self.ctx, jobs, stream)
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(stream)
            if jobs is fin_jobs:
                for r in finishing:
                    r.done_event = ev
        q.append(ev)
        return True

    def _retire(self):
        still = []
        for r in self.active:
            if r.done_event is not None and r.done_event.query():
                t_gpu = self._t0_event.elapsed_time(r.done_event) / 1e3
                r.t_done = t_gpu
                self.used -= r.out_bytes
                rec = dict(
                    rid=r.rid, arrival_s=r.arrival_s, admit_s=r.t_admit,
                    first_issue_s=r.t_first, done_s=t_gpu,
                    latency_ms=(t_gpu - r.arrival_s) * 1e3,
                    det_samples=r.det_samples, bytes=r.out_bytes,
                    n_pix=r.n_pix, K=r.K, t_total=r.t_total,
                    stream=r.stream_idx)
                self.stats.records.append(rec)
                if self.log_path:
                    with open(self.log_path, "a") as f:
                        f.write(json.dumps(rec, default=float) + "\n")
                if self.on_done:
                    self.on_done(r)
                if not self.keep_outputs:
                    r.tod = None
                self.done.append(r)
            else:
                still.append(r)
        self.active = still

    # ------------------------------------------------------------------
    def run(self, requests: List[Request], realtime=True, poll_s=2e-4):
        """Serve requests (sorted by arrival).  realtime: arrivals happen at
        their wall-clock offsets; otherwise all have arrived at start."""
        torch = self.torch
        reqs = sorted(requests, key=lambda r: (r.arrival_s, r.rid))
        if not realtime:
            for r in reqs:
                r.arrival_s = 0.0
        self.pending.extend(reqs)
        torch.cuda.synchronize()
        self._t0_event = torch.cuda.Event(enable_timing=True)
        self._t0_event.record(self.streams[0])
        torch.cuda.synchronize()
        self._t0_wall = time.perf_counter()
        while self.pending or self.active:
            now = self._now()
            self._retire()
            self._admit(now)
            issued = False
            for si in range(len(self.streams)):
                issued |= self._issue(si, now)
            if not issued:
                time.sleep(poll_s)
        torch.cuda.synchronize()
        self._retire()
        return self.stats
