"""Thin Python binding of the gtod C-ABI (argument marshalling only).

The five calls keep the C names without the prefix: sim_init, load_screen,
load_filters, simulate_tod, free.  Device memory and streams come from
PyTorch (tensors' data pointers, a torch stream's raw handle); every step
of the simulation runs in the HIP library.  `ScenarioRun` marshals a
plain-data scenario (angles, tables, stage list, source cube, ...) into the
descriptors and device buffers.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

from . import _abi
from ._abi import (JOB_ACCUMULATE, JOB_KELVIN, JOB_PHOTON_NOISE, JOB_PINK,
                   JOB_SIGNAL,
                   OBJ_CTX, OBJ_SCREEN, OBJ_SPEC, PREC_FP32, PREC_SPLIT_BF16,
                   SCAN_DAISY, SCAN_STARE, SCAN_TRAJ)


class GtodError(RuntimeError):
    def __init__(self, status: int, msg: str):
        self.status = status
        super().__init__(f"{_abi.STATUS_NAMES.get(status, status)}: {msg}")


def _check(ctx, st):
    if st != 0:
        lib = _abi.load()
        msg = lib.gtod_last_error(ctx)
        raise GtodError(st, msg.decode() if msg else "")


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


# --------------------------------------------------------------------------
# the five calls
# --------------------------------------------------------------------------
def sim_init(device=0, precision=PREC_FP32, hbm_budget_bytes=0,
             workspace_bytes=0, f_sample_hz=160.0, eta_taper=0.85,
             rho_surf_m=42e-6, eta_pol=0.5, delta_J=188e-6 * 1.602176634e-19,
             eta_pb=0.4, t_cmb_K=2.725, strict_range=False):
    lib = _abi.load()
    d = _abi.InitDesc(device=device, precision=precision,
                      flags=_abi.INIT_STRICT_RANGE if strict_range else 0,
                      hbm_budget_bytes=hbm_budget_bytes,
                      workspace_bytes=workspace_bytes,
                      f_sample_hz=f_sample_hz, eta_taper=eta_taper,
                      rho_surf_m=rho_surf_m, eta_pol=eta_pol,
                      delta_J=delta_J, eta_pb=eta_pb, t_cmb_K=t_cmb_K)
    ctx = C.c_void_p()
    _check(None, lib.gtod_sim_init(C.byref(d), C.byref(ctx)))
    return ctx


def load_screen(ctx, pwv_mm, dx_m, dy_m, ix0, iy0, h_column_m, wind_mps):
    """pwv_mm: host float64 [ny][nx] array or a CUDA float64 tensor."""
    lib = _abi.load()
    if hasattr(pwv_mm, "data_ptr"):
        ptr, mem, (ny, nx) = pwv_mm.data_ptr(), 1, tuple(pwv_mm.shape)
        keep = pwv_mm
    else:
        keep = _f64(pwv_mm)
        ptr, mem, (ny, nx) = keep.ctypes.data, 0, keep.shape
    d = _abi.ScreenDesc(pwv_mm=ptr, nx=nx, ny=ny, dx_m=dx_m, dy_m=dy_m,
                        ix0=ix0, iy0=iy0, h_column_m=h_column_m,
                        wind_mps=wind_mps, mem_kind=mem)
    sid = C.c_int32()
    _check(ctx, lib.gtod_load_screen(ctx, C.byref(d), C.byref(sid)))
    del keep
    return sid.value


_STAGE_KIND = {"reflect": _abi.STAGE_REFLECT,
               "atm_coupled": _abi.STAGE_ATM_COUPLED,
               "ohmic": _abi.STAGE_OHMIC,
               "refractive": _abi.STAGE_REFRACTIVE}
_FILT_MODE = {"lorentz": _abi.FILT_LORENTZ,
              "filterbank": _abi.FILT_FILTERBANK,
              "matrix": _abi.FILT_MATRIX}


def load_filters(ctx, nu_hz, w_hz, eta_z, pwv0_mm, dpwv_mm, t_atm_K, stages,
                 filter_mode, f_hz=None, R=None, eta_peak=None, eta_filt=None,
                 ref_pwv_mm=1.0, ref_el_rad=np.pi / 3):
    """stages: sequence of objects with the fields of workloads.Stage."""
    lib = _abi.load()
    keep = []
    nu, w, ez = _f64(nu_hz), _f64(w_hz), _f64(eta_z)
    keep += [nu, w, ez]
    F = nu.size
    arr = (_abi.Stage * max(len(stages), 1))()
    for i, st in enumerate(stages):
        eta = st.eta
        eta_ptr, eta_const = None, 1.0
        if np.ndim(eta) == 0:
            eta_const = float(eta)
        else:
            e = _f64(eta)
            keep.append(e)
            eta_ptr = e.ctypes.data
        arr[i] = _abi.Stage(kind=_STAGE_KIND[st.kind],
                            ar_coated=int(bool(st.ar_coated)), eta=eta_ptr,
                            eta_const=eta_const, t_K=st.t_K,
                            t_refl_K=st.t_refl_K, eps_ref=st.eps_ref,
                            nu_ref_hz=st.nu_ref_hz, d_m=st.d_m,
                            n_index=st.n_index, tan_delta=st.tan_delta)
    mode = _FILT_MODE[filter_mode]
    fa = [None if x is None else _f64(x) for x in (f_hz, R, eta_peak,
                                                    eta_filt)]
    keep += fa
    K = fa[3].shape[1] if mode == _abi.FILT_MATRIX else fa[0].size
    d = _abi.SpectralDesc(F=F, K=K, nu_hz=nu.ctypes.data, w_hz=w.ctypes.data,
                          n_pwv=ez.shape[0], filter_mode=mode,
                          pwv0_mm=pwv0_mm, dpwv_mm=dpwv_mm,
                          eta_z=ez.ctypes.data, t_atm_K=t_atm_K,
                          n_stage=len(stages),
                          stages=C.cast(arr, C.c_void_p),
                          f_hz=_ptr(fa[0]), R=_ptr(fa[1]),
                          eta_peak=_ptr(fa[2]), eta_filt=_ptr(fa[3]),
                          ref_pwv_mm=ref_pwv_mm, ref_el_rad=ref_el_rad)
    sid = C.c_int32()
    _check(ctx, lib.gtod_load_filters(ctx, C.byref(d), C.byref(sid)))
    return sid.value


def _enqueue(fn, ctx, jobs, stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    handle = stream.cuda_stream if hasattr(stream, "cuda_stream") else stream
    n = len(jobs)
    arr = (_abi.Job * max(n, 1))(*jobs)
    _check(ctx, fn(ctx, arr, n, C.c_void_p(handle)))


def simulate_tod(ctx, jobs: Sequence[_abi.Job], stream=None):
    """Enqueue jobs on a torch stream (default: the current stream)."""
    _enqueue(_abi.load().gtod_simulate_tod, ctx, jobs, stream)


def simulate_tod_noalloc(ctx, jobs: Sequence[_abi.Job], stream=None):
    """As simulate_tod, in the library's static per-GPU scratch: the call
    allocates no device memory (gtod_simulate_tod_noalloc)."""
    _enqueue(_abi.load().gtod_simulate_tod_noalloc, ctx, jobs, stream)


def release_stream(ctx, stream):
    """Free the workspace of a torch stream (or raw hipStream_t handle)
    after its queued work (gtod_release_stream)."""
    lib = _abi.load()
    handle = stream.cuda_stream if hasattr(stream, "cuda_stream") else stream
    _check(ctx, lib.gtod_release_stream(ctx, C.c_void_p(handle)))


def free(ctx, kind=OBJ_CTX, obj_id=0):
    lib = _abi.load()
    _check(ctx, lib.gtod_free(ctx, kind, obj_id))


# --------------------------------------------------------------------------
# utilities
# --------------------------------------------------------------------------
def memory(ctx):
    lib = _abi.load()
    u, b = C.c_uint64(), C.c_uint64()
    _check(ctx, lib.gtod_memory(ctx, C.byref(u), C.byref(b)))
    return u.value, b.value


def counters(ctx):
    """(screen clamps, table clamps, rows with elevation outside (0, pi),
    (row, bin) elements with |P - P_ref| > P / 8)"""
    lib = _abi.load()
    out = (C.c_uint64 * 4)()
    _check(ctx, lib.gtod_get_counters(ctx, out))
    return tuple(int(v) for v in out)


def spec_nep2_ref(ctx, spec_id, K):
    lib = _abi.load()
    out = np.zeros(K, dtype=np.float64)
    _check(ctx, lib.gtod_spec_nep2_ref(ctx, spec_id,
                                       out.ctypes.data_as(C.POINTER(C.c_double))))
    return out


def skydip(ctx, spec_id, K, el_rad, pwv_lo_mm, pwv_hi_mm, n,
           return_sweep=False):
    """Brightness-temperature scale of a spectral setup by a simulated
    skydip; returns (a, b) per channel (P = a + b T_b), plus the sweep's
    (p_kid, t_b) [n][K] with return_sweep.  Later KELVIN jobs of the setup
    use this scale."""
    lib = _abi.load()
    a = np.zeros(K)
    b = np.zeros(K)
    pk = np.zeros((n, K)) if return_sweep else None
    tb = np.zeros((n, K)) if return_sweep else None
    _check(ctx, lib.gtod_skydip(ctx, spec_id, el_rad, pwv_lo_mm, pwv_hi_mm,
                                n, _ptr(a), _ptr(b), _ptr(pk), _ptr(tb)))
    return (a, b, pk, tb) if return_sweep else (a, b)


def reduce(ctx, desc: _abi.ReduceDesc, stream=None):
    """Enqueue gtod_reduce (common-mode subtraction and gridding)."""
    lib = _abi.load()
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    _check(ctx, lib.gtod_reduce(ctx, C.byref(desc),
                                C.c_void_p(stream.cuda_stream)))


def simulate_to_disk(ctx, signal: _abi.Job, pink: Optional[_abi.Job], out_dir,
                     device_bytes, host_bytes=256 << 20, pwv=True,
                     pix_per_group=0):
    """Out-of-core run: the whole observation in pixel groups, streamed to
    out_dir/{tod,pwv,time}.npy.  Returns (wall s, bytes, groups, pixels
    per group)."""
    lib = _abi.load()
    d = _abi.SinkDesc(dir=str(out_dir).encode(), device_bytes=device_bytes,
                      host_bytes=host_bytes,
                      flags=_abi.SINK_PWV if pwv else 0,
                      pix_per_group=pix_per_group)
    st = (C.c_double * 4)()
    _check(ctx, lib.gtod_simulate_to_disk(
        ctx, C.byref(signal), C.byref(pink) if pink is not None else None,
        C.byref(d), st))
    return st[0], int(st[1]), int(st[2]), int(st[3])


def _stream(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def far_field(ctx, nu_hz, n_a, n_b, da_rad, db_rad, r_tel_m, t_edge_db,
              stream=None):
    """Peak-normalised far field [F][n_b][n_a] (device float32) at
    rho = sqrt((a da)^2 + (b db)^2)."""
    import torch
    lib = _abi.load()
    nu = _f64(nu_hz)
    out = torch.empty((nu.size, n_b, n_a), dtype=torch.float32, device="cuda")
    _check(ctx, lib.gtod_far_field(ctx, _ptr(nu), nu.size, n_a, n_b, da_rad,
                                   db_rad, r_tel_m, t_edge_db,
                                   out.data_ptr(), _stream(stream)))
    return out


def convolve_source(ctx, intensity, nu_hz, daz_rad, el0_rad, del_rad,
                    r_tel_m, t_edge_db, stream=None):
    """Source power cube [n_el][n_az][F] (device float32, W/Hz) from a
    specific-intensity cube of the same shape (Eq. convolve_src)."""
    import torch
    lib = _abi.load()
    nu = _f64(nu_hz)
    n_el, n_az, ld = intensity.shape
    out = torch.empty((n_el, n_az, nu.size), dtype=torch.float32,
                      device=intensity.device)
    _check(ctx, lib.gtod_convolve_source(
        ctx, intensity.data_ptr(), n_az, n_el, ld, _ptr(nu), nu.size,
        daz_rad, el0_rad, del_rad, r_tel_m, t_edge_db, out.data_ptr(),
        nu.size, _stream(stream)))
    return out


def convolve_screen(ctx, screen, dx_m, dy_m, r_tel_m, t_edge_db,
                    stream=None):
    """Footprint-smoothed PWV screen (device float64 [ny][nx])."""
    import torch
    lib = _abi.load()
    ny, nx = screen.shape
    out = torch.empty_like(screen)
    _check(ctx, lib.gtod_convolve_screen(ctx, screen.data_ptr(), nx, ny, dx_m,
                                         dy_m, r_tel_m, t_edge_db,
                                         out.data_ptr(), _stream(stream)))
    return out


def philox(ctx, ctr_dev, out_dev, n, seed, stream=None):
    lib = _abi.load()
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    _check(ctx, lib.gtod_philox(ctx, ctr_dev.data_ptr(), out_dev.data_ptr(),
                                n, seed, C.c_void_p(stream.cuda_stream)))


def profile_enable(ctx, on=True):
    lib = _abi.load()
    _check(ctx, lib.gtod_profile_enable(ctx, 1 if on else 0))


def profile_read(ctx):
    """{kernel: (total_ms, launches, work_units)} since profile_enable."""
    lib = _abi.load()
    n = len(_abi.KERNEL_NAMES)
    out = (C.c_double * (3 * n))()
    _check(ctx, lib.gtod_profile_read(ctx, out, n))
    return {k: (out[3 * i], int(out[3 * i + 1]), out[3 * i + 2])
            for i, k in enumerate(_abi.KERNEL_NAMES)}


def abi_sizes():
    lib = _abi.load()
    out = (C.c_int64 * 6)()
    lib.gtod_abi_sizes(out)
    return list(out)


# --------------------------------------------------------------------------
# scenario marshalling
# --------------------------------------------------------------------------
@dataclass
class Outputs:
    tod: object
    p_kid: object = None
    sigma: object = None
    pwv: object = None
    t0: int = 0            # first sample held
    length: int = 0        # samples held per (pixel, channel)


class ScenarioRun:
    """Loads a scenario's screen and spectral setup into a context, keeps
    its source cube and trajectory on the device, and builds jobs."""

    def __init__(self, ctx, sc, device="cuda", screen_id=None, spec_id=None,
                 cube=None):
        import torch
        self.ctx = ctx
        self.sc = sc
        sp = sc.spectral
        scr = sc.screen
        self.screen_id = screen_id if screen_id is not None else load_screen(
            ctx, scr.pwv_mm, scr.dx_m, scr.dy_m, scr.ix0, scr.iy0,
            scr.h_column_m, scr.wind_mps)
        fil = sp.filters
        self.spec_id = spec_id if spec_id is not None else load_filters(
            ctx, sp.nu_hz, sp.w_hz, sp.eta_z, sp.pwv0_mm, sp.dpwv_mm,
            sp.t_atm_K, sp.stages, fil.mode, fil.f_hz, fil.R, fil.eta_peak,
            fil.matrix, sp.ref_pwv_mm, sp.ref_el_rad)
        self.cube = cube
        if cube is None and sc.source is not None:
            self.cube = torch.from_numpy(np.ascontiguousarray(
                sc.source.cube, dtype=np.float32)).to(device)
        self.traj = None
        if sc.scan.kind == "traj":
            self.traj = torch.from_numpy(_f64(sc.scan.traj)).to(device)
        self.dphi = _f64(sc.dphi)
        self.dtheta = _f64(sc.dtheta)
        self.alpha = (None if sc.pink_alpha is None else _f64(sc.pink_alpha))
        self.pink_A = (None if getattr(sc, "pink_A", None) is None
                       else _f64(sc.pink_A))

    def alloc(self, with_p_kid=False, with_sigma=False, with_pwv=False,
              device="cuda", t0=0, length=None):
        """Output buffers for samples [t0, t0 + length) (default: all)."""
        import torch
        sc = self.sc
        length = sc.t_total if length is None else length
        shape = (sc.n_pix, sc.K, length)
        z = lambda s: torch.zeros(s, dtype=torch.float32, device=device)
        return Outputs(tod=z(shape), p_kid=z(shape) if with_p_kid else None,
                       sigma=z(shape) if with_sigma else None,
                       pwv=z((sc.n_pix, length)) if with_pwv else None,
                       t0=t0, length=length)

    def signal_job(self, out: Outputs, t_begin=0, t_end=None, precision=-1,
                   photon_noise=None, accumulate=False,
                   kelvin=False) -> _abi.Job:
        sc = self.sc
        t_end = sc.t_total if t_end is None else t_end
        noise = sc.photon_noise if photon_noise is None else photon_noise
        kind = {"stare": SCAN_STARE, "daisy": SCAN_DAISY,
                "traj": SCAN_TRAJ}[sc.scan.kind]
        j = _abi.Job(kind=JOB_SIGNAL, screen_id=self.screen_id,
                     spec_id=self.spec_id, n_pix=sc.n_pix,
                     dphi_rad=self.dphi.ctypes.data,
                     dtheta_rad=self.dtheta.ctypes.data, scan_kind=kind,
                     precision=precision, phi0_rad=sc.scan.phi0,
                     theta0_rad=sc.scan.theta0,
                     t_begin=t_begin, t_end=t_end, t_total=sc.t_total,
                     seed=sc.seed,
                     flags=(JOB_PHOTON_NOISE if noise else 0)
                     | (JOB_ACCUMULATE if accumulate else 0)
                     | (JOB_KELVIN if kelvin else 0),
                     out_t0=out.t0, out_ld=out.length,
                     tod=out.tod.data_ptr(),
                     p_kid=out.p_kid.data_ptr() if out.p_kid is not None else None,
                     sigma=out.sigma.data_ptr() if out.sigma is not None else None,
                     pwv=out.pwv.data_ptr() if out.pwv is not None else None)
        j.scan_params[0] = sc.scan.r_petal
        j.scan_params[1] = sc.scan.omega
        j.scan_params[2] = sc.scan.Omega
        if self.traj is not None:
            j.traj = self.traj.data_ptr()
        if self.cube is not None:
            s = sc.source
            j.cube = self.cube.data_ptr()
            j.n_az, j.n_el, j.cube_ld = s.n_az, s.n_el, s.cube.shape[2]
            j.az0_rad, j.daz_rad, j.el0_rad, j.del_rad = s.az0, s.daz, s.el0, s.del_
        return j

    def reduce_desc(self, tod, r_out_rad, t_star=None, maps=None,
                    map_n=31, map_half_rad=0.0, pwv=None, pwv_mean_mm=None,
                    t0=0, T=None) -> _abi.ReduceDesc:
        """Descriptor for gtod_reduce over this run's Kelvin TOD [P][K][ld]
        holding samples [t0, t0 + T); maps = (map, weight) device float64
        tensors [K][map_n][map_n]; the mean PWV comes from the pwv output
        tensor [P][len] or from pwv_mean_mm."""
        sc = self.sc
        T = tod.shape[2] if T is None else T
        kind = {"stare": SCAN_STARE, "daisy": SCAN_DAISY,
                "traj": SCAN_TRAJ}[sc.scan.kind]
        d = _abi.ReduceDesc(spec_id=self.spec_id, n_pix=sc.n_pix,
                            dphi_rad=self.dphi.ctypes.data,
                            dtheta_rad=self.dtheta.ctypes.data,
                            scan_kind=kind, theta0_rad=sc.scan.theta0,
                            t_total=sc.t_total, t0=t0, T=T,
                            ld=tod.shape[2], tod=tod.data_ptr(),
                            r_out_rad=r_out_rad,
                            pwv_mean_mm=(float("nan") if pwv_mean_mm is None
                                         else pwv_mean_mm))
        d.scan_params[0] = sc.scan.r_petal
        d.scan_params[1] = sc.scan.omega
        d.scan_params[2] = sc.scan.Omega
        if self.traj is not None:
            d.traj = self.traj.data_ptr()
        if pwv is not None:
            d.pwv = pwv.data_ptr()
            d.pwv_ld = pwv.shape[1]
            d.pwv_len = pwv.shape[1]
        if t_star is not None:
            d.t_star = t_star.data_ptr()
        if maps is not None:
            d.map, d.weight = maps[0].data_ptr(), maps[1].data_ptr()
            d.map_n = map_n
            d.map_half_rad = map_half_rad
        return d

    def pink_job(self, tod, accumulate=True, kelvin=False) -> _abi.Job:
        sc = self.sc
        return _abi.Job(kind=JOB_PINK, spec_id=self.spec_id, n_pix=sc.n_pix,
                        t_total=sc.t_total, seed=sc.seed,
                        flags=(JOB_ACCUMULATE if accumulate else 0)
                        | (JOB_KELVIN if kelvin else 0),
                        pink_alpha=self.alpha.ctypes.data,
                        pink_knee_hz=sc.pink_knee_hz,
                        pink_A=(self.pink_A.ctypes.data
                                if self.pink_A is not None else None),
                        tod=tod.data_ptr())
