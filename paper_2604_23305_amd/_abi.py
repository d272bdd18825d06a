"""ctypes mirror of include/gtod.h and the library loader.

The HIP library is required: loading fails loudly when libgtod.so has not
been built (python -m paper_2604_23305_amd.build)."""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgtod.so")

OK, EINVAL, ENOMEM, EBUDGET, ENOTFOUND, ERANGE, EDEVICE, EUNSUPPORTED, EIO = \
    0, -1, -2, -3, -4, -5, -6, -7, -8
STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EBUDGET",
                -4: "ENOTFOUND", -5: "ERANGE", -6: "EDEVICE",
                -7: "EUNSUPPORTED", -8: "EIO"}
SINK_PWV = 1
PREC_FP32, PREC_SPLIT_BF16 = 0, 1
INIT_STRICT_RANGE = 1
STAGE_REFLECT, STAGE_ATM_COUPLED, STAGE_OHMIC, STAGE_REFRACTIVE = 0, 1, 2, 3
FILT_LORENTZ, FILT_FILTERBANK, FILT_MATRIX = 0, 1, 2
JOB_SIGNAL, JOB_PINK = 0, 1
SCAN_STARE, SCAN_DAISY, SCAN_TRAJ = 0, 1, 2
JOB_PHOTON_NOISE, JOB_ACCUMULATE, JOB_KELVIN = 1, 2, 4
SKYDIP_MAX_N = 16384
OBJ_SCREEN, OBJ_SPEC, OBJ_CTX = 0, 1, 2

_dp = C.POINTER(C.c_double)
_fp = C.POINTER(C.c_float)


class InitDesc(C.Structure):
    _fields_ = [("device", C.c_int32), ("precision", C.c_int32),
                ("flags", C.c_uint32), ("reserved0", C.c_int32),
                ("hbm_budget_bytes", C.c_uint64),
                ("workspace_bytes", C.c_uint64),
                ("f_sample_hz", C.c_double), ("eta_taper", C.c_double),
                ("rho_surf_m", C.c_double), ("eta_pol", C.c_double),
                ("delta_J", C.c_double), ("eta_pb", C.c_double),
                ("t_cmb_K", C.c_double)]


class ScreenDesc(C.Structure):
    _fields_ = [("pwv_mm", C.c_void_p), ("nx", C.c_int64), ("ny", C.c_int64),
                ("dx_m", C.c_double), ("dy_m", C.c_double),
                ("ix0", C.c_double), ("iy0", C.c_double),
                ("h_column_m", C.c_double), ("wind_mps", C.c_double),
                ("mem_kind", C.c_int32), ("reserved0", C.c_int32)]


class Stage(C.Structure):
    _fields_ = [("kind", C.c_int32), ("ar_coated", C.c_int32),
                ("eta", C.c_void_p), ("eta_const", C.c_double),
                ("t_K", C.c_double), ("t_refl_K", C.c_double),
                ("eps_ref", C.c_double), ("nu_ref_hz", C.c_double),
                ("d_m", C.c_double), ("n_index", C.c_double),
                ("tan_delta", C.c_double)]


class SpectralDesc(C.Structure):
    _fields_ = [("F", C.c_int32), ("K", C.c_int32),
                ("nu_hz", C.c_void_p), ("w_hz", C.c_void_p),
                ("n_pwv", C.c_int32), ("filter_mode", C.c_int32),
                ("pwv0_mm", C.c_double), ("dpwv_mm", C.c_double),
                ("eta_z", C.c_void_p), ("t_atm_K", C.c_double),
                ("n_stage", C.c_int32), ("reserved0", C.c_int32),
                ("stages", C.c_void_p), ("f_hz", C.c_void_p),
                ("R", C.c_void_p), ("eta_peak", C.c_void_p),
                ("eta_filt", C.c_void_p), ("ref_pwv_mm", C.c_double),
                ("ref_el_rad", C.c_double)]


class Job(C.Structure):
    _fields_ = [("kind", C.c_int32), ("screen_id", C.c_int32),
                ("spec_id", C.c_int32), ("n_pix", C.c_int32),
                ("dphi_rad", C.c_void_p), ("dtheta_rad", C.c_void_p),
                ("scan_kind", C.c_int32), ("precision", C.c_int32),
                ("phi0_rad", C.c_double), ("theta0_rad", C.c_double),
                ("scan_params", C.c_double * 8),
                ("traj", C.c_void_p), ("cube", C.c_void_p),
                ("n_az", C.c_int32), ("n_el", C.c_int32),
                ("cube_ld", C.c_int64),
                ("az0_rad", C.c_double), ("daz_rad", C.c_double),
                ("el0_rad", C.c_double), ("del_rad", C.c_double),
                ("t_begin", C.c_int64), ("t_end", C.c_int64),
                ("t_total", C.c_int64), ("seed", C.c_uint64),
                ("flags", C.c_uint32), ("pix0", C.c_int32),
                ("pink_alpha", C.c_void_p), ("pink_knee_hz", C.c_double),
                ("pink_A", C.c_void_p),
                ("out_t0", C.c_int64), ("out_ld", C.c_int64),
                ("tod", C.c_void_p), ("p_kid", C.c_void_p),
                ("sigma", C.c_void_p), ("pwv", C.c_void_p)]


class ReduceDesc(C.Structure):
    _fields_ = [("spec_id", C.c_int32), ("n_pix", C.c_int32),
                ("dphi_rad", C.c_void_p), ("dtheta_rad", C.c_void_p),
                ("scan_kind", C.c_int32), ("map_n", C.c_int32),
                ("theta0_rad", C.c_double),
                ("scan_params", C.c_double * 8),
                ("traj", C.c_void_p), ("t_total", C.c_int64),
                ("t0", C.c_int64), ("T", C.c_int64), ("ld", C.c_int64),
                ("tod", C.c_void_p), ("pwv", C.c_void_p),
                ("pwv_ld", C.c_int64), ("pwv_len", C.c_int64),
                ("pwv_mean_mm", C.c_double), ("r_out_rad", C.c_double),
                ("map_half_rad", C.c_double),
                ("t_star", C.c_void_p), ("map", C.c_void_p),
                ("weight", C.c_void_p)]


class SinkDesc(C.Structure):
    _fields_ = [("dir", C.c_char_p), ("device_bytes", C.c_uint64),
                ("host_bytes", C.c_uint64), ("flags", C.c_uint32),
                ("pix_per_group", C.c_int32)]


SYMBOLS = ["gtod_sim_init", "gtod_load_screen", "gtod_load_filters",
           "gtod_simulate_tod", "gtod_free", "gtod_last_error",
           "gtod_memory", "gtod_get_counters", "gtod_spec_nep2_ref",
           "gtod_philox", "gtod_abi_sizes", "gtod_profile_enable",
           "gtod_profile_read", "gtod_skydip", "gtod_reduce",
           "gtod_simulate_to_disk", "gtod_far_field", "gtod_convolve_source",
           "gtod_convolve_screen", "gtod_simulate_tod_noalloc",
           "gtod_release_stream"]
KERNEL_NAMES = ["panel", "gemm_f32", "gemm_bf16", "pink_pass1", "pink_pass2",
                "common", "grid", "beam", "src_conv", "screen_conv"]
MAP_MAX_N = 48

_lib = None


def load():
    """Load libgtod.so and declare its signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: the HIP library must be built "
            "(python -m paper_2604_23305_amd.build); there is no fallback")
    lib = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    lib.gtod_sim_init.argtypes = [C.POINTER(InitDesc), C.POINTER(vp)]
    lib.gtod_load_screen.argtypes = [vp, C.POINTER(ScreenDesc),
                                     C.POINTER(C.c_int32)]
    lib.gtod_load_filters.argtypes = [vp, C.POINTER(SpectralDesc),
                                      C.POINTER(C.c_int32)]
    lib.gtod_simulate_tod.argtypes = [vp, C.POINTER(Job), C.c_int32, vp]
    lib.gtod_simulate_tod_noalloc.argtypes = [vp, C.POINTER(Job), C.c_int32,
                                              vp]
    lib.gtod_free.argtypes = [vp, C.c_int32, C.c_int32]
    lib.gtod_release_stream.argtypes = [vp, vp]
    lib.gtod_last_error.argtypes = [vp]
    lib.gtod_last_error.restype = C.c_char_p
    lib.gtod_memory.argtypes = [vp, C.POINTER(C.c_uint64),
                                C.POINTER(C.c_uint64)]
    lib.gtod_get_counters.argtypes = [vp, C.POINTER(C.c_uint64)]
    lib.gtod_spec_nep2_ref.argtypes = [vp, C.c_int32, C.POINTER(C.c_double)]
    lib.gtod_philox.argtypes = [vp, vp, vp, C.c_int64, C.c_uint64, vp]
    lib.gtod_abi_sizes.argtypes = [C.POINTER(C.c_int64)]
    lib.gtod_abi_sizes.restype = None
    lib.gtod_profile_enable.argtypes = [vp, C.c_int32]
    lib.gtod_profile_read.argtypes = [vp, C.POINTER(C.c_double), C.c_int32]
    lib.gtod_skydip.argtypes = [vp, C.c_int32, C.c_double, C.c_double,
                                C.c_double, C.c_int32, vp, vp, vp, vp]
    lib.gtod_reduce.argtypes = [vp, C.POINTER(ReduceDesc), vp]
    d_ = C.c_double
    lib.gtod_far_field.argtypes = [vp, vp, C.c_int32, C.c_int32, C.c_int32,
                                   d_, d_, d_, d_, vp, vp]
    lib.gtod_convolve_source.argtypes = [vp, vp, C.c_int32, C.c_int32,
                                         C.c_int64, vp, C.c_int32, d_, d_, d_,
                                         d_, d_, vp, C.c_int64, vp]
    lib.gtod_convolve_screen.argtypes = [vp, vp, C.c_int64, C.c_int64, d_, d_,
                                         d_, d_, vp, vp]
    lib.gtod_simulate_to_disk.argtypes = [vp, C.POINTER(Job), C.POINTER(Job),
                                          C.POINTER(SinkDesc),
                                          C.POINTER(C.c_double)]
    for name in SYMBOLS:
        if name not in ("gtod_last_error", "gtod_abi_sizes"):
            getattr(lib, name).restype = C.c_int32
    _lib = lib
    return lib


def struct_sizes():
    return [C.sizeof(InitDesc), C.sizeof(ScreenDesc), C.sizeof(Stage),
            C.sizeof(SpectralDesc), C.sizeof(Job), C.sizeof(ReduceDesc)]
