"""Plain-data description of one simulation (inputs only, no arithmetic).

A Scenario carries every array and parameter the simulator consumes.  The
oracle reads it directly; the GPU binding marshals the same arrays into the
C-ABI descriptors.  Angles are radians, frequencies Hz, temperatures K,
spectral powers W/Hz, PWV mm.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

E_CHARGE = 1.602176634e-19  # C (exact SI); converts the gap energy to J


@dataclass
class Telescope:
    r_tel_m: float = 5.0
    eta_taper: float = 0.85
    rho_surf_m: float = 42e-6
    eta_pol: float = 0.5


@dataclass
class KID:
    delta_J: float = 188e-6 * E_CHARGE
    eta_pb: float = 0.4


@dataclass
class Stage:
    """One optics stage after the atmosphere.

    kind: 'reflect' (eta, t_K), 'atm_coupled' (eta), 'ohmic' (eps_ref,
    nu_ref_hz, t_K) or 'refractive' (d_m, n_index, tan_delta, t_K for the
    dielectric pass, t_refl_K for the two surface passes, ar_coated).
    eta is a scalar or an [F] array."""
    kind: str
    eta: object = 1.0
    t_K: float = 0.0
    eps_ref: float = 0.0025
    nu_ref_hz: float = 840e9
    d_m: float = 0.0
    n_index: float = 1.0
    tan_delta: float = 0.0
    t_refl_K: float = 0.0
    ar_coated: bool = False


@dataclass
class Filters:
    """mode: 'lorentz', 'filterbank' (f_hz, R, eta_peak per channel) or
    'matrix' (eta_filt[F][K])."""
    mode: str
    f_hz: Optional[np.ndarray] = None
    R: Optional[np.ndarray] = None
    eta_peak: Optional[np.ndarray] = None
    matrix: Optional[np.ndarray] = None

    @property
    def K(self) -> int:
        if self.mode == "matrix":
            return int(self.matrix.shape[1])
        return int(len(self.f_hz))


@dataclass
class Spectral:
    nu_hz: np.ndarray
    w_hz: np.ndarray
    eta_z: np.ndarray          # [n_pwv][F] zenith transmission table
    pwv0_mm: float
    dpwv_mm: float
    t_atm_K: float
    stages: List[Stage]
    filters: Filters
    ref_pwv_mm: float = 1.0    # operating point of the reference row
    ref_el_rad: float = np.pi / 3

    @property
    def F(self) -> int:
        return int(self.nu_hz.size)


@dataclass
class Screen:
    pwv_mm: np.ndarray         # [ny][nx] FP64, x (wind axis) contiguous
    dx_m: float = 0.2
    dy_m: float = 0.2
    ix0: float = 32.0
    iy0: float = 0.0
    h_column_m: float = 1537.0
    wind_mps: float = 10.0


@dataclass
class Scan:
    kind: str                  # 'stare' | 'daisy' | 'traj'
    phi0: float = 0.0
    theta0: float = np.pi / 3
    r_petal: float = 0.0
    omega: float = 0.0         # petal angular frequency (rad/s)
    Omega: float = 0.0         # full-daisy angular frequency (rad/s)
    traj: Optional[np.ndarray] = None   # [t_total][2] (phi, theta)


@dataclass
class Source:
    cube: np.ndarray           # float32 [n_el][n_az][F], W/Hz
    az0: float
    daz: float
    el0: float
    del_: float

    @property
    def n_el(self):
        return int(self.cube.shape[0])

    @property
    def n_az(self):
        return int(self.cube.shape[1])


@dataclass
class Scenario:
    name: str
    f_sample_hz: float
    spectral: Spectral
    screen: Screen
    scan: Scan
    dphi: np.ndarray
    dtheta: np.ndarray
    t_total: int
    source: Optional[Source] = None
    telescope: Telescope = field(default_factory=Telescope)
    kid: KID = field(default_factory=KID)
    t_cmb_K: float = 2.725
    seed: int = 1
    photon_noise: bool = True
    pink_alpha: Optional[np.ndarray] = None   # [K]; None = no pink noise
    pink_knee_hz: float = 1.0
    # explicit per-channel 1/f levels A_k (W^2/Hz); None = knee-derived
    pink_A: Optional[np.ndarray] = None

    @property
    def n_pix(self) -> int:
        return int(self.dphi.size)

    @property
    def K(self) -> int:
        return self.spectral.filters.K

    @property
    def F(self) -> int:
        return self.spectral.F
