"""The profile request: everything that defines one n(r)/nbar computation.

A plain record, no arithmetic.  The fields mirror ``nh_request`` in
``include/nuhalo.h``; the binding marshals them into that struct.

Problem statement (arXiv:2410.08267): cosmology (Sec. II.A), halo mass and
concentration history (Sec. II.B, IV.A), optional modulation of G (Sec. IV.B),
relic mass and initial phase-space distribution (Sec. II.C, IV.B), the radius
grid and the (|p|, cos psi) momentum grid (Sec. II.D).
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import Optional

import numpy as np

# 200^(1/3) - 1: the collapse redshift of a halo virialised at z0 = 0 (Sec. II.B)
Z_FORM_PAPER = 200.0 ** (1.0 / 3.0) - 1.0

MASS_KINDS = ("zero", "paper", "exponential", "table")
CONC_KINDS = ("constant", "power", "table")
KAPPA_KINDS = ("none", "log", "paper", "constant", "table")
GEOMETRIES = ("paper", "delta200")
F0_KINDS = ("fermi_dirac", "freeze_in", "table")
METHODS = ("rk4", "dp5")
PRECISIONS = ("fp64", "fp32c")


@dataclass
class Request:
    # flat FRW background; H0 in km/s/Mpc
    H0: float = 67.7
    Omega_m: float = 0.31
    Omega_L: float = 0.69
    # halo mass history M(z)
    mass_kind: str = "exponential"   # zero | paper (xi^alpha M0) | exponential (M0 e^{-beta z})
    M0: float = 1.0e12               # Msun, mass at z = 0
    mass_alpha: float = 1.0          # paper: exponent of xi
    z_form: float = Z_FORM_PAPER     # paper: z_i of xi
    mass_beta: float = 0.8           # exponential: rate
    # concentration history c(z)
    conc_kind: str = "power"         # constant c0 | power c0 (1+z)^-gamma
    c0: float = 10.0
    conc_gamma: float = 1.0
    # G -> kappa(z) G
    kappa_kind: str = "none"         # none | log 1+a ln(1+z) | paper 1+a[z/(1+z)]^b | constant a
    kappa_a: float = 0.0
    kappa_b: float = 1.0
    geometry: str = "paper"          # paper (fixed physical r200) | delta200 (200 rhobar_m(z))
    compensated: bool = True
    # sampled histories for the "table" kinds: sample i at u_i = u_min + i (0 - u_min)/(n-1),
    # u = ln a, u_min = -ln(1 + hist_z_max); the last sample is z = 0
    hist_z_max: float = 4.0
    hist_M: Optional[np.ndarray] = None      # Msun
    hist_c: Optional[np.ndarray] = None
    hist_kappa: Optional[np.ndarray] = None
    # relic
    m_eV: float = 0.1
    f0_kind: str = "fermi_dirac"     # fermi_dirac | freeze_in | table
    T_K: float = 1.95
    # f0 "table": ln f0 at ln y = f0_ln_y0 + i f0_d_ln_y
    f0_ln_y0: float = 0.0
    f0_d_ln_y: float = 1.0
    f0_ln_f: Optional[np.ndarray] = None
    # grids
    r_kpc: np.ndarray = field(default_factory=lambda: np.geomspace(10.0, 1000.0, 10))
    y: np.ndarray = field(default_factory=lambda: np.geomspace(0.01, 100.0, 50))
    n_mu: int = 20
    mu: Optional[np.ndarray] = None   # None: Gauss-Legendre on [-1, 1] with n_mu nodes
    w_mu: Optional[np.ndarray] = None
    # integrator
    method: str = "rk4"
    n_steps: int = 1000
    rtol: float = 1.0e-8
    atol_x: Optional[float] = None    # kpc; None: rtol * 1 kpc
    atol_v: Optional[float] = None    # km/s; None: rtol * 1 km/s
    h0: float = -1.0e-3
    max_steps: int = 1_000_000
    z_end: float = 4.0
    precision: str = "fp64"           # fp64 | fp32c
    z_obs: float = 0.0                # observation redshift (the paper's z0); integration starts there

    @property
    def n_r(self) -> int:
        return int(len(self.r_kpc))

    @property
    def n_y(self) -> int:
        return int(len(self.y))

    @property
    def n_mu_eff(self) -> int:
        return int(len(self.mu)) if self.mu is not None else int(self.n_mu)

    @property
    def n_traj(self) -> int:
        return self.n_r * self.n_y * self.n_mu_eff

    def with_(self, **kw) -> "Request":
        return replace(self, **kw)
