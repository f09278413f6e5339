"""Seeded synthetic workloads shared by the tests, the benchmark and the oracle runs.

Only input construction lives here (parameter draws and grids); none of the
method's arithmetic.  Random numbers come from ``numpy.random.default_rng(seed)``.

The paper's own grids (Sec. II.D) and halo masses (Sec. III) motivate these
shapes; the paper publishes no dataset, so every workload is synthetic.

  plain_small     flat LCDM (H0 = 67.7, Om = 0.31, OL = 0.69); M(z) = 1e12 e^{-0.8 z} Msun,
                  c(z) = 10/(1+z); m = 0.1 eV, Fermi-Dirac at 1.95 K; 10 radii log-spaced
                  10 kpc - 1 Mpc x 50 y log-spaced 0.01 - 100 x 20 Gauss-Legendre mu
                  = 10 000 trajectories; RK4, 1000 equal steps in ln a, z 0 -> 4.
  plain_scale     same cosmology; M0 log-uniform in [1e11, 1e15] Msun, c0 uniform in [4, 15],
                  m uniform over {0.05, 0.1, 0.3} eV; 100 x 200 x 64 = 1.28 M trajectories;
                  Dormand-Prince 5(4), rtol 1e-8, z 0 -> 4.
  precision       plain_scale integrated in the FP32-compensated form.
  batched         heterogeneous requests: M0 log-uniform [1e11, 1e15], c0 U[4, 15],
                  m U[0.02, 0.3] eV, N_r U{16..128}, N_y U{32..256}, N_mu U{16..64}.
  serving         batched-shaped requests arriving as a Poisson process; 30 % use the
                  freeze-in f0 ~ y^-1/2 e^-y, 20 % use G(z) = G0 (1 + 0.05 ln(1+z)).
"""
from __future__ import annotations

import numpy as np

from .request import Request

R_MIN_KPC, R_MAX_KPC = 10.0, 1000.0
Y_MIN, Y_MAX = 0.01, 100.0


def _grids(n_r: int, n_y: int):
    return np.geomspace(R_MIN_KPC, R_MAX_KPC, n_r), np.geomspace(Y_MIN, Y_MAX, n_y)


def plain_small() -> Request:
    r, y = _grids(10, 50)
    return Request(
        H0=67.7, Omega_m=0.31, Omega_L=0.69,
        mass_kind="exponential", M0=1.0e12, mass_beta=0.8,
        conc_kind="power", c0=10.0, conc_gamma=1.0,
        m_eV=0.1, f0_kind="fermi_dirac", T_K=1.95,
        r_kpc=r, y=y, n_mu=20,
        method="rk4", n_steps=1000, z_end=4.0)


def plain_scale(seed: int, n_r: int = 100, n_y: int = 200, n_mu: int = 64,
                rtol: float = 1.0e-8) -> Request:
    rng = np.random.default_rng(seed)
    M0 = 10.0 ** rng.uniform(11.0, 15.0)
    c0 = rng.uniform(4.0, 15.0)
    m = float(rng.choice([0.05, 0.1, 0.3]))
    r, y = _grids(n_r, n_y)
    return Request(
        H0=67.7, Omega_m=0.31, Omega_L=0.69,
        mass_kind="exponential", M0=M0, mass_beta=0.8,
        conc_kind="power", c0=c0, conc_gamma=1.0,
        m_eV=m, f0_kind="fermi_dirac", T_K=1.95,
        r_kpc=r, y=y, n_mu=n_mu,
        method="dp5", rtol=rtol, z_end=4.0)


def precision(seed: int, **kw) -> Request:
    return plain_scale(seed, **kw).with_(precision="fp32c")


def batched(seed: int, n_req: int = 512, prec: str = "fp64", freeze_in_frac: float = 0.0,
            kappa_frac: float = 0.0):
    """n_req heterogeneous requests, all drawn from one seeded stream."""
    rng = np.random.default_rng(seed)
    reqs = []
    for _ in range(n_req):
        M0 = 10.0 ** rng.uniform(11.0, 15.0)
        c0 = rng.uniform(4.0, 15.0)
        m = rng.uniform(0.02, 0.3)
        n_r = int(rng.integers(16, 129))
        n_y = int(rng.integers(32, 257))
        n_mu = int(rng.integers(16, 65))
        fi = rng.uniform() < freeze_in_frac
        kp = rng.uniform() < kappa_frac
        r, y = _grids(n_r, n_y)
        reqs.append(Request(
            H0=67.7, Omega_m=0.31, Omega_L=0.69,
            mass_kind="exponential", M0=M0, mass_beta=0.8,
            conc_kind="power", c0=c0, conc_gamma=1.0,
            kappa_kind="log" if kp else "none", kappa_a=0.05 if kp else 0.0,
            m_eV=m, f0_kind="freeze_in" if fi else "fermi_dirac", T_K=1.95,
            r_kpc=r, y=y, n_mu=n_mu,
            method="dp5", rtol=1.0e-8, z_end=4.0, precision=prec))
    return reqs


def serving(seed: int, n_req: int, qps: float, prec: str = "fp32c"):
    """(arrival_times_s, requests): Poisson arrivals at rate qps of batched-shaped requests."""
    rng = np.random.default_rng(seed + 1_000_003)
    gaps = rng.exponential(1.0 / qps, size=n_req)
    t = np.cumsum(gaps) - gaps[0]
    reqs = batched(seed, n_req, prec=prec, freeze_in_frac=0.3, kappa_frac=0.2)
    return t, reqs


def shrink(req: Request, n_r: int, n_y: int, n_mu: int) -> Request:
    """Same physics on a smaller (r, y, mu) grid spanning the same ranges."""
    r = np.geomspace(float(req.r_kpc[0]), float(req.r_kpc[-1]), n_r)
    y = np.geomspace(float(req.y[0]), float(req.y[-1]), n_y)
    return req.with_(r_kpc=r, y=y, n_mu=n_mu, mu=None, w_mu=None)
