"""Plain FP64 CPU oracle for the n(r)/nbar profiles of arXiv:2410.08267.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark may import this module; the product library never does.  It
shares no code with the HIP path.  The trajectory integrator is the plain C
file ``nh_oracle.c`` next to this module (one trajectory at a time, closed-form
halo at every call); everything else here is NumPy/`math` written to read
against the paper:

* initial conditions (Sec. II.C): x0 = (r, 0), v0 = V (mu, sqrt(1-mu^2)),
  V = y k_B T c / m (non-relativistic v = P/m, as in Sec. II.D);
* Liouville map (Sec. II.C): f0(x0, P0, mu) = f_rel(P_i), with
  P_i / P0 = |v(u_end)| / |v0| because the EOM are mass independent;
* momentum-space quadrature, Eq. (localdensity) over Eq. (density_integral)'s
  background: n/nbar = sum_jl W_jl f(y_i) / sum_jl W_jl f(y_j), with
  W_jl = w_mu,l * y_j^3 * dlny_j (trapezoid in ln y) and Gauss-Legendre mu
  nodes on [-1, 1].  The g/(4 pi^2) and g/(2 pi^2) prefactors cancel because
  the mu weights sum to 2.
* the sums are exactly rounded (``math.fsum``), so they do not depend on an
  evaluation order.

Request objects are read by attribute name (see ``paper_2410_08267_amd.request``
for the fields); this module does not import the product package.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nh_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libnh_oracle.so")

# Constants (the paper gives only T_nu0 = 1.95 K, Sec. II.C)
K_B_EV_PER_K = 1.380649e-23 / 1.602176634e-19   # k_B / e: both exact in SI since 2019
C_KM_S = 299792.458                 # exact
T_NU0_K = 1.95

STATUS_OK, STATUS_MAXSTEPS, STATUS_UNDERFLOW, STATUS_NONFINITE = 0, 1, 2, 3

_MASS_KIND = {"zero": 0, "paper": 1, "exponential": 2, "point": 3, "table": 4}
_CONC_KIND = {"constant": 0, "power": 1, "table": 2}
_KAPPA_KIND = {"none": 0, "log": 1, "paper": 2, "constant": 3, "table": 4}
_GEOMETRY = {"paper": 0, "delta200": 1}
_METHOD = {"rk4": 0, "dp5": 1, "dp5_fixed": 2}


class _Model(ctypes.Structure):
    _fields_ = [
        ("H0_km_s_Mpc", ctypes.c_double),
        ("Omega_m", ctypes.c_double),
        ("Omega_L", ctypes.c_double),
        ("static_background", ctypes.c_int),
        ("mass_kind", ctypes.c_int),
        ("M0_Msun", ctypes.c_double),
        ("mass_alpha", ctypes.c_double),
        ("z_form", ctypes.c_double),
        ("mass_beta", ctypes.c_double),
        ("conc_kind", ctypes.c_int),
        ("c0", ctypes.c_double),
        ("conc_gamma", ctypes.c_double),
        ("kappa_kind", ctypes.c_int),
        ("kappa_a", ctypes.c_double),
        ("kappa_b", ctypes.c_double),
        ("geometry", ctypes.c_int),
        ("compensated", ctypes.c_int),
        ("z_obs", ctypes.c_double),
        ("hist_n", ctypes.c_int),
        ("hist_u_min", ctypes.c_double),
        ("hist_M", ctypes.POINTER(ctypes.c_double)),
        ("hist_c", ctypes.POINTER(ctypes.c_double)),
        ("hist_kappa", ctypes.POINTER(ctypes.c_double)),
        ("hist_hmod", ctypes.POINTER(ctypes.c_double)),
    ]


class _Integ(ctypes.Structure):
    _fields_ = [
        ("method", ctypes.c_int),
        ("n_steps", ctypes.c_int),
        ("u_start", ctypes.c_double),
        ("u_end", ctypes.c_double),
        ("rtol", ctypes.c_double),
        ("atol_x", ctypes.c_double),
        ("atol_v", ctypes.c_double),
        ("h0", ctypes.c_double),
        ("max_steps", ctypes.c_longlong),
        ("fmax", ctypes.c_double),
        ("component_scales", ctypes.c_int),
    ]


def build(force: bool = True) -> str:
    """Compile nh_oracle.c into libnh_oracle.so (plain gcc, no FMA contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.run(
            ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
             "-fno-fast-math", "-o", tmp, _SRC, "-lm"],
            check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    """The compiled oracle.  NH_ORACLE_LIB names another build of nh_oracle.c
    (the mutation test loads deliberately broken copies this way)."""
    global _lib
    if _lib is None:
        path = os.environ.get("NH_ORACLE_LIB")
        if not path:
            path = _LIB_PATH
            if not os.path.exists(path):
                build()
        L = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        L.nho_integrate.argtypes = [ctypes.POINTER(_Model), ctypes.POINTER(_Integ), ctypes.c_long,
                                    dp, ctypes.POINTER(ctypes.c_longlong),
                                    ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_int)]
        L.nho_integrate.restype = None
        L.nho_deltaM_many.argtypes = [ctypes.POINTER(_Model), ctypes.c_long, dp, dp, dp]
        L.nho_deltaM_many.restype = None
        L.nho_rhs_many.argtypes = [ctypes.POINTER(_Model), ctypes.c_long, dp, dp, dp]
        L.nho_rhs_many.restype = None
        for name in ("nho_hubble", "nho_mass", "nho_conc", "nho_kappa"):
            fn = getattr(L, name)
            fn.argtypes = [ctypes.POINTER(_Model), ctypes.c_double]
            fn.restype = ctypes.c_double
        L.nho_nfw_I.argtypes = [ctypes.c_double]
        L.nho_nfw_I.restype = ctypes.c_double
        L.nho_G_value.argtypes = []
        L.nho_G_value.restype = ctypes.c_double
        L.nho_radii.argtypes = [ctypes.POINTER(_Model), ctypes.c_double, dp, dp]
        L.nho_radii.restype = None
        _lib = L
    return _lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# --------------------------------------------------------------------------
# request -> C structs
# --------------------------------------------------------------------------

def model_of(req, static_background: bool = False) -> _Model:
    m = _Model()
    m.H0_km_s_Mpc = float(req.H0)
    m.Omega_m = float(req.Omega_m)
    m.Omega_L = float(req.Omega_L)
    m.static_background = int(bool(static_background))
    m.mass_kind = _MASS_KIND[req.mass_kind]
    m.M0_Msun = float(req.M0)
    m.mass_alpha = float(req.mass_alpha)
    m.z_form = float(req.z_form)
    m.mass_beta = float(req.mass_beta)
    m.conc_kind = _CONC_KIND[req.conc_kind]
    m.c0 = float(req.c0)
    m.conc_gamma = float(req.conc_gamma)
    m.kappa_kind = _KAPPA_KIND[req.kappa_kind]
    m.kappa_a = float(req.kappa_a)
    m.kappa_b = float(req.kappa_b)
    m.geometry = _GEOMETRY[req.geometry]
    m.compensated = int(bool(req.compensated))
    m.z_obs = float(getattr(req, "z_obs", 0.0))
    # sampled histories: the not-a-knot cubic spline through the samples in
    # u = ln a (scipy's CubicSpline), handed to the C side as its polynomial
    # pieces; the model keeps the coefficient arrays alive
    m._keep = []
    # hist_hmod: test-only sampled factor of H(z) (see nh_oracle.c); requests
    # carry it only as a probe attribute set by the tests
    arrays = [getattr(req, "hist_" + k, None) for k in ("M", "c", "kappa", "hmod")]
    if any(a is not None for a in arrays):
        from scipy.interpolate import CubicSpline
        u_min = -math.log1p(float(req.hist_z_max))
        m.hist_u_min = u_min
        for name, a in zip(("hist_M", "hist_c", "hist_kappa", "hist_hmod"), arrays):
            if a is None:
                continue
            a = np.asarray(a, dtype=np.float64)
            u = u_min + np.arange(a.size) * (0.0 - u_min) / (a.size - 1)
            pieces = np.ascontiguousarray(CubicSpline(u, a, bc_type="not-a-knot").c.T)   # (n-1, 4)
            m._keep.append(pieces)
            m.hist_n = a.size
            setattr(m, name, pieces.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return m


def u_end_of(z_end: float) -> float:
    """u = ln a at redshift z_end."""
    return -math.log1p(z_end)


def integ_of(req) -> _Integ:
    it = _Integ()
    it.method = _METHOD[req.method]
    it.n_steps = int(req.n_steps)
    it.u_start = -math.log1p(float(getattr(req, "z_obs", 0.0)))
    it.u_end = u_end_of(float(req.z_end))
    it.rtol = float(req.rtol)
    it.atol_x = float(req.rtol if req.atol_x is None else req.atol_x)
    it.atol_v = float(req.rtol if req.atol_v is None else req.atol_v)
    it.h0 = float(req.h0)
    it.max_steps = int(req.max_steps)
    return it


# --------------------------------------------------------------------------
# grids, weights and phase-space distributions
# --------------------------------------------------------------------------

def gauss_legendre(n: int):
    """Gauss-Legendre nodes and weights on [-1, 1] (mu = cos psi, Eq. density_integral)."""
    x, w = np.polynomial.legendre.leggauss(n)
    return np.asarray(x, dtype=np.float64), np.asarray(w, dtype=np.float64)


def mu_grid(req):
    if req.mu is not None:
        return np.asarray(req.mu, dtype=np.float64), np.asarray(req.w_mu, dtype=np.float64)
    return gauss_legendre(int(req.n_mu))


def y_weights(y) -> np.ndarray:
    """w_j = y_j^3 * dlny_j: trapezoid rule in ln y for int dP P^2 f(P) = T^3 int dlny y^3 f."""
    y = np.asarray(y, dtype=np.float64)
    n = y.size
    ly = np.log(y)
    d = np.empty(n)
    if n == 1:
        d[0] = 1.0
    else:
        d[0] = 0.5 * (ly[1] - ly[0])
        d[-1] = 0.5 * (ly[-1] - ly[-2])
        for j in range(1, n - 1):
            d[j] = 0.5 * (ly[j + 1] - ly[j - 1])
    return y ** 3 * d


def f0(kind: str, y):
    """Relic phase-space distribution at the start of the backward integration.

    fermi_dirac: 1/(1 + e^y) (Sec. II.C, y = P/T_nu0);
    freeze_in:   y^(-1/2) e^(-y) (normalisation cancels in n/nbar, Sec. IV.B)."""
    y = np.asarray(y, dtype=np.float64)
    with np.errstate(over="ignore"):
        if kind == "fermi_dirac":
            return 1.0 / (1.0 + np.exp(y))
        if kind == "freeze_in":
            return np.exp(-y) / np.sqrt(y)
    raise ValueError(f"unknown f0 kind {kind!r}")


def f0_of(req, y):
    """f0 of a request at y: the named distributions, or for f0_kind "table"
    exp of the sampled ln f0 (samples at ln y = f0_ln_y0 + i f0_d_ln_y): the
    cubic through four consecutive samples in Lagrange's form inside the
    sampled range (nodes i-1..i+2 around the interval, moved inward in the
    first and last one), the straight line through the two end samples
    outside it."""
    if req.f0_kind != "table":
        return f0(req.f0_kind, y)
    v = np.asarray(req.f0_ln_f, dtype=np.float64)
    n = v.size
    s = (np.log(np.asarray(y, dtype=np.float64)) - req.f0_ln_y0) / req.f0_d_ln_y
    i = np.clip(np.floor(s).astype(np.int64), 1, n - 3)
    inner = np.zeros_like(s)
    for a in (-1, 0, 1, 2):
        L = np.ones_like(s)
        for b in (-1, 0, 1, 2):
            if b != a:
                L *= (s - (i + b)) / (a - b)
        inner += L * v[i + a]
    below = v[0] + (v[1] - v[0]) * s
    above = v[n - 1] + (v[n - 1] - v[n - 2]) * (s - (n - 1))
    lnf = np.where(s < 0, below, np.where(s > n - 1, above, inner))
    with np.errstate(over="ignore"):
        return np.exp(lnf)


def velocity_per_y(m_eV: float, T_K: float) -> float:
    """Comoving speed (km/s) of a relic with y = P/T = 1: v = P/m = y k_B T c / m."""
    return K_B_EV_PER_K * T_K * C_KM_S / m_eV


# --------------------------------------------------------------------------
# trajectories
# --------------------------------------------------------------------------

def initial_state(req, r, y, mu) -> np.ndarray:
    """(N_r*N_y*N_mu, 4) initial states, index t = (k*N_y + j)*N_mu + l (Sec. II.C)."""
    r = np.asarray(r, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    mu = np.asarray(mu, dtype=np.float64)
    V = y * velocity_per_y(req.m_eV, req.T_K)
    sin = np.sqrt(1.0 - mu * mu)
    nr, ny, nm = r.size, y.size, mu.size
    st = np.zeros((nr, ny, nm, 4))
    st[..., 0] = r[:, None, None]
    st[..., 2] = V[None, :, None] * mu[None, None, :]
    st[..., 3] = V[None, :, None] * sin[None, None, :]
    return st.reshape(-1, 4)


def integrate_states(model: _Model, integ: _Integ, state: np.ndarray, threads: int | None = None):
    """Integrate every row of `state` (copied) from u = 0 to integ.u_end.

    Returns (final_state, accepted, rejected, status).  Rows are split into
    chunks run on a thread pool; ctypes releases the GIL inside the C call."""
    L = lib()
    st = np.ascontiguousarray(state, dtype=np.float64).copy()
    n = st.shape[0]
    acc = np.zeros(n, dtype=np.int64)
    rej = np.zeros(n, dtype=np.int64)
    status = np.zeros(n, dtype=np.int32)
    if n == 0:
        return st, acc, rej, status
    if threads is None:
        threads = len(os.sched_getaffinity(0))
    threads = max(1, min(threads, n))
    bounds = np.linspace(0, n, min(n, threads * 8) + 1).astype(np.int64)

    def run(i):
        a, b = int(bounds[i]), int(bounds[i + 1])
        if b <= a:
            return
        sub = st[a:b]
        L.nho_integrate(ctypes.byref(model), ctypes.byref(integ), b - a,
                        _dptr(sub),
                        acc[a:b].ctypes.data_as(ctypes.POINTER(ctypes.c_longlong)),
                        rej[a:b].ctypes.data_as(ctypes.POINTER(ctypes.c_longlong)),
                        status[a:b].ctypes.data_as(ctypes.POINTER(ctypes.c_int)))

    if threads == 1:
        for i in range(len(bounds) - 1):
            run(i)
    else:
        with ThreadPoolExecutor(max_workers=threads) as ex:
            list(ex.map(run, range(len(bounds) - 1)))
    return st, acc, rej, status


def speed_ratio(v0: np.ndarray, v1: np.ndarray) -> np.ndarray:
    """|v1| / |v0| = P_i / P0 (Liouville map, Sec. II.C); both norms by the same hypot."""
    return np.hypot(v1[:, 0], v1[:, 1]) / np.hypot(v0[:, 0], v0[:, 1])


def trajectories(req, threads: int | None = None, index=None):
    """Integrate the request's trajectories (all, or the flat indices `index`).

    Returns a dict with the flat indices, initial and final states, the speed
    ratio P_i/P0, step counts and status."""
    r = np.asarray(req.r_kpc, dtype=np.float64)
    y = np.asarray(req.y, dtype=np.float64)
    mu, _ = mu_grid(req)
    st0 = initial_state(req, r, y, mu)
    idx = np.arange(st0.shape[0]) if index is None else np.asarray(index, dtype=np.int64)
    st0 = st0[idx]
    st1, acc, rej, status = integrate_states(model_of(req), integ_of(req), st0, threads)
    return {
        "index": idx,
        "state0": st0,
        "state1": st1,
        "ratio": speed_ratio(st0[:, 2:], st1[:, 2:]),
        "accepted": acc,
        "rejected": rej,
        "status": status,
    }


def profile_from_ratio(req, ratio: np.ndarray) -> np.ndarray:
    """n/nbar per radius from the speed ratios of all trajectories (Eq. localdensity)."""
    y = np.asarray(req.y, dtype=np.float64)
    _, w_mu = mu_grid(req)
    nr, ny, nm = len(req.r_kpc), y.size, w_mu.size
    ratio = np.asarray(ratio, dtype=np.float64).reshape(nr, ny, nm)
    wy = y_weights(y)
    W = wy[:, None] * w_mu[None, :]                     # (j, l)
    f_bg = f0_of(req, np.broadcast_to(y[:, None], (ny, nm)))
    den = math.fsum((W * f_bg).ravel().tolist())
    out = np.empty(nr)
    for k in range(nr):
        yi = y[:, None] * ratio[k]
        num = math.fsum((W * f0_of(req, yi)).ravel().tolist())
        out[k] = num / den
    return out


def solve(req, threads: int | None = None):
    """Full oracle profile: integrate every trajectory, then the quadrature."""
    tr = trajectories(req, threads)
    prof = profile_from_ratio(req, tr["ratio"])
    tr["n_over_nbar"] = prof
    return tr


def integrand_from_ratio(req, ratio: np.ndarray) -> np.ndarray:
    """Direction-integrated distribution at each radius and momentum node
    (Sec. II.D, Fig. 3): out[k, j] = sum_l w_mu,l f0(y_j P_i/P0), l in order."""
    y = np.asarray(req.y, dtype=np.float64)
    _, w_mu = mu_grid(req)
    nr, ny, nm = len(req.r_kpc), y.size, w_mu.size
    ratio = np.asarray(ratio, dtype=np.float64).reshape(nr, ny, nm)
    out = np.empty((nr, ny))
    for k in range(nr):
        f = f0_of(req, y[:, None] * ratio[k])          # (j, l)
        for j in range(ny):
            out[k, j] = math.fsum((w_mu * f[j]).tolist())
    return out


def solve_masses(req, m_eV, threads: int | None = None):
    """Profiles for several relic masses from one set of trajectories (Sec. II.D:
    the equations of motion do not contain the mass).  The request's y grid at
    its own mass fixes the velocities; for mass m the same trajectories carry
    momenta y m / m_req, so mass m's profile is the quadrature of the request
    with that mass and that scaled grid.  Returns (n_mass, n_r)."""
    tr = trajectories(req, threads)
    y = np.asarray(req.y, dtype=np.float64)
    out = []
    for m in np.atleast_1d(np.asarray(m_eV, dtype=np.float64)):
        rq = req.with_(m_eV=float(m), y=y * (float(m) / req.m_eV))
        out.append(profile_from_ratio(rq, tr["ratio"]))
    return np.array(out)


# --------------------------------------------------------------------------
# direct access for the pins
# --------------------------------------------------------------------------

def deltaM(req, r, z) -> np.ndarray:
    r = np.ascontiguousarray(np.broadcast_to(np.asarray(r, dtype=np.float64), np.broadcast(r, z).shape))
    z = np.ascontiguousarray(np.broadcast_to(np.asarray(z, dtype=np.float64), r.shape))
    out = np.empty(r.shape)
    m = model_of(req)
    lib().nho_deltaM_many(ctypes.byref(m), r.size, _dptr(r), _dptr(z), _dptr(out))
    return out


def rhs(req, u, Y, static_background: bool = False) -> np.ndarray:
    u = np.ascontiguousarray(np.asarray(u, dtype=np.float64).ravel())
    Y = np.ascontiguousarray(np.asarray(Y, dtype=np.float64).reshape(-1, 4))
    out = np.empty_like(Y)
    m = model_of(req, static_background)
    lib().nho_rhs_many(ctypes.byref(m), u.size, _dptr(u), _dptr(Y), _dptr(out))
    return out


def halo_radii(req, z: float):
    R = ctypes.c_double()
    rv = ctypes.c_double()
    m = model_of(req)
    lib().nho_radii(ctypes.byref(m), float(z), ctypes.byref(R), ctypes.byref(rv))
    return R.value, rv.value


def histories(req, z):
    """(M(z), c(z), kappa(z)) of the request's halo at each redshift in z."""
    m = model_of(req)
    L = lib()
    z = np.atleast_1d(np.asarray(z, dtype=np.float64))
    M = np.array([L.nho_mass(ctypes.byref(m), float(zz)) for zz in z])
    c = np.array([L.nho_conc(ctypes.byref(m), float(zz)) for zz in z])
    k = np.array([L.nho_kappa(ctypes.byref(m), float(zz)) for zz in z])
    return M, c, k


def hubble(req, z: float) -> float:
    m = model_of(req)
    return lib().nho_hubble(ctypes.byref(m), float(z))


def nfw_I(q: float) -> float:
    return lib().nho_nfw_I(float(q))


def G_value() -> float:
    return lib().nho_G_value()
