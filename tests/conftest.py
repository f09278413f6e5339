import ctypes
import os
import subprocess
import sys

import numpy as np

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
# the mutation tests run the pins against a modified copy of the oracle package
ORACLE_ROOT = os.environ.get("NH_ORACLE_ROOT")
if ORACLE_ROOT:
    sys.path.insert(0, ORACLE_ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU oracle runs, excluded from the default CPU suite")


@pytest.fixture(scope="session")
def oracle_mod():
    from oracle import oracle as O
    if ORACLE_ROOT:
        assert os.path.realpath(O.__file__).startswith(os.path.realpath(ORACLE_ROOT)), O.__file__
    O.lib()
    return O


@pytest.fixture(scope="session")
def oracle_fma(oracle_mod, tmp_path_factory):
    """The oracle source built with FMA contraction: same arithmetic, other rounding."""
    O = oracle_mod
    so = tmp_path_factory.mktemp("fma") / "oracle_fma.so"
    subprocess.run(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=fast", "-mfma",
                    "-o", str(so), O._SRC, "-lm"], check=True)
    L = ctypes.CDLL(str(so))
    L.nho_integrate.argtypes = O.lib().nho_integrate.argtypes
    return L


class OracleProbe:
    """A request as the oracle reads it, with oracle-only probe attributes
    (hist_hmod: a sampled factor of H(z)) on top of the request's fields."""

    def __init__(self, req, **extra):
        self._req = req
        self.__dict__.update(extra)

    def __getattr__(self, name):
        return getattr(self._req, name)


def ripple_probes(req):
    """Requests whose expansion rate H(z) carries a ripple with the period of the
    library's coefficient table (3072 intervals over the integration interval):
    H -> H (1 + A (1 - cos(2 pi (s + phase)))), s the position in table
    intervals, sampled four times per period, with peaks 2A of 3e-14 and 1e-13,
    the largest interpolation errors of the table's drift and kick columns.
    That is the size and shape of a cubic table's interpolation error, and it
    reaches both the drift (1+z)^2/H and the kick.  The step control is far more
    sensitive to such a ripple than to a smooth change of the same size: its
    error estimate responds to the fifth derivative.  A request with sampled
    histories takes them resampled on the ripple's grid from the oracle's own
    splines (itself a perturbation below 1e-12)."""
    from scipy.interpolate import CubicSpline
    sampled = req.hist_M is not None or req.hist_c is not None or req.hist_kappa is not None
    z_max = req.hist_z_max if sampled else req.z_end
    u_start = -np.log1p(getattr(req, "z_obs", 0.0))
    u_end = -np.log1p(req.z_end)
    n = 4 * 3072 + 1
    u = -np.log1p(z_max) + np.arange(n) * np.log1p(z_max) / (n - 1)
    s = (u - u_end) / (u_start - u_end) * 3072.0
    base = {}
    if sampled:
        m = next(len(a) for a in (req.hist_M, req.hist_c, req.hist_kappa) if a is not None)
        uc = -np.log1p(z_max) + np.arange(m) * np.log1p(z_max) / (m - 1)
        for k in ("hist_M", "hist_c", "hist_kappa"):
            a = getattr(req, k)
            if a is not None:
                base[k] = CubicSpline(uc, np.asarray(a, dtype=np.float64), bc_type="not-a-knot")(u)
    out = []
    for amp, phase in ((1.5e-14, 0.0), (1.5e-14, 0.5), (5e-14, 0.25)):
        ripple = 1.0 + amp * (1.0 - np.cos(2.0 * np.pi * (s + phase)))
        out.append(OracleProbe(req.with_(hist_z_max=z_max, **base), hist_hmod=ripple))
    return out


@pytest.fixture(scope="session")
def sensitivity(oracle_mod, oracle_fma):
    """sensitivity(req, ref_profile): the largest relative change of the oracle's
    own profile under perturbations no larger than what separates two correct
    FP64 integrations of the request: re-rounding of the same arithmetic (the
    FMA-contracted build); relative changes of the force between 1e-14 and
    1e-12: the halo mass scaled by 1 + 1e-12, 1 + 3e-13 and 1 - 1e-14, and,
    when the request leaves G unmodulated, G scaled by 1 + 1e-12 z/(1+z) and by
    1 + 1e-12 sin(40 ln a); a ripple of the expansion rate at the period of the
    library's coefficient table with peaks of 3e-14 and 1e-13, the size and
    shape of that table's interpolation error (ripple_probes); and the first
    trial step scaled by 1 + 1e-12 and 1 - 1e-13, which shifts every later
    step.  Adaptive step control turns such differences into flipped
    accept/reject decisions, i.e. profile differences of order rtol for some
    halos; a ripple at the table period flips far more of them than a smooth
    change of the same size.  The measure is a maximum over these
    probes, computed from the oracle alone."""
    O = oracle_mod

    def dev(profile, ref):
        return float(np.max(np.abs(np.asarray(profile) / np.asarray(ref) - 1.0)))

    def f(req, ref_profile):
        if req.mass_kind == "zero":
            return 0.0
        saved = O._lib
        try:
            O._lib = oracle_fma
            worst = dev(O.solve(req)["n_over_nbar"], ref_profile)
        finally:
            O._lib = saved

        def mass(fac):
            if req.mass_kind == "table":
                return req.with_(hist_M=np.asarray(req.hist_M) * fac)
            return req.with_(M0=req.M0 * fac)
        probes = [mass(1.0 + 1e-12), mass(1.0 + 3e-13), mass(1.0 - 1e-14),
                  req.with_(h0=req.h0 * (1.0 + 1e-12)), req.with_(h0=req.h0 * (1.0 - 1e-13))]
        if req.kappa_kind == "none":
            probes.append(req.with_(kappa_kind="paper", kappa_a=1e-12, kappa_b=1.0))
            # an oscillating G(z), sampled on the request's own history grid if it has one
            n = len(req.hist_M) if req.hist_M is not None else (len(req.hist_c) if req.hist_c is not None else 257)
            z_max = req.hist_z_max if (req.hist_M is not None or req.hist_c is not None) else req.z_end
            u = -np.log1p(z_max) + np.arange(n) * np.log1p(z_max) / (n - 1)
            probes.append(req.with_(kappa_kind="table", hist_z_max=z_max, hist_kappa=1.0 + 1e-12 * np.sin(40.0 * u)))
        probes += ripple_probes(req)
        for p in probes:
            worst = max(worst, dev(O.solve(p)["n_over_nbar"], ref_profile))
        return worst
    return f
