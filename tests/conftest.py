import ctypes
import os
import subprocess
import sys

import numpy as np

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU oracle runs, excluded from the default CPU suite")


@pytest.fixture(scope="session")
def oracle_mod():
    from oracle import oracle as O
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


@pytest.fixture(scope="session")
def sensitivity(oracle_mod, oracle_fma):
    """sensitivity(req, ref_profile): the largest relative change of the oracle's
    profile under perturbations no larger than what separates two correct FP64
    integrations of the request: re-rounding of the same arithmetic (the
    FMA-contracted build), and relative changes of the force of 1e-12 (the
    device interpolates its coefficient tables to ~1e-13-1e-12): the halo mass
    scaled by 1 + 1e-12; when the request leaves G unmodulated, G scaled by
    1 + 1e-12 z/(1+z) and by 1 + 1e-12 sin(40 ln a); and the first trial
    step scaled by 1 + 1e-12, which shifts every later step.  Adaptive step control
    turns such differences into flipped accept/reject decisions, i.e. profile
    differences of order rtol, for some halos, and how much depends on the
    shape of the perturbation; parity bounds scale with this measure where it
    exceeds them."""
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
        if req.mass_kind == "table":
            heavier = req.with_(hist_M=np.asarray(req.hist_M) * (1.0 + 1e-12))
        else:
            heavier = req.with_(M0=req.M0 * (1.0 + 1e-12))
        probes = [heavier, req.with_(h0=req.h0 * (1.0 + 1e-12))]
        if req.kappa_kind == "none":
            probes.append(req.with_(kappa_kind="paper", kappa_a=1e-12, kappa_b=1.0))
            # an oscillating G(z), sampled on the request's own history grid if it has one
            n = len(req.hist_M) if req.hist_M is not None else (len(req.hist_c) if req.hist_c is not None else 257)
            z_max = req.hist_z_max if (req.hist_M is not None or req.hist_c is not None) else req.z_end
            u = -np.log1p(z_max) + np.arange(n) * np.log1p(z_max) / (n - 1)
            probes.append(req.with_(kappa_kind="table", hist_z_max=z_max, hist_kappa=1.0 + 1e-12 * np.sin(40.0 * u)))
        for p in probes:
            worst = max(worst, dev(O.solve(p)["n_over_nbar"], ref_profile))
        return worst
    return f
