"""Rounding-level conditioning of the discrete problem (CPU only).

The same oracle source built with FMA contraction (a different rounding of the
same arithmetic, as a GPU compiler produces) is compared with the plain build.
On chaotic orbits through the halo centre the speed ratios differ at O(1);
trajectories whose one-ulp sensitivity in x0, vx0, vy0 is below 1e-10 agree to
1e-9, and the profiles agree to 1e-9.  These are the tolerances the GPU parity
tests use.
"""
import ctypes
import subprocess

import numpy as np

from paper_2410_08267_amd import workloads as W


def test_fma_build_differs_only_on_ill_conditioned_orbits(oracle_mod, tmp_path):
    O = oracle_mod
    so = tmp_path / "oracle_fma.so"
    subprocess.run(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=fast", "-mfma",
                    "-o", str(so), O._SRC, "-lm"], check=True)
    fma = ctypes.CDLL(str(so))
    fma.nho_integrate.argtypes = O.lib().nho_integrate.argtypes
    req = W.plain_small()
    mu, _ = O.mu_grid(req)
    s0 = O.initial_state(req, req.r_kpc, req.y, mu)
    m, it = O.model_of(req), O.integ_of(req)
    plain = O.speed_ratio(s0[:, 2:], O.integrate_states(m, it, s0)[0][:, 2:])
    saved = O._lib
    try:
        O._lib = fma
        other = O.speed_ratio(s0[:, 2:], O.integrate_states(m, it, s0)[0][:, 2:])
    finally:
        O._lib = saved
    d = np.abs(other / plain - 1)
    sens = np.zeros(s0.shape[0])
    for col in (0, 2, 3):
        for direction in (np.inf, -np.inf):
            p = s0.copy()
            p[:, col] = np.nextafter(p[:, col], direction)
            q = O.speed_ratio(p[:, 2:], O.integrate_states(m, it, p)[0][:, 2:])
            sens = np.maximum(sens, np.abs(q / plain - 1))
    ok = sens <= 1e-10
    assert d.max() > 1e-3            # the ill-conditioned set exists
    assert ok.mean() > 0.95
    assert d[ok].max() <= 1e-9
    pa = O.profile_from_ratio(req, plain)
    pb = O.profile_from_ratio(req, other)
    assert np.abs(pa / pb - 1).max() <= 1e-9
