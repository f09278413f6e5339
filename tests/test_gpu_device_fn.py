"""The device's own elementary functions of the right-hand side, through the C
ABI (nh_device_function), against 50-digit references (mpmath):

  * the NFW mass integral I(q) = ln(1+q) - q/(1+q) (Eq. nfw, App. A), over q
    from 1e-10 to 1e4: the kernels' branch-free form sums e ln2,
    (1 - 2^e)/(1+q), s^2 (1 + 1/m) and 2(atanh s - s) with 1+q = m 2^e,
    s = (m-1)/(m+1), so its error is a few ulp of the largest of those terms,
    not of I: the bound is 12 ulp of the sum of their magnitudes (s carries up
    to ~3 ulp from the reciprocal of (m+1)(1+q) and two products, and s^2
    doubles it; where the terms cancel, just above q = sqrt(2) - 1, I is a
    twenty-fifth of their sum and the relative error reaches ~30 ulp); below
    q = sqrt(2) - 1 (e = 0) the first two terms are exactly zero, the others
    positive, and the bound is 12 ulp of I itself.  The median error is within
    4 ulp of I;
  * the power-law factor of K and Kc (Sec. IV.A, IV.B): xi^alpha of the paper's
    growth model and kappa = 1 + a [z/(1+z)]^b, from the kernels' own exp, expm1
    and log.  Bound per point: 8 ulp, plus for xi^alpha the error that 4 ulp of
    e^{-u} make through the cancellation in xi = (1 + z_f - e^{-u})/(z_f - z0)
    (any FP64 evaluation of that formula carries it).  A request with neither
    factor gives exactly 1.
"""
import math

import numpy as np
import pytest
import torch

from paper_2410_08267_amd import workloads as W

pytestmark = pytest.mark.gpu
mp = pytest.importorskip("mpmath")
mp.mp.dps = 50
EPS = 2.0 ** -53


def say(msg):
    print(f"[case] {msg}", flush=True)


@pytest.fixture(scope="module")
def ctx():
    from paper_2410_08267_amd import nuhalo as N
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = N.Context(0)
    yield c
    c.close()


def test_nfw_integral_on_the_device(ctx):
    s2m1 = math.sqrt(2.0) - 1.0
    q = np.concatenate([np.geomspace(1e-10, 1e4, 3000), np.linspace(0.3, 0.8, 500),
                        np.linspace(s2m1 - 1e-3, s2m1 + 1e-3, 400), [s2m1, 0.5, 1.0, 2.0]])
    say(f"device nfw_I at {q.size} points")
    got = ctx.device_function("nfw_I", q)
    ref = np.array([float(mp.log1p(mp.mpf(x)) - mp.mpf(x) / (1 + mp.mpf(x))) for x in q])
    e = np.frexp((1.0 + q) * math.sqrt(2.0))[1] - 1.0
    m = (1.0 + q) / 2.0 ** e
    # the magnitudes of e ln2, (1 - 2^e)/(1+q), s^2 (1 + 1/m) and
    # 2 (atanh s - s); at e = 0 the first two vanish and the others sum to I
    s = (m - 1.0) / (m + 1.0)
    t3 = np.abs(2.0 * (np.arctanh(s) - s))
    terms = np.where(e == 0.0, ref, e * math.log(2.0) + (2.0 ** e - 1.0) / (1.0 + q)
                     + s * s * (1.0 + 1.0 / m) + t3)
    err = np.abs(got / ref - 1.0) / EPS
    over = np.abs(got - ref) / (12.0 * EPS * terms)
    print(f"ulp max {err.max():.1f} median {np.median(err):.2f} at q = {q[np.argmax(err)]:.3g}; "
          f"worst fraction of the bound {over.max():.2f} at q = {q[np.argmax(over)]:.4g}", flush=True)
    assert over.max() <= 1.0 and np.median(err) <= 4.0
    assert ctx.device_function("nfw_I", np.array([0.0]))[0] == 0.0


def _variants():
    base = W.plain_scale(0).with_(mass_kind="paper", M0=1.0e14, conc_kind="constant", c0=7.0)
    return {"xi_alpha_0.5": base.with_(mass_alpha=0.5), "xi_alpha_2": base.with_(mass_alpha=2.0),
            "early_onset_z9": base.with_(z_form=9.0, mass_alpha=1.0),
            "kappa_1": base.with_(kappa_kind="paper", kappa_a=0.2, kappa_b=1.5),
            "kappa_2": base.with_(kappa_kind="paper", kappa_a=0.1, kappa_b=0.8),
            "both_z_obs": base.with_(mass_alpha=0.7, kappa_kind="paper", kappa_a=0.1, kappa_b=0.8, z_obs=0.5)}


def _reference(r, u):
    """The factor in 50-digit arithmetic from the same FP64 parameters the
    library derives (1 + z_f, 1/(z_f - z0)), and the per-point bound in ulp."""
    on_mass = r.mass_kind == "paper" and r.mass_alpha > 0 and (r.mass_alpha != 1.0 or r.z_form < r.z_end)
    on_kappa = r.kappa_kind == "paper"
    zf1, inv_dz = 1.0 + r.z_form, 1.0 / (r.z_form - r.z_obs)
    ref, tol = [], []
    for x in u:
        f, t = mp.mpf(1), 8.0
        if on_mass:
            e = mp.exp(-mp.mpf(x))
            xi = min(max((mp.mpf(zf1) - e) * mp.mpf(inv_dz), mp.mpf(0)), mp.mpf(1))
            f = xi ** mp.mpf(r.mass_alpha) if xi > 0 else mp.mpf(0)
            if xi > 0:
                t += r.mass_alpha * 4.0 * np.spacing(float(e)) * inv_dz / float(xi) / EPS
        if on_kappa:
            zr = -mp.expm1(mp.mpf(x))
            f *= 1 + (mp.mpf(r.kappa_a) * zr ** mp.mpf(r.kappa_b) if zr > 0 else 0)
        ref.append(float(f))
        tol.append(t)
    return np.array(ref), np.array(tol)


@pytest.mark.parametrize("name", sorted(_variants()))
def test_power_factor_on_the_device(ctx, name):
    r = _variants()[name]
    u = np.linspace(-math.log1p(r.z_end), -math.log1p(r.z_obs), 1500)
    say(f"device pow_factor {name} at {u.size} points")
    got = ctx.device_function("pow_factor", u, r)
    ref, tol = _reference(r, u)
    err = np.where(ref != 0.0, np.abs(got / np.where(ref != 0.0, ref, 1.0) - 1.0) / EPS, np.abs(got) / EPS)
    print(f"ulp max {err.max():.1f} (bound there {tol[np.argmax(err)]:.1f}) median {np.median(err):.2f}", flush=True)
    assert np.all(err <= tol)


def test_no_factor_is_exactly_one(ctx):
    r = W.plain_scale(0)
    u = np.linspace(-math.log1p(r.z_end), 0.0, 100)
    assert np.all(ctx.device_function("pow_factor", u, r) == 1.0)
