"""GPU parity of the HIP path against the CPU oracle, through the C ABI.

Every case names itself on stdout before it touches the GPU.

Conditioning.  Orbits that plunge through the halo centre are chaotic under a
fixed-step integrator: moving the oracle's own starting radius by one ulp
changes about 1 % of the plain-small RK4 speed ratios by more than 1e-6 (up
to 0.9) and its profile by 5e-11, and the oracle built with FMA contraction
differs from its plain build by up to 16x on those orbits
(test_conditioning.py).  Such trajectories have no unique answer at rounding
level, so per-trajectory comparisons use only the well-conditioned ones (the
oracle's one-ulp sensitivity in x0, vx0, vy0 below 1e-10), and the profiles,
which average over all of them, carry the tolerance:
  * RK4 (identical step sequence): n/nbar within 1e-9 relative; conditioned
    trajectories within 1e-8 (their sensitivity is <= 1e-10 per ulp, and the
    GPU's elementary functions round differently from the C library's by a
    few ulps on every right-hand side).
  * Dormand-Prince FP64, the gate: rtol 1e-12 on both sides, n/nbar within
    1e-9 relative, every case, no allowance.  At that tolerance the
    accept/reject decisions no longer decide the 1e-9 digit: the oracle's own
    profile moves by at most 2.6e-10 under every probe of the `sensitivity`
    measure, on every case here.
  * Dormand-Prince FP64 at rtol 1e-10 and at the production rtol 1e-8: n/nbar
    within 1e-8 relative, or within four times the oracle's own sensitivity
    where that is larger.  Adaptive step control amplifies tiny differences of
    the force into flipped accept/reject decisions, and at these tolerances
    the discrete answer itself moves by up to a few 1e-8 under 1e-14 relative
    changes of the halo mass (the oracle's rtol-1e-10 profiles are up to 4e-8
    from its converged ones); the sensitivity is measured per case from the
    oracle alone (conftest).  Conditioned trajectories agree to 1e-6.
"""
import math

import numpy as np
import pytest
import torch

from paper_2410_08267_amd import nuhalo as N
from paper_2410_08267_amd import workloads as W
from paper_2410_08267_amd.request import Z_FORM_PAPER

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[case] {msg}", flush=True)


@pytest.fixture(scope="module")
def ctx():
    from paper_2410_08267_amd import nuhalo as N
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = N.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def O():
    from oracle import oracle
    oracle.lib()
    return oracle


def rel(a, b):
    return np.abs(np.asarray(a) / np.asarray(b) - 1.0)


def conditioned(O, req, ref_ratio, index=None, tol=1e-10):
    """Mask of trajectories whose oracle speed ratio moves by <= tol when x0, vx0
    or vy0 moves by one ulp either way (six oracle runs)."""
    mu, _ = O.mu_grid(req)
    s0 = O.initial_state(req, req.r_kpc, req.y, mu)
    if index is not None:
        s0 = s0[index]
    sens = np.zeros(s0.shape[0])
    for col in (0, 2, 3):
        for direction in (np.inf, -np.inf):
            p = s0.copy()
            p[:, col] = np.nextafter(p[:, col], direction)
            s1 = O.integrate_states(O.model_of(req), O.integ_of(req), p)[0]
            sens = np.maximum(sens, rel(O.speed_ratio(p[:, 2:], s1[:, 2:]), ref_ratio))
    return sens <= tol


def gpu_ratios(ctx, req):
    """Run through nh_solve_async with a device ratio buffer; return (profile, ratios, stats)."""
    out = torch.empty(req.n_r, dtype=torch.float64, device="cuda")
    ratio = torch.empty(req.n_traj, dtype=torch.float64, device="cuda")
    ctx.solve_async(req, out, ratio)
    stats, _ = ctx.last_stats()
    torch.cuda.synchronize()
    return out.cpu().numpy(), ratio.cpu().numpy(), stats


def test_rk4_plain_small_full(ctx, O):
    req = W.plain_small()
    say(f"rk4 plain_small full grid n_traj={req.n_traj}")
    prof, ratio, stats = gpu_ratios(ctx, req)
    ref = O.solve(req)
    print("n/nbar gpu", prof, "\noracle", ref["n_over_nbar"], flush=True)
    d = rel(ratio, ref["ratio"])
    ok = conditioned(O, req, ref["ratio"])
    print(f"ratio rel diff: median {np.median(d):.2e} p99.9 {np.quantile(d, 0.999):.2e} max {d.max():.2e}; "
          f"conditioned {ok.mean():.4f}, their max {d[ok].max():.2e}")
    assert rel(prof, ref["n_over_nbar"]).max() <= 1e-9
    assert ok.mean() > 0.95
    assert d[ok].max() <= 1e-8
    assert stats["n_failed"] == 0


@pytest.mark.parametrize("method", ["rk4", "dp5"])
def test_zero_halo_is_exactly_one(ctx, method):
    req = W.shrink(W.plain_small(), 7, 13, 5).with_(mass_kind="zero", method=method)
    say(f"zero halo {method}")
    prof, ratio, _ = gpu_ratios(ctx, req)
    assert np.all(prof == 1.0)
    assert np.all(ratio == 1.0)


def test_rk4_without_exit_region_matches(ctx, O):
    """Radii far outside R: everything free streams (bit-exact ratio 1 for outgoing relics)."""
    req = W.plain_small().with_(r_kpc=np.array([5000.0, 20000.0]), y=np.geomspace(0.01, 100, 9), n_mu=7)
    say("rk4 far radii")
    prof, ratio, _ = gpu_ratios(ctx, req)
    ref = O.solve(req)
    assert rel(prof, ref["n_over_nbar"]).max() <= 1e-12
    mu, _ = O.mu_grid(req)
    out = np.tile(mu, req.n_r * req.n_y) <= 0
    assert np.all(ratio[out] == 1.0)


DP5_CASES = {
    "seed0": lambda: W.shrink(W.plain_scale(0), 12, 24, 10),
    "seed4_heavy": lambda: W.shrink(W.plain_scale(4), 12, 24, 10),
    "seed5": lambda: W.shrink(W.plain_scale(5), 9, 20, 7),
    "paper_model": lambda: W.shrink(W.plain_small(), 8, 16, 6).with_(
        method="dp5", mass_kind="paper", M0=1e14, conc_kind="constant", c0=7.0, z_end=Z_FORM_PAPER, m_eV=0.3),
    "delta200": lambda: W.shrink(W.plain_small(), 8, 16, 6).with_(method="dp5", geometry="delta200", M0=5e13),
    "kappa_freezein": lambda: W.shrink(W.plain_small(), 8, 16, 6).with_(
        method="dp5", kappa_kind="log", kappa_a=0.05, f0_kind="freeze_in", M0=2e14, m_eV=0.2),
    "uncompensated": lambda: W.shrink(W.plain_small(), 6, 12, 6).with_(method="dp5", compensated=False, M0=1e13),
    "ragged_1r_1mu": lambda: W.shrink(W.plain_scale(1), 1, 37, 1),
    "user_mu": lambda: W.shrink(W.plain_scale(2), 5, 11, 3).with_(
        mu=np.array([-0.9, -0.2, 0.1, 0.65]), w_mu=np.array([0.3, 0.6, 0.6, 0.5])),
    "tight_rtol": lambda: W.shrink(W.plain_scale(3), 6, 16, 8).with_(rtol=1e-11),
    "sampled_histories": lambda: _sampled_history(W.shrink(W.plain_scale(2), 8, 16, 6)),
    "sampled_f0": lambda: _sampled_f0(W.shrink(W.plain_scale(6), 8, 16, 6)),
    "z_obs_paper": lambda: W.shrink(W.plain_small(), 8, 16, 6).with_(
        method="dp5", mass_kind="paper", M0=1e14, conc_kind="constant", c0=7.0, m_eV=0.3, z_obs=0.5,
        z_form=1.5 * 200.0 ** (1.0 / 3.0) - 1.0, z_end=1.5 * 200.0 ** (1.0 / 3.0) - 1.0),
    "z_obs_exponential": lambda: W.shrink(W.plain_scale(1), 8, 16, 6).with_(z_obs=1.0, z_end=5.0),
    # Sec. IV.A (Fig. 4): halo growth xi^alpha and an earlier onset of growth;
    # Sec. IV.B (Fig. 5, bottom): the G modulations kappa_1 and kappa_2
    "growth_alpha_0.5": lambda: _paper_sec4(mass_alpha=0.5),
    "growth_alpha_2": lambda: _paper_sec4(mass_alpha=2.0),
    "early_onset": lambda: _paper_sec4(z_form=2.0 * Z_FORM_PAPER),
    "kappa_1": lambda: _paper_sec4(kappa_kind="paper", kappa_a=0.2, kappa_b=1.5),
    "kappa_2": lambda: _paper_sec4(kappa_kind="paper", kappa_a=0.1, kappa_b=0.8),
}


def _paper_sec4(**kw):
    """The paper's halo model with the settings of its Sec. IV studies: a relic of
    0.3 eV around a 1e15 Msun halo (Figs. 4 and 5), observed at z0 = 0 and
    integrated back to the base model's z_i."""
    return W.shrink(W.plain_small(), 6, 10, 6).with_(
        method="dp5", mass_kind="paper", M0=1e15, conc_kind="constant", c0=7.0, m_eV=0.3, z_end=Z_FORM_PAPER, **kw)


def _sampled_history(req, n=41):
    """M(z), c(z) and G(z) given as samples in u = ln a (a growth history with a wiggle)."""
    u = -math.log1p(4.0) + np.arange(n) * math.log1p(4.0) / (n - 1)
    z = np.expm1(-u)
    return req.with_(mass_kind="table", conc_kind="table", kappa_kind="table", hist_z_max=4.0,
                     hist_M=req.M0 * np.exp(-0.8 * z) * (1.0 + 0.1 * np.sin(3.0 * u)),
                     hist_c=req.c0 / (1.0 + z) ** 0.7, hist_kappa=1.0 + 0.1 * (z / (1.0 + z)) ** 1.5)


def _sampled_f0(req, n=60):
    """A two-component f0 (thermal plus a bump, Fig. 5 top) given as ln f samples in ln y;
    the grid's ends fall outside the sampled range."""
    x = math.log(0.02) + np.arange(n) * (math.log(60.0) - math.log(0.02)) / (n - 1)
    y = np.exp(x)
    f = 1.0 / (1.0 + np.exp(y)) + 0.3 * np.exp(-0.5 * ((y - 3.0) / 0.7) ** 2)
    return req.with_(f0_kind="table", f0_ln_y0=float(x[0]), f0_d_ln_y=float(x[1] - x[0]), f0_ln_f=np.log(f))


@pytest.mark.parametrize("name", sorted(DP5_CASES))
def test_dp5_fp64_gate(ctx, O, name):
    """The FP64 gate: Dormand-Prince at rtol 1e-12 on both sides, every radius
    of every case within 1e-9 of the oracle, with no allowance (the oracle's
    own profile moves by at most 2.6e-10 there under any probe)."""
    req = DP5_CASES[name]().with_(rtol=1e-12)
    say(f"dp5 gate {name} rtol 1e-12 n_traj={req.n_traj}")
    prof, _, stats = gpu_ratios(ctx, req)
    ref = O.solve(req)
    e = rel(prof, ref["n_over_nbar"]).max()
    print(f"n/nbar max rel {e:.2e}; steps gpu {stats['accepted_steps']} oracle {int(ref['accepted'].sum())}",
          flush=True)
    assert stats["n_failed"] == 0 and np.all(ref["status"] == 0)
    assert e <= 1e-9


@pytest.mark.parametrize("name", sorted(DP5_CASES))
def test_dp5_matches_oracle(ctx, O, sensitivity, name):
    """At the case's own tolerance (rtol 1e-8 for most: the production
    setting): within 1e-8, or 4x the oracle's own sensitivity where that is
    larger; per trajectory, the median speed ratio within 1e-10 and nearly all
    well-conditioned ones within 1e-6."""
    req = DP5_CASES[name]()
    say(f"dp5 {name} n_traj={req.n_traj} M0={req.M0:.3g} m={req.m_eV} rtol {req.rtol}")
    prof, ratio, stats = gpu_ratios(ctx, req)
    ref = O.solve(req)
    e = rel(prof, ref["n_over_nbar"]).max()
    d = rel(ratio, ref["ratio"])
    acc_ref = int(ref["accepted"].sum())
    ok = conditioned(O, req, ref["ratio"])
    sens = sensitivity(req, ref["n_over_nbar"]) if e > 1e-8 else float("nan")
    print(f"n/nbar max rel {e:.2e} (oracle sensitivity {sens:.2e}); "
          f"ratio median {np.median(d):.2e} p99 {np.quantile(d, 0.99):.2e} "
          f"max {d.max():.2e}; conditioned {ok.mean():.4f} p99 {np.quantile(d[ok], 0.99):.2e}; "
          f"steps gpu {stats['accepted_steps']} oracle {acc_ref} free exits {stats['free_exits']}",
          flush=True)
    assert e <= 1e-8 or e <= 4.0 * sens
    assert np.median(d) <= 1e-10
    assert np.quantile(d[ok], 0.99) <= 1e-6
    assert stats["n_failed"] == 0
    # the free-streaming exit only removes steps
    assert stats["accepted_steps"] <= acc_ref * 1.01 + 10


@pytest.mark.parametrize("name", sorted(DP5_CASES))
def test_dp5_matches_oracle_at_rtol_1e10(ctx, O, sensitivity, name):
    """The oracle's reference tolerance, rtol 1e-10, on both sides: within
    1e-8, or 4x the oracle's own sensitivity at that tolerance where that is
    larger."""
    req = DP5_CASES[name]().with_(rtol=1e-10)
    say(f"dp5 {name} at rtol {req.rtol} n_traj={req.n_traj}")
    prof, _, stats = gpu_ratios(ctx, req)
    ref = O.solve(req)["n_over_nbar"]
    e = rel(prof, ref).max()
    assert stats["n_failed"] == 0
    if e <= 1e-8:
        print(f"n/nbar max rel {e:.2e}", flush=True)
        return
    sens = sensitivity(req, ref)
    print(f"n/nbar max rel {e:.2e} (oracle sensitivity {sens:.2e})", flush=True)
    assert e <= 4.0 * sens


def test_dp5_full_size_launch_shapes_agree(ctx, O):
    """Full 100 x 200 x 64 grid of a heavy halo (seed 4) in the benchmark's launch
    shape (1024-thread workgroups, at most 64 of them, as when four profiles run
    side by side) and in the default launch: the same bits, and the profile is
    the oracle's quadrature of the GPU's own ratios.  (The whole profile against
    the oracle's: test_gpu_full_size.py.)"""
    req = W.plain_scale(4)
    say(f"dp5 full size seed 4 n_traj={req.n_traj}, 1024 threads x 64 workgroups vs default")
    ctx.set_option("block_threads", 1024)
    ctx.set_option("workgroups", 64)
    try:
        prof, ratio, stats = gpu_ratios(ctx, req)
    finally:
        ctx.set_option("block_threads", 0)
        ctx.set_option("workgroups", 0)
    assert stats["n_failed"] == 0
    prof0, ratio0, _ = gpu_ratios(ctx, req)
    assert np.array_equal(ratio0, ratio) and np.array_equal(prof0, prof)
    cpu_prof = O.profile_from_ratio(req, ratio)
    assert rel(prof, cpu_prof).max() <= 1e-13


def test_max_steps_is_reported(ctx):
    from paper_2410_08267_amd import nuhalo as N
    req = W.shrink(W.plain_scale(4), 3, 8, 4).with_(max_steps=3)
    say("dp5 max_steps=3")
    out, stats, rc = ctx.solve(req, allow_failed=True)
    assert rc == N.NH_ESTEPS
    assert stats["n_failed"] > 0
    assert np.all(np.isfinite(out))


def test_async_on_torch_stream(ctx, O):
    req = W.shrink(W.plain_scale(0), 6, 16, 8)
    say("dp5 async on a side stream")
    s = torch.cuda.Stream()
    out = torch.zeros(req.n_r, dtype=torch.float64, device="cuda")
    with torch.cuda.stream(s):
        ctx.solve_async(req, out, stream=s)
    s.synchronize()
    ref = O.solve(req)["n_over_nbar"]
    assert rel(out.cpu().numpy(), ref).max() <= 1e-8


def test_step_counts_match_oracle_without_exit(ctx, O):
    """With the free-streaming exit off, the GPU takes the oracle's step sequence:
    identical accepted/rejected counts for almost every trajectory."""
    req = W.shrink(W.plain_scale(0), 10, 20, 8)
    say("dp5 step counts, free exit off")
    ctx.set_option("free_exit", 0)
    try:
        prof, ratio, stats = gpu_ratios(ctx, req)
        acc, rej, st = ctx.trajectory_stats(req.n_traj)
    finally:
        ctx.set_option("free_exit", 1)
    ref = O.solve(req)
    same = (acc == ref["accepted"]) & (rej == ref["rejected"])
    print(f"identical step counts: {same.mean():.4f}; free exits {int(((st & 256) != 0).sum())}")
    assert np.all((st & 256) == 0)
    assert same.mean() > 0.97
    assert stats["accepted_steps"] == int(acc.sum())


@pytest.mark.parametrize("block", [128, 0])
def test_queue_order_does_not_change_results(ctx, block):
    """Every queue order is a permutation of the trajectories: identical ratios.
    With 128-thread workgroups the spread order (3) runs three full rounds of
    claims plus a partial round and a ragged last block (100650 trajectories)."""
    req = W.shrink(W.plain_scale(4), 25, 66, 61)
    say(f"dp5 queue orders 0-3, block {block}, n_traj={req.n_traj}")
    ctx.set_option("block_threads", block)
    try:
        ref = gpu_ratios(ctx, req)
        for order in (1, 2, 3):
            ctx.set_option("queue_order", order)
            got = gpu_ratios(ctx, req)
            assert np.array_equal(ref[1], got[1]), order
            assert np.array_equal(ref[0], got[0]), order
            assert got[2]["accepted_steps"] == ref[2]["accepted_steps"]
    finally:
        ctx.set_option("queue_order", 0)
        ctx.set_option("block_threads", 0)


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
@pytest.mark.parametrize("block", [512, 1024])
def test_fused_quadrature_from_finish_rings(ctx, block, prec):
    """The fused quadrature (finished trajectories wait in per-wavefront LDS
    rings of 64 and are summed a ring at a time) against the reduction of
    stored ratios: the same bits and the same step statistics.  100650
    trajectories on 8 or 16 wavefronts a workgroup: many full rings, and a
    partial one per wavefront at the end.  FP32C at 1024 threads is the build
    that re-reads the request's parameters at each use."""
    req = W.shrink(W.plain_scale(4), 25, 66, 61).with_(precision=prec)
    say(f"{prec} fused vs stored ratios, block {block}, n_traj={req.n_traj}")
    ctx.set_option("block_threads", block)
    try:
        prof, _, st = gpu_ratios(ctx, req)
        out = torch.empty(req.n_r, dtype=torch.float64, device="cuda")
        ctx.solve_async(req, out)
        fst, _ = ctx.last_stats()
        torch.cuda.synchronize()
    finally:
        ctx.set_option("block_threads", 0)
    assert np.array_equal(out.cpu().numpy(), prof)
    for key in ("accepted_steps", "rejected_steps", "n_failed", "free_exits", "max_steps_one_traj", "fp64_steps"):
        assert fst[key] == st[key], key


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_fused_quadrature_with_culled_relics(ctx, O, prec):
    """As above with App. B culls: radii from 0.3 to 12 compensation radii, so
    that many relics never reach the halo and are summed at their claim without
    a step (ratio exactly 1), beside the ring's finishers.  Fused and
    stored-ratio profiles and statistics are the same bits."""
    base = W.shrink(W.plain_scale(0), 25, 66, 61)
    R, _ = O.halo_radii(base, 0.0)
    req = base.with_(r_kpc=R * np.geomspace(0.3, 12.0, 25), precision=prec)
    say(f"{prec} fused vs stored ratios with culls, n_traj={req.n_traj}")
    ctx.set_option("block_threads", 1024)
    try:
        prof, ratio, st = gpu_ratios(ctx, req)
        acc, rej, _ = ctx.trajectory_stats(req.n_traj)
        out = torch.empty(req.n_r, dtype=torch.float64, device="cuda")
        ctx.solve_async(req, out)
        fst, _ = ctx.last_stats()
        torch.cuda.synchronize()
    finally:
        ctx.set_option("block_threads", 0)
    culled = (acc + rej) == 0
    print(f"culled {culled.sum()} of {req.n_traj}", flush=True)
    assert culled.sum() > req.n_traj // 10 and np.all(ratio[culled] == 1.0)
    assert np.array_equal(out.cpu().numpy(), prof)
    for key in ("accepted_steps", "rejected_steps", "n_failed", "free_exits", "max_steps_one_traj", "fp64_steps"):
        assert fst[key] == st[key], key


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_workgroup_cap_does_not_change_results(ctx, prec):
    """Capping a launch's workgroups (so that solves on several streams run side
    by side) changes only which lanes take which trajectories: identical ratios.
    Three 1024-thread workgroups (FP32C: its 768-thread limit) leave a ragged
    last round of claims on 100650 trajectories; two solves on two streams at
    once give the same bits again."""
    req = W.shrink(W.plain_scale(4), 25, 66, 61).with_(precision=prec)
    say(f"{prec} workgroup cap 3 and two streams, n_traj={req.n_traj}")
    ref = gpu_ratios(ctx, req)
    ctx.set_option("workgroups", 3)
    ctx.set_option("block_threads", 1024)
    try:
        got = gpu_ratios(ctx, req)
        assert np.array_equal(ref[1], got[1])
        assert np.array_equal(ref[0], got[0])
        assert got[2]["accepted_steps"] == ref[2]["accepted_steps"]
        with pytest.raises(N.NhError):
            ctx.set_option("workgroups", 0.5)
        with pytest.raises(N.NhError):
            ctx.set_option("workgroups", 70000)
        # two contexts, half the device each, on two streams at once
        ctx.set_option("workgroups", 128)
        other = N.Context(0)
        try:
            other.set_option("workgroups", 128)
            s2 = torch.cuda.Stream()
            outs = [torch.empty(req.n_r, dtype=torch.float64, device="cuda") for _ in range(2)]
            ratios = [torch.empty(req.n_traj, dtype=torch.float64, device="cuda") for _ in range(2)]
            ctx.solve_async(req, outs[0], ratio=ratios[0])
            other.solve_async(req, outs[1], ratio=ratios[1], stream=s2)
            ctx.last_stats()
            other.last_stats()
            torch.cuda.synchronize()
            for o, r in zip(outs, ratios):
                assert np.array_equal(o.cpu().numpy(), ref[0])
                assert np.array_equal(r.cpu().numpy(), ref[1])
        finally:
            other.close()
    finally:
        ctx.set_option("workgroups", 0)
        ctx.set_option("block_threads", 0)


def test_rk4_observed_at_z_obs(ctx, O):
    """Integration from z_obs > 0 (the halo's reference epoch moves with it)."""
    req = W.shrink(W.plain_small(), 6, 12, 6).with_(z_obs=0.8, z_end=3.5, M0=5e13)
    say(f"rk4 z_obs {req.z_obs} n_traj={req.n_traj}")
    prof, ratio, stats = gpu_ratios(ctx, req)
    ref = O.solve(req)
    print("n/nbar gpu", prof, "\noracle", ref["n_over_nbar"], flush=True)
    assert rel(prof, ref["n_over_nbar"]).max() <= 1e-9
    assert stats["n_failed"] == 0


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_cull_relics_that_never_reach_the_halo(ctx, O, prec):
    """App. B: a relic whose straight backward path stays outside the largest
    compensation radius feels no force (the compensated halo has no mass
    perturbation there), so it takes no steps and keeps ratio 1; the oracle,
    which integrates every trajectory, returns exactly 1 for them too."""
    base = W.shrink(W.plain_scale(0), 4, 16, 8)
    R, _ = O.halo_radii(base, 0.0)
    req = base.with_(r_kpc=R * np.array([0.5, 1.5, 4.0, 12.0]), precision=prec)
    say(f"cull {prec} radii {req.r_kpc} n_traj={req.n_traj}")
    prof, ratio, stats = gpu_ratios(ctx, req)
    acc, rej, _ = ctx.trajectory_stats(req.n_traj)
    culled = (acc + rej) == 0
    ref = O.solve(req.with_(precision="fp64"))
    print(f"culled {culled.sum()} of {req.n_traj}; free exits {stats['free_exits']}", flush=True)
    assert culled.sum() > req.n_traj // 10
    assert np.all(ratio[culled] == 1.0)
    assert np.all(ref["ratio"][culled] == 1.0)
    tol = 1e-8 if prec == "fp64" else 1e-4
    assert rel(prof, ref["n_over_nbar"]).max() <= tol


def test_masses_reuse_one_integration(ctx, O, sensitivity):
    """Sec. II.D: one integration serves every relic mass.  Mass m's profile is
    the quadrature of the scaled momentum grid over the same speed ratios; the
    request's own mass reproduces the plain solve bit for bit."""
    req = DP5_CASES["paper_model"]().with_(rtol=1e-10)
    masses = [req.m_eV, 0.1, 0.6]
    say(f"masses {masses} n_traj={req.n_traj}")
    out = torch.empty(len(masses) * req.n_r, dtype=torch.float64, device="cuda")
    ratio = torch.empty(req.n_traj, dtype=torch.float64, device="cuda")
    ctx.solve_masses(req, masses, out, ratio)
    st, _ = ctx.last_stats()
    assert st["n_failed"] == 0
    prof = out.cpu().numpy().reshape(len(masses), req.n_r)
    r = ratio.cpu().numpy()
    p0, r0, _ = gpu_ratios(ctx, req)
    assert np.array_equal(prof[0], p0) and np.array_equal(r, r0)
    ref = O.solve_masses(req, masses)
    for k, m in enumerate(masses):
        rq = req.with_(m_eV=m, y=np.asarray(req.y) * (m / req.m_eV))
        assert rel(prof[k], O.profile_from_ratio(rq, r)).max() <= 1e-13
        e = rel(prof[k], ref[k]).max()
        print(f"mass {m}: n/nbar {prof[k][:3]} max rel vs oracle {e:.2e}", flush=True)
        if e > 1e-8:
            assert e <= 4.0 * sensitivity(rq, ref[k])


def test_masses_rejects_bad_input(ctx):
    from paper_2410_08267_amd import nuhalo as N
    req = W.shrink(W.plain_small(), 3, 5, 4).with_(method="dp5")
    out = torch.empty(4 * req.n_r, dtype=torch.float64, device="cuda")
    say("masses: invalid mass lists")
    for bad in ([], [0.1, -0.2], [float("nan")]):
        with pytest.raises((N.NhError, ValueError)):
            ctx.solve_masses(req, bad, out)


def test_fp64_fma_peak_is_plausible(ctx):
    """The FMA probe measures the device's FP64 vector rate: MI355X's published
    figure is 78.6 TFLOP/s (256 CUs x 128 FP64 FLOP per clock at 2.4 GHz)."""
    say("fp64 fma peak probe")
    t = ctx.fp64_fma_peak()
    print(f"measured FP64 FMA {t:.1f} TFLOP/s", flush=True)
    assert 30.0 < t < 1.1 * 78.6


def test_integrand_output(ctx, O):
    """nh_solve_integrand: the direction-integrated distribution per radius and
    momentum node equals the oracle's quadrature of the GPU's own speed ratios,
    sums (with the y weights) to the profile, and leaves profile and ratios
    identical to nh_solve_async."""
    req = DP5_CASES["paper_model"]()
    say(f"integrand output n_traj={req.n_traj}")
    out = torch.empty(req.n_r, dtype=torch.float64, device="cuda")
    F = torch.empty(req.n_r * req.n_y, dtype=torch.float64, device="cuda")
    ratio = torch.empty(req.n_traj, dtype=torch.float64, device="cuda")
    ctx.solve_integrand(req, out, F, ratio)
    st, _ = ctx.last_stats()
    assert st["n_failed"] == 0
    prof, r, F = out.cpu().numpy(), ratio.cpu().numpy(), F.cpu().numpy().reshape(req.n_r, req.n_y)
    p0, r0, _ = gpu_ratios(ctx, req)
    assert np.array_equal(prof, p0) and np.array_equal(r, r0)
    ref = O.integrand_from_ratio(req, r)
    assert rel(F, ref).max() <= 1e-13
    wy = O.y_weights(np.asarray(req.y))
    _, w_mu = O.mu_grid(req)
    den = (wy * O.f0_of(req, np.asarray(req.y))).sum() * w_mu.sum()
    assert rel((F * wy[None, :]).sum(axis=1) / den, prof).max() <= 1e-12
    # no halo: the initial distribution times the direction weights
    z = req.with_(mass_kind="zero")
    Fz = torch.empty(req.n_r * req.n_y, dtype=torch.float64, device="cuda")
    ctx.solve_integrand(z, out, Fz)
    ctx.last_stats()
    want = O.f0_of(req, np.asarray(req.y)) * w_mu.sum()
    assert rel(Fz.cpu().numpy().reshape(req.n_r, req.n_y), want[None, :]).max() <= 1e-14


def test_more_than_2_32_trajectories(ctx):
    """Maximum sizes: 65536 x 256 x 257 = 4.31e9 trajectories (more than 2^32,
    103 GB of per-trajectory results) with no halo: every index is 64-bit and
    every one-thread-per-item grid is capped and strided.  The profile is
    exactly 1 at every radius and every trajectory is counted."""
    req = W.plain_small().with_(mass_kind="zero", method="dp5", r_kpc=np.geomspace(10.0, 1000.0, 65536),
                                y=np.geomspace(0.01, 100.0, 256), n_mu=257)
    assert req.n_traj > 2 ** 32
    say(f"zero halo at n_traj={req.n_traj}")
    out = torch.empty(req.n_r, dtype=torch.float64, device="cuda")
    ctx.solve_async(req, out)
    st, _ = ctx.last_stats()
    assert st["n_traj"] == req.n_traj and st["free_exits"] == req.n_traj
    assert st["accepted_steps"] == 0 and st["n_failed"] == 0
    assert np.all(out.cpu().numpy() == 1.0)
