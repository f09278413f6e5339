"""Batched form (nh_solve_batch) on the GPU, through the C ABI.

A request's trajectories run the same per-lane code in the batched slice
kernel as in the plain kernels, on the same table when both use the same
number of nodes (by default: FP64 keeps one 3073-node table per workgroup,
like the plain form; FP32C two 2049-node tables, its plain form's size), and
the same reduction; so a batched profile must equal the plain path's bit for
bit, whatever else shares the launch.  Against the oracle the bounds are those
of the plain paths: FP32C within 1e-4; FP64 at rtol 1e-12 within 1e-9; at
rtol 1e-10 and 1e-8 within 1e-8 relative, or four times the oracle's own
sensitivity where that is larger (the `sensitivity` fixture).
"""
import numpy as np
import pytest
import torch

from paper_2410_08267_amd import workloads as W

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


def small_mix(seed, n, prec="fp64", grid=(6, 14, 6)):
    """n batched-workload requests on small grids (the physics of the full draws)."""
    reqs = W.batched(seed, n_req=n, prec=prec, freeze_in_frac=0.3, kappa_frac=0.3)
    out = []
    for i, r in enumerate(reqs):
        nr, ny, nm = grid
        out.append(W.shrink(r, nr + i % 3, ny + (i % 4), nm + (i % 2)))
    return out


def run_batch(ctx, reqs):
    n = sum(r.n_r for r in reqs)
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    stats, rc = ctx.solve_batch(reqs, out)
    torch.cuda.synchronize()
    prof = out.cpu().numpy()
    res, k = [], 0
    for r in reqs:
        res.append(prof[k:k + r.n_r].copy())
        k += r.n_r
    return res, stats, rc


def run_plain(ctx, req):
    out = torch.empty(req.n_r, dtype=torch.float64, device="cuda")
    ctx.solve_async(req, out)
    st, _ = ctx.last_stats()
    return out.cpu().numpy(), st


class options:
    """Context options for one test, restored to their defaults afterwards."""

    def __init__(self, ctx, **kw):
        self.ctx, self.kw = ctx, kw

    def __enter__(self):
        for k, v in self.kw.items():
            self.ctx.set_option(k, v)

    def __exit__(self, *exc):
        for k in self.kw:
            self.ctx.set_option(k, 0)


def rel(a, b):
    return np.abs(np.asarray(a) / np.asarray(b) - 1.0)


# slots 0: the default (one table slot per workgroup, request parameters as
# scalars); 2: two slots with per-lane parameters (FP32C at 768 threads)
@pytest.mark.parametrize("prec,slots,nodes", [("fp64", 0, 0), ("fp64", 2, 1537), ("fp32c", 0, 0),
                                               ("fp32c", 2, 0)])
def test_batch_equals_plain_bitwise(ctx, prec, slots, nodes):
    reqs = small_mix(21, 12, prec)
    say(f"batch {prec} of {len(reqs)} vs plain, slots {slots} nodes {nodes}, n_traj {sum(r.n_traj for r in reqs)}")
    with options(ctx, batch_slots=slots, table_nodes=nodes):
        profs, stats, rc = run_batch(ctx, reqs)
        plain = [run_plain(ctx, r) for r in reqs]
    assert rc == 0
    for i, r in enumerate(reqs):
        p, st = plain[i]
        assert np.array_equal(p, profs[i]), (i, rel(p, profs[i]).max())
        assert st["accepted_steps"] == stats[i]["accepted_steps"]
        assert st["rejected_steps"] == stats[i]["rejected_steps"]
        assert st["free_exits"] == stats[i]["free_exits"]
        assert st["fp64_steps"] == stats[i]["fp64_steps"]


def test_alone_equals_in_mix(ctx):
    reqs = small_mix(5, 9)
    say("batch fp64: request 4 alone vs in a mix of 9")
    mix, _, _ = run_batch(ctx, reqs)
    alone, _, _ = run_batch(ctx, [reqs[4]])
    assert np.array_equal(alone[0], mix[4])
    # and in a different order and company
    other, _, _ = run_batch(ctx, [reqs[7], reqs[4], reqs[0]])
    assert np.array_equal(other[1], mix[4])


def mixed_kinds(rtol):
    base = W.shrink(W.plain_small(), 6, 12, 6).with_(method="dp5", rtol=rtol)
    return [
        base.with_(M0=3e13),
        base.with_(geometry="delta200", M0=5e13),
        base.with_(f0_kind="freeze_in", kappa_kind="log", kappa_a=0.05, M0=2e13),
        base.with_(compensated=False, M0=1e13),
        base.with_(mass_kind="zero"),
        W.shrink(W.plain_scale(4), 5, 12, 6).with_(rtol=rtol),
        base.with_(M0=4e13, z_obs=0.6, z_end=4.5),
        base.with_(mass_kind="table", conc_kind="table", hist_z_max=4.0,
                   hist_M=2e13 * np.exp(-0.8 * np.expm1(-np.linspace(-np.log(5.0), 0.0, 33))),
                   hist_c=8.0 / np.exp(-np.linspace(-np.log(5.0), 0.0, 33)),
                   f0_kind="table", f0_ln_y0=np.log(0.02), f0_d_ln_y=0.25,
                   f0_ln_f=-np.logaddexp(0.0, np.exp(np.log(0.02) + 0.25 * np.arange(36)))),
    ]


@pytest.mark.parametrize("rtol", [1e-12, 1e-10, 1e-8])
def test_mixed_geometry_kinds_vs_oracle(ctx, O, sensitivity, rtol):
    """Constant-R and moving-R requests in one launch (the six-column slot layout),
    freeze-in f0, G(z), an uncompensated halo, a halo-free request and one with
    sampled M(z), c(z) and f0, and one observed at z_obs > 0.  At rtol 1e-12
    within 1e-9 (the FP64 gate); at rtol 1e-10 and 1e-8 within 1e-8, or 4x the
    oracle's own sensitivity where that is larger."""
    reqs = mixed_kinds(rtol)
    say(f"batch fp64 mixed kinds vs oracle, rtol {rtol}")
    profs, stats, rc = run_batch(ctx, reqs)
    assert rc == 0
    for i, r in enumerate(reqs):
        ref = O.solve(r)["n_over_nbar"]
        e = rel(profs[i], ref).max()
        if rtol <= 1e-12:
            print(f"request {i}: max rel {e:.2e}", flush=True)
            assert e <= 1e-9, i
        elif e <= 1e-8:
            print(f"request {i}: max rel {e:.2e}", flush=True)
        else:
            sens = sensitivity(r, ref)
            print(f"request {i}: max rel {e:.2e} (oracle sensitivity {sens:.2e})", flush=True)
            assert e <= 4.0 * sens, i
    assert np.array_equal(profs[4], np.ones(reqs[4].n_r))
    assert stats[4]["accepted_steps"] == 0


def sec4_variants():
    """The paper's Sec. IV halo variants (growth xi^alpha, early onset, kappa_1 and
    kappa_2) next to a smooth request in one launch."""
    base = W.shrink(W.plain_small(), 5, 9, 6).with_(method="dp5", mass_kind="paper", M0=1e15, conc_kind="constant",
                                                    c0=7.0, m_eV=0.3, z_end=4.5)
    return [base.with_(mass_alpha=0.5), base.with_(mass_alpha=2.0), base.with_(z_form=9.0),
            base.with_(kappa_kind="paper", kappa_a=0.2, kappa_b=1.5),
            base.with_(kappa_kind="paper", kappa_a=0.1, kappa_b=0.8), W.shrink(W.plain_scale(3), 5, 9, 6)]


def test_sec4_variants_in_a_batch(ctx, O):
    """Power-law factors of the coefficients in the batched form: each request
    equals the plain path bit for bit, and the oracle within 1e-9 at rtol 1e-12."""
    reqs = [r.with_(rtol=1e-12) for r in sec4_variants()]
    say(f"batch fp64 of the Sec. IV variants, rtol 1e-12, n_traj {sum(r.n_traj for r in reqs)}")
    profs, stats, rc = run_batch(ctx, reqs)
    assert rc == 0
    for i, r in enumerate(reqs):
        p, st = run_plain(ctx, r)
        assert np.array_equal(p, profs[i]), (i, rel(p, profs[i]).max())
        e = rel(profs[i], O.solve(r)["n_over_nbar"]).max()
        print(f"request {i}: max rel {e:.2e}", flush=True)
        assert e <= 1e-9, i


@pytest.mark.parametrize("slots", [0, 2])
def test_sec4_variants_fp32c_in_a_batch(ctx, O, slots):
    """The Sec. IV variants (power-law factors: the kernels' HIST variant) in the
    FP32C form, one slot (the default, 1024 threads) and two (768): each
    request equals the plain FP32C path bit for bit, and the oracle's reference
    integration within 1e-4."""
    reqs = [r.with_(precision="fp32c") for r in sec4_variants()]
    say(f"batch fp32c of the Sec. IV variants, slots {slots}, n_traj {sum(r.n_traj for r in reqs)}")
    with options(ctx, batch_slots=slots):
        profs, stats, rc = run_batch(ctx, reqs)
    assert rc == 0
    for i, r in enumerate(reqs):
        p, st = run_plain(ctx, r)
        assert np.array_equal(p, profs[i]), (i, rel(p, profs[i]).max())
        assert st["accepted_steps"] == stats[i]["accepted_steps"]
        ref = O.solve(r.with_(precision="fp64", rtol=1e-10))["n_over_nbar"]
        e = rel(profs[i], ref).max()
        print(f"request {i}: max rel {e:.2e}", flush=True)
        assert e <= 1e-4, i


def test_batch_fp32c_vs_oracle(ctx, O):
    reqs = small_mix(33, 6, "fp32c")
    say("batch fp32c of 6 vs oracle")
    profs, stats, rc = run_batch(ctx, reqs)
    assert rc == 0
    for i, r in enumerate(reqs):
        ref = O.solve(r.with_(precision="fp64"))["n_over_nbar"]
        e = rel(profs[i], ref).max()
        print(f"request {i}: max rel {e:.2e} fp64 attempts {stats[i]['fp64_steps']}", flush=True)
        assert e <= 1e-4


def test_batch_full_size_requests_equal_plain(ctx):
    """Requests of the batched workload at their full drawn sizes: the batch
    must reproduce the plain path (itself checked against sampled oracle
    trajectories at full size) bit for bit."""
    reqs = W.batched(7, n_req=24)
    say(f"batch fp64 24 full-size requests, n_traj {sum(r.n_traj for r in reqs)}")
    profs, stats, rc = run_batch(ctx, reqs)
    assert rc == 0
    for i in (0, 5, 11, 23):
        p, st = run_plain(ctx, reqs[i])
        assert np.array_equal(p, profs[i]), (i, rel(p, profs[i]).max())
        assert st["accepted_steps"] == stats[i]["accepted_steps"]


def test_batch_rejects_mixed_precision_and_rk4(ctx):
    from paper_2410_08267_amd import nuhalo as N
    a = W.shrink(W.plain_scale(0), 3, 8, 4)
    out = torch.empty(64, dtype=torch.float64, device="cuda")
    with pytest.raises(N.NhError):
        ctx.solve_batch([a, a.with_(precision="fp32c")], out)
    with pytest.raises(N.NhError):
        ctx.solve_batch([a.with_(method="rk4", n_steps=50)], out)
    with options(ctx, batch_slots=2, table_nodes=3000):
        with pytest.raises(N.NhError):
            ctx.solve_batch([a], out)
