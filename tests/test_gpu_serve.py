"""Serving form (nh_submit / nh_poll / nh_cancel) on the GPU, through the C ABI.

The server runs the batched slice kernel in time slices and resumes
trajectories cut by a slice boundary from their saved state, so a served
profile must equal the plain path's bit for bit whatever else is being served
and however often it was interrupted.  Served profiles are also checked
against the oracle with the plain paths' bounds: FP64 within 1e-9 at rtol
1e-12 and within 1e-8 (or 4x the oracle's own sensitivity) at rtol 1e-8; FP32C
within 1e-4 of the oracle's reference integration.  Admission is by
device-memory footprint against the budget; cancellation drops a request
without disturbing the others.
"""
import time

import numpy as np
import pytest
import torch

from paper_2410_08267_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[case] {msg}", flush=True)


@pytest.fixture
def ctx():
    from paper_2410_08267_amd import nuhalo as N
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = N.Context(0)
    yield c
    c.close()


def plain(ctx, req):
    out = torch.empty(req.n_r, dtype=torch.float64, device="cuda")
    ctx.solve_async(req, out)
    st, _ = ctx.last_stats()
    return out.cpu().numpy(), st


def wait(ctx, ticket, n_r, timeout=60.0):
    t0 = time.monotonic()
    while True:
        r = ctx.poll(ticket, n_r)
        if r is not None:
            return r
        assert time.monotonic() - t0 < timeout, "ticket did not finish"
        time.sleep(0.001)


@pytest.fixture(scope="module")
def O():
    from oracle import oracle
    oracle.lib()
    return oracle


def small(seed, n, prec="fp64"):
    reqs = W.batched(seed, n_req=n, prec=prec, freeze_in_frac=0.3, kappa_frac=0.2)
    return [W.shrink(r, 5 + i % 3, 10 + i % 5, 6 + i % 2) for i, r in enumerate(reqs)]


@pytest.mark.parametrize("graph", [1, 0])
@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_served_equals_plain_bitwise_across_slices(ctx, prec, graph):
    """Short slices (200 us): most trajectories are saved and resumed many times,
    each slice a replay of the session's HIP graph (graph=1, the default, with
    the host's uploads and synchronisations between replays) or separate
    launches (graph=0)."""
    reqs = small(41, 10, prec)
    say(f"serve {prec} x{len(reqs)} slice 200 us graph {graph}")
    ctx.set_option("slice_us", 200)
    ctx.set_option("serve_graph", graph)
    tickets = [ctx.submit(r) for r in reqs]
    assert all(t is not None for t in tickets)
    res = [wait(ctx, t, r.n_r) for t, r in zip(tickets, reqs)]
    for (prof, st, rc), r in zip(res, reqs):
        assert rc == 0
        p, pst = plain(ctx, r)
        assert np.array_equal(prof, p), np.abs(prof / p - 1).max()
        assert st["accepted_steps"] == pst["accepted_steps"]
        assert st["rejected_steps"] == pst["rejected_steps"]
        assert st["latency_ms"] > 0.0
        assert st["kernel_ms"] > 0.0


def serving_mix(prec, rtol):
    """Serving-workload requests on small grids, with the serving workload's
    kinds certainly present: freeze-in f0 (Sec. IV.B), G(z) = G0 (1 + 0.05 ln(1+z)),
    both, and plain Fermi-Dirac."""
    reqs = small(57, 8, prec)
    reqs[0] = reqs[0].with_(f0_kind="freeze_in", kappa_kind="none", kappa_a=0.0)
    reqs[1] = reqs[1].with_(f0_kind="fermi_dirac", kappa_kind="log", kappa_a=0.05)
    reqs[2] = reqs[2].with_(f0_kind="freeze_in", kappa_kind="log", kappa_a=0.05)
    return [r.with_(rtol=rtol) for r in reqs]


@pytest.mark.parametrize("prec,rtol", [("fp64", 1e-12), ("fp64", 1e-8), ("fp32c", 1e-8)])
def test_served_vs_oracle(ctx, O, sensitivity, prec, rtol):
    """Continuous batching: requests arrive in waves while earlier ones are on the
    GPU, with 500 us slices; each served profile equals the same request solved
    alone on the plain path bit for bit, and the oracle within the plain paths'
    bounds."""
    reqs = serving_mix(prec, rtol)
    say(f"serve {prec} rtol {rtol} x{len(reqs)} in waves, slice 500 us, vs oracle")
    ctx.set_option("slice_us", 500)
    tickets = []
    for i, r in enumerate(reqs):
        t = ctx.submit(r)
        assert t is not None
        tickets.append(t)
        if i % 3 == 2:
            time.sleep(0.003)
    res = [wait(ctx, t, r.n_r) for t, r in zip(tickets, reqs)]
    for i, ((prof, st, rc), r) in enumerate(zip(res, reqs)):
        assert rc == 0
        assert np.array_equal(prof, plain(ctx, r)[0]), i
        if prec == "fp32c":
            ref = O.solve(r.with_(precision="fp64", rtol=1e-10))["n_over_nbar"]
            e = np.abs(prof / ref - 1).max()
            print(f"request {i} ({r.f0_kind}, kappa {r.kappa_kind}): fp32c max rel vs oracle {e:.2e}", flush=True)
            assert e <= 1e-4, i
            continue
        ref = O.solve(r)["n_over_nbar"]
        e = np.abs(prof / ref - 1).max()
        if rtol <= 1e-12:
            print(f"request {i} ({r.f0_kind}, kappa {r.kappa_kind}): max rel vs oracle {e:.2e}", flush=True)
            assert e <= 1e-9, i
        elif e > 1e-8:
            sens = sensitivity(r, ref)
            print(f"request {i}: max rel {e:.2e} (oracle sensitivity {sens:.2e})", flush=True)
            assert e <= 4.0 * sens, i
        else:
            print(f"request {i} ({r.f0_kind}, kappa {r.kappa_kind}): max rel vs oracle {e:.2e}", flush=True)


def test_served_full_size_requests(ctx):
    reqs = W.batched(3, n_req=6, prec="fp32c")
    say(f"serve fp32c full-size x6 n_traj {sum(r.n_traj for r in reqs)}")
    tickets = [ctx.submit(r) for r in reqs]
    res = [wait(ctx, t, r.n_r) for t, r in zip(tickets, reqs)]
    for i in (0, 3, 5):
        p, _ = plain(ctx, reqs[i])
        assert np.array_equal(res[i][0], p)


def test_admission_by_footprint(ctx):
    from paper_2410_08267_amd import nuhalo as N
    reqs = small(7, 3)
    fp = max(N.footprint_bytes(r) for r in reqs)
    say(f"serve admission: budget for two requests of <= {fp} bytes")
    ctx.set_budget(int(2.5 * fp))
    a = ctx.submit(reqs[0])
    b = ctx.submit(reqs[1])
    assert a is not None and b is not None
    assert ctx.submit(reqs[2]) is None           # NH_EBUSY: nothing queued
    ra = wait(ctx, a, reqs[0].n_r)
    wait(ctx, b, reqs[1].n_r)
    c = ctx.submit(reqs[2])                      # memory returned at completion
    assert c is not None
    rc_ = wait(ctx, c, reqs[2].n_r)
    assert np.array_equal(ra[0], plain(ctx, reqs[0])[0])
    assert np.array_equal(rc_[0], plain(ctx, reqs[2])[0])
    assert ctx.submit(W.plain_scale(0)) is None   # larger than the whole budget: NH_EBUSY too
    ctx.set_budget(0)


def test_cancel_isolated(ctx):
    from paper_2410_08267_amd import nuhalo as N
    big = W.plain_scale(4)
    others = small(9, 4)
    say("serve cancel: one full-size request among small ones")
    tb = ctx.submit(big)
    ts = [ctx.submit(r) for r in others]
    assert ctx.cancel(tb) == N.NH_OK
    with pytest.raises(N.NhError) as e:
        wait(ctx, tb, big.n_r)
    assert e.value.code == N.NH_ECANCELED
    for t, r in zip(ts, others):
        prof, st, rc = wait(ctx, t, r.n_r)
        assert np.array_equal(prof, plain(ctx, r)[0])
    assert ctx.cancel(123456789) == N.NH_ENOTFOUND
    with pytest.raises(N.NhError) as e:
        ctx.poll(tb, big.n_r)                     # collected once already
    assert e.value.code == N.NH_ENOTFOUND


def test_one_precision_at_a_time(ctx):
    from paper_2410_08267_amd import nuhalo as N
    a, b = small(13, 2)
    say("serve precision mismatch")
    t = ctx.submit(a)
    with pytest.raises(N.NhError) as e:
        ctx.submit(b.with_(precision="fp32c"))
    assert e.value.code == N.NH_EINVAL
    wait(ctx, t, a.n_r)
    # the server is empty again: the next request may start an FP32C session
    t2 = ctx.submit(b.with_(precision="fp32c"))
    prof, _, _ = wait(ctx, t2, b.n_r)
    assert np.array_equal(prof, plain(ctx, b.with_(precision="fp32c"))[0])
