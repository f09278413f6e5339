"""Serving form (nh_submit / nh_poll / nh_cancel) on the GPU, through the C ABI.

The server runs the batched slice kernel in time slices and resumes
trajectories cut by a slice boundary from their saved state, so a served
profile must equal the plain path's bit for bit whatever else is being served
and however often it was interrupted.  Admission is by device-memory footprint
against the budget; cancellation drops a request without disturbing the others.
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
