"""nh_solve_noalloc, the plain solve that allocates nothing (its buffers live
in the library's static device scratch), against nh_solve_async through the
C ABI: the same profile bits, two calls in a row with the second request
smaller than the first, in FP64 and FP32C, RK4 and a halo-free request; and
its refusals (too large for the scratch, sampled histories)."""
import math

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


def async_profile(ctx, req):
    out = torch.empty(req.n_r, dtype=torch.float64, device="cuda")
    ctx.solve_async(req, out)
    st, _ = ctx.last_stats()
    return out.cpu().numpy(), st


def noalloc_profile(ctx, req):
    out = torch.full((req.n_r,), float("nan"), dtype=torch.float64, device="cuda")
    ctx.solve_noalloc(req, out)
    st, _ = ctx.last_stats()
    return out.cpu().numpy(), st


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_noalloc_equals_async_twice_then_smaller(ctx, prec):
    big = W.shrink(W.plain_scale(3), 40, 48, 24).with_(precision=prec)
    small = W.shrink(W.plain_scale(5), 9, 17, 7).with_(precision=prec)
    for req in (big, small):
        say(f"noalloc {prec} n_r={req.n_r} n_traj={req.n_traj}")
        got, st = noalloc_profile(ctx, req)
        want, wst = async_profile(ctx, req)
        assert np.all(np.isfinite(got))
        assert np.array_equal(got, want), np.abs(got / want - 1).max()
        assert st["accepted_steps"] == wst["accepted_steps"]
        assert st["rejected_steps"] == wst["rejected_steps"]
        assert st["free_exits"] == wst["free_exits"]
        assert st["n_failed"] == 0


def test_noalloc_rk4_and_no_halo(ctx):
    for req in (W.shrink(W.plain_small(), 6, 12, 5), W.shrink(W.plain_small(), 4, 9, 3).with_(mass_kind="zero")):
        say(f"noalloc {req.method} mass {req.mass_kind}")
        got, st = noalloc_profile(ctx, req)
        want, _ = async_profile(ctx, req)
        assert np.array_equal(got, want)
        if req.mass_kind == "zero":
            assert np.all(got == 1.0) and st["free_exits"] == req.n_traj


def test_noalloc_refusals(ctx):
    from paper_2410_08267_amd import nuhalo as N
    say("noalloc refusals")
    out = torch.empty(8192, dtype=torch.float64, device="cuda")
    huge = W.plain_small().with_(method="dp5", y=np.geomspace(0.01, 100.0, 300000))
    with pytest.raises(N.NhError) as e:
        ctx.solve_noalloc(huge, out)
    assert e.value.code == N.NH_EINVAL
    n = 9
    u = -math.log1p(4.0) + np.arange(n) * math.log1p(4.0) / (n - 1)
    sampled = W.shrink(W.plain_small(), 3, 5, 4).with_(method="dp5", mass_kind="table", hist_z_max=4.0,
                                                       hist_M=1e12 * np.exp(-0.8 * np.expm1(-u)))
    with pytest.raises(N.NhError) as e:
        ctx.solve_noalloc(sampled, out)
    assert e.value.code == N.NH_EINVAL
    # the scratch still serves the next call
    req = W.shrink(W.plain_scale(1), 5, 8, 6)
    got, _ = noalloc_profile(ctx, req)
    assert np.array_equal(got, async_profile(ctx, req)[0])
