"""nh_autotune on the GPU, through the C ABI: the chosen configuration is one
of the candidates, becomes the context's default, and changes no result."""
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
    ratio = torch.empty(req.n_traj, dtype=torch.float64, device="cuda")
    ctx.solve_async(req, out, ratio)
    ctx.last_stats()
    return out.cpu().numpy(), ratio.cpu().numpy()


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_plain_autotune_changes_no_result(ctx, prec):
    sample = [W.shrink(W.plain_scale(s), 24, 48, 32).with_(precision=prec) for s in (100, 101)]
    req = W.shrink(W.plain_scale(3), 20, 40, 24).with_(precision=prec)
    say(f"autotune plain {prec}")
    before = plain(ctx, req)
    res = ctx.autotune(sample, "plain")
    print(res, flush=True)
    allowed = {256, 384, 512, 640, 768, 1024}
    assert res["block_threads"] in allowed
    assert res["n_tried"] == len(allowed)
    assert res["batch_slots"] == 0
    assert 0.0 < res["best_ms"] <= 1.25 * res["default_ms"]
    after = plain(ctx, req)
    assert np.array_equal(before[0], after[0]) and np.array_equal(before[1], after[1])


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_batch_autotune_changes_no_result(ctx, prec):
    reqs = W.batched(21, n_req=12, prec=prec)
    reqs = [W.shrink(r, 6 + i % 4, 12 + i % 7, 8 + i % 3) for i, r in enumerate(reqs)]
    say(f"autotune batch {prec} x{len(reqs)}")
    out = torch.empty(sum(r.n_r for r in reqs), dtype=torch.float64, device="cuda")
    ctx.solve_batch(reqs, out)
    before = out.cpu().numpy().copy()
    res = ctx.autotune(reqs, "batch")
    print(res, flush=True)
    if prec == "fp32c":
        assert res["batch_slots"] in {1, 2}
        # one slot: up to 1024 threads; two slots: up to 768
        assert res["block_threads"] in ({256, 384, 512, 768, 1024} if res["batch_slots"] == 1 else {256, 384, 512, 768})
        assert res["n_tried"] == 9
    else:
        assert res["block_threads"] in {512, 768, 1024} and res["batch_slots"] == 1
        assert res["n_tried"] == 3
    ctx.solve_batch(reqs, out)
    assert np.array_equal(out.cpu().numpy(), before)
    # and a batched profile still equals the plain one bit for bit
    p, _ = plain(ctx, reqs[2])
    off = sum(r.n_r for r in reqs[:2])
    assert np.array_equal(before[off:off + reqs[2].n_r], p)


def test_autotune_rejects_bad_samples(ctx):
    from paper_2410_08267_amd import nuhalo as N
    a = W.shrink(W.plain_small(), 3, 5, 4).with_(method="dp5")
    say("autotune: invalid samples")
    for bad, form in (([a.with_(method="rk4", n_steps=20)], "plain"),
                      ([a, a.with_(precision="fp32c")], "plain"),
                      ([a, a.with_(precision="fp32c")], "batch")):
        with pytest.raises(N.NhError) as e:
            ctx.autotune(bad, form)
        assert e.value.code == N.NH_EINVAL
