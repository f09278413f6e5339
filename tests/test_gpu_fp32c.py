"""The FP32-compensated precision form against the FP64 oracle.

Bound: max relative n/nbar error per radius <= 1e-4 against the oracle's
reference integration (Dormand-Prince at rtol 1e-10).  The FP32 path
integrates at max(rtol, 1e-7); attempts whose step falls below the promotion
threshold run in FP64.  Also reported: the error on delta = n/nbar - 1, which
is the harder measure where n/nbar is close to 1.
"""
import math

import numpy as np
import pytest
import torch

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


CASES = {
    "seed0": lambda: W.shrink(W.precision(0), 12, 24, 10),
    "seed4_heavy": lambda: W.shrink(W.precision(4), 12, 24, 10),
    "seed5": lambda: W.shrink(W.precision(5), 10, 20, 8),
    "seed9": lambda: W.shrink(W.precision(9), 10, 20, 8),
    # the paper's Sec. IV variants and a sampled history (the kernels' HIST variant)
    "growth_alpha_0.5": lambda: _sec4(mass_alpha=0.5),
    "kappa_2": lambda: _sec4(kappa_kind="paper", kappa_a=0.1, kappa_b=0.8),
    "sampled_history": lambda: _sampled(W.shrink(W.precision(2), 8, 16, 6)),
}


def _sec4(**kw):
    return W.shrink(W.plain_small(), 6, 10, 6).with_(
        method="dp5", mass_kind="paper", M0=1e15, conc_kind="constant", c0=7.0, m_eV=0.3, z_end=Z_FORM_PAPER,
        precision="fp32c", **kw)


def _sampled(req, n=41):
    u = -math.log1p(4.0) + np.arange(n) * math.log1p(4.0) / (n - 1)
    z = np.expm1(-u)
    return req.with_(mass_kind="table", conc_kind="table", hist_z_max=4.0,
                     hist_M=req.M0 * np.exp(-0.8 * z) * (1.0 + 0.1 * np.sin(3.0 * u)), hist_c=req.c0 / (1.0 + z) ** 0.7)


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("h_fp64", [0.0, 1e-4])
def test_fp32c_within_1e4_of_oracle(ctx, O, name, h_fp64):
    req = CASES[name]()
    say(f"fp32c {name} h_fp64={h_fp64} n_traj={req.n_traj} M0={req.M0:.3g} m={req.m_eV}")
    ctx.set_option("fp64_below_h", h_fp64)
    try:
        got, stats, _ = ctx.solve(req)
    finally:
        ctx.set_option("fp64_below_h", 1e-6)
    ref = O.solve(req.with_(precision="fp64", rtol=1e-10))["n_over_nbar"]
    e = np.abs(got / ref - 1)
    ed = np.abs((got - 1) - (ref - 1)) / np.maximum(np.abs(ref - 1), 1e-12)
    frac64 = stats["fp64_steps"] / max(1, stats["accepted_steps"] + stats["rejected_steps"])
    print(f"max rel err {e.max():.2e}; delta rel err max {ed.max():.2e}; fp64 attempts {frac64:.4f}; "
          f"steps {stats['accepted_steps']}", flush=True)
    assert stats["n_failed"] == 0
    assert e.max() <= 1e-4
    if h_fp64 == 0.0:
        assert stats["fp64_steps"] == 0


def test_fp32c_full_size_launch_shapes_agree(ctx):
    """Full 1.28 M-trajectory profile of a heavy halo (seed 4) in the benchmark's
    launch shape (1024-thread workgroups, at most 64 of them: the kernel built
    for four waves per SIMD), at 768 threads and in the default launch: the
    same bits.  (The whole profile against the oracle's reference integration:
    test_gpu_full_size.py.)"""
    req = W.precision(4)
    got = {}
    for block in (1024, 768):
        say(f"fp32c full size seed 4 n_traj={req.n_traj}, {block} threads x 64 workgroups")
        ctx.set_option("block_threads", block)
        ctx.set_option("workgroups", 64)
        try:
            got[block], stats, _ = ctx.solve(req)
        finally:
            ctx.set_option("block_threads", 0)
            ctx.set_option("workgroups", 0)
        assert stats["n_failed"] == 0
    say("fp32c full size seed 4, default launch")
    got0, _, _ = ctx.solve(req)
    assert np.array_equal(got0, got[1024])
    assert np.array_equal(got0, got[768])
