"""Batched restarted GMRES (one launch per DCGS2 step over all instances, graph-replayed
cycles) against the oracle's GMRES on the DCGS2 basis and against the single-instance
gmres_solve, instance by instance.

Instances differ in grid size (m = 42 .. 4,096, odd and even), velocity and restart
length (5 .. 50).  Per instance: the true relative residual reaches 1e-8, the
reported residual is the true one, the iteration count is the oracle's within one
step and the cycle count the oracle's (GMRES has many correct x, so x is checked by
its residual, not by its bits).
"""
import numpy as np
import pytest

from oracle import operators as ops
from oracle.gmres import gmres_dcgs2
from paper_2104_01253_amd import binding, synth
from tests._gpu import dev_vector, host, say, torch_cuda

pytestmark = pytest.mark.gpu

# (grid, velocity, restart, seed)
CASES = [((32, 32), (10.0, 10.0), 50, 31), ((31, 17), (10.0, 3.0), 20, 32),
         ((48, 20), (0.0, 20.0), 35, 33), ((7, 6), (1.0, 2.0), 5, 34),
         ((64, 64), (25.0, 5.0), 40, 35), ((50, 1), (8.0, 0.0), 10, 36)]


@pytest.fixture(scope="module")
def ctx():
    torch_cuda()
    c = binding.Context(0)
    yield c
    c.close()


def _setup(cases, zero=()):
    descs = [binding.stencil2d(g, 1.0, v) for g, v, _, _ in cases]
    bs = [synth.uniform_vector(g[0] * g[1], s) for g, _, _, s in cases]
    for i in zero:
        bs[i] = np.zeros_like(bs[i])
    return descs, bs, [r for _, _, r, _ in cases]


def _check(infos, xs, cases, bs, tau=1e-8):
    for i, (g, v, r, _) in enumerate(cases):
        A = ops.convection_diffusion(g, 1.0, v)
        xr, iref = gmres_dcgs2(A, bs[i], restart=r, rtol=1e-8, tau=tau)
        relres = np.linalg.norm(bs[i] - A @ xs[i]) / np.linalg.norm(bs[i])
        say("instance", i, g, "restart", r, "gpu", infos[i]["iters"], infos[i]["cycles"],
            f"{relres:.2e}", "oracle", iref["iters"], iref["cycles"])
        assert infos[i]["status"] == binding.OK and relres <= 1e-8
        assert abs(infos[i]["relres_true"] - relres) <= 1e-12
        assert abs(infos[i]["iters"] - iref["iters"]) <= 1
        assert infos[i]["cycles"] == iref["cycles"]


def _split(x, cases):
    out, o = [], 0
    for g, _, _, _ in cases:
        m = g[0] * g[1]
        out.append(x[o:o + m])
        o += m
    return out


def test_gmres_batched_vs_oracle_and_single(ctx):
    torch = torch_cuda()
    descs, bs, rs = _setup(CASES)
    x = torch.zeros(sum(b.size for b in bs), dtype=torch.float64, device="cuda")
    rc, infos = ctx.gmres_batched(descs, rs, dev_vector(np.concatenate(bs)), x, rtol=1e-8)
    assert rc == binding.OK
    xs = _split(host(x), CASES)
    _check(infos, xs, CASES, bs)
    for i, (g, v, r, _) in enumerate(CASES):
        xi = torch.zeros(g[0] * g[1], dtype=torch.float64, device="cuda")
        rc1, i1 = ctx.gmres(binding.stencil_op(g, 1.0, v), dev_vector(bs[i]), xi, restart=r,
                            rtol=1e-8)
        assert rc1 == binding.OK and abs(i1["iters"] - infos[i]["iters"]) <= 1
        assert i1["cycles"] == infos[i]["cycles"]


def test_gmres_batched_zero_rhs_warm_start_budget(ctx):
    """b = 0 gives x = 0 and OK; a warm start x0 = the solution converges at once; a
    budget of 30 steps leaves the slow instances NOT_CONVERGED after exactly 30."""
    torch = torch_cuda()
    cases = CASES[:4]
    descs, bs, rs = _setup(cases, zero=(1,))
    x = torch.full((sum(b.size for b in bs),), 3.0, dtype=torch.float64, device="cuda")
    rc, infos = ctx.gmres_batched(descs, rs, dev_vector(np.concatenate(bs)), x, rtol=1e-8)
    assert rc == binding.OK
    xs = _split(host(x), cases)
    assert np.all(xs[1] == 0.0) and infos[1]["iters"] == 0 and infos[1]["status"] == binding.OK
    # warm start from the converged iterate
    rc, infos2 = ctx.gmres_batched(descs, rs, dev_vector(np.concatenate(bs)), x, rtol=1e-8)
    assert rc == binding.OK and all(i["iters"] == 0 for i in infos2)
    x.zero_()
    rc, infos3 = ctx.gmres_batched(descs, rs, dev_vector(np.concatenate(bs)), x, rtol=1e-8,
                                   max_iters=30)
    assert rc == binding.NOT_CONVERGED
    for i, inf in enumerate(infos3):
        if i == 1:
            continue
        if infos[i]["iters"] > 30:
            assert inf["status"] == binding.NOT_CONVERGED and inf["iters"] == 30
        else:
            assert inf["status"] == binding.OK


def test_gmres_batched_forced_fallback(ctx):
    """tau = 1: every step takes the explicit norm, resolved per instance through the
    single-instance schedule; the iterations follow the oracle run with tau = 1."""
    torch = torch_cuda()
    cases = CASES[1:4]
    descs, bs, rs = _setup(cases)
    x = torch.zeros(sum(b.size for b in bs), dtype=torch.float64, device="cuda")
    ctx.set_tolerances(1.0, 1e-12)
    try:
        rc, infos = ctx.gmres_batched(descs, rs, dev_vector(np.concatenate(bs)), x, rtol=1e-8)
    finally:
        ctx.set_tolerances(1e-8, 1e-12)
    assert rc == binding.OK
    _check(infos, _split(host(x), cases), cases, bs, tau=1.0)
    for inf in infos:
        assert inf["stats"]["pyth_fallbacks"] >= inf["iters"] - inf["cycles"]
