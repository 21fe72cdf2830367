"""Batched DCGS2 Arnoldi (one launch per step over all instances, the expansion
cycle of the batched Krylov-Schur solver) against the oracle, instance by instance.

Instances differ in grid size (m = 42 .. 65,536, odd and even) and in step count
(n = 1 .. 60), so some stop while others continue, and each finishes its last
column over its own n columns.  H and Q are compared element-wise with the
oracle's DCGS2Arnoldi (each element against the norm of its reference column) at
1e-12, with the reduction count n + 2; the forced explicit-norm fallback (tau = 1)
and a breakdown instance follow the oracle's readings.
"""
import numpy as np
import pytest

from oracle import arnoldi as ar
from oracle import operators as ops
from oracle.metrics import loss_of_orthogonality, representation_error
from paper_2104_01253_amd import binding, synth
from tests._gpu import colerr, dev_vector, host, say, torch_cuda

pytestmark = pytest.mark.gpu
TOL = 1e-12

# (grid, velocity, steps, seed): the largest grid of the batched family (256^2) at
# the Krylov-Schur basis size, ragged and tiny instances, one-step and two-step ones
CASES = [((256, 256), (30.0, 20.0), 60, 21), ((31, 17), (10.0, 3.0), 17, 22),
         ((48, 48), (5.0, 45.0), 33, 23), ((7, 6), (1.0, 2.0), 5, 24),
         ((100, 3), (0.0, 20.0), 1, 25), ((63, 65), (12.0, 0.0), 60, 26),
         ((9, 11), (3.0, 3.0), 2, 27)]


@pytest.fixture(scope="module")
def ctx():
    torch_cuda()
    c = binding.Context(0)
    yield c
    c.close()


def _run(ctx, cases, r0s=None):
    descs = [binding.stencil2d(g, 1.0, v) for g, v, _, _ in cases]
    n = [k for _, _, k, _ in cases]
    if r0s is None:
        r0s = [synth.normal_vector(g[0] * g[1], s) for g, _, _, s in cases]
    bases, Hs, rc, stat, sts = ctx.arnoldi_batched(descs, n, dev_vector(np.concatenate(r0s)))
    return r0s, bases, Hs, rc, stat, sts


def test_arnoldi_batched_parity(ctx):
    r0s, bases, Hs, rc, stat, sts = _run(ctx, CASES)
    assert rc == binding.OK and np.all(stat == binding.OK)
    for b, (g, v, n, _) in enumerate(CASES):
        A = ops.convection_diffusion(g, 1.0, v)
        ref = ar.dcgs2_arnoldi(lambda x: A @ x, r0s[b], n)
        Q = host(bases[b])
        dh, dq = colerr(Hs[b], ref["H"]), colerr(Q, ref["Q"])
        say("instance", b, g, "n", n, "H colerr", dh, "Q colerr", dq)
        assert dh <= TOL and dq <= TOL
        assert sts[b]["reductions"] == ref["reductions"] == n + 2
        assert sts[b]["pyth_fallbacks"] == 0
        assert loss_of_orthogonality(Q) <= 1e-13
        assert representation_error(A, Q, Hs[b], n) <= 1e-15


def test_arnoldi_batched_forced_fallback(ctx):
    """tau = 1: every step of every instance takes the explicit norm; the batched
    launches stop each instance at its guard and the single-instance schedule
    finishes it on the instance's own buffers, as the oracle reads Sec. 3."""
    cases = CASES[1:5]
    ctx.set_tolerances(1.0, 1e-12)
    try:
        r0s, bases, Hs, rc, stat, sts = _run(ctx, cases)
    finally:
        ctx.set_tolerances(1e-8, 1e-12)
    assert rc == binding.OK
    for b, (g, v, n, _) in enumerate(cases):
        A = ops.convection_diffusion(g, 1.0, v)
        ref = ar.dcgs2_arnoldi(lambda x: A @ x, r0s[b], n, tau=1.0)
        assert sts[b]["pyth_fallbacks"] == ref["fallbacks"] == n
        assert sts[b]["reductions"] == ref["reductions"]
        assert colerr(Hs[b], ref["H"]) <= TOL and colerr(host(bases[b]), ref["Q"]) <= TOL


def test_arnoldi_batched_breakdown_instance(ctx):
    """One instance starts in a 3-dimensional invariant subspace (v = 0, three grid
    eigenvectors): it breaks down with k = 3 and exact Ritz values while the others
    run to their n."""
    nx, ny = 20, 14
    t = np.arange(1, nx + 1) / (nx + 1)
    s = np.arange(1, ny + 1) / (ny + 1)
    vec = lambda p, q: np.outer(np.sin(q * np.pi * s), np.sin(p * np.pi * t)).ravel()
    r0 = vec(1, 1) - 2.0 * vec(2, 3) + 0.5 * vec(5, 2)
    cases = [CASES[1], ((nx, ny), (0.0, 0.0), 10, 0), CASES[3]]
    r0s = [synth.normal_vector(31 * 17, 22), r0, synth.normal_vector(42, 24)]
    _, bases, Hs, rc, stat, sts = _run(ctx, cases, r0s)
    assert rc == binding.BREAKDOWN
    assert list(stat) == [binding.OK, binding.BREAKDOWN, binding.OK]
    A = ops.convection_diffusion((nx, ny), 1.0, (0.0, 0.0))
    ref = ar.dcgs2_arnoldi(lambda x: A @ x, r0, 10)
    assert ref["status"] == ar.BREAKDOWN and sts[1]["breakdown_step"] == ref["k"] == 3
    assert colerr(Hs[1][:4, :3], ref["H"][:4, :3]) <= TOL
    lam = np.sort(np.linalg.eigvals(Hs[1][:3, :3]).real)
    ev = ops.closed_form_eigenvalues((nx, ny), 1.0, (0.0, 0.0))
    for th in lam:
        assert np.min(np.abs(ev - th)) <= 1e-10 * ev[-1]
    for b in (0, 2):
        g, v, n, _ = cases[b]
        A = ops.convection_diffusion(g, 1.0, v)
        ref = ar.dcgs2_arnoldi(lambda x: A @ x, r0s[b], n)
        assert colerr(Hs[b], ref["H"]) <= TOL
