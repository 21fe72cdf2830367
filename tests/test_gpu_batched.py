"""Batched Krylov-Schur (one launch per DCGS2 step over all instances) against the
oracle, against the single-instance path, and graph replay against eager launches.

The instances are 2-D convection-diffusion operators of different grid sizes and
velocities (the batched eigenvalue family), including a ragged odd-sized grid and a
tiny instance whose first cycle already converges while the others restart.
"""
import numpy as np
import pytest

from oracle import operators as ops
from oracle.krylov_schur import krylov_schur
from paper_2104_01253_amd import binding, synth
from tests._gpu import dev_vector, say, torch_cuda

pytestmark = pytest.mark.gpu

NEV, NCV, KEEP, TOL = 6, 30, 12, 1e-9

# (grid, velocity, start-vector seed): square and rectangular grids, an odd m = 527,
# a tiny m = 42 instance, and strongly non-normal ones (cell Peclet up to 0.48)
CASES = [((24, 24), (4.0, 6.0), 11), ((31, 17), (10.0, 3.0), 12), ((40, 40), (30.0, 30.0), 13),
         ((7, 6), (1.0, 2.0), 14), ((48, 20), (0.0, 20.0), 15)]


@pytest.fixture(scope="module")
def ctx():
    torch_cuda()
    c = binding.Context(0)
    yield c
    c.close()


def _batch(cases):
    import torch
    descs = [binding.stencil2d(g, 1.0, v) for g, v, _ in cases]
    v0s = [synth.normal_vector(g[0] * g[1], s) for g, _, s in cases]
    v0 = dev_vector(np.concatenate(v0s))
    torch.cuda.synchronize()
    return descs, v0s, v0


def _by_magnitude(ev):
    return ev[np.lexsort((ev.imag, ev.real, -np.abs(ev)))]


def _eigvec_condition(grid, vel):
    """kappa(D) of the diagonal similarity that symmetrises the operator: per axis
    |a/c|^((n-1)/2) with a, c the neighbour coefficients (closed-form case)."""
    k = 1.0
    for n, v in zip(grid, vel):
        h = 1.0 / (n + 1)
        a, c = -1.0 / h**2 - v / (2 * h), -1.0 / h**2 + v / (2 * h)
        k *= abs(a / c) ** ((n - 1) / 2.0)
    return k


def _sigma_min(A, theta, iters=12):
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    M = (A.astype(complex) - theta * sp.identity(A.shape[0], dtype=complex, format="csr")).tocsc()
    lu = spla.splu(M)
    x = np.random.default_rng(0).standard_normal(A.shape[0]).astype(complex)
    s = 0.0
    for _ in range(iters):
        x /= np.linalg.norm(x)
        y = lu.solve(lu.solve(x), trans="H")
        s = np.linalg.norm(y)
        x = y
    return 1.0 / np.sqrt(s)


@pytest.mark.parametrize("host_dense", [1, 0])
def test_batched_ks_vs_oracle(ctx, host_dense):
    """Each instance converges (backward error of the partial Schur form <= tol),
    each Ritz value is an eigenvalue of a nearby matrix (sigma_min check), lies
    within kappa(V) * tol * |theta_1| of the closed-form spectrum (Bauer-Fike), and
    the restart count is close to the oracle's -- with the restart's dense work on
    host threads and on the GPU."""
    descs, v0s, v0 = _batch(CASES)
    ctx.set_tuning(binding.TUNE_BATCH_DENSE, host_dense)
    try:
        ev, rc, infos = ctx.krylov_schur_batched(descs, v0, NEV, NCV, KEEP, TOL, 200)
    finally:
        ctx.set_tuning(binding.TUNE_BATCH_DENSE, 1)
    say("batched rc", rc, [(i["status"], i["restarts"], i["resid"]) for i in infos])
    assert rc == binding.OK
    for b, (g, v, _) in enumerate(CASES):
        A = ops.convection_diffusion(g, 1.0, v)
        ref, io = krylov_schur(A, v0s[b], nev=NEV, ncv=NCV, keep=KEEP, tol=TOL)
        say("instance", b, g, v, "restarts gpu", infos[b]["restarts"], "oracle", io["restarts"])
        assert infos[b]["status"] == binding.OK and infos[b]["resid"] <= TOL
        assert abs(infos[b]["restarts"] - io["restarts"]) <= max(3, io["restarts"] // 4)
        got = _by_magnitude(ev[b])
        for th in got:
            assert _sigma_min(A, th) <= 1e-7 * abs(th), (b, th)
        exact = ops.closed_form_eigenvalues(g, 1.0, v)[::-1][:NEV + 2]
        bound = 2.0 * _eigvec_condition(g, v) * TOL * abs(exact[0]) + 1e-12 * abs(exact[0])
        for th in got:
            assert np.min(np.abs(exact - th)) <= bound, (b, th, bound)
    assert len({i["restarts"] for i in infos}) > 1      # instances leave at different cycles


def test_batched_matches_single_instance_path(ctx):
    """Batched and single-instance solvers reduce in different workgroup shapes, so
    their Ritz values agree to the accuracy both guarantee: within
    2 kappa(V) tol |theta_1| of each other (Bauer-Fike on both), for the instances
    whose eigenvector condition keeps that bound meaningful."""
    descs, v0s, v0 = _batch(CASES[:3])
    ev, rc, infos = ctx.krylov_schur_batched(descs, v0, NEV, NCV, KEEP, TOL, 200)
    assert rc == binding.OK
    for b, (g, v, _) in enumerate(CASES[:3]):
        e1, rc1, i1 = ctx.krylov_schur(binding.stencil_op(g, 1.0, v), dev_vector(v0s[b]),
                                       nev=NEV, ncv=NCV, keep=KEEP, tol=TOL, max_restarts=200)
        assert rc1 == binding.OK and i1["resid"] <= TOL
        kappa = _eigvec_condition(g, v)
        if kappa < 1e6:
            bound = 4.0 * kappa * TOL * abs(e1[0]) + 1e-12 * abs(e1[0])
            diff = np.abs(_by_magnitude(ev[b])[:, None] - _by_magnitude(e1)[None, :]).min(axis=1)
            assert np.max(diff) <= bound, (b, diff, bound)
        assert abs(i1["restarts"] - infos[b]["restarts"]) <= max(3, i1["restarts"] // 4)


def test_batched_graph_replay_is_bitwise_eager(ctx):
    descs, _, v0 = _batch(CASES)
    eg, rcg, ig = ctx.krylov_schur_batched(descs, v0, NEV, NCV, KEEP, TOL, 200, use_graph=True)
    ee, rce, ie = ctx.krylov_schur_batched(descs, v0, NEV, NCV, KEEP, TOL, 200, use_graph=False)
    assert rcg == rce == binding.OK
    assert np.array_equal(eg, ee)
    for a, b in zip(ig, ie):
        assert a["restarts"] == b["restarts"] and a["resid"] == b["resid"]
        assert a["stats"]["reductions"] == b["stats"]["reductions"]


def test_batched_single_instance_and_budget(ctx):
    descs, _, v0 = _batch(CASES[2:3])
    ev, rc, infos = ctx.krylov_schur_batched(descs, v0, NEV, NCV, KEEP, TOL, 200)
    assert rc == binding.OK and infos[0]["status"] == binding.OK
    # a budget of one restart: the tiny instance (one restart) converges, the
    # 40 x 40 one (dozens) reports NOT_CONVERGED after exactly one restart
    descs, _, v0 = _batch(CASES[2:4])
    ev, rc, infos = ctx.krylov_schur_batched(descs, v0, NEV, NCV, KEEP, TOL, 1)
    say("budget 1", [(i["status"], i["restarts"]) for i in infos])
    assert rc == binding.NOT_CONVERGED
    assert infos[0]["status"] == binding.NOT_CONVERGED and infos[0]["restarts"] == 1
    assert infos[1]["status"] == binding.OK and infos[1]["restarts"] <= 1


def test_batched_dense_work_gpu_matches_host(ctx):
    """The restart's dense work (Schur form, reordering, residual test, truncated H)
    on the GPU, one wavefront per instance, against the same algorithms on host
    threads: both converge, with Ritz values within 2 kappa(V) tol |theta_1| of each
    other and restart counts as close as between the batched and single-instance
    paths."""
    descs, _, v0 = _batch(CASES)
    ctx.set_tuning(binding.TUNE_BATCH_DENSE, 1)
    try:
        eh, rch, ih = ctx.krylov_schur_batched(descs, v0, NEV, NCV, KEEP, TOL, 200)
    finally:
        ctx.set_tuning(binding.TUNE_BATCH_DENSE, 0)
    try:
        eg, rcg, ig = ctx.krylov_schur_batched(descs, v0, NEV, NCV, KEEP, TOL, 200)
    finally:
        ctx.set_tuning(binding.TUNE_BATCH_DENSE, 1)
    say("host", [(i["status"], i["restarts"]) for i in ih], "gpu",
        [(i["status"], i["restarts"]) for i in ig])
    assert rch == rcg == binding.OK
    for b, (g, v, _) in enumerate(CASES):
        assert ig[b]["status"] == binding.OK and ig[b]["resid"] <= TOL
        # the paths round differently (fused multiply-adds on the GPU), which can
        # move an instance's convergence by a few restarts, as between the batched
        # and single-instance solvers
        assert abs(ig[b]["restarts"] - ih[b]["restarts"]) <= max(3, ih[b]["restarts"] // 4)
        kappa = _eigvec_condition(g, v)
        if kappa < 1e6:
            bound = 2.0 * kappa * TOL * abs(eh[b][0]) + 1e-12 * abs(eh[b][0])
            diff = np.abs(_by_magnitude(eg[b])[:, None] - _by_magnitude(eh[b])[None, :]).min(axis=1)
            assert np.max(diff) <= bound, (b, diff, bound)


def test_batched_every_tuned_reduce_shape(ctx):
    """Rows per reduction workgroup change only the partial-sum grouping (1 to 32
    workgroups per instance), so every value the autotuner can choose converges to
    Ritz values within 2 kappa(V) tol |theta_1| of the default's.  Two instances
    are large enough (m = 12,288 and 27,150) that their workgroup count changes
    with the setting, up to the 32-workgroup cap."""
    from paper_2104_01253_amd import autotune
    cases = CASES[:2] + [((128, 96), (5.0, 8.0), 16), ((181, 150), (12.0, 2.0), 17)]
    descs, _, v0 = _batch(cases)
    key = binding.TUNE_BATCH_REDUCE_ROWS
    default = ctx.get_tuning(key)
    ref, rc0, i0 = ctx.krylov_schur_batched(descs, v0, NEV, NCV, KEEP, TOL, 300)
    assert rc0 == binding.OK
    try:
        for rows in autotune.BATCHED_CANDIDATES[key] + (512,):
            ctx.set_tuning(key, rows)
            ev, rc, infos = ctx.krylov_schur_batched(descs, v0, NEV, NCV, KEEP, TOL, 300)
            say("rows", rows, [(i["status"], i["restarts"]) for i in infos])
            assert rc == binding.OK
            for b, (g, v, _) in enumerate(cases):
                assert infos[b]["status"] == binding.OK and infos[b]["resid"] <= TOL
                assert abs(infos[b]["restarts"] - i0[b]["restarts"]) <= max(3, i0[b]["restarts"] // 4)
                kappa = _eigvec_condition(g, v)
                if kappa < 1e6:
                    bound = 2.0 * kappa * TOL * abs(ref[b][0]) + 1e-12 * abs(ref[b][0])
                    diff = np.abs(_by_magnitude(ev[b])[:, None]
                                  - _by_magnitude(ref[b])[None, :]).min(axis=1)
                    assert np.max(diff) <= bound, (rows, b, diff, bound)
    finally:
        ctx.set_tuning(key, default)


def test_batched_ks_forced_fallback_vs_oracle(ctx):
    """tau = 1 forces the explicit-norm fallback at every DCGS2 step of every cycle:
    the batched solver resolves each through the single-instance schedule and
    converges like the oracle run with the same reading (restart counts, Ritz values
    within the Bauer-Fike bound), with one fallback per expansion step."""
    cases = CASES[:2] + CASES[3:4]
    descs, v0s, v0 = _batch(cases)
    ctx.set_tolerances(1.0, 1e-12)
    try:
        ev, rc, infos = ctx.krylov_schur_batched(descs, v0, NEV, NCV, KEEP, TOL, 200)
    finally:
        ctx.set_tolerances(1e-8, 1e-12)
    say("forced fallback", [(i["status"], i["restarts"], i["stats"]["pyth_fallbacks"])
                            for i in infos])
    assert rc == binding.OK
    for b, (g, v, _) in enumerate(cases):
        A = ops.convection_diffusion(g, 1.0, v)
        ref, io = krylov_schur(A, v0s[b], nev=NEV, ncv=NCV, keep=KEEP, tol=TOL, tau=1.0)
        assert infos[b]["status"] == binding.OK and infos[b]["resid"] <= TOL
        assert abs(infos[b]["restarts"] - io["restarts"]) <= max(3, io["restarts"] // 4)
        # every step but the continuation step of a restart takes the fallback
        steps = infos[b]["matvecs"]
        assert infos[b]["stats"]["pyth_fallbacks"] == steps - infos[b]["restarts"]
        exact = ops.closed_form_eigenvalues(g, 1.0, v)[::-1][:NEV + 2]
        bound = 2.0 * _eigvec_condition(g, v) * TOL * abs(exact[0]) + 1e-12 * abs(exact[0])
        for th in _by_magnitude(ev[b]):
            assert np.min(np.abs(exact - th)) <= bound, (b, th, bound)
