"""Per-step GPU parity: one identical state is given to the GPU (through
dcgs2_arnoldi_steps / dcgs2_qr_steps) and to the oracle's step (Alg. arnoldi,
Alg. qr), and every quantity of the step is compared with its natural scale:

  reduction   C = Q^T w (scale ||w||), beta (beta), S = Q^T v (||v||),
              sigma (||w|| ||v||), gamma (gamma)
  finalise    alpha (||w||), T or the S column (||v||/alpha, times ||w||/alpha
              for the last entry), the next breakdown scale (itself)
  update      q_{j-1} element-wise ((||w|| + ||C||)/alpha), w_j element-wise
              (||v||/alpha + ||T|| for Arnoldi, ||a|| + ||S|| for QR)
  H, K, R     each new column element-wise against its own norm.

The bound is 1e-12 everywhere (the GPU's fixed-order tree sums and the oracle's
BLAS dots differ by O(eps log m)).  Two (Arnoldi) or three (QR) consecutive steps
run on the GPU; each later step starts from the GPU's own state, the oracle's from
its own, which differ by rounding only.  With the one-pass QR schedule the update of
a step and the reduction of the next are one pass of the fused kernel, and the
second fused pass does the first one's finishing work, so every kernel of that
schedule is checked from the given state.
"""
import copy

import numpy as np
import pytest

from oracle import arnoldi as ar
from oracle import gram_schmidt as gs
from oracle import operators as ops
from paper_2104_01253_amd import binding, synth
from tests._gpu import colerr, dev_matrix, dev_vector, host, maxerr, say, torch_cuda

pytestmark = pytest.mark.gpu
TOL = 1e-12
M_BIG = 2 ** 20 + 3


@pytest.fixture(scope="module")
def ctx():
    torch_cuda()
    c = binding.Context(0)
    yield c
    c.close()


def cases(jmax_of_m):
    out = []
    for m in (63, 64, 65, 1000, M_BIG):
        for j in (2, 3, 4, 17, 64, 101):
            if j + 1 <= jmax_of_m(m):
                out.append((m, j))
    return out


def split_record(r, j):
    """GPU step record of step j: reduced values, coefficients, alpha, next scale."""
    J = j - 2
    return dict(C=r[:J], beta=r[J], sigma_x=r[J + 1], S=r[J + 2:2 * J + 2], sigma=r[2 * J + 2],
                gamma=r[2 * J + 3], T=r[2 * J + 4:3 * J + 5], alpha=r[3 * J + 5],
                rho_next=r[3 * J + 6])


def check_reduction(tag, g, C, beta, S, sigma, gamma):
    nw, nv = np.sqrt(beta), np.sqrt(gamma)
    errs = dict(C=maxerr(g["C"], C, nw), beta=abs(g["beta"] - beta) / beta,
                S=maxerr(g["S"], S, nv), sigma=abs(g["sigma"] - sigma) / (nw * nv),
                sigma_x=abs(g["sigma_x"] - sigma) / (nw * nv), gamma=abs(g["gamma"] - gamma) / gamma)
    say(tag, {k: f"{v:.1e}" for k, v in errs.items()})
    for k, v in errs.items():
        assert v <= TOL, (tag, k, v)


# ---------------------------------------------------------------- Arnoldi --------
def arnoldi_state(m, j0):
    """The oracle's expansion after step j0 - 1 on a 1-D convection-diffusion operator
    of m rows (the 5-point stencil with one grid row): Q, w, H, K and rho."""
    grid = (m, 1)
    A = ops.convection_diffusion(grid, 1.0, (20.0, 0.0))
    r0 = synth.normal_vector(m, 40 + j0)
    a = ar.DCGS2Arnoldi(lambda x: A @ x, r0, j0 + 1)
    while a.j < j0:
        assert a.step() == ar.OK
    return A, grid, a


@pytest.mark.parametrize("m,j0", cases(lambda m: m))
def test_arnoldi_two_steps_from_oracle_state(ctx, m, j0):
    A, grid, a = arnoldi_state(m, j0)
    j1 = j0 + 1
    say(f"arnoldi steps m={m} j={j0}..{j1}")
    Q = binding.colmajor_empty(m, j1 - 1)
    Q[:, :j0 - 2].copy_(torch_cuda().from_numpy(np.asfortranarray(a.Q[:, :j0 - 2])))
    w = dev_vector(a.w)
    ld = j1 + 2                                    # a leading dimension beyond j1
    H = np.zeros((ld, j1 - 1), order="F")
    K = np.zeros((ld, j1 - 1), order="F")
    H[:j1, :j0 - 3 if j0 >= 3 else 0] = a.H[:j1, :max(j0 - 3, 0)]
    K[:j1, :j0 - 2] = a.K[:j1, :j0 - 2]
    H[ld - 1, :] = 7.0                             # outside every step's rows: unchanged
    rho = a.rho_next if j0 >= 3 else 0.0
    rec, rc, st = ctx.arnoldi_steps(binding.stencil_op(grid, 1.0, (20.0, 0.0)), j0, j1, Q, w,
                                    H, K, rho)
    assert rc == binding.OK and st["reductions"] == 2 and st["pyth_fallbacks"] == 0
    ref = copy.deepcopy(a)
    ref.trace = []
    assert ref.step() == ar.OK and ref.step() == ar.OK
    Qg = host(Q)
    for r, t in zip(rec, ref.trace):
        j = t["j"]
        J = j - 2
        g = split_record(r, j)
        check_reduction(f"  step {j}", g, t["C"], t["beta"], t["S"], t["sigma"], t["gamma"])
        nw, nv, al = np.sqrt(t["beta"]), np.sqrt(t["gamma"]), t["alpha"]
        assert abs(g["alpha"] - al) / nw <= TOL
        assert maxerr(g["T"][:J], t["T"][:J], nv / al) <= TOL
        assert abs(g["T"][J] - t["T"][J]) / (nv / al * nw / al) <= TOL
        assert abs(g["rho_next"] - t["rho_next"]) / t["rho_next"] <= TOL
        # q_{j-1}
        scale_q = (nw + np.linalg.norm(t["C"])) / al
        assert maxerr(Qg[:, J], ref.Q[:, J], scale_q) <= TOL, j
        # H column j-2 (completed at step j) and K column j-1
        if j >= 3:
            assert colerr(H[:J + 1, J - 1], ref.H[:J + 1, J - 1]) <= TOL
        scale_k = np.linalg.norm(t["T"]) + np.linalg.norm(ref.H[:J + 1, :J]) * \
            np.linalg.norm(t["C"]) / al
        assert maxerr(K[:J + 1, J], ref.K[:J + 1, J], scale_k) <= TOL
    t = ref.trace[-1]
    scale_w = np.sqrt(t["gamma"]) / t["alpha"] + np.linalg.norm(t["T"])
    assert maxerr(host(w), ref.w, scale_w) <= TOL
    assert np.all(H[ld - 1, :] == 7.0)
    assert colerr(H[:j1, :j0 - 1], ref.H[:j1, :j0 - 1]) <= TOL


def test_arnoldi_steps_fallback_and_breakdown(ctx):
    """The explicit-norm fallback inside a step (tau = 1) and a breakdown step from a
    given state: the same status, counts and record as the oracle's step."""
    m, j0 = 1000, 17
    A, grid, a = arnoldi_state(m, j0)
    op = binding.stencil_op(grid, 1.0, (20.0, 0.0))
    Q = binding.colmajor_empty(m, j0)
    Q[:, :j0 - 2].copy_(torch_cuda().from_numpy(np.asfortranarray(a.Q[:, :j0 - 2])))
    w = dev_vector(a.w)
    H = np.asfortranarray(a.H[:j0 + 1, :j0].copy())
    K = np.asfortranarray(a.K[:j0 + 1, :j0].copy())
    ctx.set_tolerances(1.0, 1e-12)
    try:
        rec, rc, st = ctx.arnoldi_steps(op, j0, j0 + 1, Q, w, H, K, a.rho_next)
    finally:
        ctx.set_tolerances(1e-8, 1e-12)
    ref = copy.deepcopy(a)
    ref.tau = 1.0
    ref.trace = []
    assert ref.step() == ar.OK and ref.step() == ar.OK
    assert rc == binding.OK and st["pyth_fallbacks"] == 2 and st["reductions"] == 4
    for r, t in zip(rec, ref.trace):
        g = split_record(r, t["j"])
        assert t["fallback"]
        assert abs(g["alpha"] - t["alpha"]) / np.sqrt(t["beta"]) <= TOL
    assert maxerr(host(w), ref.w, np.linalg.norm(ref.w)) <= TOL
    # breakdown: eta so large that alpha_{j-1} <= eta rho
    w2 = dev_vector(a.w)
    H2 = np.asfortranarray(a.H[:j0 + 1, :j0].copy())
    K2 = np.asfortranarray(a.K[:j0 + 1, :j0].copy())
    ctx.set_tolerances(1e-8, 0.999)
    try:
        rec, rc, st = ctx.arnoldi_steps(op, j0, j0 + 1, Q, w2, H2, K2, a.rho_next)
    finally:
        ctx.set_tolerances(1e-8, 1e-12)
    ref = copy.deepcopy(a)
    ref.eta = 0.999
    assert ref.step() == ar.BREAKDOWN
    assert rc == binding.BREAKDOWN and st["breakdown_step"] == ref.k == j0 - 2
    assert colerr(H2[:j0 - 1, j0 - 3], ref.H[:j0 - 1, j0 - 3]) <= TOL
    assert np.all(np.isnan(rec[1]))                # the second step did not run


# ---------------------------------------------------------------- QR -------------
def qr_state(m, j0, j1):
    """The oracle's Alg. qr after step j0 - 1 on B (m x j1, kappa ~ 1e4)."""
    B = synth.tall_skinny(m, j1, 4.0, seed_g=60 + j0, seed_v=61)
    Q = np.zeros((m, j1), order="F")
    w = B[:, 0].copy()
    S_prev = np.zeros(0)
    gamma_prev = None
    R = np.zeros((j1, j1))
    for j in range(2, j0):
        rho = None if j == 2 else np.sqrt(gamma_prev)
        o = gs.dcgs2_qr_step(Q, j - 2, w, B[:, j - 1], S_prev, rho)
        assert o["status"] == gs.OK
        R[:j - 1, j - 2] = o["rcol"]
        w, S_prev, gamma_prev = o["w"], o["s_full"], o["gamma"]
    rho = np.sqrt(gamma_prev) if j0 >= 3 else 0.0
    return B, Q, w, S_prev, rho, R


@pytest.mark.parametrize("one_pass", [True, False])
@pytest.mark.parametrize("m,j0", cases(lambda m: min(m, binding.MAX_N) - 1))
def test_qr_three_steps_from_oracle_state(ctx, m, j0, one_pass):
    """Steps j0, j0+1, j0+2: with the one-pass schedule the first fused pass leaves its
    finishing work to the second, which folds it (and the third step's update is a
    plain pass)."""
    j1 = j0 + 2
    B, Qs, w0, S_prev, rho, _ = qr_state(m, j0, j1)
    say(f"qr steps m={m} j={j0}..{j1} one_pass={one_pass}")
    torch = torch_cuda()
    Bd = dev_matrix(B)
    Q = binding.colmajor_empty(m, j1 - 1)
    Q[:, :j0 - 2].copy_(torch.from_numpy(np.asfortranarray(Qs[:, :j0 - 2])))
    w = dev_vector(w0)
    R = np.full((j1 - 1, j1 - 1), 5.0, order="F")   # columns before j0-1 stay 5.0
    S = np.zeros(j1 - 1)
    S[:j0 - 2] = S_prev
    ctx.set_qr_schedule(one_pass)
    try:
        rec, rc, st = ctx.qr_steps(Bd, j0, j1, Q, w, R, S, rho)
    finally:
        ctx.set_qr_schedule(True)
    assert rc == binding.OK and st["reductions"] == 3
    # the oracle's steps from the same state
    Qo = Qs.copy(order="F")
    wo, So, rhoo = w0, S_prev, (None if j0 == 2 else rho)
    Qg = host(Q)
    for r, j in zip(rec, range(j0, j1 + 1)):
        J = j - 2
        a = B[:, j - 1]
        o = gs.dcgs2_qr_step(Qo, J, wo, a, So, rhoo)
        assert o["status"] == gs.OK
        g = split_record(r, j)
        check_reduction(f"  step {j}", g, o["C"], o["beta"], o["S"], o["sigma"], o["gamma"])
        nw, na, al = np.sqrt(o["beta"]), np.sqrt(o["gamma"]), o["alpha"]
        assert abs(g["alpha"] - al) / nw <= TOL
        assert maxerr(g["T"][:J], o["s_full"][:J], na) <= TOL
        assert abs(g["T"][J] - o["s_full"][J]) / (na * max(1.0, nw / al)) <= TOL
        assert abs(g["rho_next"] - na) / na <= TOL
        assert maxerr(Qg[:, J], Qo[:, J], (nw + np.linalg.norm(o["C"])) / al) <= TOL
        assert colerr(R[:J + 1, J], o["rcol"]) <= TOL
        wo, So, rhoo = o["w"], o["s_full"], na
    assert maxerr(host(w), wo, na + np.linalg.norm(So)) <= TOL
    assert maxerr(S, So, np.linalg.norm(So)) <= TOL
    assert np.all(R[:, :j0 - 2] == 5.0)


@pytest.mark.parametrize("one_pass", [True, False])
def test_qr_steps_fallback(ctx, one_pass):
    """tau = 1: both steps take the explicit norm; the host resumes the schedule after
    each (a step whose guard fails never reaches the fused pass)."""
    m, j0 = 20011, 9
    j1 = j0 + 1
    B, Qs, w0, S_prev, rho, _ = qr_state(m, j0, j1)
    Bd = dev_matrix(B)
    Q = binding.colmajor_empty(m, j1 - 1)
    Q[:, :j0 - 2].copy_(torch_cuda().from_numpy(np.asfortranarray(Qs[:, :j0 - 2])))
    w = dev_vector(w0)
    R = np.zeros((j1 - 1, j1 - 1), order="F")
    S = np.zeros(j1 - 1)
    S[:j0 - 2] = S_prev
    ctx.set_tolerances(1.0, 1e-12)
    ctx.set_qr_schedule(one_pass)
    try:
        rec, rc, st = ctx.qr_steps(Bd, j0, j1, Q, w, R, S, rho)
    finally:
        ctx.set_tolerances(1e-8, 1e-12)
        ctx.set_qr_schedule(True)
    assert rc == binding.OK and st["pyth_fallbacks"] == 2 and st["reductions"] == 4
    Qo = Qs.copy(order="F")
    wo, So, rhoo = w0, S_prev, rho
    for r, j in zip(rec, (j0, j1)):
        o = gs.dcgs2_qr_step(Qo, j - 2, wo, B[:, j - 1], So, rhoo, tau=1.0)
        assert o["fallback"]
        g = split_record(r, j)
        assert abs(g["alpha"] - o["alpha"]) / np.sqrt(o["beta"]) <= TOL
        assert colerr(R[:j - 1, j - 2], o["rcol"]) <= TOL
        wo, So, rhoo = o["w"], o["s_full"], np.sqrt(o["gamma"])
    assert maxerr(host(w), wo, np.linalg.norm(wo) + np.linalg.norm(So)) <= TOL
