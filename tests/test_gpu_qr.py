"""GPU parity of dcgs2_qr (Alg. qr) against the FP64 oracle, through the C ABI.

Gate: 1e-12 on the quantities that are unique at the given conditioning -- R
element-wise against the norm of its own column (colerr), (Q - Q_oracle) R_oracle /
||B|| normwise, and raw Q element-wise where kappa(B) is small (raw Q at kappa ~ 1e8
differs between any two correct implementations by ~ eps * kappa(B_{1:j}) in
column j).
"""
import numpy as np
import pytest

from oracle import gram_schmidt as gs
from oracle.metrics import loss_of_orthogonality, qr_error
from paper_2104_01253_amd import binding, synth
from tests._gpu import colerr, dev_matrix, host, say, torch_cuda

pytestmark = pytest.mark.gpu
TOL = 1e-12


@pytest.fixture(scope="module")
def ctx():
    torch_cuda()
    c = binding.Context(0)
    yield c
    c.close()


def run_qr(ctx, B, ld=None):
    Bd = dev_matrix(B, ld)
    Qd = binding.colmajor_empty(B.shape[0], B.shape[1], ld)
    R, rc, st = ctx.qr(Bd, Qd)
    return host(Qd), R, rc, st


@pytest.mark.parametrize("one_pass", [True, False])
# m = 1, 2, 63, 64 and 65: one partial tile of the one-pass kernel (64 rows with
# one-row slots, 128 with two-row slots), odd and even
@pytest.mark.parametrize("m,n,ce", [(1, 1, 2), (2, 2, 2), (63, 20, 2), (64, 17, 2), (65, 40, 2),
                                    (64, 64, 1), (1000, 1, 2), (1000, 2, 2), (1023, 3, 2),
                                    (4097, 17, 2), (4097, 17, 8), (20011, 64, 8), (3000, 100, 4),
                                    (130, 120, 2)])
def test_qr_parity_small(ctx, m, n, ce, one_pass):
    say(f"qr parity m={m} n={n} kappa=1e{ce} one_pass={one_pass}")
    B = synth.tall_skinny(m, n, ce, seed_g=100 + m, seed_v=7)
    ctx.set_qr_schedule(one_pass)
    try:
        Q, R, rc, st = run_qr(ctx, B)
    finally:
        ctx.set_qr_schedule(True)
    ref = gs.dcgs2_qr(B)
    assert rc == binding.OK and ref["status"] == 0
    assert colerr(R, ref["R"]) <= TOL
    assert np.linalg.norm((Q - ref["Q"]) @ ref["R"]) / np.linalg.norm(B) <= TOL
    if np.linalg.cond(B) <= 1e3:
        assert colerr(Q, ref["Q"]) <= TOL
    assert st["reductions"] == ref["reductions"] == (n + 1 if n > 1 else 1)
    assert loss_of_orthogonality(Q) <= 1e-13
    assert qr_error(B, Q, R) <= 1e-14


def test_qr_unaligned_leading_dimension(ctx):
    """Odd ldq/ldb: the one-row (8-byte) kernel path."""
    m, n = 5001, 12
    B = synth.tall_skinny(m, n, 3)
    Q, R, rc, _ = run_qr(ctx, B, ld=5003)
    ref = gs.dcgs2_qr(B)
    assert rc == 0
    assert colerr(R, ref["R"]) <= TOL
    assert colerr(Q, ref["Q"]) <= TOL


def test_qr_deterministic(ctx):
    B = synth.tall_skinny(300007, 30, 8)
    Q1, R1, _, _ = run_qr(ctx, B)
    Q2, R2, _, _ = run_qr(ctx, B)
    assert np.array_equal(Q1, Q2) and np.array_equal(R1, R2)


@pytest.mark.parametrize("one_pass", [True, False])
def test_qr_forced_fallback(ctx, one_pass):
    """tau = 1 forces the explicit-norm branch at every step (host-resumed)."""
    B = synth.tall_skinny(7000, 15, 4)
    ctx.set_tolerances(1.0, 1e-12)
    ctx.set_qr_schedule(one_pass)
    try:
        Q, R, rc, st = run_qr(ctx, B)
    finally:
        ctx.set_tolerances(1e-8, 1e-12)
        ctx.set_qr_schedule(True)
    ref = gs.dcgs2_qr(B, tau=1.0)
    assert rc == 0
    assert st["pyth_fallbacks"] == ref["fallbacks"] == 14
    assert st["reductions"] == ref["reductions"]
    assert colerr(R, ref["R"]) <= TOL
    assert colerr(Q, ref["Q"]) <= TOL


def test_qr_breakdown(ctx):
    B = synth.tall_skinny(2000, 8, 2)
    B[:, 3] = B[:, 0] - 2.0 * B[:, 2]
    Q, R, rc, st = run_qr(ctx, B)
    ref = gs.dcgs2_qr(B)
    assert rc == binding.BREAKDOWN and ref["status"] == gs.BREAKDOWN
    assert st["breakdown_step"] == ref["k"] == 3
    assert colerr(R[:3, :4], ref["R"][:3, :4]) <= TOL
    assert colerr(Q[:, :3], ref["Q"][:, :3]) <= TOL


def test_qr_nonfinite(ctx):
    B = synth.tall_skinny(500, 6, 2)
    B[17, 4] = np.nan
    _, _, rc, st = run_qr(ctx, B)
    assert rc == binding.NONFINITE
    assert st["breakdown_step"] == gs.dcgs2_qr(B)["k"] == 3


@pytest.fixture(scope="module")
def full_size():
    """The tall-skinny workload at full size (m = 2,000,000, n = 100, kappa ~ 1e8) and
    the oracle's factorisation of it, computed once for the tests below."""
    m, n = 2_000_000, 100
    say("generating B 2e6 x 100")
    B = synth.tall_skinny(m, n, 8.0)
    say("oracle qr")
    return B, gs.dcgs2_qr(B)


def test_qr_full_size_kappa_1e8(ctx, full_size):
    """Full size with the default launch shapes."""
    B, ref = full_size
    n = B.shape[1]
    say("gpu qr")
    Q, R, rc, st = run_qr(ctx, B)
    assert rc == 0 and st["reductions"] == n + 1
    assert colerr(R, ref["R"]) <= TOL
    dq = np.linalg.norm((Q - ref["Q"]) @ ref["R"]) / np.linalg.norm(B)
    say("dQ R", dq)
    assert dq <= TOL
    loo = loss_of_orthogonality(Q)
    say("loo", loo)
    assert loo <= 1e-13


def test_qr_full_size_kappa_1e2(ctx):
    """Full size on the well-conditioned matrix (singular values logspace(0, -2)):
    against the oracle, with the orthogonality DCGS2 reaches there (the oracle's
    own loss of orthogonality on this matrix is 1.9e-14, its representation error
    3.1e-16)."""
    m, n = 2_000_000, 100
    say("generating B 2e6 x 100, kappa ~ 1e2")
    B = synth.tall_skinny(m, n, 2.0)
    say("oracle qr")
    ref = gs.dcgs2_qr(B)
    say("gpu qr")
    Q, R, rc, st = run_qr(ctx, B)
    assert rc == 0 and st["reductions"] == n + 1
    assert colerr(R, ref["R"]) <= TOL
    dq = np.linalg.norm((Q - ref["Q"]) @ ref["R"]) / np.linalg.norm(B)
    loo = loss_of_orthogonality(Q)
    rre = np.linalg.norm(B - Q @ R) / np.linalg.norm(B)
    say("dQ R", dq, "loo", loo, "rre", rre)
    assert dq <= TOL and loo <= 1e-13 and rre <= 1e-15


def test_qr_full_size_every_tuned_shape(ctx, full_size):
    """Full size under every launch-shape combination the autotuner can choose, so
    the configuration the benchmark times is among those checked."""
    from paper_2104_01253_amd import autotune
    import itertools
    B, ref = full_size
    n = B.shape[1]
    Bd = dev_matrix(B)
    Qd = binding.colmajor_empty(B.shape[0], n)
    keys = list(autotune.CANDIDATES)
    try:
        for combo in itertools.product(*(autotune.CANDIDATES[k] for k in keys)):
            for k, v in zip(keys, combo):
                ctx.set_tuning(k, v)
            R, rc, st = ctx.qr(Bd, Qd)
            Q = host(Qd)
            dq = np.linalg.norm((Q - ref["Q"]) @ ref["R"]) / np.linalg.norm(B)
            say("shape", dict(zip(keys, combo)), "R colerr", colerr(R, ref["R"]), "dQ R", dq)
            assert rc == 0 and st["reductions"] == n + 1
            assert colerr(R, ref["R"]) <= TOL and dq <= TOL
    finally:
        for k in keys:
            ctx.set_tuning(k, {binding.TUNE_FUSED_PAIR_SLOTS: 16}.get(k, 0))


@pytest.mark.parametrize("m,n,ce", [(4097, 17, 2), (20011, 64, 8)])
def test_cgs2_comparator_parity(ctx, m, n, ce):
    """The CGS2 comparator against the oracle's Alg. cgs2 (three reductions per column)."""
    B = synth.tall_skinny(m, n, ce, seed_g=300 + m, seed_v=5)
    Bd = dev_matrix(B)
    Qd = binding.colmajor_empty(m, n)
    R, rc, st = ctx.cgs2_qr(Bd, Qd)
    Qr, Rr, red = gs.cgs2_qr(B)
    assert rc == 0 and st["reductions"] == red == 3 * (n - 1) + 1
    assert colerr(R, Rr) <= TOL
    assert np.linalg.norm((host(Qd) - Qr) @ Rr) / np.linalg.norm(B) <= TOL
    assert loss_of_orthogonality(host(Qd)) <= 1e-13


@pytest.mark.parametrize("m,n,ce", [(4097, 17, 2), (20011, 40, 2), (3001, 12, 6)])
def test_mgs_comparator_parity(ctx, m, n, ce):
    """The MGS comparator against the oracle's MGS: n(n+1)/2 reductions; R and Q to
    1e-12 at kappa ~ 1e2; at kappa ~ 1e6 both lose orthogonality at the MGS rate
    O(eps kappa) (Tab. loss_of_orth) while R stays a backward-stable factor."""
    B = synth.tall_skinny(m, n, ce, seed_g=500 + m, seed_v=5)
    Bd = dev_matrix(B)
    Qd = binding.colmajor_empty(m, n)
    R, rc, st = ctx.mgs_qr(Bd, Qd)
    Qr, Rr, red = gs.mgs_qr(B)
    Q = host(Qd)
    assert rc == 0 and st["reductions"] == red == n * (n + 1) // 2
    assert colerr(R, Rr) <= (TOL if ce <= 2 else 1e-9)
    assert qr_error(B, Q, R) <= 1e-14
    if ce <= 2:
        assert colerr(Q, Qr) <= TOL
    else:
        lo_gpu, lo_ref = loss_of_orthogonality(Q), loss_of_orthogonality(Qr)
        say("mgs LOO gpu", lo_gpu, "oracle", lo_ref)
        assert 1e-13 < lo_gpu < 1e-6 and 0.1 < lo_gpu / lo_ref < 10


@pytest.mark.parametrize("min_j", [8, 200])
@pytest.mark.parametrize("m,n,ce", [(1000, 2, 2), (4097, 17, 8), (20011, 64, 8), (3000, 100, 4)])
def test_qr_hybrid_schedule_parity(ctx, m, n, ce, min_j):
    """One-pass schedule with the first min_j steps as separate update and
    reduction passes (min_j beyond n: every step separate); the forced-fallback
    path resumes inside the hybrid schedule too."""
    say(f"qr hybrid m={m} n={n} min_j={min_j}")
    B = synth.tall_skinny(m, n, ce, seed_g=300 + m, seed_v=9)
    ref = gs.dcgs2_qr(B)
    ctx.set_tuning(binding.TUNE_FUSED_MIN_J, min_j)
    try:
        Q, R, rc, st = run_qr(ctx, B)
        ctx.set_tolerances(1.0, 1e-12)
        Qf, Rf, rcf, stf = run_qr(ctx, B)
    finally:
        ctx.set_tolerances(1e-8, 1e-12)
        ctx.set_tuning(binding.TUNE_FUSED_MIN_J, 0)
    assert rc == 0 and st["reductions"] == ref["reductions"]
    assert colerr(R, ref["R"]) <= TOL
    assert np.linalg.norm((Q - ref["Q"]) @ ref["R"]) / np.linalg.norm(B) <= TOL
    reff = gs.dcgs2_qr(B, tau=1.0)
    assert rcf == 0 and stf["pyth_fallbacks"] == reff["fallbacks"]
    assert colerr(Rf, reff["R"]) <= TOL


@pytest.mark.parametrize("one_pass", [True, False])
@pytest.mark.parametrize("gmax,m,n", [(1, 20011, 40), (3, 20011, 40), (37, 4097, 17),
                                      (1024, 600000, 12)])
def test_qr_reduction_grid_parity(ctx, gmax, m, n, one_pass):
    """The fixed-order sum of the per-workgroup partials for grids of 1 to 1024
    workgroups (a single chunk, chunks of unequal length, more workgroups than
    threads per value): parity with the oracle, and the same result twice."""
    say(f"qr reduction grid gmax={gmax} m={m} n={n} one_pass={one_pass}")
    B = synth.tall_skinny(m, n, 6, seed_g=500 + gmax, seed_v=11)
    ref = gs.dcgs2_qr(B)
    ctx.set_tuning(binding.TUNE_REDUCE_GRID, gmax)
    ctx.set_qr_schedule(one_pass)
    try:
        Q, R, rc, st = run_qr(ctx, B)
        Q2, R2, _, _ = run_qr(ctx, B)
    finally:
        ctx.set_tuning(binding.TUNE_REDUCE_GRID, 0)
        ctx.set_qr_schedule(True)
    assert rc == 0 and st["reductions"] == ref["reductions"]
    assert colerr(R, ref["R"]) <= TOL
    assert np.linalg.norm((Q - ref["Q"]) @ ref["R"]) / np.linalg.norm(B) <= TOL
    assert np.array_equal(Q, Q2) and np.array_equal(R, R2)


@pytest.mark.parametrize("m,n", [(6000, 126), (6000, 127), (3001, 127), (6000, 128), (2600, 200)])
def test_qr_one_pass_size_limits(ctx, m, n):
    """Around the one-pass limit: n = 127 takes J up to 125, sixteen basis slots per
    wavefront (two-row slots for even m, one-row slots for odd m); n >= 128 runs the
    two-pass schedule."""
    say(f"qr size limits m={m} n={n}")
    B = synth.tall_skinny(m, n, 4, seed_g=700 + n, seed_v=13)
    ref = gs.dcgs2_qr(B)
    Q, R, rc, st = run_qr(ctx, B)
    assert rc == 0 and st["reductions"] == ref["reductions"] == n + 1
    assert colerr(R, ref["R"]) <= TOL
    assert np.linalg.norm((Q - ref["Q"]) @ ref["R"]) / np.linalg.norm(B) <= TOL
    assert loss_of_orthogonality(Q) <= 1e-13


@pytest.mark.parametrize("m,n", [(20011, 40), (20011, 100), (4097, 17)])
def test_qr_sixteen_wavefront_workgroups(ctx, m, n):
    """FUSED_WAVES = 16: 16-wavefront workgroups with one-row slots (at most eight basis
    slots per wavefront)."""
    B = synth.tall_skinny(m, n, 6, seed_g=800 + n, seed_v=17)
    ref = gs.dcgs2_qr(B)
    ctx.set_tuning(binding.TUNE_FUSED_WAVES, 16)
    try:
        Q, R, rc, st = run_qr(ctx, B)
    finally:
        ctx.set_tuning(binding.TUNE_FUSED_WAVES, 8)
    assert rc == 0 and st["reductions"] == ref["reductions"]
    assert colerr(R, ref["R"]) <= TOL
    assert np.linalg.norm((Q - ref["Q"]) @ ref["R"]) / np.linalg.norm(B) <= TOL


def test_qr_longest_basis(ctx):
    """n = DCGS2_MAX_N (1024 columns, two-pass schedule): the finishing kernel's LDS grows
    with the basis (about 90 KB at this n)."""
    m, n = 4000, binding.MAX_N
    say(f"qr longest basis m={m} n={n}")
    B = synth.tall_skinny(m, n, 4, seed_g=1100, seed_v=23)
    ref = gs.dcgs2_qr(B)
    Q, R, rc, st = run_qr(ctx, B)
    assert rc == 0 and st["reductions"] == ref["reductions"] == n + 1
    assert colerr(R, ref["R"]) <= TOL
    assert np.linalg.norm((Q - ref["Q"]) @ ref["R"]) / np.linalg.norm(B) <= TOL
    assert loss_of_orthogonality(Q) <= 1e-13


@pytest.mark.parametrize("m", [20012, 4096])
def test_qr_last_slot_past_the_basis(ctx, m):
    """n = 100 (FP64, two-row slots): for J not a multiple of eight a wavefront's last slot
    lies past the basis and must contribute exactly zero; wavefronts 0, 1 and 2 form the
    products of q, w' and a_{j+1}; J = 89..97 hold twelve and thirteen slots."""
    B = synth.tall_skinny(m, 100, 6, seed_g=1200 + m, seed_v=29)
    ref = gs.dcgs2_qr(B)
    Q, R, rc, st = run_qr(ctx, B)
    assert rc == 0 and st["reductions"] == ref["reductions"]
    assert colerr(R, ref["R"]) <= TOL
    assert np.linalg.norm((Q - ref["Q"]) @ ref["R"]) / np.linalg.norm(B) <= TOL
    assert loss_of_orthogonality(Q) <= 1e-13
