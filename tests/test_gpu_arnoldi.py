"""GPU parity of dcgs2_arnoldi (Alg. arnoldi) and the matvec, through the C ABI.

Gate: H and Q element-wise against the oracle, each element against the norm of its
own column (colerr), at 1e-12; plus orthogonality and the Arnoldi relation."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import arnoldi as ar
from oracle import operators as ops
from oracle.metrics import loss_of_orthogonality, representation_error
from paper_2104_01253_amd import binding, synth
from tests._gpu import colerr, dev_vector, host, relnorm, say, torch_cuda

pytestmark = pytest.mark.gpu
TOL = 1e-12


@pytest.fixture(scope="module")
def ctx():
    torch_cuda()
    c = binding.Context(0)
    yield c
    c.close()


def run_arnoldi(ctx, op, r0, n, ld=None):
    Q = binding.colmajor_empty(op.m, n + 1, ld)
    H, rc, st = ctx.arnoldi(op, dev_vector(r0), n, Q)
    return host(Q), H, rc, st


@pytest.mark.parametrize("grid,vel", [((32, 32), (10.0, 10.0)), ((31, 29), (3.0, 40.0)),
                                      ((7, 5, 3), (1.0, 2.0, 3.0)), ((40, 33, 17), (10., 10., 10.)),
                                      ((1000, 1), (5.0, 0.0)), ((1, 1000), (0.0, 5.0)),
                                      ((1, 1, 50), (0.0, 0.0, 2.0)), ((3, 1, 7), (1.0, 0.0, 4.0)),
                                      ((129, 65, 9), (7.0, 3.0, 1.0)),
                                      ((128, 128, 128), (10.0, 10.0, 10.0))])
def test_matvec_parity(ctx, grid, vel):
    torch = torch_cuda()
    A = ops.convection_diffusion(grid, 1.0, vel)
    op = binding.stencil_op(grid, 1.0, vel)
    x = synth.normal_vector(A.shape[0], 3)
    y = torch.empty(A.shape[0], dtype=torch.float64, device="cuda")
    ctx.apply(op, dev_vector(x), y)
    ref = A @ x
    assert np.max(np.abs(host(y) - ref)) <= 1e-13 * np.max(np.abs(A).sum(axis=1)) * np.max(np.abs(x))


def test_csr_matvec_parity(ctx):
    torch = torch_cuda()
    A = sp.random(3001, 3001, density=0.003, random_state=4, format="csr") + sp.eye(3001)
    A = A.tocsr()
    A.sort_indices()
    rp = torch.from_numpy(A.indptr.astype(np.int32)).cuda()
    ci = torch.from_numpy(A.indices.astype(np.int32)).cuda()
    va = torch.from_numpy(A.data.astype(np.float64)).cuda()
    op = binding.csr_op(rp, ci, va)
    x = synth.normal_vector(3001, 5)
    y = torch.empty(3001, dtype=torch.float64, device="cuda")
    ctx.apply(op, dev_vector(x), y)
    assert relnorm(host(y), A @ x) <= 1e-14


def test_config1_parity():
    """2-D convection-diffusion 32x32, v=(10,10), 50 steps, r0 ~ N(0,1) seed 0."""
    torch_cuda()
    prob, r0, n = synth.arnoldi_cd2d_32()
    A = ops.convection_diffusion(prob.grid, prob.D, prob.vel)
    with binding.Context(0) as c:
        Q, H, rc, st = run_arnoldi(c, binding.stencil_op(prob.grid, prob.D, prob.vel), r0, n)
    ref = ar.dcgs2_arnoldi(lambda x: A @ x, r0, n)
    assert rc == 0 and st["reductions"] == ref["reductions"] == n + 2
    say("H colerr", colerr(H, ref["H"]), "Q colerr", colerr(Q, ref["Q"]))
    assert colerr(H, ref["H"]) <= TOL
    assert colerr(Q, ref["Q"]) <= TOL
    assert loss_of_orthogonality(Q) <= 1e-13
    assert representation_error(A, Q, H, n) <= 1e-15


@pytest.mark.parametrize("grid,n", [((5, 4), 1), ((5, 4), 2), ((9, 7), 3), ((33, 31), 17),
                                    ((12, 11, 9), 40), ((64, 64, 3), 64)])
def test_arnoldi_parity_shapes(ctx, grid, n):
    vel = (10.0,) * len(grid)
    A = ops.convection_diffusion(grid, 1.0, vel)
    r0 = synth.normal_vector(A.shape[0], 11)
    Q, H, rc, st = run_arnoldi(ctx, binding.stencil_op(grid, 1.0, vel), r0, n)
    ref = ar.dcgs2_arnoldi(lambda x: A @ x, r0, n)
    assert rc == 0
    assert colerr(H, ref["H"]) <= TOL
    assert colerr(Q, ref["Q"]) <= TOL
    assert st["reductions"] == n + 2


def test_arnoldi_csr_operator_and_odd_ld(ctx):
    torch = torch_cuda()
    g = np.random.default_rng(8)
    A = (sp.random(2501, 2501, density=0.004, random_state=9, format="csr") + 4 * sp.eye(2501)).tocsr()
    rp = torch.from_numpy(A.indptr.astype(np.int32)).cuda()
    ci = torch.from_numpy(A.indices.astype(np.int32)).cuda()
    va = torch.from_numpy(A.data.astype(np.float64)).cuda()
    r0 = g.standard_normal(2501)
    Q, H, rc, _ = run_arnoldi(ctx, binding.csr_op(rp, ci, va), r0, 30, ld=2503)
    ref = ar.dcgs2_arnoldi(lambda x: A @ x, r0, 30)
    assert rc == 0
    assert colerr(H, ref["H"]) <= TOL and colerr(Q, ref["Q"]) <= TOL


def test_arnoldi_forced_fallback(ctx):
    prob, r0, _ = synth.arnoldi_cd2d_32()
    A = ops.convection_diffusion(prob.grid, prob.D, prob.vel)
    ctx.set_tolerances(1.0, 1e-12)
    try:
        Q, H, rc, st = run_arnoldi(ctx, binding.stencil_op(prob.grid, prob.D, prob.vel), r0, 20)
    finally:
        ctx.set_tolerances(1e-8, 1e-12)
    ref = ar.dcgs2_arnoldi(lambda x: A @ x, r0, 20, tau=1.0)
    assert rc == 0 and st["pyth_fallbacks"] == ref["fallbacks"] == 20
    assert st["reductions"] == ref["reductions"]
    assert colerr(H, ref["H"]) <= TOL and colerr(Q, ref["Q"]) <= TOL


def test_arnoldi_breakdown_invariant_subspace(ctx):
    torch = torch_cuda()
    lam = np.arange(1.0, 201.0)
    A = sp.diags(lam).tocsr()
    rp = torch.from_numpy(A.indptr.astype(np.int32)).cuda()
    ci = torch.from_numpy(A.indices.astype(np.int32)).cuda()
    va = torch.from_numpy(A.data.astype(np.float64)).cuda()
    r0 = np.zeros(200)
    r0[[4, 50, 120]] = [1.0, -2.0, 0.5]
    Q, H, rc, st = run_arnoldi(ctx, binding.csr_op(rp, ci, va), r0, 10)
    ref = ar.dcgs2_arnoldi(lambda x: A @ x, r0, 10)
    assert rc == binding.BREAKDOWN and st["breakdown_step"] == ref["k"] == 3
    say("breakdown H colerr", colerr(H[:4, :3], ref["H"][:4, :3]))
    assert colerr(H[:4, :3], ref["H"][:4, :3]) <= TOL
    assert colerr(Q[:, :3], ref["Q"][:, :3]) <= TOL
    ritz = np.sort(np.linalg.eigvals(H[:3, :3]).real)
    assert np.allclose(ritz, [5.0, 51.0, 121.0], rtol=1e-12)


def test_arnoldi_nonfinite(ctx):
    prob, r0, _ = synth.arnoldi_cd2d_32()
    r0 = r0.copy()
    r0[7] = np.nan
    _, _, rc, st = run_arnoldi(ctx, binding.stencil_op(prob.grid, prob.D, prob.vel), r0, 5)
    assert rc == binding.NONFINITE and st["breakdown_step"] == 0


def test_arnoldi_deterministic(ctx):
    prob = synth.cd3d(64)
    r0 = synth.uniform_vector(prob.m, 3)
    op = binding.stencil_op(prob.grid, prob.D, prob.vel)
    Q1, H1, _, _ = run_arnoldi(ctx, op, r0, 30)
    Q2, H2, _, _ = run_arnoldi(ctx, op, r0, 30)
    assert np.array_equal(Q1, Q2) and np.array_equal(H1, H2)


def test_arnoldi_full_size_128cube(ctx):
    """The Arnoldi workload at full size: 3-D 128^3 (m = 2,097,152), n = 100 steps."""
    prob, b = synth.gmres_cd3d(128)
    A = ops.convection_diffusion(prob.grid, prob.D, prob.vel)
    n = 100
    say("gpu arnoldi 128^3 n=100")
    Q, H, rc, st = run_arnoldi(ctx, binding.stencil_op(prob.grid, prob.D, prob.vel), b, n)
    assert rc == 0 and st["reductions"] == n + 2
    say("oracle arnoldi 128^3 n=100")
    ref = ar.dcgs2_arnoldi(lambda x: A @ x, b, n)
    dh, dq = colerr(H, ref["H"]), colerr(Q, ref["Q"])
    say("H colerr", dh, "Q colerr", dq)
    assert dh <= TOL and dq <= TOL
    loo = loss_of_orthogonality(Q)
    say("loo", loo)
    assert loo <= 1e-13
    assert representation_error(A, Q, H, n) <= 1e-15


@pytest.mark.parametrize("gmax", [1, 37, 1024])
def test_arnoldi_reduction_grid_parity(ctx, gmax):
    """Arnoldi with 1, 37 and (at this size) 1024 reduction workgroups against the
    oracle: the finishing kernel's fixed-order sums for every grid shape."""
    prob = synth.cd3d(84)                  # m = 592,704: the default sizing reaches 1024
    A = ops.convection_diffusion(prob.grid, prob.D, prob.vel)
    r0 = synth.uniform_vector(prob.m, 5)
    n = 12
    say(f"arnoldi reduction grid gmax={gmax}")
    ctx.set_tuning(binding.TUNE_REDUCE_GRID, gmax)
    try:
        Q, H, rc, st = run_arnoldi(ctx, binding.stencil_op(prob.grid, prob.D, prob.vel), r0, n)
    finally:
        ctx.set_tuning(binding.TUNE_REDUCE_GRID, 0)
    ref = ar.dcgs2_arnoldi(lambda x: A @ x, r0, n)
    assert rc == 0 and st["reductions"] == n + 2
    assert colerr(H, ref["H"]) <= TOL
    assert colerr(Q, ref["Q"]) <= TOL


@pytest.mark.parametrize("grid,vel,bits,ld", [((32, 32), (10.0, 10.0), 64, None),
                                              ((31, 29), (3.0, 40.0), 64, None),
                                              ((40, 33, 17), (10.0, 10.0, 10.0), 64, None),
                                              ((40, 33, 17), (10.0, 10.0, 10.0), 32, None),
                                              ((36, 20), (5.0, 1.0), 64, 777),
                                              ((36, 20), (5.0, 1.0), 32, 780),
                                              ((128, 128, 128), (10.0, 10.0, 10.0), 64, None),
                                              ((128, 128, 128), (10.0, 10.0, 10.0), 32, None)])
def test_matvec_fold_and_update_grid_bitwise(ctx, grid, vel, bits, ld):
    """Launch shapes change no bit: the matvec inside the reduction pass against the
    separate matvec kernel, and update passes over 1, 7, 256 and 65536 slabs, give
    the same Q and H, with an FP64 or FP32 basis and with a padded (odd) leading
    dimension.  With an even m and an even leading dimension the folded pass runs (no
    matvec launches)."""
    torch = torch_cuda()
    op = binding.stencil_op(grid, 1.0, vel)
    m = op.m
    n = 12 if m > 100000 else 30
    r0 = synth.uniform_vector(m, 8)
    runs = {}
    for fold, ugrid in [(1, 0), (0, 0), (1, 1), (1, 7), (0, 256), (1, 65536)]:
        say(f"arnoldi {grid} bits={bits} ld={ld} fold={fold} update_grid={ugrid}")
        ctx.set_tuning(binding.TUNE_MATVEC_FOLD, fold)
        ctx.set_tuning(binding.TUNE_UPDATE_GRID, ugrid)
        try:
            ctx.profile(True)
            ctx.profile_read(reset=True)
            Qd = binding.colmajor_empty(m, n + 1, ld,
                                        dtype=torch.float32 if bits == 32 else None)
            H, rc, st = ctx.arnoldi(op, dev_vector(r0), n, Qd)
            Q = host(Qd)
            prof = ctx.profile_read(reset=True)
            ctx.profile(False)
        finally:
            ctx.set_tuning(binding.TUNE_MATVEC_FOLD, 1)
            ctx.set_tuning(binding.TUNE_UPDATE_GRID, 0)
        assert rc == 0 and st["reductions"] == n + 2
        spmv = prof.get("spmv", {}).get("launches", 0)
        if fold == 1 and m % 2 == 0 and (ld is None or ld % 2 == 0):
            assert spmv == 0
        if fold == 0:
            assert spmv >= n
        runs[(fold, ugrid)] = (Q, H)
    Q0, H0 = runs[(1, 0)]
    for key, (Q, H) in runs.items():
        assert np.array_equal(Q, Q0) and np.array_equal(H, H0), key


def test_arnoldi_longest_basis(ctx):
    """n = DCGS2_MAX_N (1024 steps) on a 48 x 48 grid (m = 2304): orthogonality and the
    Arnoldi relation over the whole basis, and the first 64 columns element-wise
    against the oracle (later columns of so long a Krylov basis are sensitive to
    rounding far beyond the gate, in any two implementations)."""
    grid, vel = (48, 48), (10.0, 10.0)
    A = ops.convection_diffusion(grid, 1.0, vel)
    op = binding.stencil_op(grid, 1.0, vel)
    n = binding.MAX_N
    r0 = synth.normal_vector(A.shape[0], 17)
    say(f"arnoldi longest basis m={A.shape[0]} n={n}")
    Q, H, rc, st = run_arnoldi(ctx, op, r0, n)
    assert rc == 0 and st["reductions"] == n + 2
    ref = ar.dcgs2_arnoldi(lambda x: A @ x, r0, 64)
    assert colerr(H[:65, :64], ref["H"][:65, :64]) <= TOL
    assert colerr(Q[:, :65], ref["Q"][:, :65]) <= TOL
    loo = loss_of_orthogonality(Q)
    rre = representation_error(A, Q, H, n)
    say("loo", loo, "rre", rre)
    assert loo <= 1e-12
    assert rre <= 1e-15
